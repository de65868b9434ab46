// FP64 CPU oracle: pseudopotential multiphase lattice Boltzmann step with the multiphase
// curved wetting boundary of Yao, Liu, Zhong & Wen, "Multiphase curved boundary condition in
// lattice Boltzmann method" (arXiv 2203.04508).
//
// TEST INFRASTRUCTURE ONLY. Tests, the package smoke check and the CPU-baseline leg of the
// benchmark load this library; the HIP product path never does, and the two share no code.
//
// It is written to be read against the paper: doubles, plain loops over nodes and directions,
// each step of the method in its own function, no blocking and no fusion.
//
//   lattice            D2Q9 velocities in the column order of the moment matrix M (Sec. 2.1, eq. 2);
//                      D3Q19 for the 3-D runs (not in the paper; listed below)
//   equilibrium        eq. 14 with c_s^2 = 1/3
//   forcing            exact difference method, eq. 13
//   collision          eq. 4 with S = I/tau (single relaxation time), or in 2-D the paper's
//                      multiple-relaxation-time form: eqs. 1-4 with the moment matrix of eq. 2, the
//                      listed moment equilibria and S of eq. 3; streaming eq. 5
//   body force         optional uniform acceleration g: F = F_nonideal + rho g (the drop-impact
//                      runs of Sec. 4.5 use gravity); it enters eq. 13 and eqs. 16-17 with the rest
//   nonideal force     pseudopotential with an EOS-based effective mass (the model class named in
//                      Sec. 1): psi = sqrt(2 (p_EOS - rho c_s^2) / G), F = -G psi(x) sum_i w^_i psi(x+e_i) e_i,
//                      Carnahan-Starling p_EOS
//   wall density       eq. 15 restricted to the first solid layer, times a wettability factor phi
//   chemical-potential model (2-D, the paper's own, Sec. 2.2-2.3): Peng-Robinson EOS (eq. 10),
//                      mu = k^2 mu_PR(rho) - kappa lap(rho) (eqs. 11-12), F = -rho grad mu + grad rho / 3
//                      (eq. 9) with fourth-order central differences, densities on two solid layers
//                      by eq. 15 and an assigned chemical potential on them (the wettability)
//   curved boundary    eq. 16 (0 <= q < 1/2), eq. 17 (1/2 <= q <= 1)       (Sec. 3.1)
//   mass modification  eq. 18                                              (Sec. 3.2)
//   comparison schemes the paper measures the present one against (Secs. 1, 4): linear
//                      interpolation bounce-back (eqs. 16-17 without the forcing term, no eq. 18),
//                      the same with eq. 18, and halfway bounce-back; all four coincide at q = 1/2
//
// Geometry is exact integer arithmetic in units of 2^-16 lattice spacings: node classification,
// the fluid-solid link list and each link's q = q_fixed / 2^16 (first point of the link segment
// that lies inside or on a shape).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <type_traits>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr int MAXQ = 19;
constexpr int64_t ONE = 65536;  // one lattice spacing in fixed point

struct Lat {
    int dim = 2, Q = 9;
    int e[MAXQ][3] = {};
    double w[MAXQ] = {};    // lattice weights of eq. 14
    double wf[MAXQ] = {};   // interaction-force stencil weights, sum_i wf_i e_i e_i^T = I
    int opp[MAXQ] = {};
};

Lat make_lat(int dim) {
    Lat L;
    L.dim = dim;
    if (dim == 2) {
        // columns of M (eq. 2): rows j_x and j_y give the x and y components of e_i
        static const int E[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                                    {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
        L.Q = 9;
        for (int i = 0; i < 9; ++i) { L.e[i][0] = E[i][0]; L.e[i][1] = E[i][1]; L.e[i][2] = 0; }
    } else {
        // D3Q19: rest, the 6 axis vectors, the 12 edge vectors; opposite pairs sit side by side
        static const int E[19][3] = {{0, 0, 0},
            {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
            {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
            {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
            {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
        L.Q = 19;
        for (int i = 0; i < 19; ++i) for (int k = 0; k < 3; ++k) L.e[i][k] = E[i][k];
    }
    for (int i = 0; i < L.Q; ++i) {
        int n2 = L.e[i][0] * L.e[i][0] + L.e[i][1] * L.e[i][1] + L.e[i][2] * L.e[i][2];
        if (dim == 2) {
            L.w[i] = n2 == 0 ? 4.0 / 9.0 : (n2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
            L.wf[i] = n2 == 0 ? 0.0 : (n2 == 1 ? 1.0 / 3.0 : 1.0 / 12.0);
        } else {
            L.w[i] = n2 == 0 ? 1.0 / 3.0 : (n2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
            L.wf[i] = n2 == 0 ? 0.0 : (n2 == 1 ? 1.0 / 6.0 : 1.0 / 12.0);
        }
        for (int j = 0; j < L.Q; ++j)
            if (L.e[j][0] == -L.e[i][0] && L.e[j][1] == -L.e[i][1] && L.e[j][2] == -L.e[i][2]) L.opp[i] = j;
    }
    return L;
}

}  // namespace

extern "C" {

typedef struct {
    int32_t dim, nx, ny, nz;  // nz = 1 for dim 2
    double tau;               // single relaxation time (S = I/tau in eq. 4)
    double G;                 // interaction strength of the pseudopotential force (negative)
    double eos_a, eos_b, eos_R, eos_T;  // Carnahan-Starling parameters and temperature
} or_params;

}  // extern "C"

namespace {

// ----------------------------------------------------------------------------------------
// dual numbers with K tangent directions (forward-mode reference derivatives)
// ----------------------------------------------------------------------------------------
constexpr int KD = 4;
struct Dual {
    double v = 0;
    double d[KD] = {};
    Dual() = default;
    Dual(double x) : v(x) {}
};
inline Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v); for (int k = 0; k < KD; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v); for (int k = 0; k < KD; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
inline Dual operator-(const Dual& a) { Dual r(-a.v); for (int k = 0; k < KD; ++k) r.d[k] = -a.d[k]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v); for (int k = 0; k < KD; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) { Dual r(a.v / b.v); for (int k = 0; k < KD; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v); return r; }
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(const Dual& a, double b) { Dual r(a.v * b); for (int k = 0; k < KD; ++k) r.d[k] = a.d[k] * b; return r; }
inline Dual operator*(double a, const Dual& b) { return b * a; }
inline Dual operator/(const Dual& a, double b) { Dual r(a.v / b); for (int k = 0; k < KD; ++k) r.d[k] = a.d[k] / b; return r; }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
inline Dual& operator+=(Dual& a, const Dual& b) { a = a + b; return a; }
inline Dual sqrt(const Dual& a) { double s = std::sqrt(a.v); Dual r(s); for (int k = 0; k < KD; ++k) r.d[k] = a.d[k] / (2.0 * s); return r; }
inline Dual log(const Dual& a) { Dual r(std::log(a.v)); for (int k = 0; k < KD; ++k) r.d[k] = a.d[k] / a.v; return r; }
inline Dual tanh(const Dual& a) { double t = std::tanh(a.v); Dual r(t); for (int k = 0; k < KD; ++k) r.d[k] = a.d[k] * (1.0 - t * t); return r; }
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline bool finite(double x) { return std::isfinite(x); }
inline bool finite(const Dual& x) { return std::isfinite(x.v); }

// ----------------------------------------------------------------------------------------
// thermodynamics: Carnahan-Starling EOS and the pseudopotential
// ----------------------------------------------------------------------------------------
template <class R>
R p_eos(const or_params& P, R rho) {
    R eta = rho * (P.eos_b / 4.0);
    R one_m = 1.0 - eta;
    return rho * (P.eos_R * P.eos_T) * (1.0 + eta + eta * eta - eta * eta * eta) / (one_m * one_m * one_m)
           - P.eos_a * rho * rho;
}

// The pressure of the pseudopotential model is rho c_s^2 + G psi^2 / 2 (c = 1); equating it with
// p_EOS fixes psi.  Returns false when rho <= 0 or the square root argument is negative.
template <class R>
bool psi_of(const or_params& P, R rho, R* psi) {
    if (!(val(rho) > 0.0)) { *psi = R(0.0); return false; }
    R arg = 2.0 * (p_eos(P, rho) - rho / 3.0) / P.G;
    if (!(val(arg) >= 0.0)) { *psi = R(0.0); return false; }
    using std::sqrt;
    *psi = sqrt(arg);
    return true;
}

// eq. 14: second-order equilibrium, c_s^2 = 1/3
template <class R>
void equilibrium(const Lat& L, R rho, const R u[3], R out[]) {
    R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < L.Q; ++i) {
        R eu = u[0] * double(L.e[i][0]) + u[1] * double(L.e[i][1]) + u[2] * double(L.e[i][2]);
        out[i] = L.w[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

// ---- Peng-Robinson equation of state and its chemical potential (eqs. 10-11)
struct PR {
    double a = 2.0 / 49.0, b = 2.0 / 21.0, R = 1.0, T = 0.0, omega = 0.344;
    double alpha = 1.0;  // alpha(T), set by pr_set
};

// critical point of eq. 10 (alpha = 1): with x = b rho, dp/drho = 0 gives
//   R T b / a = (1 - x)^2 (2x + 2x^2) / (1 + 2x - x^2)^2,
// and d2p/drho2 = 0 along it reduces to x^3 + x^2 + x - 1/3 = 0, whose real root (Cardano) is
//   x_c = (-1 + cbrt(8 + 6 sqrt 2) + cbrt(8 - 6 sqrt 2)) / 3 = 0.25307...
inline void pr_critical(double a, double b, double R, double* Tc, double* rhoc) {
    const double s2 = std::sqrt(2.0);
    const double x = (-1.0 + std::cbrt(8.0 + 6.0 * s2) + std::cbrt(8.0 - 6.0 * s2)) / 3.0;
    const double d = 1.0 + 2.0 * x - x * x;
    *rhoc = x / b;
    *Tc = (1.0 - x) * (1.0 - x) * (2.0 * x + 2.0 * x * x) / (d * d) * a / (b * R);
}

inline void pr_set(PR& E) {
    double Tc, rc;
    pr_critical(E.a, E.b, E.R, &Tc, &rc);
    const double m = 0.37464 + 1.54226 * E.omega - 0.26992 * E.omega * E.omega;
    const double s = 1.0 + m * (1.0 - std::sqrt(E.T / Tc));
    E.alpha = s * s;
}

inline double pr_p(const PR& E, double r) {  // eq. 10
    const double br = E.b * r;
    return r * E.R * E.T / (1.0 - br) - E.a * E.alpha * r * r / (1.0 + 2.0 * br - br * br);
}

// eq. 11 without the gradient term; false outside 0 < rho < 1/b
template <class R>
inline bool pr_mu(const PR& E, R r, R* mu) {
    using std::log;
    const R br = E.b * r;
    if (!(val(r) > 0.0) || !(val(br) < 1.0)) return false;
    const double s2 = std::sqrt(2.0), aa = E.a * E.alpha;
    *mu = E.R * E.T * log(r / (1.0 - br)) - aa / (2.0 * s2 * E.b) * log((s2 - 1.0 + br) / (s2 + 1.0 - br)) +
          E.R * E.T / (1.0 - br) - aa * r / (1.0 + 2.0 * br - br * br);
    return true;
}

// the chemical-potential model's settings (Sec. 2.2, eq. 12): mesh scaling k, gradient coefficient
struct ChemPot {
    bool on = false;
    PR eos;
    double k = 1.0, kappa = 0.0;
};

// fourth-order central differences along an axis: derivative and second derivative from the values
// at offsets -2 .. +2
template <class R>
inline R d1_4(R m2, R m1, R p1, R p2) { return (8.0 * (p1 - m1) - (p2 - m2)) / 12.0; }
template <class R>
inline R d2_4(R m2, R m1, R c, R p1, R p2) {
    return (16.0 * (p1 + m1) - (p2 + m2) - 30.0 * c) / 12.0;
}

// eq. 2: D2Q9 moment matrix; rows rho, e, epsilon, j_x, q_x, j_y, q_y, p_xx, p_xy, columns the
// velocities in the order of make_lat
const double MRT_M[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

// inverse of an n x n matrix by Gauss-Jordan elimination with partial pivoting
void invert(int n, const double* A, double* Ainv) {
    std::vector<double> a(A, A + n * n), b(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) b[i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r) if (std::fabs(a[r * n + c]) > std::fabs(a[piv * n + c])) piv = r;
        for (int k = 0; k < n; ++k) { std::swap(a[c * n + k], a[piv * n + k]); std::swap(b[c * n + k], b[piv * n + k]); }
        const double d = a[c * n + c];
        for (int k = 0; k < n; ++k) { a[c * n + k] /= d; b[c * n + k] /= d; }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double m = a[r * n + c];
            for (int k = 0; k < n; ++k) { a[r * n + k] -= m * a[c * n + k]; b[r * n + k] -= m * b[c * n + k]; }
        }
    }
    for (int i = 0; i < n * n; ++i) Ainv[i] = b[i];
}

// the multiple-relaxation-time collision of eqs. 1-4 (D2Q9): the relaxation rates of eq. 3 and M^-1
struct Mrt {
    bool on = false;
    double s[9] = {};
    double Minv[9][9] = {};
};

// eq. 1-4 for one node: f~ = f - M^-1 S (m - m_eq) with m = M f and the equilibria of Sec. 2.1
// (q_y^eq read as -j_y, like q_x^eq); the eq. 13 term is added by the caller
template <class R>
void mrt_relax(const Mrt& T, const R f[9], R out[9]) {
    R m[9];
    for (int k = 0; k < 9; ++k) {
        m[k] = 0.0;
        for (int i = 0; i < 9; ++i) m[k] += MRT_M[k][i] * f[i];
    }
    const R rho = m[0], jx = m[3], jy = m[5];
    const R jj = (jx * jx + jy * jy) / rho;
    const R meq[9] = {rho, -2.0 * rho + 3.0 * jj, rho - 3.0 * jj, jx, -jx, jy, -jy,
                      (jx * jx - jy * jy) / rho, jx * jy / rho};
    R d[9];
    for (int k = 0; k < 9; ++k) d[k] = T.s[k] * (m[k] - meq[k]);
    for (int i = 0; i < 9; ++i) {
        R c = 0.0;
        for (int k = 0; k < 9; ++k) c += T.Minv[i][k] * d[k];
        out[i] = f[i] - c;
    }
}

// eq. 13: exact-difference forcing term F_i = f^eq(rho, u + dt F / rho) - f^eq(rho, u), dt = 1
template <class R>
void edm_terms(const Lat& L, R rho, const R u[3], const R F[3], R out[]) {
    R a[MAXQ], b[MAXQ];
    R us[3];
    for (int k = 0; k < 3; ++k) us[k] = u[k] + F[k] / rho;
    equilibrium(L, rho, us, a);
    equilibrium(L, rho, u, b);
    for (int i = 0; i < L.Q; ++i) out[i] = a[i] - b[i];
}

// eqs. 16 and 17 for one link; F_i is the eq. 13 term of direction i at x1 and time t.
// x2_fluid selects the fallback when the second fluid node behind x1 is solid (q < 1/2 only):
// the link is then treated by halfway bounce-back, the q = 1/2 case of the same scheme.
template <class R>
R curved_bc(double q, bool x2_fluid, R ft_i_x1, R ft_i_x2, R ft_ibar_x1, R F_i) {
    if (q < 0.5) {
        if (!x2_fluid) return ft_i_x1;
        return (2.0 * q) * ft_i_x1 + (1.0 - 2.0 * q) * ft_i_x2 + (1.0 - 2.0 * q) * F_i;
    }
    return (1.0 / (2.0 * q)) * ft_i_x1 + ((2.0 * q - 1.0) / (2.0 * q)) * ft_ibar_x1
           + ((2.0 * q - 1.0) / (2.0 * q)) * F_i;
}

// ----------------------------------------------------------------------------------------
// grid helpers
// ----------------------------------------------------------------------------------------
struct Grid {
    int dim, n[3];
    int64_t N;
    explicit Grid(const or_params& P) : dim(P.dim) {
        n[0] = P.nx; n[1] = P.ny; n[2] = dim == 3 ? P.nz : 1;
        N = int64_t(n[0]) * n[1] * n[2];
    }
    int64_t lin(int x, int y, int z) const { return x + int64_t(n[0]) * (y + int64_t(n[1]) * z); }
    void coords(int64_t id, int c[3]) const {
        c[0] = int(id % n[0]); c[1] = int((id / n[0]) % n[1]); c[2] = int(id / (int64_t(n[0]) * n[1]));
    }
    static int wrap(int a, int m) { a %= m; return a < 0 ? a + m : a; }
    int64_t shift(int64_t id, const int d[3], int sign) const {
        int c[3];
        coords(id, c);
        for (int k = 0; k < 3; ++k) c[k] = wrap(c[k] + sign * d[k], n[k]);
        return lin(c[0], c[1], c[2]);
    }
};

// ----------------------------------------------------------------------------------------
// exact geometry in 2^-16 units
// ----------------------------------------------------------------------------------------
enum { SHAPE_BALL = 1, SHAPE_BAND_Y = 2 };
enum { CLS_EQ16 = 0, CLS_HBB = 1, CLS_EQ17 = 2 };
constexpr uint32_t NOHIT = 0xFFFFFFFFu;

struct Shape {
    int64_t kind, c[3], r, lo, hi, group;
};

Shape load_shape(const int64_t* s) {
    Shape h;
    h.kind = s[0]; h.c[0] = s[1]; h.c[1] = s[2]; h.c[2] = s[3]; h.r = s[4]; h.lo = s[5]; h.hi = s[6]; h.group = s[7];
    return h;
}

// periodic minimum image of d on a ring of length Lf: result in [-Lf/2, Lf/2)
int64_t min_image(int64_t d, int64_t Lf) {
    d %= Lf;
    if (d < 0) d += Lf;
    if (d >= Lf / 2) d -= Lf;
    return d;
}

int64_t pmod(int64_t a, int64_t m) { a %= m; return a < 0 ? a + m : a; }

// strict interior test of the lattice node at integer coordinates c
bool node_inside(const Grid& g, const Shape& s, const int c[3]) {
    if (s.kind == SHAPE_BALL) {
        __int128 acc = 0;
        for (int k = 0; k < g.dim; ++k) {
            int64_t d = min_image(int64_t(c[k]) * ONE - s.c[k], int64_t(g.n[k]) * ONE);
            acc += (__int128)d * d;
        }
        return acc < (__int128)s.r * s.r;
    }
    int64_t Ly = int64_t(g.n[1]) * ONE;
    return pmod(int64_t(c[1]) * ONE - s.lo, Ly) < s.hi - s.lo;
}

// First n in [0, 2^16] for which X1 + n e lies inside or on shape s; NOHIT if none.
// For a ball the squared distance along the segment is the convex quadratic
// f(n) = A n^2 + B n + C; its smaller root is estimated in double and then settled by exact
// integer sign tests.
uint32_t first_hit(const Grid& g, const Shape& s, const int c1[3], const int e[3]) {
    if (s.kind == SHAPE_BALL) {
        int64_t d[3] = {0, 0, 0};
        for (int k = 0; k < g.dim; ++k) d[k] = min_image(int64_t(c1[k]) * ONE - s.c[k], int64_t(g.n[k]) * ONE);
        __int128 A = 0, B = 0, C = -(__int128)s.r * s.r;
        for (int k = 0; k < g.dim; ++k) {
            A += e[k] * e[k];
            B += (__int128)2 * d[k] * e[k];
            C += (__int128)d[k] * d[k];
        }
        auto f = [&](int64_t n) { return A * n * n + B * n + C; };
        if (f(0) <= 0) return 0;
        if (B >= 0) return NOHIT;  // f increases on n >= 0
        __int128 disc = B * B - 4 * A * C;
        if (disc < 0) return NOHIT;
        double root = (-double(B) - std::sqrt(double(disc))) / (2.0 * double(A));
        int64_t n = int64_t(std::ceil(root));
        if (n < 0) n = 0;
        while (n > 0 && f(n - 1) <= 0) --n;
        // step forward while still on the decreasing branch and outside
        while (f(n) > 0 && 2 * A * n + B < 0) ++n;
        if (f(n) > 0 || n > ONE) return NOHIT;
        return uint32_t(n);
    }
    // periodic band along y: inside-or-on iff (Y - lo) mod Ly <= hi - lo
    int64_t Ly = int64_t(g.n[1]) * ONE;
    int64_t H = s.hi - s.lo;
    int64_t r = pmod(int64_t(c1[1]) * ONE - s.lo, Ly);
    if (r <= H) return 0;
    int64_t n;
    if (e[1] > 0) n = Ly - r;        // reaches the band's lower face (r wraps to 0)
    else if (e[1] < 0) n = r - H;    // reaches the band's upper face
    else return NOHIT;
    return n <= ONE ? uint32_t(n) : NOHIT;
}

// lattice range of a ball's bounding box, widened by `pad` nodes
void ball_box(const Shape& s, int k, int pad, int* lo, int* hi) {
    int64_t a = s.c[k] - s.r, b = s.c[k] + s.r;
    int64_t fa = a >= 0 ? a / ONE : -((-a + ONE - 1) / ONE);
    int64_t fb = b >= 0 ? b / ONE : -((-b + ONE - 1) / ONE);
    *lo = int(fa) - pad;
    *hi = int(fb) + 1 + pad;
}

// ----------------------------------------------------------------------------------------
// the simulation state
// ----------------------------------------------------------------------------------------
template <class R>
struct Sim {
    or_params P;
    Lat L;
    Grid g;
    std::vector<uint8_t> solid;
    std::vector<int64_t> link0;     // CSR: links of node x are link0[x] .. link0[x+1]-1
    std::vector<int32_t> lk_dir;
    std::vector<uint32_t> lk_q;
    std::vector<int64_t> wall_of;   // wall index of a first-layer solid node, -1 otherwise
    std::vector<int64_t> wall_nodes;
    std::vector<R> phi;             // wettability factor per wall node
    // state at time t
    std::vector<R> ft;    // post-collision populations f~_i(x, t), SoA [Q][N]
    std::vector<R> rho;   // rho(x, t)
    std::vector<R> u;     // u(x, t) = j / rho, [3][N]
    std::vector<R> F;     // nonideal force F(x, t), [3][N]
    // work
    std::vector<R> fn, psi;
    R dm_last = R(0.0);
    int64_t n_domain = 0;
    int bc_mode = 0;  // 0 present scheme, 1 IBC, 2 MIBC, 3 halfway bounce-back
    Mrt mrt;          // multiple-relaxation-time collision (2-D) when mrt.on
    double grav[3] = {0.0, 0.0, 0.0};  // body acceleration
    ChemPot cp;                         // chemical-potential model when cp.on (2-D)
    std::vector<int8_t> layer;          // solid layer of each node: 0 fluid, 1, 2 (eq. 15), 3 deeper
    std::vector<R> mu_s;                // assigned chemical potential per first-layer wall node
    std::vector<R> mu;                  // chemical potential field (fluid nodes and solid layers 1-2)

    explicit Sim(const or_params& p) : P(p), L(make_lat(p.dim)), g(p) {}

    bool fluid(int64_t x) const { return solid[x] == 0; }

    int64_t link_of(int64_t x, int dir) const {
        for (int64_t l = link0[x]; l < link0[x + 1]; ++l) if (lk_dir[l] == dir) return l;
        return -1;
    }

    // S1-S6: from pre-collision populations fpre at time t to the post-collision state
    void collide(const std::vector<R>& fpre) {
        const int64_t N = g.N;
        const int Q = L.Q;
        // S1: density and velocity
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < N; ++x) {
            if (!fluid(x)) continue;
            R r = 0.0, j[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < Q; ++i) {
                r += fpre[i * N + x];
                for (int k = 0; k < 3; ++k) j[k] += fpre[i * N + x] * double(L.e[i][k]);
            }
            rho[x] = r;
            for (int k = 0; k < 3; ++k) u[k * N + x] = j[k] / r;
        }
        if (cp.on) {
            chempot_force();
            collide_with_force(fpre);
            return;
        }
        // S2 + S3: pseudopotential on fluid nodes; wall nodes take psi of their virtual density
        int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
        for (int64_t x = 0; x < N; ++x) {
            if (fluid(x)) {
                if (!psi_of(P, rho[x], &psi[x])) ++bad;
            } else if (wall_of[x] >= 0) {
                // eq. 15, first layer: lattice-weighted mean of the fluid neighbours' density
                R num = 0.0;
                double den = 0.0;
                for (int i = 1; i < Q; ++i) {
                    int64_t y = g.shift(x, L.e[i], +1);
                    if (fluid(y)) { num += L.w[i] * rho[y]; den += L.w[i]; }
                }
                R rho_w = phi[wall_of[x]] * (num / den);
                if (!psi_of(P, rho_w, &psi[x])) ++bad;
            } else {
                psi[x] = 0.0;
            }
        }
        n_domain += bad;
        // S4 - S6: force, exact-difference forcing term, single-relaxation-time collision
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < N; ++x) {
            if (!fluid(x)) continue;
            R s[3] = {0.0, 0.0, 0.0};
            for (int i = 1; i < Q; ++i) {
                int64_t y = g.shift(x, L.e[i], +1);
                for (int k = 0; k < 3; ++k) s[k] += L.wf[i] * psi[y] * double(L.e[i][k]);
            }
            R Fx[3], ux[3];
            for (int k = 0; k < 3; ++k) {
                Fx[k] = -P.G * psi[x] * s[k] + rho[x] * grav[k];
                F[k * N + x] = Fx[k];
                ux[k] = u[k * N + x];
            }
            R feq[MAXQ], Fi[MAXQ];
            edm_terms(L, rho[x], ux, Fx, Fi);
            if (mrt.on) {
                R f[9], o[9];
                for (int i = 0; i < 9; ++i) f[i] = fpre[i * N + x];
                mrt_relax(mrt, f, o);
                for (int i = 0; i < 9; ++i) ft[i * N + x] = o[i] + Fi[i];
                continue;
            }
            equilibrium(L, rho[x], ux, feq);
            for (int i = 0; i < Q; ++i) {
                R f = fpre[i * N + x];
                ft[i * N + x] = f - (f - feq[i]) / P.tau + Fi[i];
            }
        }
    }

    // S5 - S6 with the force F(x, t) already in F: exact-difference forcing term and collision
    void collide_with_force(const std::vector<R>& fpre) {
        const int64_t N = g.N;
        const int Q = L.Q;
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < N; ++x) {
            if (!fluid(x)) continue;
            R Fx[3], ux[3];
            for (int k = 0; k < 3; ++k) { Fx[k] = F[k * N + x]; ux[k] = u[k * N + x]; }
            R feq[MAXQ], Fi[MAXQ];
            edm_terms(L, rho[x], ux, Fx, Fi);
            if (mrt.on) {
                R f[9], o[9];
                for (int i = 0; i < 9; ++i) f[i] = fpre[i * N + x];
                mrt_relax(mrt, f, o);
                for (int i = 0; i < 9; ++i) ft[i * N + x] = o[i] + Fi[i];
                continue;
            }
            equilibrium(L, rho[x], ux, feq);
            for (int i = 0; i < Q; ++i) {
                R f = fpre[i * N + x];
                ft[i * N + x] = f - (f - feq[i]) / P.tau + Fi[i];
            }
        }
    }

    // value of field v at x + m e_k (axis k)
    R at_axis(const std::vector<R>& v, int64_t x, int k, int m) const {
        int d[3] = {0, 0, 0};
        d[k] = m;
        return v[g.shift(x, d, +1)];
    }

    // Secs. 2.2-2.3: densities on the two solid layers (eq. 15), the chemical potential (eq. 12) on
    // fluid nodes and the assigned one on the layers, the nonideal force (eq. 9) with fourth-order
    // central differences, plus the body force
    void chempot_force() {
        const int64_t N = g.N;
        const int Q = L.Q;
        for (int lay = 1; lay <= 2; ++lay) {
#pragma omp parallel for schedule(static)
            for (int64_t x = 0; x < N; ++x) {
                if (layer[x] != lay) continue;
                R num = 0.0;
                double den = 0.0;
                for (int i = 1; i < Q; ++i) {
                    const int64_t y = g.shift(x, L.e[i], +1);
                    if (layer[y] == lay - 1) { num += L.w[i] * rho[y]; den += L.w[i]; }
                }
                rho[x] = num / den;
            }
        }
        const double k2 = cp.k * cp.k;
        int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
        for (int64_t x = 0; x < N; ++x) {
            if (layer[x] == 0) {
                R m0 = 0.0;
                if (!pr_mu(cp.eos, rho[x], &m0)) ++bad;
                R lap = 0.0;
                for (int k = 0; k < g.dim; ++k)
                    lap += d2_4(at_axis(rho, x, k, -2), at_axis(rho, x, k, -1), rho[x], at_axis(rho, x, k, 1), at_axis(rho, x, k, 2));
                mu[x] = k2 * m0 - cp.kappa * lap;
            } else if (layer[x] == 1) {
                mu[x] = mu_s[wall_of[x]];
            } else if (layer[x] == 2) {
                // the assigned potential of the first-layer neighbours, weighted as in eq. 15
                R num = 0.0;
                double den = 0.0;
                for (int i = 1; i < Q; ++i) {
                    const int64_t y = g.shift(x, L.e[i], +1);
                    if (layer[y] == 1) { num += L.w[i] * mu_s[wall_of[y]]; den += L.w[i]; }
                }
                mu[x] = num / den;
            } else {
                mu[x] = 0.0;
            }
        }
        n_domain += bad;
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < N; ++x) {
            if (!fluid(x)) continue;
            for (int k = 0; k < 3; ++k) {
                R Fk = rho[x] * grav[k];
                if (k < g.dim) {
                    const R gm = d1_4(at_axis(mu, x, k, -2), at_axis(mu, x, k, -1), at_axis(mu, x, k, 1), at_axis(mu, x, k, 2));
                    const R gr = d1_4(at_axis(rho, x, k, -2), at_axis(rho, x, k, -1), at_axis(rho, x, k, 1), at_axis(rho, x, k, 2));
                    Fk += -rho[x] * gm + gr / 3.0;
                }
                F[k * N + x] = Fk;
            }
        }
    }

    // eq. 13 term of direction i at node x from the stored moments of time t
    R force_term(int64_t x, int i) const {
        const int64_t N = g.N;
        R ux[3], Fx[3], Fi[MAXQ];
        for (int k = 0; k < 3; ++k) { ux[k] = u[k * N + x]; Fx[k] = F[k * N + x]; }
        edm_terms(L, rho[x], ux, Fx, Fi);
        return Fi[i];
    }

    // S7-S9: streaming (eq. 5), curved boundary (eqs. 16-17), mass modification (eq. 18)
    void stream_and_bounce() {
        const int64_t N = g.N;
        const int Q = L.Q;
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < N; ++x) {
            if (!fluid(x)) continue;
            for (int i = 0; i < Q; ++i) {
                int64_t src = g.shift(x, L.e[i], -1);
                if (fluid(src)) {
                    fn[i * N + x] = ft[i * N + src];
                    continue;
                }
                // the population arriving along e_i left x along e_j (j = opposite of i) and met the wall
                int j = L.opp[i];
                int64_t l = link_of(x, j);
                double q = double(lk_q[l]) / double(ONE);
                int64_t x2 = g.shift(x, L.e[j], -1);
                R ft_j_x2 = fluid(x2) ? ft[j * N + x2] : R(0.0);
                if (bc_mode == 3) {
                    // halfway bounce-back: the wall sits midway whatever q is
                    fn[i * N + x] = ft[j * N + x];
                } else {
                    // IBC and MIBC interpolate without the nonideal-force term
                    const R Fj = bc_mode == 0 ? force_term(x, j) : R(0.0);
                    fn[i * N + x] = curved_bc(q, fluid(x2), ft[j * N + x], ft_j_x2, ft[i * N + x], Fj);
                }
            }
        }
        R total = 0.0;
        if (bc_mode == 1) {  // plain IBC: no mass modification
            dm_last = total;
            return;
        }
        // eq. 18: every boundary-fluid node keeps the outflow-inflow difference of its links in f_0
        for (int64_t x = 0; x < N; ++x) {
            if (!fluid(x) || link0[x] == link0[x + 1]) continue;
            R dm = 0.0;
            for (int64_t l = link0[x]; l < link0[x + 1]; ++l) {
                int j = lk_dir[l];
                dm += ft[j * N + x] - fn[L.opp[j] * N + x];
            }
            fn[x] = fn[x] + dm;
            total += dm;
        }
        dm_last = total;
    }

    void step() {
        stream_and_bounce();
        collide(fn);
    }
};

template <class R>
int build_sim(Sim<R>* S, const uint8_t* solid, const int64_t* lk_node, const int32_t* lk_dir,
              const uint32_t* lk_q, int64_t nlinks) {
    const Grid& g = S->g;
    const Lat& L = S->L;
    const int64_t N = g.N;
    S->solid.assign(solid, solid + N);
    S->link0.assign(N + 1, 0);
    for (int64_t l = 0; l < nlinks; ++l) {
        if (lk_node[l] < 0 || lk_node[l] >= N) return -1;
        if (l > 0 && (lk_node[l] < lk_node[l - 1] || (lk_node[l] == lk_node[l - 1] && lk_dir[l] <= lk_dir[l - 1]))) return -1;
        if (lk_dir[l] < 1 || lk_dir[l] >= L.Q || lk_q[l] > uint32_t(ONE)) return -1;
        S->link0[lk_node[l] + 1]++;
    }
    for (int64_t x = 0; x < N; ++x) S->link0[x + 1] += S->link0[x];
    S->lk_dir.assign(lk_dir, lk_dir + nlinks);
    S->lk_q.assign(lk_q, lk_q + nlinks);
    // every fluid-solid neighbour pair must be a link, and every link such a pair
    int64_t mismatch = 0;
#pragma omp parallel for schedule(static) reduction(+ : mismatch)
    for (int64_t x = 0; x < N; ++x) {
        for (int i = 1; i < L.Q; ++i) {
            bool need = S->fluid(x) && !S->fluid(g.shift(x, L.e[i], +1));
            bool have = S->link_of(x, i) >= 0;
            if (need != have) ++mismatch;
        }
    }
    if (mismatch) return -1;
    // first-layer wall nodes (a fluid neighbour), numbered in ascending linear index
    std::vector<uint8_t> is_wall(N, 0);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        if (S->fluid(x)) continue;
        for (int i = 1; i < L.Q; ++i)
            if (S->fluid(g.shift(x, L.e[i], +1))) { is_wall[x] = 1; break; }
    }
    S->wall_of.assign(N, -1);
    S->wall_nodes.clear();
    for (int64_t x = 0; x < N; ++x)
        if (is_wall[x]) { S->wall_of[x] = int64_t(S->wall_nodes.size()); S->wall_nodes.push_back(x); }
    S->phi.assign(S->wall_nodes.size(), R(1.0));
    // solid layers for eq. 15: 1 = a fluid neighbour, 2 = a layer-1 neighbour, 3 = deeper
    S->layer.assign(N, 0);
    for (int64_t x = 0; x < N; ++x) if (!S->fluid(x)) S->layer[x] = S->wall_of[x] >= 0 ? 1 : 3;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        if (S->layer[x] != 3) continue;
        for (int i = 1; i < L.Q; ++i)
            if (S->layer[g.shift(x, L.e[i], +1)] == 1) { S->layer[x] = 2; break; }
    }
    S->mu_s.assign(S->wall_nodes.size(), R(0.0));
    S->mu.assign(N, R(0.0));
    S->ft.assign(size_t(L.Q) * N, R(0.0));
    S->fn.assign(size_t(L.Q) * N, R(0.0));
    S->rho.assign(N, R(0.0));
    S->psi.assign(N, R(0.0));
    S->u.assign(3 * N, R(0.0));
    S->F.assign(3 * N, R(0.0));
    return 0;
}

// Observables of the differentiation growth, from the stored state f~(x, T) (density
// rho(x) = sum_i f~_i(x, T) over fluid nodes):
//   kind 0  centre of mass in x, sum_x X (rho - rho_v) / sum_x (rho - rho_v), X the node's x index;
//           prm[0] = rho_v
//   kind 1  smooth wetted length, sum over links (x1, j) of |e_j| (1 + tanh((rho(x1) - rho_mid) / delta)) / 2;
//           prm[0] = rho_mid, prm[1] = delta
//   kind 2  total mass, sum_x rho
template <class R>
R loss_of(const Sim<R>& S, int kind, const double* prm) {
    const int64_t N = S.g.N;
    const int Q = S.L.Q;
    R a = 0.0, b = 0.0;
    for (int64_t x = 0; x < N; ++x) {
        if (!S.fluid(x)) continue;
        R r = 0.0;
        for (int i = 0; i < Q; ++i) r = r + S.ft[i * N + x];
        if (kind == 0) {
            const double X = double(x % S.g.n[0]);
            a = a + X * (r - prm[0]);
            b = b + (r - prm[0]);
        } else if (kind == 1) {
            using std::tanh;
            for (int64_t l = S.link0[x]; l < S.link0[x + 1]; ++l) {
                const int* e = S.L.e[S.lk_dir[l]];
                const double len = std::sqrt(double(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]));
                a = a + len * 0.5 * (1.0 + tanh((r - prm[0]) / prm[1]));
            }
        } else {
            a = a + r;
        }
    }
    return kind == 0 ? a / b : a;
}

struct Handle {
    int kind;  // 0 double, 1 dual
    void* sim;
};

}  // namespace

// ========================================================================================
// C entry points (ctypes)
// ========================================================================================
extern "C" {

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

// timing helper: the number of threads later parallel loops use (no effect on the arithmetic,
// which is per node)
void or_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

// ---- lattice and pointwise pieces (used by the pins) ----
int or_lattice(int dim, int32_t* e, double* w, double* wf, int32_t* opp) {
    Lat L = make_lat(dim);
    for (int i = 0; i < L.Q; ++i) {
        for (int k = 0; k < 3; ++k) e[3 * i + k] = L.e[i][k];
        w[i] = L.w[i]; wf[i] = L.wf[i]; opp[i] = L.opp[i];
    }
    return L.Q;
}

void or_equilibrium(int dim, double rho, const double* u, double* out) {
    Lat L = make_lat(dim);
    double uu[3] = {u[0], u[1], dim == 3 ? u[2] : 0.0};
    equilibrium(L, rho, uu, out);
}

void or_edm_terms(int dim, double rho, const double* u, const double* F, double* out) {
    Lat L = make_lat(dim);
    double uu[3] = {u[0], u[1], dim == 3 ? u[2] : 0.0};
    double FF[3] = {F[0], F[1], dim == 3 ? F[2] : 0.0};
    edm_terms(L, rho, uu, FF, out);
}

double or_p_eos(const or_params* P, double rho) { return p_eos(*P, rho); }

double or_psi(const or_params* P, double rho) {
    double s;
    return psi_of(*P, rho, &s) ? s : std::nan("");
}

double or_curved_bc(double q, int x2_fluid, double ft_i_x1, double ft_i_x2, double ft_ibar_x1, double F_i) {
    return curved_bc(q, x2_fluid != 0, ft_i_x1, ft_i_x2, ft_ibar_x1, F_i);
}

// ---- geometry ----
int or_classify(const or_params* P, const int64_t* shapes, int64_t nshape, uint8_t* solid) {
    Grid g(*P);
    std::memset(solid, 0, size_t(g.N));
    for (int64_t s = 0; s < nshape; ++s) {
        Shape h = load_shape(shapes + 8 * s);
        if (h.kind == SHAPE_BALL) {
            if (h.r <= 0) return -1;
            for (int k = 0; k < g.dim; ++k) if (2 * h.r >= int64_t(g.n[k]) * ONE) return -1;
            int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
            for (int k = 0; k < g.dim; ++k) ball_box(h, k, 0, &lo[k], &hi[k]);
            for (int z = lo[2]; z < hi[2]; ++z)
                for (int y = lo[1]; y < hi[1]; ++y)
                    for (int x = lo[0]; x < hi[0]; ++x) {
                        int c[3] = {Grid::wrap(x, g.n[0]), Grid::wrap(y, g.n[1]), g.dim == 3 ? Grid::wrap(z, g.n[2]) : 0};
                        if (node_inside(g, h, c)) solid[g.lin(c[0], c[1], c[2])] = 1;
                    }
        } else if (h.kind == SHAPE_BAND_Y) {
            if (h.hi <= h.lo || h.hi - h.lo >= int64_t(g.n[1]) * ONE) return -1;
            for (int64_t id = 0; id < g.N; ++id) {
                int c[3];
                g.coords(id, c);
                if (node_inside(g, h, c)) solid[id] = 1;
            }
        } else {
            return -1;
        }
    }
    return 0;
}

int64_t or_count_links(const or_params* P, const uint8_t* solid) {
    Grid g(*P);
    Lat L = make_lat(P->dim);
    int64_t n = 0;
    for (int64_t x = 0; x < g.N; ++x) {
        if (solid[x]) continue;
        for (int i = 1; i < L.Q; ++i) if (solid[g.shift(x, L.e[i], +1)]) ++n;
    }
    return n;
}

// Links (x1, i) with x1 fluid and x1 + e_i solid, in (node, direction) order, with
// q_fixed = the first n for which x1 + n e_i / 2^16 is inside or on any shape, and the class
// used by the step: eq. 16 (q < 1/2, x2 = x1 - e_i fluid), halfway bounce-back (q < 1/2, x2 solid)
// or eq. 17 (q >= 1/2).
int or_fill_links(const or_params* P, const int64_t* shapes, int64_t nshape, const uint8_t* solid,
                  int64_t* node, int32_t* dir, int32_t* cls, uint32_t* qfix, int64_t cap) {
    Grid g(*P);
    Lat L = make_lat(P->dim);
    std::vector<int64_t> first(g.N + 1, 0);
    int64_t n = 0;
    for (int64_t x = 0; x < g.N; ++x) {
        first[x] = n;
        if (solid[x]) continue;
        for (int i = 1; i < L.Q; ++i) {
            if (!solid[g.shift(x, L.e[i], +1)]) continue;
            if (n >= cap) return -2;
            node[n] = x; dir[n] = i; qfix[n] = NOHIT;
            ++n;
        }
    }
    first[g.N] = n;
    auto visit = [&](const Shape& h, int64_t x) {
        if (solid[x] || first[x] == first[x + 1]) return;
        int c[3];
        g.coords(x, c);
        for (int64_t l = first[x]; l < first[x + 1]; ++l) {
            uint32_t hit = first_hit(g, h, c, L.e[dir[l]]);
            if (hit < qfix[l]) qfix[l] = hit;
        }
    };
    for (int64_t s = 0; s < nshape; ++s) {
        Shape h = load_shape(shapes + 8 * s);
        if (h.kind == SHAPE_BALL) {
            int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
            for (int k = 0; k < g.dim; ++k) ball_box(h, k, 1, &lo[k], &hi[k]);
            for (int z = lo[2]; z < hi[2]; ++z)
                for (int y = lo[1]; y < hi[1]; ++y)
                    for (int x = lo[0]; x < hi[0]; ++x)
                        visit(h, g.lin(Grid::wrap(x, g.n[0]), Grid::wrap(y, g.n[1]), g.dim == 3 ? Grid::wrap(z, g.n[2]) : 0));
        } else {
            for (int64_t x = 0; x < g.N; ++x) visit(h, x);
        }
    }
    for (int64_t l = 0; l < n; ++l) {
        if (qfix[l] == NOHIT) return -3;  // the solid neighbour lies in no shape: inconsistent input
        if (qfix[l] >= uint32_t(ONE / 2)) cls[l] = CLS_EQ17;
        else cls[l] = solid[g.shift(node[l], L.e[dir[l]], -1)] ? CLS_HBB : CLS_EQ16;
    }
    return 0;
}

int64_t or_wall_nodes(const or_params* P, const uint8_t* solid, int64_t* out, int64_t cap) {
    Grid g(*P);
    Lat L = make_lat(P->dim);
    int64_t n = 0;
    for (int64_t x = 0; x < g.N; ++x) {
        if (!solid[x]) continue;
        for (int i = 1; i < L.Q; ++i)
            if (!solid[g.shift(x, L.e[i], +1)]) {
                if (out && n < cap) out[n] = x;
                ++n;
                break;
            }
    }
    return n;
}

// ---- simulation (double) ----
void* or_sim_create(const or_params* P, const uint8_t* solid, const int64_t* lk_node, const int32_t* lk_dir,
                    const uint32_t* lk_q, int64_t nlinks) {
    if (P->dim != 2 && P->dim != 3) return nullptr;
    if (!(P->tau > 0.5) || !(P->G < 0.0)) return nullptr;
    auto* S = new Sim<double>(*P);
    if (build_sim(S, solid, lk_node, lk_dir, lk_q, nlinks) != 0) { delete S; return nullptr; }
    return S;
}

void or_sim_destroy(void* h) { delete static_cast<Sim<double>*>(h); }

// multiple-relaxation-time collision for later collisions (D2Q9 only): S of eq. 3 with the given
// s_e, s_epsilon, s_q, and s_nu = 1/tau; each rate in (0, 2)
extern "C++" {
template <class R>
static int set_mrt(Sim<R>* S, double se, double seps, double sq) {
    if (S->L.Q != 9) return -1;
    for (double r : {se, seps, sq})
        if (!(r > 0.0 && r < 2.0)) return -1;
    const double snu = 1.0 / S->P.tau;
    const double rates[9] = {1.0, se, seps, 1.0, sq, 1.0, sq, snu, snu};
    for (int k = 0; k < 9; ++k) S->mrt.s[k] = rates[k];
    invert(9, &MRT_M[0][0], &S->mrt.Minv[0][0]);
    S->mrt.on = true;
    return 0;
}
}  // extern "C++"
int or_sim_set_mrt(void* h, double se, double seps, double sq) { return set_mrt(static_cast<Sim<double>*>(h), se, seps, sq); }

// the chemical-potential model (2-D) for later collisions: PR parameters a, b, R, temperature T,
// acentric factor omega, mesh scaling k and gradient coefficient kappa (eqs. 9-12)
extern "C++" {
template <class RR>
static int set_chempot(Sim<RR>* S, double a, double b, double R, double T, double omega, double k, double kappa) {
    if (S->L.dim != 2) return -1;
    if (!(a > 0.0 && b > 0.0 && R > 0.0 && T > 0.0 && k > 0.0 && kappa >= 0.0) || !std::isfinite(omega)) return -1;
    S->cp.eos.a = a;
    S->cp.eos.b = b;
    S->cp.eos.R = R;
    S->cp.eos.T = T;
    S->cp.eos.omega = omega;
    pr_set(S->cp.eos);
    S->cp.k = k;
    S->cp.kappa = kappa;
    S->cp.on = true;
    return 0;
}
}  // extern "C++"
int or_sim_set_chempot(void* h, double a, double b, double R, double T, double omega, double k, double kappa) {
    return set_chempot(static_cast<Sim<double>*>(h), a, b, R, T, omega, k, kappa);
}
int or_dsim_set_chempot(void* h, double a, double b, double R, double T, double omega, double k, double kappa) {
    return set_chempot(static_cast<Sim<Dual>*>(h), a, b, R, T, omega, k, kappa);
}
// assigned wall chemical potentials of the dual-number simulation, with tangents dmu[k * n_wall + w]
int or_dsim_set_mu_wall(void* h, const double* mu_s, const double* dmu) {
    auto* S = static_cast<Sim<Dual>*>(h);
    const size_t nw = S->mu_s.size();
    for (size_t w = 0; w < nw; ++w) {
        if (!std::isfinite(mu_s[w])) return -1;
        Dual v(mu_s[w]);
        if (dmu) for (int k = 0; k < KD; ++k) v.d[k] = dmu[k * nw + w];
        S->mu_s[w] = v;
    }
    return 0;
}

// assigned chemical potential of each first-layer wall node (the wettability, Sec. 2.3)
int or_sim_set_mu_wall(void* h, const double* mu_s) {
    auto* S = static_cast<Sim<double>*>(h);
    for (size_t w = 0; w < S->mu_s.size(); ++w) {
        if (!std::isfinite(mu_s[w])) return -1;
        S->mu_s[w] = mu_s[w];
    }
    return 0;
}

// density and chemical potential of every node as the last collision saw them (fluid nodes and
// the two solid layers; deeper solid nodes 0), chemical-potential model only
int or_sim_cp_fields(void* h, double* rho, double* mu) {
    auto* S = static_cast<Sim<double>*>(h);
    if (!S->cp.on) return -1;
    for (int64_t x = 0; x < S->g.N; ++x) {
        rho[x] = S->layer[x] <= 2 ? S->rho[x] : 0.0;
        mu[x] = S->layer[x] <= 2 ? S->mu[x] : 0.0;
    }
    return 0;
}

// eqs. 10-11 and the critical point of eq. 10, for tests
double or_pr_p(double a, double b, double R, double T, double omega, double rho) {
    PR E;
    E.a = a; E.b = b; E.R = R; E.T = T; E.omega = omega;
    pr_set(E);
    return pr_p(E, rho);
}
double or_pr_mu(double a, double b, double R, double T, double omega, double rho) {
    PR E;
    E.a = a; E.b = b; E.R = R; E.T = T; E.omega = omega;
    pr_set(E);
    double m = std::nan("");
    pr_mu(E, rho, &m);
    return m;
}
void or_pr_critical(double a, double b, double R, double* Tc, double* rhoc) { pr_critical(a, b, R, Tc, rhoc); }

// uniform body acceleration for later collisions (components beyond the lattice's dimension are 0)
extern "C++" {
template <class R>
static int set_gravity(Sim<R>* S, double gx, double gy, double gz) {
    if (!std::isfinite(gx) || !std::isfinite(gy) || !std::isfinite(gz)) return -1;
    if (S->L.dim == 2 && gz != 0.0) return -1;
    S->grav[0] = gx;
    S->grav[1] = gy;
    S->grav[2] = gz;
    return 0;
}
}  // extern "C++"
int or_sim_set_gravity(void* h, double gx, double gy, double gz) { return set_gravity(static_cast<Sim<double>*>(h), gx, gy, gz); }

// boundary scheme of later steps: 0 present (eqs. 16-18), 1 IBC, 2 MIBC, 3 halfway bounce-back
int or_sim_set_bc_mode(void* h, int mode) {
    if (mode < 0 || mode > 3) return -1;
    static_cast<Sim<double>*>(h)->bc_mode = mode;
    return 0;
}

int64_t or_sim_n_wall(void* h) { return int64_t(static_cast<Sim<double>*>(h)->wall_nodes.size()); }

int or_sim_set_phi(void* h, const double* phi) {
    auto* S = static_cast<Sim<double>*>(h);
    for (size_t w = 0; w < S->phi.size(); ++w) {
        if (!(phi[w] > 0.0)) return -1;
        S->phi[w] = phi[w];
    }
    return 0;
}

static int finish(Sim<double>* S) {
    if (S->n_domain) return -4;
    for (int64_t x = 0; x < S->g.N; ++x)
        if (S->fluid(x))
            for (int i = 0; i < S->L.Q; ++i)
                if (!std::isfinite(S->ft[i * S->g.N + x])) return -5;
    return 0;
}

// pre-collision populations f(x, t) (SoA [Q][N]; solid entries ignored) -> post-collision state at t
int or_sim_set_f(void* h, const double* fpre) {
    auto* S = static_cast<Sim<double>*>(h);
    std::vector<double> f(fpre, fpre + size_t(S->L.Q) * S->g.N);
    S->n_domain = 0;
    S->collide(f);
    return finish(S);
}

// f(x, 0) = f^eq(rho0, u0) (eq. 14), then the first collision
int or_sim_init_eq(void* h, const double* rho0, const double* u0) {
    auto* S = static_cast<Sim<double>*>(h);
    const int64_t N = S->g.N;
    std::vector<double> f(size_t(S->L.Q) * N, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        if (!S->fluid(x)) continue;
        double uu[3] = {0, 0, 0}, fe[MAXQ];
        if (u0) for (int k = 0; k < S->g.dim; ++k) uu[k] = u0[k * N + x];
        equilibrium(S->L, rho0[x], uu, fe);
        for (int i = 0; i < S->L.Q; ++i) f[i * N + x] = fe[i];
    }
    S->n_domain = 0;
    S->collide(f);
    return finish(S);
}

int or_sim_step(void* h, int64_t nsteps, double* dm_hist) {
    auto* S = static_cast<Sim<double>*>(h);
    S->n_domain = 0;
    for (int64_t t = 0; t < nsteps; ++t) {
        S->step();
        if (dm_hist) dm_hist[t] = S->dm_last;
        if (S->n_domain) return -4;
    }
    return finish(S);
}

void or_sim_get_f(void* h, double* f) {
    auto* S = static_cast<Sim<double>*>(h);
    std::memcpy(f, S->ft.data(), S->ft.size() * sizeof(double));
}

// rho(x, t) and the physical velocity v = u + F / (2 rho) (Sec. 2.2, after eq. 14), SoA [dim][N];
// F (nullable) receives the nonideal force
void or_sim_moments(void* h, double* rho, double* v, double* F) {
    auto* S = static_cast<Sim<double>*>(h);
    const int64_t N = S->g.N;
    for (int64_t x = 0; x < N; ++x) {
        bool fl = S->fluid(x);
        rho[x] = fl ? S->rho[x] : 0.0;
        for (int k = 0; k < S->g.dim; ++k) {
            v[k * N + x] = fl ? S->u[k * N + x] + S->F[k * N + x] / (2.0 * S->rho[x]) : 0.0;
            if (F) F[k * N + x] = fl ? S->F[k * N + x] : 0.0;
        }
    }
}

// total mass: sum over fluid nodes of the stored populations, with Neumaier's compensated
// summation so that the sum itself is exact to a few ulps at any lattice size
double or_sim_mass(void* h) {
    auto* S = static_cast<Sim<double>*>(h);
    double sum = 0.0, comp = 0.0;
    for (int64_t x = 0; x < S->g.N; ++x) {
        if (!S->fluid(x)) continue;
        for (int i = 0; i < S->L.Q; ++i) {
            const double v = S->ft[i * S->g.N + x];
            const double t = sum + v;
            if (std::fabs(sum) >= std::fabs(v)) comp += (sum - t) + v;
            else comp += (v - t) + sum;
            sum = t;
        }
    }
    return sum + comp;
}

double or_sim_dm_last(void* h) { return static_cast<Sim<double>*>(h)->dm_last; }

int or_sim_loss(void* h, int kind, const double* prm, double* out) {
    if (kind < 0 || kind > 2) return -1;
    *out = loss_of(*static_cast<Sim<double>*>(h), kind, prm);
    return 0;
}

// ---- forward-mode derivatives: dual numbers carrying KD tangent directions ----
// The wettability factors carry the tangents, every step propagates them exactly (to rounding),
// and a loss returns its value and its KD directional derivatives: the reference gradient for
// the hand-written reverse mode, obtained with no transposition at all.
int or_dual_kd(void) { return KD; }

void* or_dsim_create(const or_params* P, const uint8_t* solid, const int64_t* lk_node, const int32_t* lk_dir,
                     const uint32_t* lk_q, int64_t nlinks) {
    if (P->dim != 2 && P->dim != 3) return nullptr;
    if (!(P->tau > 0.5) || !(P->G < 0.0)) return nullptr;
    auto* S = new Sim<Dual>(*P);
    if (build_sim(S, solid, lk_node, lk_dir, lk_q, nlinks) != 0) { delete S; return nullptr; }
    return S;
}

void or_dsim_destroy(void* h) { delete static_cast<Sim<Dual>*>(h); }

// phi[w] with tangents dphi[k * n_wall + w], k < KD (dphi nullable: no tangents)
int or_dsim_set_phi(void* h, const double* phi, const double* dphi) {
    auto* S = static_cast<Sim<Dual>*>(h);
    const size_t nw = S->phi.size();
    for (size_t w = 0; w < nw; ++w) {
        if (!(phi[w] > 0.0)) return -1;
        Dual v(phi[w]);
        if (dphi) for (int k = 0; k < KD; ++k) v.d[k] = dphi[k * nw + w];
        S->phi[w] = v;
    }
    return 0;
}

static int dfinish(Sim<Dual>* S) {
    if (S->n_domain) return -4;
    for (int64_t x = 0; x < S->g.N; ++x)
        if (S->fluid(x))
            for (int i = 0; i < S->L.Q; ++i)
                if (!finite(S->ft[i * S->g.N + x])) return -5;
    return 0;
}

// the collision, body force and boundary scheme of the dual-number simulation (as or_sim_set_*)
int or_dsim_set_mrt(void* h, double se, double seps, double sq) { return set_mrt(static_cast<Sim<Dual>*>(h), se, seps, sq); }
int or_dsim_set_gravity(void* h, double gx, double gy, double gz) {
    return set_gravity(static_cast<Sim<Dual>*>(h), gx, gy, gz);
}
int or_dsim_set_bc_mode(void* h, int mode) {
    if (mode < 0 || mode > 3) return -1;
    static_cast<Sim<Dual>*>(h)->bc_mode = mode;
    return 0;
}

int or_dsim_init_eq(void* h, const double* rho0) {
    auto* S = static_cast<Sim<Dual>*>(h);
    const int64_t N = S->g.N;
    std::vector<Dual> f(size_t(S->L.Q) * N, Dual(0.0));
    for (int64_t x = 0; x < N; ++x) {
        if (!S->fluid(x)) continue;
        Dual uu[3] = {0.0, 0.0, 0.0}, fe[MAXQ];
        equilibrium(S->L, Dual(rho0[x]), uu, fe);
        for (int i = 0; i < S->L.Q; ++i) f[i * N + x] = fe[i];
    }
    S->n_domain = 0;
    S->collide(f);
    return dfinish(S);
}

int or_dsim_step(void* h, int64_t nsteps) {
    auto* S = static_cast<Sim<Dual>*>(h);
    S->n_domain = 0;
    for (int64_t t = 0; t < nsteps; ++t) {
        S->step();
        if (S->n_domain) return -4;
    }
    return dfinish(S);
}

// out[0] = loss value, out[1 + k] = its derivative along tangent k
int or_dsim_loss(void* h, int kind, const double* prm, double* out) {
    if (kind < 0 || kind > 2) return -1;
    Dual L = loss_of(*static_cast<Sim<Dual>*>(h), kind, prm);
    out[0] = L.v;
    for (int k = 0; k < KD; ++k) out[1 + k] = L.d[k];
    return 0;
}

// wall nodes (ascending linear index) and their eq. 15 density rho_ave(s) at time t, before the
// wettability factor
int64_t or_sim_wall_rho(void* h, int64_t* nodes, double* rho_ave) {
    auto* S = static_cast<Sim<double>*>(h);
    const int64_t nw = int64_t(S->wall_nodes.size());
    for (int64_t w = 0; w < nw; ++w) {
        int64_t x = S->wall_nodes[w];
        double num = 0.0, den = 0.0;
        for (int i = 1; i < S->L.Q; ++i) {
            int64_t y = S->g.shift(x, S->L.e[i], +1);
            if (S->fluid(y)) { num += S->L.w[i] * S->rho[y]; den += S->L.w[i]; }
        }
        if (nodes) nodes[w] = x;
        if (rho_ave) rho_ave[w] = num / den;
    }
    return nw;
}

}  // extern "C"
