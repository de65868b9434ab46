// Reverse mode of the step: the hand-written discrete adjoint of the map from the post-collision
// state of time t to that of time t+1, and of the first collision from the equilibrium start.
// Together with checkpointed recomputation of the forward states (api layer) it gives the exact
// gradient (to rounding) of a loss of the final state with respect to the wettability of every wall
// node: the factor phi (pseudopotential model) or the assigned chemical potential (chemical-potential
// model, whose transposes follow the pseudopotential ones below).
//
// State.  The forward step reads, besides the populations g(t), the forcing term F_j(x, t) of
// eq. 13 on every fluid-solid link (eqs. 16-17 use it one step later), so the state is the pair
// (g, R) with R the per-link forcing terms; its adjoint is (lambda, lambda_R).  The step keeps
// the forcing terms of each boundary node in its boundary record (rho and du = F / rho among them);
// the reverse sweep takes F = rho du from the record of each state and recomputes R from F and the
// node's own populations.
//
// Forward step, per fluid node x (f = g + w rho_ref in the shifted storages):
//   streaming, eq. 5:     p_i(x) = f_i(x - e_i)                           (x - e_i fluid)
//   link (x, j), i = opp j: p_i(x) = B_j = c1 f_j(x) + c2 o + c3 R_j(x)     (eqs. 16-17)
//        eq. 16: c1 = 2q, c2 = c3 = 1 - 2q, o = f_j(x - e_j); bounce-back: c1 = 1, c2 = c3 = 0;
//        eq. 17: c1 = 1/(2q), c2 = c3 = 1 - 1/(2q), o = f_opp(j)(x)
//   eq. 18:               p_0(x) += sum_links (f_j(x) - B_j)
//   the comparison schemes weight the forcing term R by kF and the eq. 18 sum by k18 (0 or 1)
//   collision, with E_i(rho, m) = w_i (rho + 3 e_i.m + (4.5 (e_i.m)^2 - 1.5 m.m) / rho), the
//   equilibrium of eq. 14 written with the momentum m = rho u, and K = M^-1 S M (eqs. 1-4; BGK:
//   K = I / tau):
//        g' = (I - K) p + (K - I) E(rho, j) + E(rho, j + F),   R'_i = E_i(rho, j + F) - E_i(rho, j)
//   (the MRT equilibria are M E(rho, j)), rho = sum p, j = sum p e, F = -G psi(x) sum_k w^_k
//   psi(x + e_k) e_k + rho g, psi = psi(rho) on fluid nodes and psi(phi_s rho_ave(s)) on wall
//   nodes s, rho_ave the eq. 15 weighted mean of the fluid neighbours' densities.
// The kernels below apply the transposes of these maps in reverse order; every scatter of the
// forward map becomes a gather, so each output is written by exactly one thread and the result is
// deterministic.
#include "kernels_common.h"

namespace mcb {
namespace {

template <class C>
__device__ inline C wgt(int L, int i) {
    if (L == 0) return i == 0 ? C(4.0 / 9.0) : (i < 5 ? C(1.0 / 9.0) : C(1.0 / 36.0));
    return i == 0 ? C(1.0 / 3.0) : (i < 7 ? C(1.0 / 18.0) : C(1.0 / 36.0));
}
// interaction-force stencil weights, sum_i w^_i e_i e_i^T = I
__device__ inline double wforce(int L, int i) {
    if (L == 0) return i < 5 ? 1.0 / 3.0 : 1.0 / 12.0;
    return i < 7 ? 1.0 / 6.0 : 1.0 / 12.0;
}

// a node's lattice position (32-bit arithmetic: N < 2^31) and its periodic neighbours
struct Pos {
    int x, y, z;
};
__device__ inline Pos pos_of(const GridDev& g, int64_t x) {
    const uint32_t u = uint32_t(x), nx = uint32_t(g.nx), nxy = nx * uint32_t(g.ny);
    const uint32_t z = u / nxy, r = u - z * nxy, y = r / nx;
    return {int(r - y * nx), int(y), int(z)};
}
__device__ inline int64_t nbr_at(const GridDev& g, int L, const Pos& p, int i, int sign) {
    return int64_t(wrap1(p.x + sign * c_ex[L][i], g.nx)) +
           int64_t(g.nx) * (wrap1(p.y + sign * c_ey[L][i], g.ny) + int64_t(g.ny) * wrap1(p.z + sign * c_ez[L][i], g.nz));
}
__device__ inline int64_t nbr(const GridDev& g, int L, int64_t x, int i, int sign) { return nbr_at(g, L, pos_of(g, x), i, sign); }

// opposite direction, a compile-time constant inside unrolled loops (D2Q9 pairs 1-3, 2-4, 5-7, 6-8;
// D3Q19 pairs 2k-1, 2k)
template <int L>
__host__ __device__ constexpr int opp(int i) {
    return L == 0 ? (i == 0 ? 0 : (i < 5 ? (i + 1) % 4 + 1 : (i - 3) % 4 + 5)) : (i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1));
}
static_assert(opp<0>(1) == 3 && opp<0>(2) == 4 && opp<0>(3) == 1 && opp<0>(4) == 2 && opp<0>(5) == 7 &&
                  opp<0>(6) == 8 && opp<0>(7) == 5 && opp<0>(8) == 6 && opp<0>(0) == 0,
              "D2Q9 opposites");
static_assert(opp<1>(1) == 2 && opp<1>(2) == 1 && opp<1>(17) == 18 && opp<1>(18) == 17 && opp<1>(0) == 0,
              "D3Q19 opposites");

struct AdjDev {
    GridDev g;
    int L;                       // 0: D2Q9, 1: D3Q19
    const int32_t* tag;          // node tags (see the step kernels)
    const uint32_t* nmask;       // 3-D link bits
    const int32_t* bn_link0;     // 2-D first link of each boundary node
    const double* phi;           // wettability factor per wall node
    int fs;                      // stride of the boundary records
    double tau, G, RT, a, b4, rho_ref;
    double kF, k18;              // boundary scheme: weights of the forcing term and of eq. 18
    double grav[3];              // body acceleration
    int mrt;                     // 1: K = M^-1 S M with msc[k] = s_k / |row k of M|^2 (D2Q9)
    double msc[9];
    // chemical-potential model (D2Q9): solid layers, eq. 12 and the Peng-Robinson potential
    int cp;
    const int8_t* layer;
    double k2, kappa, pRT, pb, pclog, paal;
};

// D2Q9 moment matrix of eq. 2 (rows rho, e, epsilon, j_x, q_x, j_y, q_y, p_xx, p_xy); its rows are
// orthogonal, so M^-1 = M^T diag(1 / |row k|^2)
__device__ constexpr int kM2[9][9] = {{1, 1, 1, 1, 1, 1, 1, 1, 1},     {-4, -1, -1, -1, -1, 2, 2, 2, 2},
                                      {4, -2, -2, -2, -2, 1, 1, 1, 1},  {0, 1, 0, -1, 0, 1, -1, -1, 1},
                                      {0, -2, 0, 2, 0, 1, -1, -1, 1},   {0, 0, 1, 0, -1, 1, 1, -1, -1},
                                      {0, 0, -2, 0, 2, 1, 1, -1, -1},   {0, 1, -1, 1, -1, 0, 0, 0, 0},
                                      {0, 0, 0, 0, 0, 1, -1, 1, -1}};

// boundary index of a boundary node's tag
__device__ inline int64_t bidx(const AdjDev& A, int tg) { return A.L == 0 ? int64_t(tg >> 8) : int64_t(tg - 1); }

// link bits (bit j-1: x + e_j solid) of a fluid node, and the record slot of its link j
__device__ inline uint32_t link_bits(const AdjDev& A, int64_t x, int tg) {
    if (tg <= 0) return 0u;
    return A.L == 0 ? uint32_t(tg) & 0xFFu : A.nmask[x];
}
__device__ inline int64_t link_slot(const AdjDev& A, int tg, uint32_t mask, int j) {
    (void)mask;
    if (A.L == 0) return int64_t(tg >> 8) * Q2_LINKS + (j - 1);
    return int64_t(tg - 1) * Q3_LINKS + (j - 1);
}

// Carnahan-Starling pressure and its derivative
__device__ inline void p_eos(const AdjDev& A, double rho, double* p, double* dp) {
    const double eta = rho * A.b4, om = 1.0 - eta;
    const double h = 1.0 + eta + eta * eta - eta * eta * eta, dh = 1.0 + 2.0 * eta - 3.0 * eta * eta;
    const double om3 = om * om * om;
    *p = rho * A.RT * h / om3 - A.a * rho * rho;
    *dp = A.RT * (h / om3 + rho * A.b4 * (dh / om3 + 3.0 * h / (om3 * om))) - 2.0 * A.a * rho;
}
// psi(rho) = sqrt(2 (p - rho/3) / G) and d psi / d rho
__device__ inline void psi_d(const AdjDev& A, double rho, double* psi, double* dpsi) {
    double p, dp;
    p_eos(A, rho, &p, &dp);
    const double arg = 2.0 * (p - rho / 3.0) / A.G;
    const double s = arg > 0.0 ? sqrt(arg) : 0.0;
    *psi = s;
    *dpsi = s > 0.0 ? (dp - 1.0 / 3.0) / (A.G * s) : 0.0;
}

template <class S>
__device__ inline double ldf(const S* g, const AdjDev& A, int i, int64_t x) {
    return double(ldp<S, float>(g, i, A.g.N, x)) + wgt<double>(A.L, i) * A.rho_ref;
}
template <>
__device__ inline double ldf<double>(const double* g, const AdjDev& A, int i, int64_t x) {
    return g[i * A.g.N + x] + wgt<double>(A.L, i) * A.rho_ref;
}

// ---- 1: pre-collision populations p and density of time t+1 (recomputed from (g, R) of time t);
// pull = 0: p = f^eq(rho0, 0), the first collision's input.  Q is a template parameter so that
// every direction loop unrolls and the per-node arrays live in registers.
template <class S, class RC, int Q>
__global__ __launch_bounds__(256) void k_recompute(AdjDev A, const S* __restrict__ gt, const RC* __restrict__ la, const RC* __restrict__ Fv,
                            int pull, const double* __restrict__ rho0, double* __restrict__ p, double* __restrict__ rho) {
    constexpr int L = Q == 9 ? 0 : 1;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < A.g.N; x += int64_t(gridDim.x) * blockDim.x) {
        const int tg = A.tag[x];
        if (tg < 0) continue;
        double v[Q];
        if (!pull) {
#pragma unroll
            for (int i = 0; i < Q; ++i) v[i] = wgt<double>(L, i) * rho0[x];
        } else {
            const Pos ps = pos_of(A.g, x);
            double pl[Q];  // the pulled values (the links replace some entries of v below)
#pragma unroll
            for (int i = 0; i < Q; ++i) pl[i] = ldf<S>(gt, A, i, nbr_at(A.g, L, ps, i, -1));
#pragma unroll
            for (int i = 0; i < Q; ++i) v[i] = pl[i];
            const uint32_t m = link_bits(A, x, tg);
            if (m) {
                double fo[Q];  // the node's own populations
#pragma unroll
                for (int i = 0; i < Q; ++i) fo[i] = ldf<S>(gt, A, i, x);
                // forcing terms of time t: rho and rho u + F from the node's own populations
                double r0 = 0.0, m0[3] = {0, 0, 0}, F0[3] = {0, 0, 0};
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    r0 += fo[i];
                    m0[0] += fo[i] * c_ex[L][i];
                    m0[1] += fo[i] * c_ey[L][i];
                    m0[2] += fo[i] * c_ez[L][i];
                }
                const int64_t b = bidx(A, tg);
                // F = rho du from the forcing terms at the head of the boundary record
                for (int k = 0; k < A.g.dim; ++k) F0[k] = double(Fv[b * A.fs]) * double(Fv[b * A.fs + 1 + k]);
                for (int k = 0; k < 3; ++k) m0[k] -= F0[k];
                double dm = 0.0;
#pragma unroll
                for (int j = 1; j < Q; ++j) {
                    if (!((m >> (j - 1)) & 1u)) continue;
                    const int64_t sl = link_slot(A, tg, m, j);
                    const double a = double(la[sl]);
                    // R_j = E_j(rho, m + F) - E_j(rho, m), E the equilibrium in momentum form
                    const double w = wgt<double>(L, j);
                    const double e[3] = {double(c_ex[L][j]), double(c_ey[L][j]), double(c_ez[L][j])};
                    const double m1[3] = {m0[0] + F0[0], m0[1] + F0[1], m0[2] + F0[2]};
                    const double em0 = e[0] * m0[0] + e[1] * m0[1] + e[2] * m0[2];
                    const double em1 = e[0] * m1[0] + e[1] * m1[1] + e[2] * m1[2];
                    const double mm0 = m0[0] * m0[0] + m0[1] * m0[1] + m0[2] * m0[2];
                    const double mm1 = m1[0] * m1[0] + m1[1] * m1[1] + m1[2] * m1[2];
                    const double Fj = w * (3.0 * (em1 - em0) + (4.5 * (em1 * em1 - em0 * em0) - 1.5 * (mm1 - mm0)) / r0);
                    const double fj = fo[j];
                    // x2 = x - e_j: its value is the one pulled into direction j
                    const double o = a < 0.0 ? fo[opp<L>(j)] : (A.tag[nbr_at(A.g, L, ps, j, -1)] >= 0 ? pl[j] : 0.0);
                    const double c1 = fabs(a), c2 = 1.0 - c1;
                    const double B = c1 * fj + c2 * (o + A.kF * Fj);
                    v[opp<L>(j)] = B;
                    dm += fj - B;
                }
                v[0] += A.k18 * dm;
            }
        }
        double r = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            p[i * A.g.N + x] = v[i];
            r += v[i];
        }
        rho[x] = r;
    }
}

// ---- 2: psi, d psi / d rho; wall nodes also keep rho_ave and the weight sum of eq. 15
template <int Q>
__global__ __launch_bounds__(256) void k_psi(AdjDev A, const double* __restrict__ rho, double* __restrict__ psi,
                                             double* __restrict__ dpsi, double* __restrict__ rave, double* __restrict__ den) {
    constexpr int L = Q == 9 ? 0 : 1;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < A.g.N; x += int64_t(gridDim.x) * blockDim.x) {
        const int tg = A.tag[x];
        double s = 0.0, ds = 0.0;
        if (tg >= 0) {
            psi_d(A, rho[x], &s, &ds);
        } else if (tg <= -2) {
            // every neighbour's tag and density at once; the solid ones are dropped by selection
            const Pos ps = pos_of(A.g, x);
            int ty[Q];
            double ry[Q];
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int64_t y = nbr_at(A.g, L, ps, i, +1);
                ty[i] = A.tag[y];
                ry[i] = rho[y];
            }
            double num = 0.0, dn = 0.0;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                num += ty[i] >= 0 ? wgt<double>(L, i) * ry[i] : 0.0;
                dn += ty[i] >= 0 ? wgt<double>(L, i) : 0.0;
            }
            const double ra = num / dn;
            psi_d(A, A.phi[-tg - 2] * ra, &s, &ds);
            rave[x] = ra;
            den[x] = dn;
        }
        psi[x] = s;
        dpsi[x] = ds;
    }
}

// ---- 3: transposed collision.  lam1 = adjoint of g'(t+1), lamR1 = adjoint of R(t+1) (per link
// slot).  Gives pbar = adjoint of p through the direct and (rho, j) dependences, and Fbar.
template <int Q>
__global__ __launch_bounds__(256) void k_collide_T(AdjDev A, const double* __restrict__ p, const double* __restrict__ rho,
                            const double* __restrict__ psi, const double* __restrict__ lam1,
                            const double* __restrict__ lamR1, double* __restrict__ pbar, double* __restrict__ Fbar,
                            double* __restrict__ Fv, const double* __restrict__ Fin) {
    constexpr int L = Q == 9 ? 0 : 1;
    const int64_t N = A.g.N;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < N; x += int64_t(gridDim.x) * blockDim.x) {
        const int tg = A.tag[x];
        if (tg < 0) continue;
        const double r = rho[x];
        double pv[Q], la[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            pv[i] = p[i * N + x];
            la[i] = lam1[i * N + x];
        }
        double j[3] = {0, 0, 0}, S[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            j[0] += pv[i] * c_ex[L][i];
            j[1] += pv[i] * c_ey[L][i];
            j[2] += pv[i] * c_ez[L][i];
        }
        if (!Fin) {
            const Pos ps = pos_of(A.g, x);
            double pn[Q];
#pragma unroll
            for (int k = 1; k < Q; ++k) pn[k] = psi[nbr_at(A.g, L, ps, k, +1)];
#pragma unroll
            for (int k = 1; k < Q; ++k) {
                const double w = wforce(L, k) * pn[k];
                S[0] += w * c_ex[L][k];
                S[1] += w * c_ey[L][k];
                S[2] += w * c_ez[L][k];
            }
        }
        const double gp = Fin ? 0.0 : -A.G * psi[x];
        // chemical-potential model: the whole force (body force included) comes recomputed in Fin
        const double F[3] = {Fin ? Fin[x] : gp * S[0] + r * A.grav[0], Fin ? Fin[N + x] : gp * S[1] + r * A.grav[1],
                             Fin ? Fin[2 * N + x] : gp * S[2] + r * A.grav[2]};
        // lt = (I - K)^T lambda: the adjoint of the direct dependence on p
        double lt[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) lt[i] = la[i];
        bool bgk = true;
        if constexpr (Q == 9) {
            if (A.mrt) {
                bgk = false;
                double mu[9];
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    double v = 0.0;
#pragma unroll
                    for (int i = 0; i < 9; ++i) v += kM2[k][i] * lt[i];
                    mu[k] = A.msc[k] * v;
                }
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    double v = 0.0;
#pragma unroll
                    for (int k = 0; k < 9; ++k) v += kM2[k][i] * mu[k];
                    lt[i] -= v;
                }
            }
        }
        if (bgk) {
#pragma unroll
            for (int i = 0; i < Q; ++i) lt[i] *= 1.0 - 1.0 / A.tau;
        }
        const double m1[3] = {j[0] + F[0], j[1] + F[1], j[2] + F[2]};
        const double mm0 = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
        const double mm1 = m1[0] * m1[0] + m1[1] * m1[1] + m1[2] * m1[2];
        const uint32_t msk = link_bits(A, x, tg);
        double rr[Q];  // adjoint of the forcing term on each link (0 without a link)
        rr[0] = 0.0;
#pragma unroll
        for (int i = 1; i < Q; ++i) rr[i] = ((msk >> (i - 1)) & 1u) ? lamR1[link_slot(A, tg, msk, i)] : 0.0;
        double rb = 0.0, jb[3] = {0, 0, 0}, Fb[3] = {0, 0, 0};
        const double ir = 1.0 / r, ir2 = ir * ir;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double al = la[i] + rr[i];  // on E_i(rho, j + F)
            const double be = -lt[i] - rr[i];  // on E_i(rho, j): (K - I)^T lambda
            const double w = wgt<double>(L, i);
            const double e[3] = {double(c_ex[L][i]), double(c_ey[L][i]), double(c_ez[L][i])};
            const double em0 = e[0] * j[0] + e[1] * j[1] + e[2] * j[2];
            const double em1 = e[0] * m1[0] + e[1] * m1[1] + e[2] * m1[2];
            // d E / d rho and d E / d m at (rho, m)
            rb += al * w * (1.0 - (4.5 * em1 * em1 - 1.5 * mm1) * ir2) + be * w * (1.0 - (4.5 * em0 * em0 - 1.5 * mm0) * ir2);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double d1 = al * w * (3.0 * e[k] + (9.0 * em1 * e[k] - 3.0 * m1[k]) * ir);
                const double d0 = be * w * (3.0 * e[k] + (9.0 * em0 * e[k] - 3.0 * j[k]) * ir);
                jb[k] += d1 + d0;
                Fb[k] += d1;
            }
        }
        // the body force depends on rho: F = ... + rho g
        rb += Fb[0] * A.grav[0] + Fb[1] * A.grav[1] + Fb[2] * A.grav[2];
#pragma unroll
        for (int i = 0; i < Q; ++i)
            pbar[i * N + x] = lt[i] + rb + c_ex[L][i] * jb[0] + c_ey[L][i] * jb[1] + c_ez[L][i] * jb[2];
        for (int k = 0; k < 3; ++k) {
            Fbar[k * N + x] = Fb[k];
            Fv[k * N + x] = F[k];
        }
    }
}

// ---- 4: transposed force stencil and psi.  Fluid y: rbar = psi'(rho) psibar; wall s:
// rho_w-bar = psi'(rho_w) psibar, dphi += rho_w-bar rho_ave, qbar = rho_w-bar phi / den (to be
// spread over the fluid neighbours with their lattice weights).
template <int Q>
__global__ __launch_bounds__(256) void k_psi_T(AdjDev A, const double* __restrict__ psi, const double* __restrict__ dpsi,
                                               const double* __restrict__ rave, const double* __restrict__ den,
                                               const double* __restrict__ Fbar, double* __restrict__ rbar,
                                               double* __restrict__ qbar, double* __restrict__ dphi) {
    constexpr int L = Q == 9 ? 0 : 1;
    const int64_t N = A.g.N;
    for (int64_t y = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; y < N; y += int64_t(gridDim.x) * blockDim.x) {
        const int tg = A.tag[y];
        if (tg == -1) continue;
        const Pos ps = pos_of(A.g, y);
        double pb = 0.0;
        if (tg >= 0) {
            // own force: F(y) = -G psi(y) S(y)
            double pn[Q];
#pragma unroll
            for (int k = 1; k < Q; ++k) pn[k] = psi[nbr_at(A.g, L, ps, k, +1)];
            double S[3] = {0, 0, 0};
#pragma unroll
            for (int k = 1; k < Q; ++k) {
                const double w = wforce(L, k) * pn[k];
                S[0] += w * c_ex[L][k];
                S[1] += w * c_ey[L][k];
                S[2] += w * c_ez[L][k];
            }
            pb += -A.G * (Fbar[y] * S[0] + Fbar[N + y] * S[1] + Fbar[2 * N + y] * S[2]);
        }
        // the fluid neighbours x = y - e_k whose force uses psi(y) = psi(x + e_k): every neighbour's
        // tag, psi and force adjoint at once, the non-fluid ones dropped by selection
        int tx[Q];
        double px[Q], fx[Q][3];
#pragma unroll
        for (int k = 1; k < Q; ++k) {
            const int64_t x = nbr_at(A.g, L, ps, k, -1);
            tx[k] = A.tag[x];
            px[k] = psi[x];
            fx[k][0] = Fbar[x];
            fx[k][1] = Fbar[N + x];
            fx[k][2] = Fbar[2 * N + x];
        }
#pragma unroll
        for (int k = 1; k < Q; ++k) {
            const double fe = fx[k][0] * c_ex[L][k] + fx[k][1] * c_ey[L][k] + fx[k][2] * c_ez[L][k];
            pb += tx[k] >= 0 ? -A.G * px[k] * wforce(L, k) * fe : 0.0;
        }
        if (tg >= 0) {
            rbar[y] = dpsi[y] * pb;
        } else {
            const int w = -tg - 2;
            const double rwb = dpsi[y] * pb;
            dphi[w] += rwb * rave[y];
            qbar[y] = rwb * A.phi[w] / den[y];
        }
    }
}

// ---- chemical-potential model (D2Q9): forward fields of the recomputed state and the transposes of
// the force (eq. 9), the potential (eq. 12 with the Peng-Robinson mu of eq. 11), and the two solid
// layers of eq. 15.  Fourth-order central differences: d/dx v = sum_m c_m v(x + m), m = -2..2,
// c = (1, -8, 0, 8, -1) / 12; d2/dx2 v = sum_m d_m v(x + m), d = (-1, 16, -30, 16, -1) / 12.
__device__ inline double cdc(int m) { return m == -2 ? 1.0 / 12.0 : m == -1 ? -8.0 / 12.0 : m == 1 ? 8.0 / 12.0 : m == 2 ? -1.0 / 12.0 : 0.0; }
__device__ inline double cdd(int m) { return (m == -2 || m == 2) ? -1.0 / 12.0 : (m == -1 || m == 1) ? 16.0 / 12.0 : -30.0 / 12.0; }

// node x + m e_k (k = 0: x axis, 1: y axis), periodic
__device__ inline int64_t axn(const GridDev& g, int64_t x, int k, int m) {
    const int cx = int(x % g.nx), cy = int(x / g.nx);
    return k == 0 ? int64_t(cy) * g.nx + wrap1(cx + m, g.nx) : int64_t(wrap1(cy + m, g.ny)) * g.nx + cx;
}

__global__ void k_cpa_layer(AdjDev A, double* __restrict__ rho, int lay) {
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < A.g.N; x += int64_t(gridDim.x) * blockDim.x) {
        if (A.layer[x] != lay) continue;
        double num = 0.0, den = 0.0;
        for (int i = 1; i < 9; ++i) {
            const int64_t y = nbr(A.g, 0, x, i, +1);
            if (A.layer[y] == lay - 1) {
                num += wgt<double>(0, i) * rho[y];
                den += wgt<double>(0, i);
            }
        }
        rho[x] = num / den;
    }
}

// mu_PR of eq. 11 (without the gradient term) and its derivative
__device__ inline double pr_mu0(const AdjDev& A, double r) {
    const double br = A.pb * r, s2 = 1.4142135623730951;
    return A.pRT * log(r / (1.0 - br)) - A.pclog * log((s2 - 1.0 + br) / (s2 + 1.0 - br)) + A.pRT / (1.0 - br) -
           A.paal * r / (1.0 + 2.0 * br - br * br);
}
__device__ inline double pr_dmu0(const AdjDev& A, double r) {
    const double br = A.pb * r, om = 1.0 - br, D = 1.0 + 2.0 * br - br * br;
    return A.pRT / (r * om) + A.pRT * A.pb / (om * om) - A.paal / D - A.paal * (1.0 + br * br) / (D * D);
}

// the assigned potential of layer-2 node t: eq. 15 mean of its wall-node neighbours' values
__device__ inline double l2_den(const AdjDev& A, int64_t t) {
    double den = 0.0;
    for (int i = 1; i < 9; ++i)
        if (A.layer[nbr(A.g, 0, t, i, +1)] == 1) den += wgt<double>(0, i);
    return den;
}

__global__ void k_cpa_mu(AdjDev A, const double* __restrict__ rho, double* __restrict__ mu) {
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < A.g.N; x += int64_t(gridDim.x) * blockDim.x) {
        const int lay = A.layer[x];
        double m = 0.0;
        if (lay == 0) {
            double lap = 0.0;
            for (int k = 0; k < 2; ++k)
                for (int d = -2; d <= 2; ++d) lap += cdd(d) * rho[axn(A.g, x, k, d)];
            m = A.k2 * pr_mu0(A, rho[x]) - A.kappa * lap;
        } else if (lay == 1) {
            m = A.phi[-A.tag[x] - 2];
        } else if (lay == 2) {
            double num = 0.0;
            for (int i = 1; i < 9; ++i) {
                const int64_t s = nbr(A.g, 0, x, i, +1);
                if (A.layer[s] == 1) num += wgt<double>(0, i) * A.phi[-A.tag[s] - 2];
            }
            m = num / l2_den(A, x);
        }
        mu[x] = m;
    }
}

__global__ void k_cpa_force(AdjDev A, const double* __restrict__ rho, const double* __restrict__ mu, double* __restrict__ F) {
    const int64_t N = A.g.N;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < N; x += int64_t(gridDim.x) * blockDim.x) {
        if (A.layer[x] != 0) continue;
        for (int k = 0; k < 3; ++k) {
            double f = rho[x] * A.grav[k];
            if (k < 2) {
                double gm = 0.0, gr = 0.0;
                for (int d = -2; d <= 2; ++d) {
                    if (d == 0) continue;
                    const int64_t y = axn(A.g, x, k, d);
                    gm += cdc(d) * mu[y];
                    gr += cdc(d) * rho[y];
                }
                f += -rho[x] * gm + gr / 3.0;
            }
            F[k * N + x] = f;
        }
    }
}

// F-bar -> mu-bar and rho-bar on every node of the stencils (fluid and both layers), gathered from
// the fluid nodes x = y - m e_k whose force reads y; the body force's rho dependence is taken by the
// transposed collision
__global__ void k_cpa_force_T(AdjDev A, const double* __restrict__ rho, const double* __restrict__ mu,
                              const double* __restrict__ Fbar, double* __restrict__ mub, double* __restrict__ rhob) {
    const int64_t N = A.g.N;
    for (int64_t y = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; y < N; y += int64_t(gridDim.x) * blockDim.x) {
        double mb = 0.0, rb = 0.0;
        if (A.layer[y] <= 2) {
            for (int k = 0; k < 2; ++k)
                for (int d = -2; d <= 2; ++d) {
                    if (d == 0) continue;
                    const int64_t x = axn(A.g, y, k, -d);
                    if (A.layer[x] != 0) continue;
                    const double fb = Fbar[k * N + x];
                    mb -= fb * rho[x] * cdc(d);
                    rb += fb * cdc(d) / 3.0;
                }
            if (A.layer[y] == 0)
                for (int k = 0; k < 2; ++k) {
                    double gm = 0.0;
                    for (int d = -2; d <= 2; ++d)
                        if (d != 0) gm += cdc(d) * mu[axn(A.g, y, k, d)];
                    rb -= Fbar[k * N + y] * gm;
                }
        }
        mub[y] = mb;
        rhob[y] = rb;
    }
}

// mu-bar -> rho-bar (eq. 12 on fluid nodes: the Peng-Robinson slope and the transposed Laplacian)
// and -> the assigned potentials of the wall nodes (their own mu and the layer-2 means)
__global__ void k_cpa_mu_T(AdjDev A, const double* __restrict__ rho, const double* __restrict__ mub, double* __restrict__ rhob,
                           double* __restrict__ dmus) {
    for (int64_t z = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; z < A.g.N; z += int64_t(gridDim.x) * blockDim.x) {
        const int lay = A.layer[z];
        if (lay > 2) continue;
        double add = 0.0;
        for (int k = 0; k < 2; ++k)
            for (int d = -2; d <= 2; ++d) {
                const int64_t x = axn(A.g, z, k, -d);
                if (A.layer[x] == 0) add -= A.kappa * cdd(d) * mub[x];
            }
        if (lay == 0) add += mub[z] * A.k2 * pr_dmu0(A, rho[z]);
        rhob[z] += add;
        if (lay == 1) {
            double g = mub[z];
            for (int i = 1; i < 9; ++i) {
                const int64_t t = nbr(A.g, 0, z, i, +1);
                if (A.layer[t] == 2) g += mub[t] * wgt<double>(0, i) / l2_den(A, t);
            }
            dmus[-A.tag[z] - 2] += g;
        }
    }
}

// layer 2 -> layer 1 (eq. 15: rho(t) = sum w rho(s) / den over t's wall-node neighbours s)
__global__ void k_cpa_l2_T(AdjDev A, double* __restrict__ rhob) {
    for (int64_t s = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; s < A.g.N; s += int64_t(gridDim.x) * blockDim.x) {
        if (A.layer[s] != 1) continue;
        double add = 0.0;
        for (int i = 1; i < 9; ++i) {
            const int64_t t = nbr(A.g, 0, s, i, +1);
            if (A.layer[t] == 2) add += rhob[t] * wgt<double>(0, i) / l2_den(A, t);
        }
        rhob[s] += add;
    }
}

// hand the fluid rho-bar and the wall nodes' rho-bar / den (layer 1 -> fluid through eq. 15) to the
// transposed density sum
__global__ void k_cpa_prep(AdjDev A, const double* __restrict__ rhob, double* __restrict__ rbar, double* __restrict__ qbar) {
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < A.g.N; x += int64_t(gridDim.x) * blockDim.x) {
        const int lay = A.layer[x];
        rbar[x] = lay == 0 ? rhob[x] : 0.0;
        double q = 0.0;
        if (lay == 1) {
            double den = 0.0;
            for (int i = 1; i < 9; ++i)
                if (A.layer[nbr(A.g, 0, x, i, +1)] == 0) den += wgt<double>(0, i);
            q = rhob[x] / den;
        }
        qbar[x] = q;
    }
}

// ---- 5: density adjoint into pbar (rho = sum_i p_i)
template <int Q>
__global__ __launch_bounds__(256) void k_rho_T(AdjDev A, const double* __restrict__ rbar, const double* __restrict__ qbar,
                                               double* __restrict__ pbar) {
    constexpr int L = Q == 9 ? 0 : 1;
    const int64_t N = A.g.N;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < N; x += int64_t(gridDim.x) * blockDim.x) {
        if (A.tag[x] < 0) continue;
        const Pos ps = pos_of(A.g, x);
        // wall nodes s = x - e_k average rho(x) = rho(s + e_k) with weight w_k: every neighbour's tag
        // and value at once, the other nodes dropped by selection
        int ts[Q];
        double qs[Q];
#pragma unroll
        for (int k = 1; k < Q; ++k) {
            const int64_t s = nbr_at(A.g, L, ps, k, -1);
            ts[k] = A.tag[s];
            qs[k] = qbar[s];
        }
        double rb = rbar[x];
#pragma unroll
        for (int k = 1; k < Q; ++k) rb += ts[k] <= -2 ? wgt<double>(L, k) * qs[k] : 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) pbar[i * N + x] += rb;
    }
}

// ---- 6: transposed streaming, boundary condition and eq. 18: lambda(t) and lambda_R(t).
// With Bbar_j(x) = pbar_opp(j)(x) - pbar_0(x) the adjoint of a boundary value, f_i(y) is used by
//   the pull into p_i(y + e_i) (y + e_i fluid);
//   its own link (y, i): c1 Bbar_i(y) + pbar_0(y) (eq. 18 adds f_i(y) to p_0);
//   eq. 16 of the link (y + e_i, i) as o = f_i(x - e_i): c2 Bbar_i(y + e_i);
//   eq. 17 of the link (y, opp i) as o = f_i(y): c2 Bbar_opp(i)(y);
// and R_j(y) by its own link only: c3 Bbar_j(y).
template <class RC, int Q>
__global__ __launch_bounds__(256) void k_stream_T(AdjDev A, const RC* __restrict__ rec, const double* __restrict__ pbar,
                                                  double* __restrict__ lam0, double* __restrict__ lamR0) {
    // rec: the link coefficients a per slot
    constexpr int L = Q == 9 ? 0 : 1;
    const int64_t N = A.g.N;
    for (int64_t y = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; y < N; y += int64_t(gridDim.x) * blockDim.x) {
        const int tg = A.tag[y];
        if (tg < 0) {
#pragma unroll
            for (int i = 0; i < Q; ++i) lam0[i * N + y] = 0.0;
            continue;
        }
        const uint32_t m = link_bits(A, y, tg);
        const Pos ps = pos_of(A.g, y);
        // the node's own adjoints and, per direction, the neighbour y + e_i's tag and adjoint, all at once
        double pby[Q], pxi[Q];
        int64_t xs[Q];
        int txs[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) pby[i] = pbar[i * N + y];
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            xs[i] = nbr_at(A.g, L, ps, i, +1);
            txs[i] = A.tag[xs[i]];
            pxi[i] = pbar[i * N + xs[i]];
        }
        const double pb0 = pby[0], pz = A.k18 * pb0;  // eq. 18 carries the adjoint of p_0 (if applied)
        lam0[y] = pb0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            double acc;
            if ((m >> (i - 1)) & 1u) {
                const int64_t sl = link_slot(A, tg, m, i);
                const double c1 = fabs(double(rec[sl]));
                const double Bb = pby[opp<L>(i)] - pz;
                acc = c1 * Bb + pz;
                lamR0[sl] = A.kF * (1.0 - c1) * Bb;
            } else {
                acc = pxi[i];
                const uint32_t mx = link_bits(A, xs[i], txs[i]);
                if ((mx >> (i - 1)) & 1u) {
                    const double ax = double(rec[link_slot(A, txs[i], mx, i)]);
                    if (ax > 0.0) acc += (1.0 - ax) * (pbar[opp<L>(i) * N + xs[i]] - A.k18 * pbar[xs[i]]);
                }
            }
            const int io = opp<L>(i);
            if ((m >> (io - 1)) & 1u) {
                const double ao = double(rec[link_slot(A, tg, m, io)]);
                if (ao < 0.0) acc += (1.0 + ao) * (pby[i] - pz);
            }
            lam0[i * N + y] = acc;
        }
    }
}

// ---- loss of the final state: deterministic two-pass reduction, then its gradient
__device__ inline double wave_sum(double v) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

template <class S>
__device__ inline double node_rho(const AdjDev& A, const S* g, int64_t x) {
    double r = 0.0;
    for (int i = 0; i < A.g.Q; ++i) r += ldf<S>(g, A, i, x);
    return r;
}

__device__ inline double link_len(int L, int j) {
    const int n2 = c_ex[L][j] * c_ex[L][j] + c_ey[L][j] * c_ey[L][j] + c_ez[L][j] * c_ez[L][j];
    return n2 == 1 ? 1.0 : (n2 == 2 ? 1.4142135623730951 : 1.7320508075688772);
}

template <class S>
__global__ __launch_bounds__(256) void k_loss_partial(AdjDev A, const S* __restrict__ g, int kind, double p0, double p1,
                                                      double* __restrict__ part) {
    double a = 0.0, b = 0.0;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < A.g.N; x += int64_t(gridDim.x) * blockDim.x) {
        const int tg = A.tag[x];
        if (tg < 0) continue;
        const double r = node_rho<S>(A, g, x);
        if (kind == 0) {
            a += double(x % A.g.nx) * (r - p0);
            b += r - p0;
        } else if (kind == 1) {
            const uint32_t m = link_bits(A, x, tg);
            for (int j = 1; j < A.g.Q; ++j)
                if ((m >> (j - 1)) & 1u) a += link_len(A.L, j) * 0.5 * (1.0 + tanh((r - p0) / p1));
        } else {
            a += r;
        }
    }
    __shared__ double sa[4], sb[4];
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sa[w] = a;
        sb[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[blockIdx.x] = sa[0] + sa[1] + sa[2] + sa[3];
        part[gridDim.x + blockIdx.x] = sb[0] + sb[1] + sb[2] + sb[3];
    }
}

__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double sa[4], sb[4];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        a += part[k];
        b += part[n + k];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sa[w] = a;
        sb[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = sa[0] + sa[1] + sa[2] + sa[3];
        out[1] = sb[0] + sb[1] + sb[2] + sb[3];
    }
}

// lambda(T) = dloss * d loss / d g(T) (every population of a node enters through its density);
// lambda_R(T) = 0.  sums = {a, b} of the reduction (kind 0: loss = a / b).
template <class S>
__global__ void k_loss_grad(AdjDev A, const S* __restrict__ g, int kind, double p0, double p1, const double* __restrict__ sums,
                            double dloss, double* __restrict__ lam) {
    const int64_t N = A.g.N;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < N; x += int64_t(gridDim.x) * blockDim.x) {
        const int tg = A.tag[x];
        double d = 0.0;
        if (tg >= 0) {
            if (kind == 0) {
                d = (double(x % A.g.nx) - sums[0] / sums[1]) / sums[1];
            } else if (kind == 1) {
                const double th = tanh((node_rho<S>(A, g, x) - p0) / p1);
                const uint32_t m = link_bits(A, x, tg);
                for (int j = 1; j < A.g.Q; ++j)
                    if ((m >> (j - 1)) & 1u) d += link_len(A.L, j) * 0.5 * (1.0 - th * th) / p1;
            } else {
                d = 1.0;
            }
        }
        for (int i = 0; i < A.g.Q; ++i) lam[i * N + x] = dloss * d;
    }
}

inline unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    return unsigned(b < 1 ? 1 : b);
}

AdjDev make_dev(const mcb_ctx* c) {
    AdjDev A;
    A.g = c->g;
    A.L = c->g.dim == 2 ? 0 : 1;
    A.tag = reinterpret_cast<const int32_t*>(c->lat + c->L.tag);
    A.nmask = reinterpret_cast<const uint32_t*>(c->lat + c->L.nmask);
    A.bn_link0 = reinterpret_cast<const int32_t*>(c->lk + c->L.bn_link0);
    A.phi = reinterpret_cast<const double*>(c->lk + c->L.wl_phi);
    A.fs = int(c->L.rec_stride);
    A.tau = c->p.tau;
    A.G = c->p.G;
    A.RT = c->p.eos_R * c->p.eos_T;
    A.a = c->p.eos_a;
    A.b4 = c->p.eos_b / 4.0;
    A.rho_ref = c->p.precision == MCB_F64 ? 0.0 : c->p.rho_ref;
    A.kF = c->p.bc_mode == MCB_BC_PRESENT ? 1.0 : 0.0;
    A.k18 = c->p.bc_mode == MCB_BC_IBC ? 0.0 : 1.0;
    for (int k = 0; k < 3; ++k) A.grav[k] = c->p.gravity[k];
    A.mrt = c->p.collision == MCB_COLL_MRT ? 1 : 0;
    const double sn = 1.0 / c->p.tau;
    const double rate[9] = {1.0, c->p.s_e, c->p.s_eps, 1.0, c->p.s_q, 1.0, c->p.s_q, sn, sn};
    const double norm[9] = {9.0, 36.0, 36.0, 6.0, 12.0, 6.0, 12.0, 4.0, 4.0};
    for (int k = 0; k < 9; ++k) A.msc[k] = rate[k] / norm[k];
    A.cp = c->p.model == MCB_MODEL_CHEMPOT ? 1 : 0;
    A.layer = reinterpret_cast<const int8_t*>(c->lat + c->L.cp_layer);
    A.k2 = c->p.cp_k * c->p.cp_k;
    A.kappa = c->p.cp_kappa;
    A.pRT = c->p.eos_R * c->p.eos_T;
    A.pb = c->p.eos_b;
    A.paal = A.cp ? pr_aalpha(c->p.eos_a, c->p.eos_b, c->p.eos_R, c->p.eos_T, c->p.pr_omega) : 0.0;
    A.pclog = A.paal / (2.0 * std::sqrt(2.0) * c->p.eos_b);
    return A;
}

template <class S, class RC>
hipError_t adj_step_t(mcb_ctx* c, const AdjWork& w, const void* gt, const void* fv, int pull, const double* lam1,
                      const double* lamR1, double* lam0, double* lamR0) {
    const AdjDev A = make_dev(c);
    const unsigned G = grid_for(c->g.N);
    const RC* rec = reinterpret_cast<const RC*>(c->lk + c->L.lk_a);
    // boundary records of time t: rho and du = F / rho lead each record
    const RC* Fv = static_cast<const RC*>(fv);
    if (c->g.dim == 2)
        hipLaunchKernelGGL((k_recompute<S, RC, 9>), dim3(G), dim3(256), 0, c->stream, A, static_cast<const S*>(gt), rec, Fv,
                           pull, w.rho0, w.p, w.rho);
    else
        hipLaunchKernelGGL((k_recompute<S, RC, 19>), dim3(G), dim3(256), 0, c->stream, A, static_cast<const S*>(gt), rec, Fv,
                           pull, w.rho0, w.p, w.rho);
    const auto collide_T = c->g.dim == 2 ? k_collide_T<9> : k_collide_T<19>;
    const bool d2 = c->g.dim == 2;
    if (!A.cp)
        hipLaunchKernelGGL(d2 ? k_psi<9> : k_psi<19>, dim3(G), dim3(256), 0, c->stream, A, w.rho, w.psi, w.dpsi, w.rave, w.den);
    if (A.cp) {
        // chemical-potential model: layer densities, mu and F of the recomputed state, then the
        // transposed collision, force, potential and layers (mu in psi, mu-bar in dpsi, rho-bar in rave)
        hipLaunchKernelGGL(k_cpa_layer, dim3(G), dim3(256), 0, c->stream, A, w.rho, 1);
        hipLaunchKernelGGL(k_cpa_layer, dim3(G), dim3(256), 0, c->stream, A, w.rho, 2);
        hipLaunchKernelGGL(k_cpa_mu, dim3(G), dim3(256), 0, c->stream, A, w.rho, w.psi);
        hipLaunchKernelGGL(k_cpa_force, dim3(G), dim3(256), 0, c->stream, A, w.rho, w.psi, w.Fv);
        hipLaunchKernelGGL(collide_T, dim3(G), dim3(256), 0, c->stream, A, w.p, w.rho, w.psi, lam1, lamR1, w.pbar, w.Fbar,
                           w.Fv, w.Fv);
        hipLaunchKernelGGL(k_cpa_force_T, dim3(G), dim3(256), 0, c->stream, A, w.rho, w.psi, w.Fbar, w.dpsi, w.rave);
        hipLaunchKernelGGL(k_cpa_mu_T, dim3(G), dim3(256), 0, c->stream, A, w.rho, w.dpsi, w.rave, w.dphi);
        hipLaunchKernelGGL(k_cpa_l2_T, dim3(G), dim3(256), 0, c->stream, A, w.rave);
        hipLaunchKernelGGL(k_cpa_prep, dim3(G), dim3(256), 0, c->stream, A, w.rave, w.rbar, w.qbar);
    } else {
        hipLaunchKernelGGL(collide_T, dim3(G), dim3(256), 0, c->stream, A, w.p, w.rho, w.psi, lam1, lamR1, w.pbar, w.Fbar, w.Fv,
                           nullptr);
        hipLaunchKernelGGL(d2 ? k_psi_T<9> : k_psi_T<19>, dim3(G), dim3(256), 0, c->stream, A, w.psi, w.dpsi, w.rave, w.den,
                           w.Fbar, w.rbar, w.qbar, w.dphi);
    }
    if (pull) {
        hipLaunchKernelGGL(d2 ? k_rho_T<9> : k_rho_T<19>, dim3(G), dim3(256), 0, c->stream, A, w.rbar, w.qbar, w.pbar);
        const auto stream_T = d2 ? k_stream_T<RC, 9> : k_stream_T<RC, 19>;
        hipLaunchKernelGGL(stream_T, dim3(G), dim3(256), 0, c->stream, A, rec, w.pbar, lam0, lamR0);
    }
    return hipGetLastError();
}

template <class S>
hipError_t adj_loss_t(mcb_ctx* c, const AdjWork& w, const void* g, int kind, const double* prm, double dloss, double* lam) {
    const AdjDev A = make_dev(c);
    hipLaunchKernelGGL((k_loss_partial<S>), dim3(MON_BLOCKS), dim3(256), 0, c->stream, A, static_cast<const S*>(g), kind, prm[0],
                       prm[1], w.part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, c->stream, w.part, MON_BLOCKS, w.sums);
    if (lam)
        hipLaunchKernelGGL((k_loss_grad<S>), dim3(grid_for(c->g.N)), dim3(256), 0, c->stream, A, static_cast<const S*>(g), kind,
                           prm[0], prm[1], w.sums, dloss, lam);
    return hipGetLastError();
}

}  // namespace

hipError_t adj_step(mcb_ctx* c, const AdjWork& w, const void* gt, const void* rec, int pull, const double* lam1,
                    const double* lamR1, double* lam0, double* lamR0) {
    switch (c->p.precision) {
        case MCB_F64: return adj_step_t<double, double>(c, w, gt, rec, pull, lam1, lamR1, lam0, lamR0);
        case MCB_F32S: return adj_step_t<float, float>(c, w, gt, rec, pull, lam1, lamR1, lam0, lamR0);
        default: return adj_step_t<__half, float>(c, w, gt, rec, pull, lam1, lamR1, lam0, lamR0);
    }
}

hipError_t adj_loss(mcb_ctx* c, const AdjWork& w, const void* g, int kind, const double* prm, double dloss, double* lam) {
    switch (c->p.precision) {
        case MCB_F64: return adj_loss_t<double>(c, w, g, kind, prm, dloss, lam);
        case MCB_F32S: return adj_loss_t<float>(c, w, g, kind, prm, dloss, lam);
        default: return adj_loss_t<__half>(c, w, g, kind, prm, dloss, lam);
    }
}

}  // namespace mcb
