// D3Q19 time step in two kernels: pull-streaming (eq. 5), density, the pseudopotential with
// first-layer wall densities (eq. 15), the interaction force, and the single-relaxation-time
// collision with exact-difference forcing (eqs. 4, 13-14), with the curved boundary condition
// (eqs. 16-17) and the mass correction of eq. 18 at boundary-fluid nodes.
//
// Why two kernels.  The force at x needs psi on the 18 neighbours of x, and psi of a wall node needs
// the density of its own fluid neighbours (eq. 15), so a tile that computed densities from its own
// pulls would have to pull a ring two nodes deep around every tile face.  In three dimensions that
// ring costs more than the whole density field: the density pass below pulls every node once and
// writes one value per node, and the collision pass then pulls only the nodes it owns, reading
// the density ring (one value per node) through L2.
//
// Density pass (k_rho3d), one lane per node: rho(x, t+1) = sum of the pulled populations.  At a
// boundary node the populations that eqs. 16-17 supply and the eq. 18 correction cancel in this
// sum -- f_in enters once and is subtracted once from f_0 -- leaving the node's own f~_j(x, t) for
// each link j, while the slot pulled from the solid neighbour holds 0 (solid nodes store zeros).
// So rho = sum of the pulled populations + sum over links of f~_j(x, t), the latter kept in the
// node's boundary record by its collision.  Without eq. 18 (IBC) nothing cancels: the pass forms
// each link's f_in from the record, the link coefficients and the pulled values, as the collision
// pass will, and adds it.  The pass writes rho for fluid nodes, -phi/(weight of the fluid neighbours)
// for wall nodes (the eq. 15 factor; the sign marks the wall) and 0 for the other solid nodes, so
// the collision pass needs no tags for the ring.
//
// Collision pass (k_step3d): a workgroup of 32 x 8 lanes owns a 32 x 8 column tile of the x-y
// plane (whole cache lines of each population row) over a segment of D planes in z, and marches
// along z.  Iteration k writes the density of the 36 x 12 region around the tile for plane
// q = z0 - 2 + k (issued one iteration earlier) into a 3-plane LDS ring, computes psi of the
// 34 x 10 region for plane q - 1 into a second 3-plane ring, and collides plane q - 2 with the
// force from the psi ring.  Each lane pulls only its own node (one plane ahead), applies eqs. 16-18
// from the boundary record in registers, and its collision hands the pulled density back exactly
// (f_0 takes the rounding).
#include "kernels_common.h"

namespace mcb {
namespace {

constexpr int TX = 32, TY = 8, NT = TX * TY;           // lanes (and output columns) of a tile
constexpr int RX = TX + 4, RY = TY + 4, NR = RX * RY;  // density region: two columns out
constexpr int PX = TX + 2, PY = TY + 2, NP = PX * PY;  // psi region: one column out
constexpr int NRL = (NR + NT - 1) / NT, NPL = (NP + NT - 1) / NT;  // region entries per lane

// D3Q19: rest, the six axis vectors, the twelve edge vectors; opposite pairs side by side
__device__ constexpr int kEx3[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ constexpr int kEy3[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int kEz3[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

// D3Q19 weights
template <class C>
__device__ inline C w19(int i) {
    return i == 0 ? C(1.0 / 3.0) : (i < 7 ? C(1.0 / 18.0) : C(1.0 / 36.0));
}

__device__ inline int zinc(int z, int nz) { return z == nz - 1 ? 0 : z + 1; }
__device__ inline int zdec(int z, int nz) { return z == 0 ? nz - 1 : z - 1; }
__device__ inline int wrapn(int a, int n) { return ((a % n) + n) % n; }

// e.(x, y, z) for a lattice vector of components 0 and +-1, folded when the components are
// constants (a product with 0 cannot be dropped under IEEE rules)
template <class C>
__device__ __forceinline__ C edot3(int ex, int ey, int ez, C x, C y, C z) {
    const C tx = ex > 0 ? x : -x, ty = ey > 0 ? y : -y, tz = ez > 0 ? z : -z;
    const C a = ex == 0 ? ty : (ey == 0 ? tx : tx + ty);  // D3Q19: at most two components are set
    return ez == 0 ? a : ((ex == 0 && ey == 0) ? tz : a + tz);
}

// ================================================================ density pass

template <class S, class C>
struct RhoArgs {
    const S* fa;                 // post-collision populations of time t, SoA [19][N]
    const int32_t* tag;          // >0: boundary index + 1; 0 fluid; -1 solid; -2-w wall w
    const C* rin;                // boundary records of time t
    const C* la;                 // link coefficients, Q3_LINKS per boundary node (IBC only)
    const C* fac;                // eq. 15 factor per wall node
    C* rho;                      // out, per node
    int32_t* flags;
    int nx, ny, nz, nbx;
    C rho_ref;
    int ibc;                     // boundary scheme without eq. 18: links' f_in summed explicitly
};

// One lane per node, workgroups of 256 consecutive nodes of an x-row.  PULL = false sums the
// node's own populations (the collision that starts a run).
template <class S, class C, bool PULL>
__global__ __launch_bounds__(256) void k_rho3d(RhoArgs<S, C> a) {
    constexpr uint32_t s = sizeof(S);
    const int bx = int(blockIdx.x) % a.nbx, row = int(blockIdx.x) / a.nbx;
    const int y = row % a.ny, z = row / a.ny;
    const int x = bx * 256 + int(threadIdx.x);
    const bool on = x < a.nx;
    const uint32_t nxy = uint32_t(a.nx) * uint32_t(a.ny), N = nxy * uint32_t(a.nz);
    const __amdgpu_buffer_rsrc_t fa = make_res(a.fa, uint64_t(kMixed<S> ? 20 : 19) * N * s);
    const __amdgpu_buffer_rsrc_t tagr = make_res(a.tag, uint64_t(N) * 4);
    const uint32_t node = uint32_t(z) * nxy + uint32_t(y) * a.nx + uint32_t(x);
    const int tg = ld_i32(tagr, on ? node * 4u : OOB);
    const int xm = x == 0 ? a.nx - 1 : x - 1, xp = x >= a.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? a.ny - 1 : y - 1, yp = y == a.ny - 1 ? 0 : y + 1;
    const int zm = zdec(z, a.nz), zp = zinc(z, a.nz);
    const int xs[3] = {xp, x, xm}, ys[3] = {yp, y, ym}, zs[3] = {zp, z, zm};  // upstream of e = -1, 0, +1
    C fv[19];
    // FP16 storage: the rest population (own node) in FP32, the others from half plane i + 1 on
    if (kMixed<S>) fv[0] = Buf<float>::ld(fa, on ? node * 4u : OOB);
#pragma unroll
    for (int i = kMixed<S> ? 1 : 0; i < 19; ++i) {
        const uint32_t src =
            PULL ? uint32_t(zs[kEz3[i] + 1]) * nxy + uint32_t(ys[kEy3[i] + 1]) * uint32_t(a.nx) + uint32_t(xs[kEx3[i] + 1]) : node;
        fv[i] = Buf<S>::ld(fa, on ? (uint32_t(i + (kMixed<S> ? 1 : 0)) * N + src) * s : OOB);
    }
    C rs = C(0);
#pragma unroll
    for (int i = 0; i < 19; ++i) rs += fv[i];
    if (PULL && on && tg > 0) {
        const C* rec = a.rin + size_t(tg - 1) * REC3;
        if (!a.ibc) {
            // boundary node: its own f~_j(x, t) on each link (the slot pulled from the solid node holds 0)
            rs += rec[RF3 + 18];
        } else {
            // IBC (no forcing term, no eq. 18): the f_in of each link j, which replaces the zero
            // pulled into slot opp(j) -- eq. 16 from the value pulled from x2 into slot j, eq. 17
            // from the node's own opposite population
            const C* ca = a.la + size_t(tg - 1) * Q3_LINKS;
            for (int j = 1; j < 19; ++j) {
                const C c = ca[j - 1];
                if (!(c < C(1.5))) continue;
                const C c1 = c < C(0) ? -c : c, c2 = C(1) - c1;
                const int jo = (j & 1) ? j + 1 : j - 1;
                C o = c < C(0) ? rec[RF3 + jo - 1] : fv[j];
                o = c2 != C(0) ? o : C(0);
                rs += Buf<S>::round(c1 * rec[RF3 + j - 1] + c2 * o);
            }
        }
    }
    if (!on) return;
    C out;
    if (tg >= 0) {
        out = rs + a.rho_ref;
        if (!(out > C(0))) atomicOr(&a.flags[FLAG_DOMAIN], 1);
    } else {
        out = tg == -1 ? C(0) : -a.fac[-tg - 2];
    }
    a.rho[node] = out;
}

// ================================================================ collision pass

template <class S, class C>
struct Args3 {
    const S* fa;                 // post-collision populations of time t, SoA [19][N]
    S* fb;                       // post-collision populations of time t+1
    const int32_t* tag;          // >0: boundary index + 1; 0 fluid; -1 solid; -2-w wall w
    const uint32_t* nmask;       // link bits of each boundary node (bit j-1: x + e_j solid)
    const C* rho;                // density pass output (rho; -eq. 15 factor at wall nodes; 0 solid)
    const C* rin;                // boundary records of time t, REC3 per boundary node
    C* rout;                     // boundary records of time t+1
    const C* la;                 // link coefficients, Q3_LINKS per boundary node (NO_LINK: none)
    int32_t* flags;
    uint32_t n_bnodes;
    int nx, ny, nz, D, ntx, nty, nblocks;
    C tau_inv, G, rho_ref;
    C kF, k18;                   // boundary scheme: weights of the forcing term and of eq. 18
    C gx, gy, gz;                // body acceleration: F = F_nonideal + rho g, so du = F / rho gains g
    Eos<C> eos;
};

// Eqs. 16-18 at a boundary node (bnd) from its record of time t (rec: forcing terms and the
// populations 1..18) and link coefficients (ca): replaces the populations pulled from solid
// neighbours by f_in (see the two-dimensional kernel for the three cases) and corrects the rest
// population; returns the correction and, in res, what rounding f_0 + correction to the compute type
// dropped.  Lanes that are not boundary nodes keep f and return zeros;
// directions in which no lane of the wave has a link are skipped.  LOAD: rec and ca are loaded
// here, from rin at byte offset roff and la at aoff, in two halves, each just before its directions
// (keeps the FP64 kernel within its registers).  kF = 0 drops the forcing term (MIBC); halfway
// bounce-back is a = 1 on every link; k18 = 0 drops eq. 18 (IBC).
template <class S, class C, bool LOAD>
__device__ __forceinline__ C apply_links3(bool bnd, C (&rec)[RF3 + 18], C (&ca)[18], C (&f)[19], __amdgpu_buffer_rsrc_t rin,
                                          uint32_t roff, __amdgpu_buffer_rsrc_t la, uint32_t aoff, C kF, C k18, C& res) {
    constexpr int H1 = RF3 + 8, A1 = 8;  // first half: forcing terms, f~_1..f~_8; directions 1..8
    if (LOAD) {
        C h[H1], g[A1];
        ld_vec(rin, roff, h);
        ld_vec(la, aoff, g);
#pragma unroll
        for (int i = 0; i < H1; ++i) rec[i] = h[i];
#pragma unroll
        for (int i = 0; i < A1; ++i) ca[i] = g[i];
    }
    const C rho = rec[0] * kF, dux = rec[1], duy = rec[2], duz = rec[3];
    const C sx = rec[4], sy = rec[5], sz = rec[6], duu = rec[7];
    // each slot opp(j) is replaced at most once, and never one that a later eq. 16 link reads (its
    // x2 = x - e_j is fluid, while a replaced slot was pulled from a solid node)
    double ds = 0.0;
    auto link = [&](int j) {
        const C a = ca[j - 1];
        const bool lk = bnd && a < C(1.5);
        if (__builtin_amdgcn_ballot_w64(lk)) {
            const C c1 = a < C(0) ? -a : a, c2 = C(1) - c1;
            // eq. 13 term of direction j
            const C ed = edot3<C>(kEx3[j], kEy3[j], kEz3[j], dux, duy, duz);
            const C es = edot3<C>(kEx3[j], kEy3[j], kEz3[j], sx, sy, sz);
            const C Fj = w19<C>(j) * rho * (C(3) * ed + C(4.5) * ed * es - duu);
            const int jo = (j & 1) ? j + 1 : j - 1;  // opposite direction
            C o = a < C(0) ? rec[RF3 + jo - 1] : f[j];
            o = c2 != C(0) ? o : C(0);
            const C fin = Buf<S>::round(c1 * rec[RF3 + j - 1] + c2 * (o + Fj));
            ds += lk ? double(rec[RF3 + j - 1]) - double(fin) : 0.0;
            f[jo] = lk ? fin : f[jo];
        }
    };
#pragma unroll
    for (int j = 1; j <= A1; ++j) link(j);
    if (LOAD) {
        __builtin_amdgcn_sched_barrier(0);
        C h[RF3 + 18 - H1], g[18 - A1];
        ld_vec(rin, roff + uint32_t(H1 * sizeof(C)), h);
        ld_vec(la, aoff + uint32_t(A1 * sizeof(C)), g);
#pragma unroll
        for (int i = 0; i < RF3 + 18 - H1; ++i) rec[H1 + i] = h[i];
#pragma unroll
        for (int i = 0; i < 18 - A1; ++i) ca[A1 + i] = g[i];
    }
#pragma unroll
    for (int j = A1 + 1; j < 19; ++j) link(j);
    ds *= double(k18);
    const double f0 = double(f[0]) + ds;
    f[0] = C(f0);
    res = C(f0 - double(f[0]));
    return C(ds);
}

// Per-workgroup state of the plane march.
template <class S, class C>
struct March3 {
    __amdgpu_buffer_rsrc_t fa, fb, tag, nmask, rho, rin, rout, la;
    int nz;
    uint32_t ns;        // bytes per population array (N nodes)
    uint32_t pb;        // bytes per z-plane of one population array
    uint32_t p4, pc;    // bytes per z-plane of a 4-byte and of a compute-type node array
    uint32_t own4;      // byte offset of this lane's column in a 4-byte node array plane (OOB: none)
    uint32_t vxy[9];    // byte offsets of the columns (x + dx, y + dy), index 3 (dy + 1) + dx + 1
    uint32_t xcol0;     // FP16 storage: byte offset of the column in the FP32 rest-population plane
    uint32_t ro[NRL];   // byte offsets of this lane's density-region columns (OOB: none)
    int pj[NPL];        // LDS index (density region) of this lane's psi-region columns (-1: none)
    bool out_col;
};

// Issue the loads of the nineteen populations arriving at plane z of this lane's column (eq. 5),
// from x - e_i; PULL = false reads the node's own populations.  on = false: loads nothing.
template <class S, class C, bool PULL>
__device__ __forceinline__ void pull_plane(const March3<S, C>& M, int z, bool on, C (&f)[19]) {
    const uint32_t z0b = uint32_t(z) * M.pb;
    const uint32_t zmb = uint32_t(zdec(z, M.nz)) * M.pb;
    const uint32_t zpb = uint32_t(zinc(z, M.nz)) * M.pb;
    const uint32_t zof[3] = {zpb, z0b, zmb};  // upstream plane for e_z = -1, 0, +1
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        if (kMixed<S> && i == 0) {
            // FP16 storage: the rest population (own node) in FP32 at twice the half offsets
            f[0] = Buf<float>::ld(M.fa, on ? M.xcol0 : OOB, z0b * 2u);
            continue;
        }
        const uint32_t vo = on ? (PULL ? M.vxy[(1 - kEy3[i]) * 3 + (1 - kEx3[i])] : M.vxy[4]) : OOB;
        const uint32_t so = uint32_t(i + (kMixed<S> ? 1 : 0)) * M.ns + (PULL ? zof[kEz3[i] + 1] : z0b);
        f[i] = Buf<S>::ld(M.fa, vo, so);
    }
}

// boundary record of time t (the part the pull uses) and link coefficients of a boundary node
// (tg > 0; other lanes get zeros)
template <class S, class C>
__device__ __forceinline__ void ld_rec(const March3<S, C>& M, int tg, C (&rec)[RF3 + 18], C (&ca)[18]) {
    constexpr uint32_t sc = sizeof(C);
    const uint32_t bi = uint32_t(tg - 1);
    ld_vec(M.rin, tg > 0 ? bi * (REC3 * sc) : OOB, rec);
    ld_vec(M.la, tg > 0 ? bi * (Q3_LINKS * sc) : OOB, ca);
}

template <class S, class C, bool PULL, bool PF>
__global__ __launch_bounds__(NT) void k_step3d(Args3<S, C> a) {
    // XCD-aware order: consecutive logical tiles (neighbours in x) go to the same XCD (one L2)
    const int bid = blockIdx.x;
    const int per = a.nblocks >> 3, rem = a.nblocks & 7;
    const int xcd = bid & 7, k8 = bid >> 3;
    const int logical = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k8;
    const int sx = logical % a.ntx, rest = logical / a.ntx;
    const int sy = rest % a.nty, sz = rest / a.nty;
    __shared__ C s_rho[3][NR];
    __shared__ C s_psi[3][NP];
    constexpr uint32_t s = sizeof(S), sc = sizeof(C);

    March3<S, C> M;
    const int t = threadIdx.x;
    const int lx = t % TX, ly = t / TX;
    const int x0 = sx * TX, y0 = sy * TY;
    const int z0 = sz * a.D;
    const int Dv = min(a.D, a.nz - z0);
    M.nz = a.nz;
    const uint32_t nxy = uint32_t(a.nx) * uint32_t(a.ny);
    M.ns = nxy * uint32_t(a.nz) * s;
    M.pb = nxy * s;
    M.p4 = nxy * 4u;
    M.pc = nxy * sc;
    const int cx = x0 + lx, cy = y0 + ly;
    M.out_col = cx < a.nx && cy < a.ny;
    M.own4 = M.out_col ? (uint32_t(cy) * a.nx + cx) * 4u : OOB;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx)
            M.vxy[(dy + 1) * 3 + dx + 1] =
                M.out_col ? (uint32_t(wrap1(cy + dy, a.ny)) * a.nx + wrap1(cx + dx, a.nx)) * s : OOB;
    // density region (RX x RY columns from (x0 - 2, y0 - 2)) and psi region (PX x PY columns from
    // (x0 - 1, y0 - 1)): NRL and NPL entries per lane, periodic
#pragma unroll
    for (int h = 0; h < NRL; ++h) {
        const int r = t + h * NT;
        M.ro[h] = r < NR ? (uint32_t(wrapn(y0 - 2 + r / RX, a.ny)) * a.nx + wrapn(x0 - 2 + r % RX, a.nx)) * sc : OOB;
    }
#pragma unroll
    for (int h = 0; h < NPL; ++h) {
        const int r = t + h * NT;
        M.pj[h] = r < NP ? (r / PX + 1) * RX + (r % PX + 1) : -1;
    }
    const int iters = Dv + 4;
    M.fa = make_res(a.fa, uint64_t(kMixed<S> ? 20 : 19) * M.ns);
    M.fb = make_res(a.fb, uint64_t(kMixed<S> ? 20 : 19) * M.ns);
    M.xcol0 = M.out_col ? (uint32_t(cy) * a.nx + cx) * 4u : OOB;
    M.tag = make_res(a.tag, uint64_t(nxy) * a.nz * 4);
    M.nmask = make_res(a.nmask, uint64_t(nxy) * a.nz * 4);
    M.rho = make_res(a.rho, uint64_t(nxy) * a.nz * sc);
    M.rin = make_res(a.rin, uint64_t(a.n_bnodes) * REC3 * sc);
    M.rout = make_res(a.rout, uint64_t(a.n_bnodes) * REC3 * sc);
    M.la = make_res(a.la, uint64_t(a.n_bnodes) * Q3_LINKS * sc);
    bool bad = false;

    // Iteration k: density of plane q = z0 - 2 + k into the LDS ring, psi of plane q - 1, collision
    // of plane p = q - 2.  Ring slots follow k modulo 3: plane q in slot k % 3.
    int zq = wrapn(z0 - 2, a.nz);            // plane q of the current iteration
    C rr[NRL];                               // density region of plane q (in flight)
#pragma unroll
    for (int h = 0; h < NRL; ++h) rr[h] = Buf<C>::ld(M.rho, M.ro[h], uint32_t(zq) * M.pc);
    C fC[19], fN[19];                        // populations of planes p (arrived) and p + 1 (in flight)
#pragma unroll
    for (int i = 0; i < 19; ++i) fC[i] = fN[i] = C(0);
    C recC[RF3 + 18], aC[18], recN[RF3 + 18], aN[18];
#pragma unroll
    for (int i = 0; i < RF3 + 18; ++i) recC[i] = recN[i] = C(0);
#pragma unroll
    for (int i = 0; i < 18; ++i) aC[i] = aN[i] = C(0);
    int tgC = -1, tgN = -1;                  // tags of planes p and p + 1
    uint32_t mkC = 0, mkN = 0;               // link bits of planes p and p + 1 (boundary nodes)
    for (int k = 0; k < iters; ++k) {
        const int s0 = k % 3, s1 = (k + 2) % 3, s2 = (k + 1) % 3;  // slots of planes q, q - 1, q - 2
        const int zq1 = zinc(zq, a.nz), zqm = zdec(zq, a.nz);
        // ---- density of plane q to LDS; issue the density region of plane q + 1, the populations
        // of plane p + 1 = q - 1 and the tag of plane p + 2 = q
#pragma unroll
        for (int h = 0; h < NRL; ++h)
            if (M.ro[h] != OOB) s_rho[s0][t + h * NT] = rr[h];
#pragma unroll
        for (int h = 0; h < NRL; ++h) rr[h] = Buf<C>::ld(M.rho, k + 1 < iters ? M.ro[h] : OOB, uint32_t(zq1) * M.pc);
        pull_plane<S, C, PULL>(M, zqm, k >= 3 && k < Dv + 3, fN);
        const int tgNN = ld_i32(M.tag, k >= 2 && k < Dv + 2 ? M.own4 : OOB, uint32_t(zq) * M.p4);
        __syncthreads();
        // ---- psi of plane q - 1 (wall nodes: eq. 15, the negated value holding the factor; other
        // solid nodes 0)
        if (k >= 2) {
#pragma unroll
            for (int h = 0; h < NPL; ++h) {
                const int c = M.pj[h];
                if (c >= 0) {
                    const C rc = s_rho[s1][c];
                    C rn = rc;
                    if (rc < C(0)) {
                        C num = C(0);
                        const int pl[3] = {s2, s1, s0};
#pragma unroll
                        for (int i = 1; i < 19; ++i) {
                            const C w = i < 7 ? C(1.0 / 18.0) : C(1.0 / 36.0);
                            const C v = s_rho[pl[kEz3[i] + 1]][c + kEx3[i] + RX * kEy3[i]];
                            num += w * (v > C(0) ? v : C(0));
                        }
                        rn = -rc * num;
                    }
                    s_psi[s1][t + h * NT] = rc == C(0) ? C(0) : psi_val(rn, a.eos, &bad);
                }
            }
        }
        __syncthreads();
        // ---- collision of plane p = q - 2
        if (k >= 4) {
            const bool coll = M.out_col && tgC >= 0;
            C dsC = C(0);
            C erC = C(0);
            if (PULL && __any(tgC > 0)) {
                // without the prefetch (FP64) the record and the coefficients are loaded here
                const uint32_t bi = uint32_t(tgC - 1);
                dsC = apply_links3<S, C, !PF>(tgC > 0, recC, aC, fC, M.rin, tgC > 0 ? bi * (REC3 * sc) : OOB, M.la,
                                              tgC > 0 ? bi * (Q3_LINKS * sc) : OOB, a.kF, a.k18, erC);
            }
            C out[19];
            C rho = C(0), dux = C(0), duy = C(0), duz = C(0), sx2 = C(0), sy2 = C(0), sz2 = C(0), duu15 = C(0);
#pragma unroll
            for (int i = 0; i < 19; ++i) out[i] = C(0);
            if (__any(coll)) {
                // the node's density at t+1 from its pulled values; the collision hands all of it
                // back, with f_0 taking the rounding
                MassAcc<S, C> rs_acc = MassAcc<S, C>(erC);  // what rounding kept out of f_0 (apply_links3)
#pragma unroll
                for (int i = 0; i < 19; ++i) rs_acc += MassAcc<S, C>(fC[i]);
                const C rs = C(rs_acc);
                const int pc = (ly + 1) * PX + (lx + 1);
                auto P = [&](int dx, int dy, int dz) {
                    const int sp = dz < 0 ? s0 : (dz > 0 ? s1 : s2);  // planes p - 1, p + 1, p
                    return s_psi[sp][pc + dx + PX * dy];
                };
                // F = -G psi(x) sum_i w^_i psi(x + e_i) e_i, w^ = 1/6 (axes), 1/12 (edges)
                const C gp = -a.G * P(0, 0, 0);
                const C exy1 = P(1, 1, 0) - P(-1, -1, 0), exy2 = P(1, -1, 0) - P(-1, 1, 0);
                const C exz1 = P(1, 0, 1) - P(-1, 0, -1), exz2 = P(1, 0, -1) - P(-1, 0, 1);
                const C eyz1 = P(0, 1, 1) - P(0, -1, -1), eyz2 = P(0, 1, -1) - P(0, -1, 1);
                const C Fx = gp * (C(1.0 / 6.0) * (P(1, 0, 0) - P(-1, 0, 0)) + C(1.0 / 12.0) * (exy1 + exy2 + exz1 + exz2));
                const C Fy = gp * (C(1.0 / 6.0) * (P(0, 1, 0) - P(0, -1, 0)) + C(1.0 / 12.0) * (exy1 - exy2 + eyz1 + eyz2));
                const C Fz = gp * (C(1.0 / 6.0) * (P(0, 0, 1) - P(0, 0, -1)) + C(1.0 / 12.0) * (exz1 - exz2 + eyz1 - eyz2));

                rho = rs + a.rho_ref;
                const C irho = rcp(coll ? rho : C(1));
                const C jx = (fC[1] - fC[2]) + (fC[7] - fC[8]) + (fC[9] - fC[10]) + (fC[11] - fC[12]) + (fC[13] - fC[14]);
                const C jy = (fC[3] - fC[4]) + (fC[7] - fC[8]) - (fC[9] - fC[10]) + (fC[15] - fC[16]) + (fC[17] - fC[18]);
                const C jz = (fC[5] - fC[6]) + (fC[11] - fC[12]) - (fC[13] - fC[14]) + (fC[15] - fC[16]) - (fC[17] - fC[18]);
                const C ux = jx * irho, uy = jy * irho, uz = jz * irho;
                dux = Fx * irho + a.gx;
                duy = Fy * irho + a.gy;
                duz = Fz * irho + a.gz;
                const C ti = a.tau_inv, omc = C(1) - ti;
                // per direction: out_i = f_i (1 - 1/tau) + w_i [rs/tau + rho (sym_i +- anti_i)] with
                //   sym  = (4.5 (e.u)^2 - 1.5 u^2) / tau + 4.5 (e.du)(e.(2u + du)) - 1.5 du.(2u + du)
                //   anti = 3 (e.u / tau + e.du)
                // (eq. 14 equilibrium, eq. 13 forcing term, eq. 4 with S = I / tau)
                const C uu15 = C(1.5) * (ux * ux + uy * uy + uz * uz);
                sx2 = C(2) * ux + dux;
                sy2 = C(2) * uy + duy;
                sz2 = C(2) * uz + duz;
                duu15 = C(1.5) * (dux * sx2 + duy * sy2 + duz * sz2);
                const C c0 = -(ti * uu15 + duu15);
                const C trs = ti * rs;
                auto pair = [&](int ip, int im, C w, C eu, C ed, C es) {
                    const C sym = ti * C(4.5) * eu * eu + C(4.5) * ed * es + c0;
                    const C anti = C(3) * (ti * eu + ed);
                    const C base = w * (trs + rho * sym);
                    const C wra = w * rho * anti;
                    out[ip] = fC[ip] * omc + base + wra;
                    out[im] = fC[im] * omc + base - wra;
                };
                constexpr C wa = C(1.0 / 18.0), we = C(1.0 / 36.0);
                pair(1, 2, wa, ux, dux, sx2);
                pair(3, 4, wa, uy, duy, sy2);
                pair(5, 6, wa, uz, duz, sz2);
                pair(7, 8, we, ux + uy, dux + duy, sx2 + sy2);
                pair(9, 10, we, ux - uy, dux - duy, sx2 - sy2);
                pair(11, 12, we, ux + uz, dux + duz, sx2 + sz2);
                pair(13, 14, we, ux - uz, dux - duz, sx2 - sz2);
                pair(15, 16, we, uy + uz, duy + duz, sy2 + sz2);
                pair(17, 18, we, uy - uz, duy - duz, sy2 - sz2);
                // the collision conserves mass: f_0 is the density minus the other outputs as stored
                MassAcc<S, C> rest = 0;
#pragma unroll
                for (int i = 1; i < 19; ++i) {
                    out[i] = Buf<S>::round(out[i]);
                    rest += MassAcc<S, C>(out[i]);
                }
                out[0] = C(rs_acc - rest);
            }
            // Every output column stores, solid nodes included (zeros: the density pass and the
            // links read 0 from them), so rows are written whole.
            const uint32_t xst = M.out_col ? uint32_t(zdec(zqm, a.nz)) * M.pb + M.vxy[4] : OOB;
#pragma unroll
            for (int i = 0; i < 19; ++i) {
                if (kMixed<S> && i == 0)
                    Buf<float>::st_nt(M.fb, xst == OOB ? OOB : xst * 2u, coll ? out[0] : C(0));
                else
                    Buf<S>::st_nt(M.fb, sat_add(xst, uint32_t(i + (kMixed<S> ? 1 : 0)) * M.ns), coll ? out[i] : C(0));
            }
            // boundary record of time t+1: the forcing terms, the populations as stored, the eq. 18
            // correction
            if (__any(coll && tgC > 0)) {
                C rv[REC3];
                rv[0] = rho;
                rv[1] = dux;
                rv[2] = duy;
                rv[3] = duz;
                rv[4] = sx2;
                rv[5] = sy2;
                rv[6] = sz2;
                rv[7] = duu15;
#pragma unroll
                for (int i = 1; i < 19; ++i) rv[RF3 + i - 1] = out[i];  // rounded to the storage format above
                // the node's own populations on its links, for the density pass of the next step
                C sl = C(0);
#pragma unroll
                for (int j = 1; j < 19; ++j) sl += ((mkC >> (j - 1)) & 1u) ? out[j] : C(0);
                rv[RF3 + 18] = sl;
                rv[RF3 + 19] = dsC;
                st_vec(M.rout, (coll && tgC > 0) ? uint32_t(tgC - 1) * (REC3 * sc) : OOB, rv);
            }
        }
        // ---- boundary record and link coefficients of plane p + 1 (PF), issued once those of plane
        // p are used up, only by waves that hold a boundary node in it
        if (PF && PULL && __any(tgN > 0)) ld_rec(M, tgN, recN, aN);
        if (__any(tgN > 0)) mkN = uint32_t(ld_i32(M.nmask, tgN > 0 ? M.own4 : OOB, uint32_t(zqm) * M.p4));
        // plane p + 1 becomes plane p
#pragma unroll
        for (int i = 0; i < 19; ++i) fC[i] = fN[i];
        if (PF) {
#pragma unroll
            for (int i = 0; i < RF3 + 18; ++i) recC[i] = recN[i];
#pragma unroll
            for (int i = 0; i < 18; ++i) aC[i] = aN[i];
        }
        tgC = tgN;
        tgN = tgNN;
        mkC = mkN;
        zq = zq1;
    }
    if (bad) atomicOr(&a.flags[FLAG_DOMAIN], 1);
}

template <class S, class C>
hipError_t launch_step3d(mcb_ctx* c, const void* fcur, const void* rcur, void* fnext, void* rnext, bool pull) {
    C* rho = reinterpret_cast<C*>(c->lat + c->L.rho3);
    {
        RhoArgs<S, C> r;
        r.fa = static_cast<const S*>(fcur);
        r.tag = reinterpret_cast<const int32_t*>(c->lat + c->L.tag);
        r.rin = static_cast<const C*>(rcur);
        r.la = reinterpret_cast<const C*>(c->lk + c->L.lk_a);
        r.ibc = c->p.bc_mode == MCB_BC_IBC ? 1 : 0;
        r.fac = reinterpret_cast<const C*>(c->lk + c->L.wl_fac);
        r.rho = rho;
        r.flags = reinterpret_cast<int32_t*>(c->lat + c->L.flags);
        r.nx = c->p.nx;
        r.ny = c->p.ny;
        r.nz = c->p.nz;
        r.nbx = (r.nx + 255) / 256;
        r.rho_ref = c->p.precision == MCB_F64 ? C(0) : C(c->p.rho_ref);
        const int64_t nb = int64_t(r.nbx) * r.ny * r.nz;
        if (pull)
            hipLaunchKernelGGL((k_rho3d<S, C, true>), dim3(unsigned(nb)), dim3(256), 0, c->stream, r);
        else
            hipLaunchKernelGGL((k_rho3d<S, C, false>), dim3(unsigned(nb)), dim3(256), 0, c->stream, r);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    Args3<S, C> a;
    a.fa = static_cast<const S*>(fcur);
    a.fb = static_cast<S*>(fnext);
    a.tag = reinterpret_cast<const int32_t*>(c->lat + c->L.tag);
    a.nmask = reinterpret_cast<const uint32_t*>(c->lat + c->L.nmask);
    a.rho = rho;
    a.rin = static_cast<const C*>(rcur);
    a.rout = static_cast<C*>(rnext);
    a.la = reinterpret_cast<const C*>(c->lk + c->L.lk_a);
    a.flags = reinterpret_cast<int32_t*>(c->lat + c->L.flags);
    a.n_bnodes = uint32_t(c->n_bnodes > 0 ? c->n_bnodes : 0);
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.nz = c->p.nz;
    a.ntx = (a.nx + TX - 1) / TX;
    a.nty = (a.ny + TY - 1) / TY;
    // segment depth: short segments, about twelve rounds of resident workgroups (about 8 planes for
    // 256^3): the planes in flight then spread over the lattice instead of marching in step, which
    // measured faster here than deep segments or a single resident round; the ring of four extra
    // density planes per segment costs one value per node each
    constexpr bool PF = sizeof(C) == 4;
    int* occ = c->occ + 4;  // slots 4, 5 (a context runs one storage type)
    const int cap = pull ? resident_blocks(c, k_step3d<S, C, true, PF>, NT, &occ[1])
                         : resident_blocks(c, k_step3d<S, C, false, PF>, NT, &occ[0]);
    const int64_t tiles = int64_t(a.ntx) * a.nty;
    const int64_t per = 12 * cap / tiles > 0 ? 12 * cap / tiles : 1;  // segments per tile column
    int D = int((a.nz + per - 1) / per);
    if (D < 4) D = 4;
    a.D = D;
    a.nblocks = a.ntx * a.nty * ((a.nz + D - 1) / D);
    a.tau_inv = C(1.0 / c->p.tau);
    a.G = C(c->p.G);
    a.rho_ref = c->p.precision == MCB_F64 ? C(0) : C(c->p.rho_ref);
    a.kF = c->p.bc_mode == MCB_BC_PRESENT ? C(1) : C(0);
    a.k18 = c->p.bc_mode == MCB_BC_IBC ? C(0) : C(1);
    a.gx = C(c->p.gravity[0]);
    a.gy = C(c->p.gravity[1]);
    a.gz = C(c->p.gravity[2]);
    a.eos.RT = C(c->p.eos_R * c->p.eos_T);
    a.eos.a = C(c->p.eos_a);
    a.eos.b4 = C(c->p.eos_b / 4.0);
    a.eos.two_over_G = C(2.0 / c->p.G);
    if (pull)
        hipLaunchKernelGGL((k_step3d<S, C, true, PF>), dim3(a.nblocks), dim3(NT), 0, c->stream, a);
    else
        hipLaunchKernelGGL((k_step3d<S, C, false, PF>), dim3(a.nblocks), dim3(NT), 0, c->stream, a);
    return hipGetLastError();
}

}  // namespace

hipError_t step3d(mcb_ctx* c, const void* fcur, const void* rcur, void* fnext, void* rnext, bool pull) {
    switch (c->p.precision) {
        case MCB_F64: return launch_step3d<double, double>(c, fcur, rcur, fnext, rnext, pull);
        case MCB_F32S: return launch_step3d<float, float>(c, fcur, rcur, fnext, rnext, pull);
        default: return launch_step3d<__half, float>(c, fcur, rcur, fnext, rnext, pull);
    }
}

}  // namespace mcb
