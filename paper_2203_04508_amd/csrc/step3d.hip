// D3Q19 bulk of a time step: the fused kernel of the D2Q9 path carried to three dimensions --
// pull-streaming (eq. 5), density, the pseudopotential with first-layer wall densities (eq. 15),
// the interaction force, and the single-relaxation-time collision with exact-difference forcing
// (eqs. 4, 13-14), with the curved boundary condition (eqs. 16-17) and the mass correction of
// eq. 18 at boundary-fluid nodes.  As in two dimensions, the collision of a boundary node writes a
// contiguous boundary record (the terms of its forcing, its post-collision populations as stored,
// the eq. 18 correction), and the pull of the next step reads it with the node's link coefficients
// in a few wide loads and replaces the populations pulled from solid neighbours by the eq. 16-17
// values.
//
// Layout: a workgroup of 32 x 16 lanes covers a 32 x 16 column tile of the x-y plane -- 28 x 12
// output columns and two halo columns on every side -- over a segment of D planes in z, and
// marches along z one plane per iteration.  Each iteration
//   A  reduces the populations pulled for plane r to rho and puts rho and the node tag into a
//      4-plane LDS ring;
//   B  computes psi of plane r-1 (wall nodes: eq. 15 average over their fluid neighbours, times
//      phi) into a second 4-plane ring;
//   C  evaluates the force stencil for plane r-2 from the psi ring, collides the populations
//      pulled two iterations earlier (kept in registers) and stores them; boundary nodes also
//      store their boundary record.
// The populations of plane r+1 and the tags of plane r+3 are in flight while plane r is processed.
// The lane part of every pull address is one of nine loop-invariant column offsets and the plane
// part a wave-uniform scalar, so the loads need no address arithmetic.
#include "kernels_common.h"

namespace mcb {
namespace {

constexpr int TX = 32, TY = 16, NT = TX * TY;  // lanes of a tile
constexpr int OX = TX - 4, OY = TY - 4;        // output columns of a tile

// D3Q19: rest, the six axis vectors, the twelve edge vectors; opposite pairs side by side
__device__ constexpr int kEx3[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ constexpr int kEy3[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int kEz3[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

template <class S, class C>
struct Args3 {
    const S* fa;                 // post-collision populations of time t, SoA [19][N]
    S* fb;                       // post-collision populations of time t+1
    const int32_t* tag;          // >0: boundary index + 1; 0 fluid; -1 solid; -2-w wall w
    const C* rin;                // boundary records of time t, REC3 per boundary node
    C* rout;                     // boundary records of time t+1
    const C* la;                 // link coefficients, Q3_LINKS per boundary node (NO_LINK: none)
    const C* fac;                // eq. 15 factor per wall node: phi / weight of its fluid neighbours
    int32_t* flags;
    uint32_t n_bnodes, n_wall;
    int nx, ny, nz, D, ntx, nty, nblocks;
    C tau_inv, G, rho_ref;
    Eos<C> eos;
};

// Per-workgroup state of the plane march.
template <class S, class C>
struct March3 {
    Args3<S, C> a;
    __amdgpu_buffer_rsrc_t fa, fb, tag, rin, rout, la, fac;
    C (*s_rho)[NT];
    C (*s_psi)[NT];
    int (*s_tag)[NT];
    int t, nz, z0, iters, zc;
    uint32_t ns;       // bytes per population array (N nodes)
    uint32_t pb;       // bytes per z-plane of one population array
    uint32_t p4;       // bytes per z-plane of a 4-byte node array
    uint32_t own4;     // byte offset of this lane's column in a 4-byte node array plane
    uint32_t vxy[9];   // byte offsets of the columns (x + dx, y + dy), index 3 (dy + 1) + dx + 1
    bool out_col, inner;
    int tgA, tgB, tgC, tg_r, tg_r1, tg_r2;  // tags of planes r-2, r-1, r (history) and r+1, r+2
    C phA, phB;                      // eq. 15 factors of planes r-1 and r (wall lanes)
    C recN[RF3 + 18], aN[18];        // boundary record (the part the pull uses) and link coefficients
                                     // of plane r+1 (PF)
    C dsA, dsB, dsC;                 // eq. 18 corrections applied to planes r-2, r-1, r
    bool bad;
};

__device__ inline int zinc(int z, int nz) { return z == nz - 1 ? 0 : z + 1; }

// Issue the loads of the nineteen populations arriving at plane z of this lane's column (eq. 5),
// from x - e_i; PULL = false reads the node's own populations.
template <class S, class C, bool PULL>
__device__ __forceinline__ void pull_plane(const March3<S, C>& M, int z, C f[19]) {
    const uint32_t z0b = uint32_t(z) * M.pb;
    const uint32_t zmb = uint32_t(z == 0 ? M.nz - 1 : z - 1) * M.pb;
    const uint32_t zpb = uint32_t(z == M.nz - 1 ? 0 : z + 1) * M.pb;
    const uint32_t zof[3] = {zpb, z0b, zmb};  // upstream plane for e_z = -1, 0, +1
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const uint32_t vo = PULL ? M.vxy[(1 - kEy3[i]) * 3 + (1 - kEx3[i])] : M.vxy[4];
        const uint32_t so = uint32_t(i) * M.ns + (PULL ? zof[kEz3[i] + 1] : z0b);
        f[i] = Buf<S>::ld(M.fa, vo, so);
    }
}

// boundary record of time t and link coefficients of a boundary node (tg > 0; other lanes get zeros)
template <class S, class C>
__device__ __forceinline__ void ld_rec(const March3<S, C>& M, int tg, C (&rec)[RF3 + 18], C (&ca)[18]) {
    constexpr uint32_t sc = sizeof(C);
    const uint32_t bi = uint32_t(tg - 1);
    ld_vec(M.rin, tg > 0 ? bi * (REC3 * sc) : OOB, rec);
    ld_vec(M.la, tg > 0 ? bi * (Q3_LINKS * sc) : OOB, ca);
}

// D3Q19 weights
template <class C>
__device__ inline C w19(int i) {
    return i == 0 ? C(1.0 / 3.0) : (i < 7 ? C(1.0 / 18.0) : C(1.0 / 36.0));
}

// e.(x, y, z) for a lattice vector of components 0 and +-1, folded when the components are
// constants (a product with 0 cannot be dropped under IEEE rules)
template <class C>
__device__ __forceinline__ C edot3(int ex, int ey, int ez, C x, C y, C z) {
    const C tx = ex > 0 ? x : -x, ty = ey > 0 ? y : -y, tz = ez > 0 ? z : -z;
    const C a = ex == 0 ? ty : (ey == 0 ? tx : tx + ty);  // D3Q19: at most two components are set
    return ez == 0 ? a : ((ex == 0 && ey == 0) ? tz : a + tz);
}

// Eqs. 16-18 at a boundary node (bnd) from its record of time t (rec) and link coefficients (ca):
// replaces the populations pulled from solid neighbours by f_in (see the two-dimensional kernel for
// the three cases) and corrects the rest population; returns the correction.  Lanes that are not
// boundary nodes keep f and return 0; directions in which no lane of the wave has a link are
// skipped.  LOAD: rec and ca are loaded here, from rin at byte offset roff and la at aoff, in two
// halves, each just before its directions (keeps the FP64 kernel within its registers).
template <class S, class C, bool LOAD>
__device__ __forceinline__ C apply_links3(bool bnd, C (&rec)[RF3 + 18], C (&ca)[18], C (&f)[19], __amdgpu_buffer_rsrc_t rin,
                                          uint32_t roff, __amdgpu_buffer_rsrc_t la, uint32_t aoff) {
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
    const C rho = rec[0], dux = rec[1], duy = rec[2], duz = rec[3];
    const C sx = rec[4], sy = rec[5], sz = rec[6], duu = rec[7];
    // each slot opp(j) is replaced at most once, and never one that a later eq. 16 link reads (its
    // x2 = x - e_j is fluid, while a replaced slot was pulled from a solid node)
    C ds = C(0);
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
            ds += lk ? rec[RF3 + j - 1] - fin : C(0);
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
    f[0] += ds;
    return ds;
}

// One plane of the march (iteration k, plane r = z0 - 2 + k).  fC holds the pulled populations
// of plane r, fB and fA those of planes r-1 and r-2; the populations of plane r+1 go to fN (PF),
// else plane r is pulled into fC at the start of the iteration.
template <class S, class C, bool PULL, bool PF>
__device__ __forceinline__ void march_plane(March3<S, C>& M, int k, C (&fA)[19], C (&fB)[19], C (&fC)[19],
                                            C (&fN)[19]) {
    const Args3<S, C>& a = M.a;
    const int t = M.t;
    constexpr uint32_t sc = sizeof(C);
    const int slot = k & 3;
    M.tgA = M.tgB; M.tgB = M.tgC; M.tgC = M.tg_r;
    M.dsA = M.dsB; M.dsB = M.dsC;
    const int tgA = M.tgA;
    C recC[RF3 + 18], aC[18];  // record and coefficients of plane r
#pragma unroll
    for (int i = 0; i < RF3 + 18; ++i) recC[i] = M.recN[i];
#pragma unroll
    for (int i = 0; i < 18; ++i) aC[i] = M.aN[i];
    const bool coll = k >= 4 && M.out_col && tgA >= 0;
    const int zA = ((M.z0 - 4 + k) % M.nz + M.nz) % M.nz;
    const uint32_t xAb = uint32_t(zA) * M.pb + M.vxy[4];  // byte offset of (x, y, zA) in a population array
    // eq. 15 factor of a wall node of plane r-1 (psi below), loaded with that plane's pull
    const C phv = M.phA;
    __builtin_amdgcn_sched_barrier(0);
    // ---- plane r+1 populations and wettability factors (PF, else plane r), tags of plane r+3.
    // The tags run three planes ahead of the pull: the loads that depend on a tag then wait for
    // nothing newer than plane r-1, and the pulls of planes r and r+1 are in flight together.
    {
        const int z1 = zinc(M.zc, M.nz), z2 = zinc(z1, M.nz), z3 = zinc(z2, M.nz);
        const int tgp = PF ? M.tg_r1 : M.tg_r;
        if (PF) {
            pull_plane<S, C, PULL>(M, z1, fN);
        } else {
            pull_plane<S, C, PULL>(M, M.zc, fC);
        }
        const C phN = Buf<C>::ld(M.fac, tgp <= -2 ? uint32_t(-tgp - 2) * sc : OOB);
        const int tg3 = ld_i32(M.tag, M.own4, uint32_t(z3) * M.p4);
        M.tg_r = M.tg_r1;
        M.tg_r1 = M.tg_r2;
        M.tg_r2 = tg3;
        M.zc = z1;
        if (PF) {
            M.phA = M.phB;
            M.phB = phN;
        } else {
            M.phA = phN;  // plane r, used at the next iteration as plane r-1
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    // ---- A: links (eqs. 16-18) and density of plane r
    {
        M.dsC = C(0);
        if (PULL && __any(M.tgC > 0)) {
            // without the prefetch (FP64) the record and the coefficients are loaded here, when the
            // plane's pull is in
            const uint32_t bi = uint32_t(M.tgC - 1);
            M.dsC = apply_links3<S, C, !PF>(M.tgC > 0, recC, aC, fC, M.rin, M.tgC > 0 ? bi * (REC3 * sc) : OOB, M.la,
                                            M.tgC > 0 ? bi * (Q3_LINKS * sc) : OOB);
        }
        C sr = C(0);
#pragma unroll
        for (int i = 0; i < 19; ++i) sr += fC[i];
        M.s_rho[slot][t] = M.tgC >= 0 ? sr + a.rho_ref : C(0);
        M.s_tag[slot][t] = M.tgC;
    }
    // PF: boundary record and link coefficients of plane r+1 (tag M.tg_r by now), issued once those
    // of plane r are used up (so the two sets never hold registers together), a whole iteration
    // before they are needed
    // (only by waves that hold a boundary node in that plane: 16-byte loads cost address cycles even
    // for lanes out of bounds; the registers keep stale values exactly where the next iteration does
    // not read them)
    if (PF && PULL && __any(M.tg_r > 0)) ld_rec(M, M.tg_r, M.recN, M.aN);
    __syncthreads();
    // ---- B: psi of plane r - 1
    if (k >= 2 && M.inner) {
        const int s_mid = (k - 1) & 3, s_lo = (k - 2) & 3;
        const int tg = M.s_tag[s_mid][t];
        C rho_n;
        if (tg >= -1) {
            rho_n = M.s_rho[s_mid][t];
        } else {
            // wall node: eq. 15 over the first layer -- the weighted sum of the neighbours' density
            // (solid neighbours hold 0 in the ring) times phi / (weight of the fluid neighbours)
            C num = C(0);
            const int pl[3] = {s_lo, s_mid, slot};
#pragma unroll
            for (int i = 1; i < 19; ++i) {
                const C w = i < 7 ? C(1.0 / 18.0) : C(1.0 / 36.0);
                num += w * M.s_rho[pl[kEz3[i] + 1]][t + kEx3[i] + TX * kEy3[i]];
            }
            rho_n = phv * num;
        }
        M.s_psi[s_mid][t] = tg == -1 ? C(0) : psi_val(rho_n, a.eos, &M.bad);
    }
    __syncthreads();
    // ---- C: force and collision of plane r - 2; colliding lanes store.  Waves that hold no
    // output column skip the arithmetic but still issue the (out-of-bounds) stores.
    C out[19];
    // forcing terms, kept for the boundary record
    C rho = C(0), dux = C(0), duy = C(0), duz = C(0), sx2 = C(0), sy2 = C(0), sz2 = C(0), duu15 = C(0);
#pragma unroll
    for (int i = 0; i < 19; ++i) out[i] = C(0);
    if (__any(coll)) {
        // the node's density at t+1 from the pulled values; the collision hands all of it back,
        // with f_0 taking the rounding
        C rs = C(0);
#pragma unroll
        for (int i = 0; i < 19; ++i) rs += fA[i];
        const int sl = (k - 3) & 3, sm = (k - 2) & 3, sh = (k - 1) & 3;
        const int lx = t % TX, ly = t / TX;
        const int tc = min(max(ly, 1), TY - 2) * TX + min(max(lx, 1), TX - 2);
        auto P = [&](int dx, int dy, int dz) {
            const int sp = dz < 0 ? sl : (dz > 0 ? sh : sm);
            return M.s_psi[sp][tc + dx + TX * dy];
        };
        // F = -G psi(x) sum_i w^_i psi(x + e_i) e_i, w^ = 1/6 (axes), 1/12 (edges)
        const C gp = -a.G * M.s_psi[sm][tc];
        const C exy1 = P(1, 1, 0) - P(-1, -1, 0), exy2 = P(1, -1, 0) - P(-1, 1, 0);
        const C exz1 = P(1, 0, 1) - P(-1, 0, -1), exz2 = P(1, 0, -1) - P(-1, 0, 1);
        const C eyz1 = P(0, 1, 1) - P(0, -1, -1), eyz2 = P(0, 1, -1) - P(0, -1, 1);
        const C Fx = gp * (C(1.0 / 6.0) * (P(1, 0, 0) - P(-1, 0, 0)) + C(1.0 / 12.0) * (exy1 + exy2 + exz1 + exz2));
        const C Fy = gp * (C(1.0 / 6.0) * (P(0, 1, 0) - P(0, -1, 0)) + C(1.0 / 12.0) * (exy1 - exy2 + eyz1 + eyz2));
        const C Fz = gp * (C(1.0 / 6.0) * (P(0, 0, 1) - P(0, 0, -1)) + C(1.0 / 12.0) * (exz1 - exz2 + eyz1 - eyz2));

        rho = rs + a.rho_ref;
        const C irho = rcp(coll ? rho : C(1));
        const C jx = (fA[1] - fA[2]) + (fA[7] - fA[8]) + (fA[9] - fA[10]) + (fA[11] - fA[12]) + (fA[13] - fA[14]);
        const C jy = (fA[3] - fA[4]) + (fA[7] - fA[8]) - (fA[9] - fA[10]) + (fA[15] - fA[16]) + (fA[17] - fA[18]);
        const C jz = (fA[5] - fA[6]) + (fA[11] - fA[12]) - (fA[13] - fA[14]) + (fA[15] - fA[16]) - (fA[17] - fA[18]);
        const C ux = jx * irho, uy = jy * irho, uz = jz * irho;
        dux = Fx * irho;
        duy = Fy * irho;
        duz = Fz * irho;
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
            out[ip] = fA[ip] * omc + base + wra;
            out[im] = fA[im] * omc + base - wra;
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
        C rest = C(0);
#pragma unroll
        for (int i = 1; i < 19; ++i) {
            out[i] = Buf<S>::round(out[i]);
            rest += out[i];
        }
        out[0] = rs - rest;
    }
    // Every output column stores, solid nodes included (zeros: the pull replaces what it takes
    // from them), so rows are written without holes.  A lane that does not store starts from OOB;
    // the saturating add keeps it out of bounds.
    const uint32_t xst = (k >= 4 && M.out_col) ? xAb : OOB;
#pragma unroll
    for (int i = 0; i < 19; ++i) Buf<S>::st(M.fb, sat_add(xst, uint32_t(i) * M.ns), coll ? out[i] : C(0));
    // boundary record of time t+1: the forcing terms, the populations as stored, the eq. 18
    // correction
    {
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
        rv[RF3 + 18] = Buf<S>::round(out[0]);
        rv[RF3 + 19] = M.dsA;
        if (__any(coll && tgA > 0)) st_vec(M.rout, (coll && tgA > 0) ? uint32_t(tgA - 1) * (REC3 * sc) : OOB, rv);
    }
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
    __shared__ C s_rho[4][NT];
    __shared__ C s_psi[4][NT];
    __shared__ int s_tag[4][NT];
    constexpr uint32_t s = sizeof(S);

    March3<S, C> M;
    M.a = a;
    // lane t covers column (x0 - 2 + t % 32, y0 - 2 + t / 32); the lanes two or more columns in
    // from every tile edge own the outputs, the outer lanes are halo (psi needs rho two nodes out,
    // through the wall nodes)
    const int x0 = sx * OX, y0 = sy * OY;
    M.z0 = sz * a.D;
    const int Wv = min(OX, a.nx - x0), Hv = min(OY, a.ny - y0), Dv = min(a.D, a.nz - M.z0);
    M.t = threadIdx.x;
    const int lx = M.t % TX, ly = M.t / TX;
    M.nz = a.nz;
    const uint32_t nxy = uint32_t(a.nx) * uint32_t(a.ny);
    M.ns = nxy * uint32_t(a.nz) * s;
    M.pb = nxy * s;
    M.p4 = nxy * 4u;
    const int cx = ((x0 - 2 + lx) % a.nx + a.nx) % a.nx;
    const int cy = ((y0 - 2 + ly) % a.ny + a.ny) % a.ny;
    M.own4 = (uint32_t(cy) * a.nx + cx) * 4u;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx)
            M.vxy[(dy + 1) * 3 + dx + 1] = (uint32_t(wrap1(cy + dy, a.ny)) * a.nx + wrap1(cx + dx, a.nx)) * s;
    M.out_col = lx >= 2 && lx < 2 + Wv && ly >= 2 && ly < 2 + Hv;
    M.inner = lx >= 1 && lx < TX - 1 && ly >= 1 && ly < TY - 1;
    M.iters = Dv + 4;
    M.s_rho = s_rho;
    M.s_psi = s_psi;
    M.s_tag = s_tag;
    M.fa = make_res(a.fa, uint64_t(19) * M.ns);
    M.fb = make_res(a.fb, uint64_t(19) * M.ns);
    M.tag = make_res(a.tag, uint64_t(nxy) * a.nz * 4);
    M.rin = make_res(a.rin, uint64_t(a.n_bnodes) * REC3 * sizeof(C));
    M.rout = make_res(a.rout, uint64_t(a.n_bnodes) * REC3 * sizeof(C));
    M.la = make_res(a.la, uint64_t(a.n_bnodes) * Q3_LINKS * sizeof(C));
    M.fac = make_res(a.fac, uint64_t(a.n_wall) * sizeof(C));
    M.tgA = M.tgB = M.tgC = -1;
    M.dsA = M.dsB = M.dsC = C(0);
#pragma unroll
    for (int i = 0; i < RF3 + 18; ++i) M.recN[i] = C(0);
#pragma unroll
    for (int i = 0; i < 18; ++i) M.aN[i] = C(0);
    M.bad = false;
    // prologue: tags of planes r and r+1, populations of plane r (PF)
    C fA[19], fB[19], fC[19], fN[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) fA[i] = fB[i] = fC[i] = fN[i] = C(0);
    M.zc = ((M.z0 - 2) % a.nz + a.nz) % a.nz;
    M.tg_r = ld_i32(M.tag, M.own4, uint32_t(M.zc) * M.p4);
    M.tg_r1 = ld_i32(M.tag, M.own4, uint32_t(zinc(M.zc, a.nz)) * M.p4);
    M.tg_r2 = ld_i32(M.tag, M.own4, uint32_t(zinc(zinc(M.zc, a.nz), a.nz)) * M.p4);
    M.phA = C(0);
    M.phB = C(0);
    if (PF) {
        pull_plane<S, C, PULL>(M, M.zc, fC);
        if (PULL) ld_rec(M, M.tg_r, M.recN, M.aN);
        M.phB = Buf<C>::ld(M.fac, M.tg_r <= -2 ? uint32_t(-M.tg_r - 2) * sizeof(C) : OOB);
    }
    // the register sets rotate by copies (an unrolled rotation costs the allocator far more)
    for (int k = 0; k < M.iters; ++k) {
        march_plane<S, C, PULL, PF>(M, k, fA, fB, fC, fN);
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            fA[i] = fB[i];
            fB[i] = fC[i];
            if (PF) fC[i] = fN[i];
        }
    }
    if (M.bad) atomicOr(&a.flags[FLAG_DOMAIN], 1);
}

template <class S, class C>
hipError_t launch_step3d(mcb_ctx* c, const void* fcur, const void* rcur, void* fnext, void* rnext, bool pull) {
    Args3<S, C> a;
    a.fa = static_cast<const S*>(fcur);
    a.fb = static_cast<S*>(fnext);
    a.tag = reinterpret_cast<const int32_t*>(c->lat + c->L.tag);
    a.rin = static_cast<const C*>(rcur);
    a.rout = static_cast<C*>(rnext);
    a.la = reinterpret_cast<const C*>(c->lk + c->L.lk_a);
    a.fac = reinterpret_cast<const C*>(c->lk + c->L.wl_fac);
    a.flags = reinterpret_cast<int32_t*>(c->lat + c->L.flags);
    a.n_bnodes = uint32_t(c->n_bnodes > 0 ? c->n_bnodes : 0);
    a.n_wall = uint32_t(c->n_wall > 0 ? c->n_wall : 0);
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.nz = c->p.nz;
    a.ntx = (a.nx + OX - 1) / OX;
    a.nty = (a.ny + OY - 1) / OY;
    // segment depth: deep segments amortise the four ramp planes; shallow ones fill the chip
    int D = 64;
    while (D > 8 && int64_t(a.ntx) * a.nty * ((a.nz + D - 1) / D) < 1536) D >>= 1;
    a.D = D;
    a.nblocks = a.ntx * a.nty * ((a.nz + D - 1) / D);
    a.tau_inv = C(1.0 / c->p.tau);
    a.G = C(c->p.G);
    a.rho_ref = c->p.precision == MCB_F64 ? C(0) : C(c->p.rho_ref);
    a.eos.RT = C(c->p.eos_R * c->p.eos_T);
    a.eos.a = C(c->p.eos_a);
    a.eos.b4 = C(c->p.eos_b / 4.0);
    a.eos.two_over_G = C(2.0 / c->p.G);
    constexpr bool PF = sizeof(C) == 4;
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
