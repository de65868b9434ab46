// D2Q9 bulk of a time step: one fused kernel -- pull-streaming (eq. 5), density, the
// pseudopotential with first-layer wall densities (eq. 15), the interaction force, and the
// single-relaxation-time collision with exact-difference forcing (eqs. 4, 13-14), and at
// boundary-fluid nodes the curved boundary condition (eqs. 16-17) with the mass correction of
// eq. 18.
//
// Boundary nodes.  For a link (x, j) (x fluid, x + e_j solid) the population entering x along
// opp(j) at t+1 is
//   f_in = c1 f~_j(x, t) + c2 (o + F_j(x, t)),
//   eq. 16 (q < 1/2, x2 = x - e_j fluid): c1 = 2q,      c2 = 1 - 2q,       o = f~_j(x2, t)
//   eq. 17 (q >= 1/2):                    c1 = 1/(2q),  c2 = 1 - 1/(2q),   o = f~_opp(j)(x, t)
//   bounce-back (q < 1/2, x2 solid):      c1 = 1,       c2 = 0,
// and eq. 18 adds sum_links (f~_j(x, t) - f_in) to the rest population of x.  The pull of x already
// brings f~_j(x2, t) (population j arrives from x - e_j); what else the links need is the node's own
// post-collision populations and the exact-difference forcing term F_j(x, t) of eq. 13.  The
// collision of every boundary node writes its populations and the terms F_j is made of (rho,
// du = F / rho, s = 2u + du, 1.5 du.s) into a contiguous boundary record; the pull of the next step
// reads the record with the node's link coefficients in a few wide loads and applies the links in
// registers, replacing the populations pulled from solid nodes.  Records alternate between two
// buffers with the lattice buffers, since halo lanes of neighbouring workgroups read a node's
// record of time t while its owner writes that of t+1.
//
// Layout: a workgroup of W lanes (one or four waves) covers W consecutive columns -- W - 4 output
// columns and two halo columns on each side -- over a segment of H rows, and marches up the
// segment one row per iteration.  Each iteration
//   A  reduces the populations pulled for the current row to rho and puts rho and the node tag
//      into a 4-row LDS ring;
//   B  computes psi one row behind (wall nodes: eq. 15 average of their fluid neighbours times
//      phi) into a second 4-row LDS ring;
//   C  two rows behind, evaluates the force stencil from the psi ring and collides the populations
//      pulled two iterations earlier (kept in registers), then stores them; boundary nodes also
//      store their boundary record.
// Per bulk node only the populations (read once, written once) and a 4-byte tag reach HBM; rho and
// psi live in LDS.  Halo rows and columns are re-pulled by the neighbouring workgroup and hit in L2
// or the Infinity Cache.  The populations of the next row and the tag of the row after it are in
// flight while a row is processed, with the wettability factors of that row's wall nodes.  Every
// global access is a bounds-checked buffer instruction
// (no load or store sits in a divergent branch, so the wait counters stay exact), and the lane
// part of a pull address is loop-invariant, the row part a wave-uniform scalar: each vector
// memory instruction moves a full row of one population with no address arithmetic.
#include "kernels_common.h"

namespace mcb {
namespace {

template <class S, class C>
struct Args2 {
    const S* fa;                 // post-collision populations of time t, SoA [9][N]
    S* fb;                       // post-collision populations of time t+1
    const int32_t* tag;          // >0: (boundary index << 8) | link bits; 0 fluid; -1 solid; -2-w wall w
    const C* rin;                // boundary records of time t, REC2 per boundary node
    C* rout;                     // boundary records of time t+1
    const C* la;                 // link coefficients, Q2_LINKS per boundary node (NO_LINK: none)
    const C* fac;                // eq. 15 factor per wall node: phi / weight of its fluid neighbours
    int32_t* flags;
    uint32_t n_bnodes, n_wall;
    int nx, ny, H, nsx, nblocks;
    C tau_inv, G, rho_ref;
    C kF, k18;                   // boundary scheme: weight of the forcing term, of eq. 18 (0 or 1)
    C s_e, s_eps, s_q;           // rates of the multiple-relaxation-time collision (eq. 3)
    C gx, gy;                    // body acceleration: F = F_nonideal + rho g, so du = F / rho gains g
    Eos<C> eos;
};

// D2Q9 weights
template <class C>
__device__ inline C w9(int i) {
    return i == 0 ? C(4.0 / 9.0) : (i < 5 ? C(1.0 / 9.0) : C(1.0 / 36.0));
}

__device__ constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
__device__ constexpr int kEx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kEy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Per-workgroup state of the row march.
template <class S, class C, int W>
struct March {
    Args2<S, C> a;
    __amdgpu_buffer_rsrc_t fa, fb, tag, rin, rout, la, fac;
    C (*s_rho)[W];
    C (*s_psi)[W];
    int (*s_tag)[W];
    int t, p, nx, ny, y0, iters;   // lane, its column's position in the LDS rows
    uint32_t n, ns, xcol_b[3];   // nodes, bytes per population array, columns x-1, x, x+1
    uint32_t xcol0;              // FP16 storage: byte offset of column x in the FP32 rest-population plane
    uint32_t tag_b;              // byte offset of the column in the tag array (OOB for idle lanes)
    bool out_col;
    // pipeline registers: tags of rows r-2, r-1, r; row r+1 and the tag of r+2 in flight
    int tgA, tgB, tgC;
    int rr, rr1, tg_cur, tg_nxt, tg_nxt2;  // rows r+1, r+2 and the tags of r+1, r+2, r+3 (in flight)
    C phA, phB;       // eq. 15 factors of rows r-1 and r (wall lanes; issued with their pull)
    C recN[RF2 + 8], aN[Q2_LINKS];  // boundary record (the part the pull uses) and link coefficients of
                                    // row r+1 (in flight)
    C dsA, dsB, dsC;             // eq. 18 corrections applied to rows r-2, r-1, r
    C erA, erB, erC;             // and the residuals of adding them to f_0 (see apply_links)
    bool bad;
};

// Issue the loads of the nine populations arriving at row r of this lane's column (eq. 5), from
// x - e_i; PULL = false reads the node's own populations (the collision that starts a run).
// on = false: loads nothing (zeros).
template <class S, class C, int W, bool PULL>
__device__ __forceinline__ void pull_row(const March<S, C, W>& M, int r, bool on, C f[9]) {
    constexpr uint32_t s = sizeof(S);
    const uint32_t rows = uint32_t(M.nx) * s;
    const uint32_t r0 = uint32_t(r) * rows;
    const uint32_t rm = uint32_t(r == 0 ? M.ny - 1 : r - 1) * rows;
    const uint32_t rp = uint32_t(r == M.ny - 1 ? 0 : r + 1) * rows;
    const uint32_t rowof[3] = {rp, r0, rm};  // upstream row of e_y = -1, 0, +1
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (kMixed<S> && i == 0) {
            // FP16 storage: the rest population (own node) in FP32 at twice the half offsets
            f[0] = Buf<float>::ld(M.fa, on ? M.xcol0 : OOB, r0 * 2u);
            continue;
        }
        const uint32_t vo = on ? (PULL ? M.xcol_b[1 - kEx[i]] : M.xcol_b[1]) : OOB;
        const uint32_t so = uint32_t(i + (kMixed<S> ? 1 : 0)) * M.ns + (PULL ? rowof[kEy[i] + 1] : r0);
        f[i] = Buf<S>::ld(M.fa, vo, so);
    }
}

// e.(x, y) for a lattice vector of components 0 and +-1, folded when the components are constants
// (a product with 0 cannot be dropped under IEEE rules)
template <class C>
__device__ __forceinline__ C edot(int ex, int ey, C x, C y) {
    const C tx = ex > 0 ? x : -x, ty = ey > 0 ? y : -y;
    return ex == 0 ? ty : (ey == 0 ? tx : tx + ty);
}

// Eqs. 16-18 at a boundary node (bnd) from its record of time t (rec) and link coefficients (ca):
// replaces the populations pulled from solid neighbours by f_in and corrects the rest population;
// returns the correction and, in res, what rounding f_0 + correction to the compute type dropped.
// Lanes that are not boundary nodes keep f and return zeros.  Directions in which no lane of the wave has a link are
// skipped.  kF and k18 select the scheme: 1 and 1 the present one, 0 and 0 linear interpolation
// bounce-back (no forcing term, no eq. 18), 0 and 1 the same with eq. 18; halfway bounce-back is
// a = 1 on every link.
template <class S, class C>
__device__ __forceinline__ C apply_links(bool bnd, const C (&rec)[RF2 + 8], const C (&ca)[Q2_LINKS], C (&f)[9], C kF,
                                         C k18, C& res) {
    const C rho = rec[0] * kF, dux = rec[1], duy = rec[2], sx = rec[3], sy = rec[4], duu = rec[5];
    const C* fo = rec + RF2 - 1;  // own post-collision populations 1 .. 8
    // each slot opp(j) is replaced at most once, and never one that a later eq. 16 link reads (its
    // x2 = x - e_j is fluid, while a replaced slot was pulled from a solid node)
    double ds = 0.0;
#pragma unroll
    for (int j = 1; j < 9; ++j) {
        const C a = ca[j - 1];
        const bool lk = bnd && a < C(1.5);
        if (__builtin_amdgcn_ballot_w64(lk)) {
            const C c1 = a < C(0) ? -a : a, c2 = C(1) - c1;
            // eq. 13 term of direction j: w rho [3 e.du + 4.5 (e.du)(e.s) - 1.5 du.s]
            const C ed = edot<C>(kEx[j], kEy[j], dux, duy);
            const C es = edot<C>(kEx[j], kEy[j], sx, sy);
            const C Fj = w9<C>(j) * rho * (C(3) * ed + C(4.5) * ed * es - duu);
            C o = a < C(0) ? fo[kOpp[j]] : f[j];
            o = c2 != C(0) ? o : C(0);
            // rounded to the storage format, as the value would be stored; eq. 18 takes it so
            const C fin = Buf<S>::round(c1 * fo[j] + c2 * (o + Fj));
            ds += lk ? double(fo[j]) - double(fin) : 0.0;
            f[kOpp[j]] = lk ? fin : f[kOpp[j]];
        }
    }
    ds *= double(k18);
    const double f0 = double(f[0]) + ds;
    f[0] = C(f0);
    res = C(f0 - double(f[0]));
    return C(ds);
}

// Collision of one node (eq. 4, or eqs. 1-4 when MRT; eq. 13 forcing, eq. 14 equilibrium) from its
// pulled populations fA (stored format: shifted by w_i rho_ref), their sum rs_acc and the force
// (Fx, Fy) without the body force.  Writes the post-collision populations rounded to the storage
// format, f_0 taking the rounding so that the node keeps its mass exactly, and the forcing terms
// the boundary record carries.  coll = false (lanes that collide nothing) keeps the arithmetic finite.
template <class S, class C, bool MRT>
__device__ __forceinline__ void collide9(const Args2<S, C>& a, bool coll, const C (&fA)[9], MassAcc<S, C> rs_acc, C Fx, C Fy,
                                         C (&out)[9], C& rho, C& dux, C& duy, C& sx2, C& sy2, C& duu15) {
    const C rs = C(rs_acc);
    rho = rs + a.rho_ref;
    const C irho = rcp(coll ? rho : C(1));
    const C jx = fA[1] - fA[3] + fA[5] - fA[6] - fA[7] + fA[8];
    const C jy = fA[2] - fA[4] + fA[5] + fA[6] - fA[7] - fA[8];
    const C ux = jx * irho, uy = jy * irho;
    dux = Fx * irho + a.gx;
    duy = Fy * irho + a.gy;
    const C ti = a.tau_inv, omc = C(1) - ti;
    // per direction: out_i = f_i (1 - 1/tau) + w_i [rs/tau + rho (sym_i +- anti_i)] with
    //   sym  = (4.5 (e.u)^2 - 1.5 u^2) / tau + 4.5 (e.du)(e.(2u + du)) - 1.5 du.(2u + du)
    //   anti = 3 (e.u / tau + e.du)
    // (eq. 14 equilibrium, eq. 13 forcing term, eq. 4 with S = I / tau)
    const C uu15 = C(1.5) * (ux * ux + uy * uy);
    sx2 = C(2) * ux + dux;
    sy2 = C(2) * uy + duy;
    duu15 = C(1.5) * (dux * sx2 + duy * sy2);
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
    if constexpr (!MRT) {
        pair(1, 3, C(1.0 / 9.0), ux, dux, sx2);
        pair(2, 4, C(1.0 / 9.0), uy, duy, sy2);
        pair(5, 7, C(1.0 / 36.0), ux + uy, dux + duy, sx2 + sy2);
        pair(6, 8, C(1.0 / 36.0), uy - ux, duy - dux, sy2 - sx2);
    } else {
        // eqs. 1-4 with the moment matrix of eq. 2: the six non-conserved moments of the stored
        // populations (the shift w_i rho_ref has moments rho_ref, -2 rho_ref, rho_ref, 0, ...,
        // folded in through rs), relaxed at the eq. 3 rates toward the Sec. 2.1 equilibria
        // (q^eq = -j); M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
        const C s14 = fA[1] + fA[2] + fA[3] + fA[4], s58 = fA[5] + fA[6] + fA[7] + fA[8];
        const C jj = rho * (ux * ux + uy * uy);
        const C de = a.s_e * (C(-4) * fA[0] - s14 + C(2) * s58 + C(2) * rs - C(3) * jj) * C(1.0 / 36.0);
        const C dp = a.s_eps * (C(4) * fA[0] - C(2) * s14 + s58 - rs + C(3) * jj) * C(1.0 / 36.0);
        const C dx = a.s_q * (C(-2) * (fA[1] - fA[3]) + (fA[5] - fA[6] - fA[7] + fA[8]) + jx) * C(1.0 / 12.0);
        const C dy = a.s_q * (C(-2) * (fA[2] - fA[4]) + (fA[5] + fA[6] - fA[7] - fA[8]) + jy) * C(1.0 / 12.0);
        const C dxx = ti * (fA[1] - fA[2] + fA[3] - fA[4] - rho * (ux * ux - uy * uy)) * C(0.25);
        const C dxy = ti * (fA[5] - fA[6] + fA[7] - fA[8] - rho * ux * uy) * C(0.25);
        // out = f - M^-1 S (m - m_eq) + F_i, F_i the eq. 13 term, by opposite pairs
        auto mpair = [&](int ip, int im, C w, C ed, C es, C sym, C anti) {
            const C wr = w * rho;
            const C fs = wr * (C(4.5) * ed * es - duu15) + sym;
            const C fa = wr * C(3) * ed + anti;
            out[ip] = fA[ip] + fs + fa;
            out[im] = fA[im] + fs - fa;
        };
        const C e1 = de + C(2) * dp, e2 = C(2) * de + dp;
        mpair(1, 3, C(1.0 / 9.0), dux, sx2, e1 - dxx, C(2) * dx);
        mpair(2, 4, C(1.0 / 9.0), duy, sy2, e1 + dxx, C(2) * dy);
        mpair(5, 7, C(1.0 / 36.0), dux + duy, sx2 + sy2, -(e2 + dxy), -(dx + dy));
        mpair(6, 8, C(1.0 / 36.0), duy - dux, sy2 - sx2, -(e2 - dxy), -(dy - dx));
    }
    // collision conserves mass (the equilibrium and the forcing term of eq. 13 have zero net
    // mass): set f_0 to the density minus the other eight outputs as stored, so the rounding of
    // the lattice weights and of the storage format cannot bias the total mass
    MassAcc<S, C> rest = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        out[i] = Buf<S>::round(out[i]);
        rest += MassAcc<S, C>(out[i]);
    }
    out[0] = C(rs_acc - rest);
}

// One row of the march (iteration k, row r = y0 - 2 + k).  fC holds the pulled populations of row
// r, fB and fA those of rows r-1 and r-2, fN those of row r+1 (in flight); the populations of row
// r+2 are issued into fP.
template <class S, class C, int W, int OUT, bool PULL, bool MRT>
__device__ __forceinline__ void march_row(March<S, C, W>& M, int k, C (&fA)[9], C (&fB)[9], C (&fC)[9], C (&fN)[9],
                                          C (&fP)[9]) {
    const Args2<S, C>& a = M.a;
    const int t = M.p, nx = M.nx, ny = M.ny;  // LDS rows are indexed by column position
    constexpr uint32_t s = sizeof(S), sc = sizeof(C);
    const int slot = k & 3;
    M.tgA = M.tgB; M.tgB = M.tgC; M.tgC = M.tg_cur;
    M.dsA = M.dsB; M.dsB = M.dsC;
    M.erA = M.erB; M.erB = M.erC;
    C recC[RF2 + 8], aC[Q2_LINKS];  // record and coefficients of row r (arrived with its pull)
#pragma unroll
    for (int i = 0; i < RF2 + 8; ++i) recC[i] = M.recN[i];
#pragma unroll
    for (int i = 0; i < Q2_LINKS; ++i) aC[i] = M.aN[i];
    const int tgA = M.tgA;
    const bool coll = k >= 4 && M.out_col && tgA >= 0;
    const int yA = ((M.y0 - 4 + k) % ny + ny) % ny;
    const uint32_t xAb = (uint32_t(yA) * nx) * s + M.xcol_b[1];  // byte offset of (x, yA) in a plane
    // eq. 15 factor of a wall node of row r-1 (psi below), loaded with that row's pull
    const C phv = M.phA;
    __builtin_amdgcn_sched_barrier(0);
    // ---- row r+2 populations, row r+1 wettability factors, row r+3 tags.  The pulls run two rows
    // ahead (rows r+1 and r+2 are in flight together), the tags three: the loads that depend on a
    // tag then wait for nothing newer than row r-1.  Rows past the segment are not pulled.
    {
        const bool more = k + 1 < M.iters;
        M.rr = M.rr1;
        M.rr1 = M.rr == ny - 1 ? 0 : M.rr + 1;
        const int r3 = M.rr1 == ny - 1 ? 0 : M.rr1 + 1;
        M.tg_cur = more ? M.tg_nxt : -1;
        M.tg_nxt = M.tg_nxt2;
        pull_row<S, C, W, PULL>(M, M.rr1, k + 2 < M.iters, fP);
        const C phN = Buf<C>::ld(M.fac, M.tg_cur <= -2 ? uint32_t(-M.tg_cur - 2) * sc : OOB);
        M.tg_nxt2 = ld_i32(M.tag, k + 3 < M.iters ? M.tag_b : OOB, uint32_t(r3) * (nx * 4u));
        M.phA = M.phB;
        M.phB = phN;
    }
    __builtin_amdgcn_sched_barrier(0);
    // ---- A: links (eqs. 16-18) and density of row r
    {
        M.dsC = C(0);
        M.erC = C(0);
        if (PULL && __any(M.tgC > 0)) M.dsC = apply_links<S, C>(M.tgC > 0, recC, aC, fC, a.kF, a.k18, M.erC);
        C sr = C(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) sr += fC[i];
        M.s_rho[slot][t] = M.tgC >= 0 ? sr + a.rho_ref : C(0);
        M.s_tag[slot][t] = M.tgC;
    }
    // boundary record and link coefficients of row r+1, issued once those of row r are used up (so
    // the two sets never hold registers together), a whole iteration before they are needed; only
    // by waves that hold a boundary node in that row (16-byte loads cost address cycles even for
    // lanes out of bounds), so the registers keep stale values exactly where the next iteration
    // does not read them
    if (PULL && __any(M.tg_cur > 0)) {
        const uint32_t bi = uint32_t(M.tg_cur >> 8);
        ld_vec(M.rin, M.tg_cur > 0 ? bi * (REC2 * sc) : OOB, M.recN);
        ld_vec(M.la, M.tg_cur > 0 ? bi * (Q2_LINKS * sc) : OOB, M.aN);
    }
    __syncthreads();
    // ---- B: psi of row r - 1
    if (k >= 2 && t >= 1 && t <= OUT + 2) {
        const int s_mid = (k - 1) & 3, s_lo = (k - 2) & 3;
        const int tg = M.s_tag[s_mid][t];
        C rho_n;
        if (tg >= -1) {
            rho_n = M.s_rho[s_mid][t];
        } else {
            // wall node: eq. 15 over the first layer -- the weighted sum of the neighbours' density
            // (solid neighbours hold 0 in the ring) times phi / (weight of the fluid neighbours)
            C num = C(0);
            const int rows[3] = {s_lo, s_mid, slot};
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    const C w = (dx == 0 || dy == 0) ? C(1.0 / 9.0) : C(1.0 / 36.0);
                    num += w * M.s_rho[rows[dy + 1]][t + dx];
                }
            rho_n = phv * num;
        }
        M.s_psi[s_mid][t] = tg == -1 ? C(0) : psi_val(rho_n, a.eos, &M.bad);
    }
    __syncthreads();
    // ---- C: force and collision of row r - 2; colliding lanes store (computed in every iteration:
    // in the first four, which collide nothing, the results are discarded, and there is no branch
    // around the stores)
    C out[9];
    C rho, dux, duy, sx2, sy2, duu15;  // forcing terms, kept for the boundary record
    {
        // the node's density at t+1 from the pulled values; the collision hands all of it back,
        // with f_0 taking the rounding
        MassAcc<S, C> rs_acc = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) rs_acc += MassAcc<S, C>(fA[i]);
        rs_acc += MassAcc<S, C>(M.erA);  // the part of the eq. 18 correction that rounding kept out of f_0
        const int sl = (k - 3) & 3, sm = (k - 2) & 3, sh = (k - 1) & 3;
        const int tc = t < 1 ? 1 : (t > OUT + 2 ? OUT + 2 : t);
        const C p0 = M.s_psi[sm][tc];
        const C pE = M.s_psi[sm][tc + 1], pW = M.s_psi[sm][tc - 1];
        const C pN = M.s_psi[sh][tc], pS = M.s_psi[sl][tc];
        const C pNE = M.s_psi[sh][tc + 1], pNW = M.s_psi[sh][tc - 1];
        const C pSW = M.s_psi[sl][tc - 1], pSE = M.s_psi[sl][tc + 1];
        // F = -G psi(x) sum_i w^_i psi(x + e_i) e_i, w^ = 1/3 (axes), 1/12 (diagonals)
        const C gp = -a.G * p0;
        const C Fx = gp * (C(1.0 / 3.0) * (pE - pW) + C(1.0 / 12.0) * (pNE - pNW - pSW + pSE));
        const C Fy = gp * (C(1.0 / 3.0) * (pN - pS) + C(1.0 / 12.0) * (pNE + pNW - pSW - pSE));

        collide9<S, C, MRT>(a, coll, fA, rs_acc, Fx, Fy, out, rho, dux, duy, sx2, sy2, duu15);
    }
    // Every output column stores, solid nodes included (zeros: the pull replaces what it takes
    // from them), so rows are written without holes and every cache line whole.  A lane that does
    // not store starts from OOB; the saturating add keeps it out of bounds.
    const uint32_t xst = (k >= 4 && M.out_col) ? xAb : OOB;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (kMixed<S> && i == 0)
            Buf<float>::st_nt(M.fb, xst == OOB ? OOB : xst * 2u, coll ? out[0] : C(0));
        else
            Buf<S>::st_nt(M.fb, sat_add(xst, uint32_t(i + (kMixed<S> ? 1 : 0)) * M.ns), coll ? out[i] : C(0));
    }
    // boundary record of time t+1: the forcing terms, the populations as stored, the eq. 18
    // correction
    {
        C rv[REC2];
        rv[0] = rho;
        rv[1] = dux;
        rv[2] = duy;
        rv[3] = sx2;
        rv[4] = sy2;
        rv[5] = duu15;
#pragma unroll
        for (int i = 1; i < 9; ++i) rv[RF2 + i - 1] = out[i];  // rounded to the storage format above
        rv[RF2 + 8] = kMixed<S> ? out[0] : Buf<S>::round(out[0]);
        rv[RF2 + 9] = M.dsA;
        if (__any(coll && tgA > 0)) st_vec(M.rout, (coll && tgA > 0) ? uint32_t(tgA >> 8) * (REC2 * sc) : OOB, rv);
    }
}

template <class S, class C, int W, int OUT, bool PULL, bool MRT>
__global__ __launch_bounds__(W) void k_step2d(Args2<S, C> a) {
    // XCD-aware order: consecutive logical tiles go to the same XCD (one L2)
    const int bid = blockIdx.x;
    const int per = a.nblocks >> 3, rem = a.nblocks & 7;
    const int xcd = bid & 7, k8 = bid >> 3;
    const int logical = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k8;
    const int sx = logical % a.nsx, sy = logical / a.nsx;
    __shared__ C s_rho[4][W];
    __shared__ C s_psi[4][W];
    __shared__ int s_tag[4][W];
    constexpr uint32_t s = sizeof(S), sc = sizeof(C);

    March<S, C, W> M;
    M.a = a;
    // The strip's OUT output columns x0 .. x0 + OUT - 1 go to lanes 0 .. OUT - 1, so that every
    // wave's loads and stores of a row start on a cache line when OUT is a multiple of the line
    // (32 FP32 or 64 FP16 values); the two halo columns on either side (psi needs rho two columns
    // out, through the wall nodes) go to lanes OUT .. OUT + 3, and further lanes idle.  The LDS
    // rows are indexed by position p = column - (x0 - 2).
    const int x0 = sx * OUT;
    M.y0 = sy * a.H;
    const int Wv = min(OUT, a.nx - x0), Hv = min(a.H, a.ny - M.y0);
    M.t = threadIdx.x;
    const int t = M.t;
    M.p = t < OUT + 2 ? t + 2 : (t < OUT + 4 ? t - OUT - 2 : t);
    const bool live = t < OUT + 4;
    M.nx = a.nx;
    M.ny = a.ny;
    M.n = uint32_t(a.nx) * uint32_t(a.ny);
    const int cx = ((x0 - 2 + M.p) % a.nx + a.nx) % a.nx;
    M.xcol_b[0] = live ? uint32_t(cx == 0 ? a.nx - 1 : cx - 1) * s : OOB;
    M.xcol_b[1] = live ? uint32_t(cx) * s : OOB;
    M.xcol_b[2] = live ? uint32_t(cx == a.nx - 1 ? 0 : cx + 1) * s : OOB;
    M.tag_b = live ? uint32_t(cx) * 4u : OOB;
    M.out_col = t < Wv;
    M.iters = Hv + 4;
    M.s_rho = s_rho;
    M.s_psi = s_psi;
    M.s_tag = s_tag;
    M.fa = make_res(a.fa, uint64_t(kMixed<S> ? 10 : 9) * M.n * s);
    M.fb = make_res(a.fb, uint64_t(kMixed<S> ? 10 : 9) * M.n * s);
    M.xcol0 = live ? uint32_t(cx) * 4u : OOB;
    M.tag = make_res(a.tag, uint64_t(M.n) * 4);
    M.rin = make_res(a.rin, uint64_t(a.n_bnodes) * REC2 * sizeof(C));
    M.rout = make_res(a.rout, uint64_t(a.n_bnodes) * REC2 * sizeof(C));
    M.la = make_res(a.la, uint64_t(a.n_bnodes) * Q2_LINKS * sizeof(C));
    M.ns = M.n * s;
    M.fac = make_res(a.fac, uint64_t(a.n_wall) * sizeof(C));
    M.tgA = M.tgB = M.tgC = -1;
    M.dsA = M.dsB = M.dsC = C(0);
    M.erA = M.erB = M.erC = C(0);
    M.bad = false;
    // row march: the populations of rows r+1 and r+2 are in flight while row r is reduced to rho,
    // row r-1 to psi and row r-2 collided; five register sets rotate
    C f0[9], f1[9], f2[9], f3[9], f4[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f0[i] = f1[i] = f4[i] = C(0);
    M.rr = ((M.y0 - 2) % a.ny + a.ny) % a.ny;
    M.tg_cur = ld_i32(M.tag, M.tag_b, uint32_t(M.rr) * (a.nx * 4u));
    M.rr1 = M.rr == a.ny - 1 ? 0 : M.rr + 1;
    M.tg_nxt = ld_i32(M.tag, M.tag_b, uint32_t(M.rr1) * (a.nx * 4u));
    M.tg_nxt2 = ld_i32(M.tag, M.tag_b, uint32_t(M.rr1 == a.ny - 1 ? 0 : M.rr1 + 1) * (a.nx * 4u));
    pull_row<S, C, W, PULL>(M, M.rr, true, f2);
    pull_row<S, C, W, PULL>(M, M.rr1, true, f3);
#pragma unroll
    for (int i = 0; i < RF2 + 8; ++i) M.recN[i] = C(0);
#pragma unroll
    for (int i = 0; i < Q2_LINKS; ++i) M.aN[i] = C(0);
    if (PULL) {
        const uint32_t bi = uint32_t(M.tg_cur >> 8);
        ld_vec(M.rin, M.tg_cur > 0 ? bi * (REC2 * sc) : OOB, M.recN);
        ld_vec(M.la, M.tg_cur > 0 ? bi * (Q2_LINKS * sc) : OOB, M.aN);
    }
    M.phA = C(0);
    M.phB = Buf<C>::ld(M.fac, M.tg_cur <= -2 ? uint32_t(-M.tg_cur - 2) * sc : OOB);
    int k = 0;
    for (; k + 5 <= M.iters; k += 5) {
        march_row<S, C, W, OUT, PULL, MRT>(M, k + 0, f0, f1, f2, f3, f4);
        march_row<S, C, W, OUT, PULL, MRT>(M, k + 1, f1, f2, f3, f4, f0);
        march_row<S, C, W, OUT, PULL, MRT>(M, k + 2, f2, f3, f4, f0, f1);
        march_row<S, C, W, OUT, PULL, MRT>(M, k + 3, f3, f4, f0, f1, f2);
        march_row<S, C, W, OUT, PULL, MRT>(M, k + 4, f4, f0, f1, f2, f3);
    }
    const int left = M.iters - k;  // uniform
    if (left > 0) march_row<S, C, W, OUT, PULL, MRT>(M, k + 0, f0, f1, f2, f3, f4);
    if (left > 1) march_row<S, C, W, OUT, PULL, MRT>(M, k + 1, f1, f2, f3, f4, f0);
    if (left > 2) march_row<S, C, W, OUT, PULL, MRT>(M, k + 2, f2, f3, f4, f0, f1);
    if (left > 3) march_row<S, C, W, OUT, PULL, MRT>(M, k + 3, f3, f4, f0, f1, f2);
    if (M.bad) atomicOr(&a.flags[FLAG_DOMAIN], 1);
}

template <class S, class C, int W, int OUT>
hipError_t launch_w(mcb_ctx* c, const void* fcur, const void* rcur, void* fnext, void* rnext, bool pull) {
    const bool mrt = c->p.collision == MCB_COLL_MRT;
    Args2<S, C> a;
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
    a.nsx = (a.nx + OUT - 1) / OUT;
    // segment height: long segments amortise the four halo rows; short ones fill the chip.  Wide
    // strips: as many segments as the device holds in a number of resident rounds -- four with
    // FP32 storage (the shorter segments' extra halo rows cost less than the march loses when every
    // workgroup moves in step with the others), one with FP16 storage, whose arithmetic is the limit
    // and grows with the halo rows, and with FP64; one-wave strips (small lattices): enough
    // workgroups to fill the chip several times over.
    int H;
    if (W == 64) {
        H = 64;
        while (H > 8 && int64_t(a.nsx) * ((a.ny + H - 1) / H) < 8192) H >>= 1;
    } else {
        // a context runs one storage type and one strip width, so four slots cover its variants
        int* occ = c->occ;
        const int cap = pull ? (mrt ? resident_blocks(c, k_step2d<S, C, W, OUT, true, true>, W, &occ[3])
                                    : resident_blocks(c, k_step2d<S, C, W, OUT, true, false>, W, &occ[1]))
                             : (mrt ? resident_blocks(c, k_step2d<S, C, W, OUT, false, true>, W, &occ[2])
                                    : resident_blocks(c, k_step2d<S, C, W, OUT, false, false>, W, &occ[0]));
        const int rounds = sizeof(S) == 4 ? 4 : 1;
        const int per = rounds * cap / a.nsx > 0 ? rounds * cap / a.nsx : 1;  // segments per strip
        H = (a.ny + per - 1) / per;
        if (H < 16) H = 16;
    }
    a.H = H;
    a.nblocks = a.nsx * ((a.ny + H - 1) / H);
    a.tau_inv = C(1.0 / c->p.tau);
    a.G = C(c->p.G);
    a.rho_ref = c->p.precision == MCB_F64 ? C(0) : C(c->p.rho_ref);
    a.kF = c->p.bc_mode == MCB_BC_PRESENT ? C(1) : C(0);
    a.k18 = c->p.bc_mode == MCB_BC_IBC ? C(0) : C(1);
    a.s_e = C(c->p.s_e);
    a.s_eps = C(c->p.s_eps);
    a.s_q = C(c->p.s_q);
    a.gx = C(c->p.gravity[0]);
    a.gy = C(c->p.gravity[1]);
    a.eos.RT = C(c->p.eos_R * c->p.eos_T);
    a.eos.a = C(c->p.eos_a);
    a.eos.b4 = C(c->p.eos_b / 4.0);
    a.eos.two_over_G = C(2.0 / c->p.G);
    if (pull && !mrt)
        hipLaunchKernelGGL((k_step2d<S, C, W, OUT, true, false>), dim3(a.nblocks), dim3(W), 0, c->stream, a);
    else if (pull)
        hipLaunchKernelGGL((k_step2d<S, C, W, OUT, true, true>), dim3(a.nblocks), dim3(W), 0, c->stream, a);
    else if (!mrt)
        hipLaunchKernelGGL((k_step2d<S, C, W, OUT, false, false>), dim3(a.nblocks), dim3(W), 0, c->stream, a);
    else
        hipLaunchKernelGGL((k_step2d<S, C, W, OUT, false, true>), dim3(a.nblocks), dim3(W), 0, c->stream, a);
    return hipGetLastError();
}

template <class S, class C>
hipError_t launch_step2d(mcb_ctx* c, const void* fcur, const void* rcur, void* fnext, void* rnext, bool pull) {
    // one-wave strips keep small lattices busy; on large lattices the strips are a whole number of
    // cache lines wide (224 FP32 / FP64 columns, 192 FP16 columns), so that no line is shared
    // between strips or written in parts
    if (c->g.N <= (int64_t(1) << 21)) return launch_w<S, C, 64, 60>(c, fcur, rcur, fnext, rnext, pull);
    if (sizeof(S) == 2) return launch_w<S, C, 256, 192>(c, fcur, rcur, fnext, rnext, pull);
    return launch_w<S, C, 256, 224>(c, fcur, rcur, fnext, rnext, pull);
}

// ---------------------------------------------------------------- chemical-potential model (2-D)
// The paper's multiphase model (Secs. 2.2-2.3): the force needs the density and the chemical
// potential two nodes away on each axis, and the chemical potential itself the density two nodes
// away.  A step runs as one march (k_cp_march below) that keeps the fields of a few rows in LDS.
// The pass kernels that follow compute the same fields over the whole lattice, one stage each
// (density with eqs. 16-18, the two solid layers of eq. 15, the chemical potential of eq. 12), for
// the velocity output, which needs them at every node.
template <class S, class C>
struct ArgsCP {
    Args2<S, C> a;
    C* rho;                 // density of the step: fluid nodes and solid layers 1-2
    C* mu;                  // chemical potential of the step: fluid nodes and solid layers 1-2
    const int8_t* layer;    // 0 fluid, 1 wall node, 2 second solid layer, 3 deeper
    const double* mus;      // assigned chemical potential per wall node
    C k2, kappa;            // eq. 12: k^2 and kappa
    C RT, b, c_log, aal;    // eq. 11: R T, b, a alpha / (2 sqrt 2 b), a alpha
};

// the populations pulled into node (cx, cy) (PULL; otherwise its own stored ones)
template <class S, class C, bool PULL>
__device__ __forceinline__ void pull_pops(const Args2<S, C>& a, int64_t N, int cx, int cy, C (&f)[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int sx = PULL ? wrap1(cx - kEx[i], a.nx) : cx, sy = PULL ? wrap1(cy - kEy[i], a.ny) : cy;
        f[i] = ldp<S, C>(a.fa, i, N, int64_t(sy) * a.nx + sx);
    }
}

// eqs. 16-18 on pulled populations f of a node with tag tg; ds = the eq. 18 correction
template <class S, class C, bool PULL>
__device__ __forceinline__ void pull_links(const Args2<S, C>& a, int tg, C (&f)[9], C& ds, C& res) {
    ds = C(0);
    res = C(0);
    if (PULL) {
        const bool bnd = tg > 0;
        if (__any(bnd)) {
            C rec[RF2 + 8], ca[Q2_LINKS];
            const int64_t bi = bnd ? int64_t(tg >> 8) : 0;
#pragma unroll
            for (int k = 0; k < RF2 + 8; ++k) rec[k] = bnd ? a.rin[bi * REC2 + k] : C(0);
#pragma unroll
            for (int k = 0; k < Q2_LINKS; ++k) ca[k] = bnd ? a.la[bi * Q2_LINKS + k] : C(NO_LINK);
            ds = apply_links<S, C>(bnd, rec, ca, f, a.kF, a.k18, res);
        }
    }
}

// eqs. 16-18 from a boundary record and link coefficients loaded beforehand (lanes that are not
// boundary nodes ignore theirs)
template <class S, class C, bool PULL>
__device__ __forceinline__ void links_from(const Args2<S, C>& a, int tg, C (&f)[9], const C (&rec)[RF2 + 8],
                                           const C (&ca)[Q2_LINKS], C& ds, C& res) {
    ds = C(0);
    res = C(0);
    if (PULL && __any(tg > 0)) ds = apply_links<S, C>(tg > 0, rec, ca, f, a.kF, a.k18, res);
}

// pulled populations of node (cx, cy) (PULL; otherwise its own stored ones), with eqs. 16-18 at
// boundary nodes; ds = the eq. 18 correction.  Solid nodes hold zeros, which the links replace.
template <class S, class C, bool PULL>
__device__ __forceinline__ int pull_node(const Args2<S, C>& a, int64_t N, int cx, int cy, C (&f)[9], C& ds, C& res) {
    const int tg = a.tag[int64_t(cy) * a.nx + cx];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int sx = PULL ? wrap1(cx - kEx[i], a.nx) : cx, sy = PULL ? wrap1(cy - kEy[i], a.ny) : cy;
        f[i] = ldp<S, C>(a.fa, i, N, int64_t(sy) * a.nx + sx);
    }
    ds = C(0);
    res = C(0);
    if (PULL) {
        const bool bnd = tg > 0;
        if (__any(bnd)) {
            C rec[RF2 + 8], ca[Q2_LINKS];
            const int64_t bi = bnd ? int64_t(tg >> 8) : 0;
#pragma unroll
            for (int k = 0; k < RF2 + 8; ++k) rec[k] = bnd ? a.rin[bi * REC2 + k] : C(0);
#pragma unroll
            for (int k = 0; k < Q2_LINKS; ++k) ca[k] = bnd ? a.la[bi * Q2_LINKS + k] : C(NO_LINK);
            ds = apply_links<S, C>(bnd, rec, ca, f, a.kF, a.k18, res);
        }
    }
    return tg;
}

// the passes over the lattice give each workgroup 256 columns of one row (blockIdx.x) of row blockIdx.y
template <class S, class C, bool PULL>
__global__ __launch_bounds__(256) void k_cp_rho(ArgsCP<S, C> p) {
    const Args2<S, C>& a = p.a;
    const int cx = blockIdx.x * 256 + threadIdx.x, cy = blockIdx.y;
    if (cx >= a.nx) return;
    const int64_t N = int64_t(a.nx) * a.ny, x = int64_t(cy) * a.nx + cx;
    C f[9], ds;
    C res;
    const int tg = pull_node<S, C, PULL>(a, N, cx, cy, f, ds, res);
    MassAcc<S, C> rs = MassAcc<S, C>(res);
#pragma unroll
    for (int i = 0; i < 9; ++i) rs += MassAcc<S, C>(f[i]);
    p.rho[x] = tg >= 0 ? C(rs) + a.rho_ref : C(0);
}

// eq. 15 for one solid layer (its n nodes in list): the lattice-weighted mean over the neighbours
// in the layer above
template <class S, class C>
__global__ __launch_bounds__(256) void k_cp_layer(ArgsCP<S, C> p, const int32_t* __restrict__ list, int64_t n, int lay) {
    const int nx = p.a.nx, ny = p.a.ny;
    for (int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; j < n; j += int64_t(gridDim.x) * blockDim.x) {
        const uint32_t x = uint32_t(list[j]);  // N < 2^31
        const int cx = int(x % uint32_t(nx)), cy = int(x / uint32_t(nx));
        // every neighbour's layer and density are loaded before any is used (one round trip), the
        // terms of the other layers are dropped by selection, so the sum keeps the direction order
        int8_t ly[8];
        C rv[8];
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const uint32_t y = uint32_t(wrap1(cy + kEy[i], ny)) * uint32_t(nx) + uint32_t(wrap1(cx + kEx[i], nx));
            ly[i - 1] = p.layer[y];
            rv[i - 1] = p.rho[y];
        }
        C num = C(0), den = C(0);
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const bool in = ly[i - 1] == lay - 1;
            num += in ? w9<C>(i) * rv[i - 1] : C(0);
            den += in ? w9<C>(i) : C(0);
        }
        p.rho[x] = num / den;
    }
}

// fourth-order central differences along an axis from the values at offsets -2 .. +2
template <class C>
__device__ __forceinline__ C cd1(C m2, C m1, C p1, C p2) {
    return (C(8) * (p1 - m1) - (p2 - m2)) * C(1.0 / 12.0);
}
template <class C>
__device__ __forceinline__ C cd2(C m2, C m1, C c, C p1, C p2) {
    return (C(16) * (p1 + m1) - (p2 + m2) - C(30) * c) * C(1.0 / 12.0);
}

// rows of one lane in the chemical-potential pass
constexpr int CP_MU_ROWS = 4;

__device__ __forceinline__ int wrapm(int v, int n) {
    const int r = v % n;
    return r < 0 ? r + n : r;
}

// chemical potential on the fluid nodes: eq. 12 with the Peng-Robinson mu of eq. 11 (the solid
// layers' values depend on the assigned ones alone and are written when those are set:
// k_cp_mu_solid).  A lane takes CP_MU_ROWS rows of one column (the workgroup 256 columns of rows
// blockIdx.y * CP_MU_ROWS ...): the column's densities over those rows and two more on either side
// serve every y stencil, and all the loads of the lane are issued before any is used.
template <class S, class C>
__global__ __launch_bounds__(256) void k_cp_mu(ArgsCP<S, C> p) {
    constexpr int R = CP_MU_ROWS;
    const int nx = p.a.nx, ny = p.a.ny;
    const C s2 = C(1.4142135623730951);
    const int cx = blockIdx.x * 256 + threadIdx.x, cy0 = blockIdx.y * R;
    if (cx >= nx) return;
    uint32_t col[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) col[d] = uint32_t(wrap1(cx + d - 2, nx));
    C cv[R + 4];  // column cx, rows cy0 - 2 .. cy0 + R + 1 (periodic)
#pragma unroll
    for (int j = 0; j < R + 4; ++j) cv[j] = p.rho[uint32_t(wrapm(cy0 - 2 + j, ny)) * uint32_t(nx) + col[2]];
    uint32_t rowb[R];
    bool fluid[R];
    C xv[R][4];  // per row: columns cx - 2, cx - 1, cx + 1, cx + 2
#pragma unroll
    for (int j = 0; j < R; ++j) {
        rowb[j] = uint32_t(cy0 + j < ny ? cy0 + j : cy0) * uint32_t(nx);
        fluid[j] = (p.layer[rowb[j] + col[2]] == 0) & (cy0 + j < ny);  // rows past the lattice: never stored
        xv[j][0] = p.rho[rowb[j] + col[0]];
        xv[j][1] = p.rho[rowb[j] + col[1]];
        xv[j][2] = p.rho[rowb[j] + col[3]];
        xv[j][3] = p.rho[rowb[j] + col[4]];
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const C r = cv[j + 2];
        const C rf = fluid[j] ? r : C(1);  // a harmless stand-in density where nothing is stored
        const C br = p.b * rf;
        if (fluid[j] && (!(rf > C(0)) || !(br < C(1)))) atomicOr(&p.a.flags[FLAG_DOMAIN], 1);
        const C iq = rcp(C(1) - br);
        const C m0 = p.RT * log(rf * iq) - p.c_log * log((s2 - C(1) + br) * rcp(s2 + C(1) - br)) +
                     p.RT * iq - p.aal * rf * rcp(C(1) + C(2) * br - br * br);
        C lap = C(0);
        lap += cd2(xv[j][0], xv[j][1], r, xv[j][2], xv[j][3]);
        lap += cd2(cv[j], cv[j + 1], r, cv[j + 3], cv[j + 4]);
        if (fluid[j]) p.mu[rowb[j] + cx] = p.k2 * m0 - p.kappa * lap;
    }
}

// chemical potential of the solid nodes: the assigned value on the wall nodes (the first solid
// layer), on the second layer the eq. 15 mean of its wall-node neighbours' assigned values, zero
// deeper; fluid nodes are left to k_cp_mu
template <class C>
__global__ __launch_bounds__(256) void k_cp_mu_solid(int nx, int ny, const int8_t* __restrict__ layer,
                                                     const int32_t* __restrict__ tag, const double* __restrict__ mus,
                                                     C* __restrict__ mu) {
    const int64_t N = int64_t(nx) * ny;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < N; x += int64_t(gridDim.x) * blockDim.x) {
        const int lay = layer[x];
        if (lay == 0) continue;
        C m = C(0);
        if (lay == 1) {
            m = C(mus[-tag[x] - 2]);
        } else if (lay == 2) {
            const int cx = int(x % nx), cy = int(x / nx);
            C num = C(0), den = C(0);
            for (int i = 1; i < 9; ++i) {
                const int64_t y = int64_t(wrap1(cy + kEy[i], ny)) * nx + wrap1(cx + kEx[i], nx);
                if (layer[y] == 1) {
                    num += w9<C>(i) * C(mus[-tag[y] - 2]);
                    den += w9<C>(i);
                }
            }
            m = num / den;
        }
        mu[x] = m;
    }
}

// ---------------------------------------------------------------- chemical-potential step in one march
// The collision of a node needs mu and rho two nodes away on each axis (eq. 9), mu of a fluid node
// rho two nodes away (eq. 12), the second solid layer's density the first layer's around it, and
// the first layer's the fluid densities around it (eq. 15): densities up to six nodes away.  A
// workgroup marches a strip of W lanes -- OUT output columns on lanes 0 .. OUT - 1 (whole cache
// lines), HC = (W - OUT) / 2 halo columns on either side -- up a segment of H rows.  LDS rings are
// indexed by the strip position p = column - (x0 - HC).  Iteration k, row r = y0 - 6 + k:
//   1  the density of row r from its pulled populations, with the node's solid layer and tag,
//      into rings.  Where eq. 18 applies, the links' f_in and the correction cancel in the sum
//      (f_in enters once and is subtracted once from f_0), leaving the node's own post-collision
//      populations on its links, whose sum its record holds; without eq. 18 (IBC) eqs. 16-17 run;
//   2  the first solid layer's density in row r - 1 (eq. 15: mean over the fluid neighbours);
//   3  the second layer's in row r - 2 (mean over the first-layer neighbours);
//   4  mu of row r - 4: eq. 12 on fluid nodes, the assigned values on the solid layers;
//   5  the collision of row r - 6: its populations pulled again with its boundary record and link
//      coefficients (issued one iteration earlier; the population lines were read six rows
//      earlier, so they come from the cache), eqs. 16-18, the eq. 9 force from the rings, the
//      collision, the store and the boundary record.
// Each phase narrows the columns it can serve by its stencil (1, 1, 2, 2): HC >= 6 covers it.  The
// per-node arithmetic and its order are those of the pass kernels above, which still produce the
// fields for the velocity output (cp_fields).
//
// Every load runs one iteration ahead of its use, and every iteration issues the same loads and
// stores in the same order: through buffer resources, a lane with nothing to load or store gets
// the offset OOB (a load reads zeros, a store is dropped), the rows past the segment are loaded
// all the same, and the collision rows before the first store at OOB.  The compiler counts the
// memory operations in flight in issue order; one that only some paths issue makes it wait, where
// the paths join, for every operation issued since, the prefetches of the next rows included.
// For the same reason the loop body ends with phase 1 of the next row, and the first row's
// phase 1 runs before the loop with every load it made waited for.
// Ring depths (rows): the densities of rows r - 8 .. r + 1 are in use at once (phase 5 reads
// r - 8 while a wave ahead writes r + 1 in the next row's phase 1), the tags of r - 5 and r + 1,
// the chemical potentials of r - 8 .. r - 4 (phase 4 writes the next one after every read of the
// oldest).  25.5 KB of LDS per 256-lane workgroup in FP32, so the VGPRs decide the occupancy.
constexpr int CP_RING = 10, CP_TRING = 8, CP_MRING = 5;

// Waves per SIMD: FP32 arithmetic with MRT fits 96 VGPRs without spilling, five waves (BGK would
// spill); FP64 fits 168 with a 20-28 byte spill, three waves instead of two (measured faster)
template <class S, class C, int W, int OUT, bool PULL, bool MRT>
__global__ __launch_bounds__(W, (sizeof(C) == 4 && MRT) ? 5 : (sizeof(C) == 8 ? 3 : 2)) void k_cp_march(ArgsCP<S, C> p) {
    constexpr int HC = (W - OUT) / 2;
    static_assert(HC >= 6, "six halo columns on either side");
    constexpr uint32_t s = sizeof(S), sc = sizeof(C), P0 = kMixed<S> ? 1 : 0;
    const Args2<S, C>& a = p.a;
    const int nx = a.nx, ny = a.ny;
    const uint32_t n = uint32_t(nx) * uint32_t(ny);  // the lattice fits the 32-bit buffer offsets
    const uint32_t ns = n * s, rows = uint32_t(nx) * s;
    // XCD-aware order, as in the pseudopotential step: each XCD takes a contiguous run of strips and
    // segments, so the strip-edge lines that neighbouring workgroups both read stay in one L2
    const int bid = blockIdx.x;
    const int per = a.nblocks >> 3, rem = a.nblocks & 7;
    const int xcd = bid & 7, k8 = bid >> 3;
    const int logical = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k8;
    const int sx = logical % a.nsx, sy = logical / a.nsx;
    const int x0 = sx * OUT, y0 = sy * a.H;
    const int Wv = min(OUT, nx - x0), Hv = min(a.H, ny - y0);
    const int t = threadIdx.x;
    const int pp = t < OUT + HC ? t + HC : t - OUT - HC;  // strip position of this lane's column
    const int cx = wrapm(x0 - HC + pp, nx);
    const bool out_col = t < Wv;
    __shared__ C s_rho[CP_RING][W];
    __shared__ int8_t s_lay[CP_RING][W];
    __shared__ int s_tag[CP_TRING][W];
    __shared__ C s_mu[CP_MRING][W];
    const __amdgpu_buffer_rsrc_t rfa = make_res(a.fa, uint64_t(9 + P0) * ns);
    const __amdgpu_buffer_rsrc_t rfb = make_res(a.fb, uint64_t(9 + P0) * ns);
    const __amdgpu_buffer_rsrc_t rtag = make_res(a.tag, uint64_t(n) * 4);
    const __amdgpu_buffer_rsrc_t rin = make_res(a.rin, uint64_t(a.n_bnodes) * REC2 * sc);
    const __amdgpu_buffer_rsrc_t rout = make_res(a.rout, uint64_t(a.n_bnodes) * REC2 * sc);
    const __amdgpu_buffer_rsrc_t rla = make_res(a.la, uint64_t(a.n_bnodes) * Q2_LINKS * sc);
    const __amdgpu_buffer_rsrc_t rmu = make_res(p.mu, uint64_t(n) * sc);
    const uint32_t xb[3] = {uint32_t(wrap1(cx - 1, nx)) * s, uint32_t(cx) * s, uint32_t(wrap1(cx + 1, nx)) * s};
    const C s2 = C(1.4142135623730951);
    const int iters = Hv + 12;
    // the sum of a boundary node's own populations on its links, which the density adds where
    // eq. 18 applies, sits in its record (the collision below puts it there); its address comes
    // from the node's tag, so the tags run one row further ahead than the pulls
    const bool link_sum = PULL && a.k18 != C(0);
    bool bad = false;

    // the populations arriving at row r of this lane's column (eq. 5), from x - e_i (PULL; otherwise
    // the node's own)
    auto pull = [&](int r, C (&f)[9]) {
        const uint32_t r0 = uint32_t(r) * rows;
        const uint32_t rowof[3] = {uint32_t(r == ny - 1 ? 0 : r + 1) * rows, r0,
                                   uint32_t(r == 0 ? ny - 1 : r - 1) * rows};  // upstream row of e_y = -1, 0, +1
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            if (kMixed<S> && i == 0) {
                f[0] = Buf<float>::ld(rfa, xb[1] * 2u, r0 * 2u);  // FP16 storage: the rest population in FP32
                continue;
            }
            const uint32_t vo = PULL ? xb[1 - kEx[i]] : xb[1];
            const uint32_t so = uint32_t(i + P0) * ns + (PULL ? rowof[kEy[i] + 1] : r0);
            f[i] = Buf<S>::ld(rfa, vo, so);
        }
    };
    auto tag_at = [&](int r) { return ld_i32(rtag, uint32_t(cx) * 4u, uint32_t(r) * uint32_t(nx) * 4u); };
    auto lsum_of = [&](int tg) {
        return Buf<C>::ld(rin, link_sum && tg > 0 ? uint32_t(tg >> 8) * (REC2 * sc) + (RF2 + 8) * sc : OOB);
    };

    // loads one iteration ahead: the density row's pull, layer and link sum, the tag of the row
    // after it; the collision row's pull, record and coefficients; the assigned chemical potential
    // of the next mu row's solid nodes
    C fD[9], fR[9], recR[RF2 + 8], aR[Q2_LINKS];
    int tgD, tgA, tgR;
    int8_t lyD;
    C slD, muN = C(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) fR[i] = C(0);
#pragma unroll
    for (int i = 0; i < RF2 + 8; ++i) recR[i] = C(0);
#pragma unroll
    for (int i = 0; i < Q2_LINKS; ++i) aR[i] = C(0);

    // ---- 1: the density of row y0 - 6 + j from the loads above, into ring slot j
    auto density = [&](int j) {
        MassAcc<S, C> rs;
        if (!PULL || a.k18 != C(0)) {
            rs = MassAcc<S, C>(0);
#pragma unroll
            for (int i = 0; i < 9; ++i) rs += MassAcc<S, C>(fD[i]);
            if (PULL) rs += MassAcc<S, C>(slD);  // zero off the boundary
        } else {
            C ds, res;
            pull_links<S, C, PULL>(a, tgD, fD, ds, res);
            rs = MassAcc<S, C>(res);
#pragma unroll
            for (int i = 0; i < 9; ++i) rs += MassAcc<S, C>(fD[i]);
        }
        s_rho[j % CP_RING][pp] = tgD >= 0 ? C(rs) + a.rho_ref : C(0);
        s_lay[j % CP_RING][pp] = lyD;
        s_tag[j % CP_TRING][pp] = tgD;
    };
    {
        const int rf = wrapm(y0 - 6, ny);
        pull(rf, fD);
        tgD = tag_at(rf);
        lyD = p.layer[int64_t(rf) * nx + cx];
        tgA = tag_at(wrapm(y0 - 5, ny));
        slD = lsum_of(tgD);
        density(0);
        asm volatile("" ::"v"(tgA));  // waited for here: nothing from before the loop is in flight in it
    }

    for (int k = 0; k < iters; ++k) {
        const int r = wrapm(y0 - 6 + k, ny);
        auto slot = [&](int d) { return (k - d + 16 * CP_RING) % CP_RING; };  // ring slot of row r - d
        auto mslot = [&](int d) { return (k - d + 16 * CP_MRING) % CP_MRING; };
        // the next density row r + 1: its pull, layer and link sum; the tag of row r + 2
        {
            const int r1 = r == ny - 1 ? 0 : r + 1;
            pull(r1, fD);
            lyD = p.layer[int64_t(r1) * nx + cx];
            tgD = tgA;
            slD = lsum_of(tgD);
            tgA = tag_at(r1 == ny - 1 ? 0 : r1 + 1);
        }
        __syncthreads();
        // ---- 2: first solid layer of row r - 1 (eq. 15 over the fluid neighbours)
        if (k >= 1 && pp >= 1 && pp < W - 1 && s_lay[slot(1)][pp] == 1) {
            C num = C(0), den = C(0);
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                const int sl = slot(1 - kEy[i]);  // row r - 1 + e_y
                const bool in = s_lay[sl][pp + kEx[i]] == 0;
                const C v = s_rho[sl][pp + kEx[i]];
                num += in ? w9<C>(i) * v : C(0);
                den += in ? w9<C>(i) : C(0);
            }
            s_rho[slot(1)][pp] = num / den;
        }
        __syncthreads();
        // ---- 3: second solid layer of row r - 2 (over the first-layer neighbours)
        if (k >= 3 && pp >= 2 && pp < W - 2 && s_lay[slot(2)][pp] == 2) {
            C num = C(0), den = C(0);
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                const int sl = slot(2 - kEy[i]);
                const bool in = s_lay[sl][pp + kEx[i]] == 1;
                const C v = s_rho[sl][pp + kEx[i]];
                num += in ? w9<C>(i) * v : C(0);
                den += in ? w9<C>(i) : C(0);
            }
            s_rho[slot(2)][pp] = num / den;
        }
        __syncthreads();
        // ---- 4: chemical potential of row r - 4 (eq. 12 with the Peng-Robinson mu of eq. 11 on
        // fluid nodes; the solid layers keep their assigned values)
        if (k >= 6 && pp >= 4 && pp < W - 4) {
            const int lay = s_lay[slot(4)][pp];
            C m;
            if (lay == 0) {
                const C rc = s_rho[slot(4)][pp];
                const C br = p.b * rc;
                if (!(rc > C(0)) || !(br < C(1))) bad = true;
                const C rf = rc > C(0) && br < C(1) ? rc : C(1);  // a harmless stand-in past the domain
                const C brf = p.b * rf;
                const C iq = rcp(C(1) - brf);
                const C m0 = p.RT * log(rf * iq) - p.c_log * log((s2 - C(1) + brf) * rcp(s2 + C(1) - brf)) +
                             p.RT * iq - p.aal * rf * rcp(C(1) + C(2) * brf - brf * brf);
                C lap = C(0);
                lap += cd2(s_rho[slot(4)][pp - 2], s_rho[slot(4)][pp - 1], rc, s_rho[slot(4)][pp + 1], s_rho[slot(4)][pp + 2]);
                lap += cd2(s_rho[slot(6)][pp], s_rho[slot(5)][pp], rc, s_rho[slot(3)][pp], s_rho[slot(2)][pp]);
                m = p.k2 * m0 - p.kappa * lap;
            } else {
                m = muN;  // loaded where the same test held (below, one iteration earlier)
            }
            s_mu[mslot(4)][pp] = m;
        }
        // the assigned potential of the solid nodes of row r - 3 (their layers are in the ring); a
        // lane at OOB may read any word, which the test above never takes
        {
            const bool want = k + 1 >= 6 && pp >= 4 && pp < W - 4 && s_lay[slot(3)][pp] != 0;
            muN = Buf<C>::ld(rmu, want ? uint32_t(cx) * sc : OOB, uint32_t(wrapm(r - 3, ny)) * uint32_t(nx) * sc);
        }
        __syncthreads();
        // ---- 5: collision of row r - 6 (pulled again, issued one iteration earlier)
        {
            C out[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) out[i] = C(0);
            uint32_t xst = OOB;
            if (k >= 12) {
                const int rc6 = wrapm(r - 6, ny);
                auto R = [&](int dx, int dy) { return s_rho[slot(6 - dy)][pp + dx]; };
                auto U = [&](int dx, int dy) { return s_mu[mslot(6 - dy)][pp + dx]; };
                C ds, res;
                const int tg = tgR;
                C f[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) f[i] = fR[i];
                links_from<S, C, PULL>(a, tg, f, recR, aR, ds, res);
                const bool coll = out_col && tg >= 0;
                MassAcc<S, C> rs = MassAcc<S, C>(res);
#pragma unroll
                for (int i = 0; i < 9; ++i) rs += MassAcc<S, C>(f[i]);
                C Fx = C(0), Fy = C(0);
                if (out_col) {
                    const C rr = R(0, 0);
                    Fx = -rr * cd1(U(-2, 0), U(-1, 0), U(1, 0), U(2, 0)) + cd1(R(-2, 0), R(-1, 0), R(1, 0), R(2, 0)) / C(3);
                    Fy = -rr * cd1(U(0, -2), U(0, -1), U(0, 1), U(0, 2)) + cd1(R(0, -2), R(0, -1), R(0, 1), R(0, 2)) / C(3);
                }
                C o[9];
                C rho, dux, duy, sx2, sy2, duu15;
                collide9<S, C, MRT>(a, coll, f, rs, coll ? Fx : C(0), coll ? Fy : C(0), o, rho, dux, duy, sx2, sy2, duu15);
#pragma unroll
                for (int i = 0; i < 9; ++i) out[i] = coll ? o[i] : C(0);
                xst = out_col ? uint32_t(rc6) * rows + xb[1] : OOB;
                // the boundary record, by the waves that hold a boundary node (its stores follow
                // every load that a later wait is for, so they may be skipped)
                if (__any(coll && tg > 0)) {
                    C rv[REC2];
                    rv[0] = rho;
                    rv[1] = dux;
                    rv[2] = duy;
                    rv[3] = sx2;
                    rv[4] = sy2;
                    rv[5] = duu15;
#pragma unroll
                    for (int i = 1; i < 9; ++i) rv[RF2 + i - 1] = out[i];
                    // the populations on the node's links (tag bits 0 .. 7), summed in the order
                    // the density of the next step would sum them from the slots above
                    C sl = C(0);
#pragma unroll
                    for (int j = 0; j < 8; ++j) sl += ((tg >> j) & 1) ? out[j + 1] : C(0);
                    rv[RF2 + 8] = sl;
                    rv[RF2 + 9] = ds;
                    st_vec(rout, coll && tg > 0 ? uint32_t(tg >> 8) * (REC2 * sc) : OOB, rv);
                }
            }
            // every output column stores, solid nodes included (zeros)
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if (kMixed<S> && i == 0)
                    Buf<float>::st_nt(rfb, xst == OOB ? OOB : xst * 2u, out[0]);
                else
                    Buf<S>::st_nt(rfb, sat_add(xst, uint32_t(i + P0) * ns), out[i]);
            }
        }
        // the collision row of the next iteration, r - 5: its tag from the ring (row r - 5 was the
        // density row five iterations ago; before the first collision row the slot may hold what
        // nothing wrote, so the tag is taken as solid there), its pull, record and coefficients
        {
            tgR = k + 1 >= 12 ? s_tag[(k + 3) % CP_TRING][pp] : -1;
            pull(wrapm(r - 5, ny), fR);
            // only waves that hold a boundary node in that row load them (16-byte loads cost
            // address cycles even at OOB); elsewhere the registers keep values nothing reads
            if (PULL && __any(tgR > 0)) {
                const bool bnd = tgR > 0;
                const uint32_t bo = uint32_t(tgR >> 8);
                ld_vec(rin, bnd ? bo * (REC2 * sc) : OOB, recR);
                ld_vec(rla, bnd ? bo * (Q2_LINKS * sc) : OOB, aR);
            }
        }
        density(k + 1);  // row r + 1 (the last iteration's is never read)
    }
    if (bad) atomicOr(&a.flags[FLAG_DOMAIN], 1);
}

inline unsigned cp_grid(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    return unsigned(b < 1 ? 1 : b);
}


// the arguments of the chemical-potential kernels for one step from fcur / rcur to fnext / rnext
template <class S, class C>
ArgsCP<S, C> cp_args(mcb_ctx* c, const void* fcur, const void* rcur, void* fnext, void* rnext) {
    ArgsCP<S, C> p;
    Args2<S, C>& a = p.a;
    a.fa = static_cast<const S*>(fcur);
    a.fb = static_cast<S*>(fnext);
    a.tag = reinterpret_cast<const int32_t*>(c->lat + c->L.tag);
    a.rin = static_cast<const C*>(rcur);
    a.rout = static_cast<C*>(rnext);
    a.la = reinterpret_cast<const C*>(c->lk + c->L.lk_a);
    a.fac = nullptr;
    a.flags = reinterpret_cast<int32_t*>(c->lat + c->L.flags);
    a.n_bnodes = uint32_t(c->n_bnodes > 0 ? c->n_bnodes : 0);
    a.n_wall = uint32_t(c->n_wall > 0 ? c->n_wall : 0);
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.H = a.nsx = a.nblocks = 0;
    a.tau_inv = C(1.0 / c->p.tau);
    a.G = C(0);
    a.rho_ref = c->p.precision == MCB_F64 ? C(0) : C(c->p.rho_ref);
    a.kF = c->p.bc_mode == MCB_BC_PRESENT ? C(1) : C(0);
    a.k18 = c->p.bc_mode == MCB_BC_IBC ? C(0) : C(1);
    a.s_e = C(c->p.s_e);
    a.s_eps = C(c->p.s_eps);
    a.s_q = C(c->p.s_q);
    a.gx = C(c->p.gravity[0]);
    a.gy = C(c->p.gravity[1]);
    a.eos = Eos<C>{};
    p.rho = reinterpret_cast<C*>(c->lat + c->L.cp_rho);
    p.mu = reinterpret_cast<C*>(c->lat + c->L.cp_mu);
    p.layer = reinterpret_cast<const int8_t*>(c->lat + c->L.cp_layer);
    p.mus = reinterpret_cast<const double*>(c->lk + c->L.wl_phi);
    const double T = c->p.eos_T, Tc = pr_tc(c->p.eos_a, c->p.eos_b, c->p.eos_R);
    const double om = c->p.pr_omega, mm = 0.37464 + 1.54226 * om - 0.26992 * om * om;
    const double sa = 1.0 + mm * (1.0 - std::sqrt(T / Tc));
    const double aal = c->p.eos_a * sa * sa;
    p.k2 = C(c->p.cp_k * c->p.cp_k);
    p.kappa = C(c->p.cp_kappa);
    p.RT = C(c->p.eos_R * T);
    p.b = C(c->p.eos_b);
    p.c_log = C(aal / (2.0 * std::sqrt(2.0) * c->p.eos_b));
    p.aal = C(aal);
    return p;
}

// The density and chemical-potential fields of a collision from the populations fpre (pulled with
// eqs. 16-18 from the records rpre when pull) into the context's field buffers: the pass kernels.
// The march keeps the fields in LDS; the velocity output asks for them through cp_fields.
template <class S, class C>
hipError_t cp_fields_t(mcb_ctx* c, const void* fpre, const void* rpre, bool pull) {
    ArgsCP<S, C> p = cp_args<S, C>(c, fpre, rpre, nullptr, nullptr);
    const dim3 grid(unsigned((c->p.nx + 255) / 256), unsigned(c->p.ny)), blk(256);
    if (pull)
        hipLaunchKernelGGL((k_cp_rho<S, C, true>), grid, blk, 0, c->stream, p);
    else
        hipLaunchKernelGGL((k_cp_rho<S, C, false>), grid, blk, 0, c->stream, p);
    if (c->n_wall > 0)
        hipLaunchKernelGGL((k_cp_layer<S, C>), dim3(cp_grid(c->n_wall)), blk, 0, c->stream, p,
                           reinterpret_cast<const int32_t*>(c->lk + c->L.wl_node), c->n_wall, 1);
    if (c->n_l2 > 0)
        hipLaunchKernelGGL((k_cp_layer<S, C>), dim3(cp_grid(c->n_l2)), blk, 0, c->stream, p,
                           reinterpret_cast<const int32_t*>(c->lat + c->L.cp_l2), c->n_l2, 2);
    hipLaunchKernelGGL((k_cp_mu<S, C>), dim3(grid.x, unsigned((c->p.ny + CP_MU_ROWS - 1) / CP_MU_ROWS)), blk, 0,
                       c->stream, p);
    return hipGetLastError();
}

template <class S, class C, int W, int OUT>
hipError_t launch_cp_w(mcb_ctx* c, const void* fcur, const void* rcur, void* fnext, void* rnext, bool pull) {
    ArgsCP<S, C> p = cp_args<S, C>(c, fcur, rcur, fnext, rnext);
    Args2<S, C>& a = p.a;
    const bool mrt = c->p.collision == MCB_COLL_MRT;
    a.nsx = (a.nx + OUT - 1) / OUT;
    // segment height: the whole grid resident at once (the twelve halo rows of a segment are then
    // spread over as few segments as the device allows), at least 32 rows
    int* occ = c->occ;  // slots 0, 1 (the pseudopotential step's; a context runs one model)
    const int cap = mrt ? resident_blocks(c, k_cp_march<S, C, W, OUT, true, true>, W, &occ[1])
                        : resident_blocks(c, k_cp_march<S, C, W, OUT, true, false>, W, &occ[0]);
    const int per = cap / a.nsx > 0 ? cap / a.nsx : 1;
    int H = (a.ny + per - 1) / per;
    if (H < 32) H = 32;
    a.H = H;
    a.nblocks = a.nsx * ((a.ny + H - 1) / H);
    const dim3 grid(unsigned(a.nblocks)), blk(W);
    if (pull && mrt)
        hipLaunchKernelGGL((k_cp_march<S, C, W, OUT, true, true>), grid, blk, 0, c->stream, p);
    else if (pull)
        hipLaunchKernelGGL((k_cp_march<S, C, W, OUT, true, false>), grid, blk, 0, c->stream, p);
    else if (mrt)
        hipLaunchKernelGGL((k_cp_march<S, C, W, OUT, false, true>), grid, blk, 0, c->stream, p);
    else
        hipLaunchKernelGGL((k_cp_march<S, C, W, OUT, false, false>), grid, blk, 0, c->stream, p);
    return hipGetLastError();
}

template <class S, class C>
hipError_t launch_cp(mcb_ctx* c, const void* fcur, const void* rcur, void* fnext, void* rnext, bool pull) {
    // as for the pseudopotential step: one-wave strips keep small lattices busy, large lattices take
    // strips of whole cache lines (224 FP32 / FP64 columns, 192 FP16) with 16 halo columns a side
    if (c->g.N <= (int64_t(1) << 21)) return launch_cp_w<S, C, 64, 52>(c, fcur, rcur, fnext, rnext, pull);
    if (sizeof(S) == 2) return launch_cp_w<S, C, 256, 192>(c, fcur, rcur, fnext, rnext, pull);
    return launch_cp_w<S, C, 256, 224>(c, fcur, rcur, fnext, rnext, pull);
}

}  // namespace

hipError_t cp_fields(mcb_ctx* c, const void* fpre, const void* rpre, bool pull) {
    switch (c->p.precision) {
        case MCB_F64: return cp_fields_t<double, double>(c, fpre, rpre, pull);
        case MCB_F32S: return cp_fields_t<float, float>(c, fpre, rpre, pull);
        default: return cp_fields_t<__half, float>(c, fpre, rpre, pull);
    }
}

hipError_t cp_wall_mu(mcb_ctx* c) {
    if (c->p.model != MCB_MODEL_CHEMPOT) return hipSuccess;
    const int8_t* layer = reinterpret_cast<const int8_t*>(c->lat + c->L.cp_layer);
    const int32_t* tag = reinterpret_cast<const int32_t*>(c->lat + c->L.tag);
    const double* mus = reinterpret_cast<const double*>(c->lk + c->L.wl_phi);
    const dim3 grid(cp_grid(c->g.N)), blk(256);
    if (c->p.precision == MCB_F64)
        hipLaunchKernelGGL(k_cp_mu_solid<double>, grid, blk, 0, c->stream, c->p.nx, c->p.ny, layer, tag, mus,
                           reinterpret_cast<double*>(c->lat + c->L.cp_mu));
    else
        hipLaunchKernelGGL(k_cp_mu_solid<float>, grid, blk, 0, c->stream, c->p.nx, c->p.ny, layer, tag, mus,
                           reinterpret_cast<float*>(c->lat + c->L.cp_mu));
    return hipGetLastError();
}

hipError_t step2d(mcb_ctx* c, const void* fcur, const void* rcur, void* fnext, void* rnext, bool pull) {
    if (c->p.model == MCB_MODEL_CHEMPOT) {
        switch (c->p.precision) {
            case MCB_F64: return launch_cp<double, double>(c, fcur, rcur, fnext, rnext, pull);
            case MCB_F32S: return launch_cp<float, float>(c, fcur, rcur, fnext, rnext, pull);
            default: return launch_cp<__half, float>(c, fcur, rcur, fnext, rnext, pull);
        }
    }
    switch (c->p.precision) {
        case MCB_F64: return launch_step2d<double, double>(c, fcur, rcur, fnext, rnext, pull);
        case MCB_F32S: return launch_step2d<float, float>(c, fcur, rcur, fnext, rnext, pull);
        default: return launch_step2d<__half, float>(c, fcur, rcur, fnext, rnext, pull);
    }
}

}  // namespace mcb
