// D2Q9 hot path: one fused kernel per time step -- pull-streaming (eq. 5), the multiphase curved
// boundary on every fluid-solid link (eqs. 16-17) with the mass modification (eq. 18), density,
// the pseudopotential with first-layer wall densities (eq. 15), the interaction force, and the
// single-relaxation-time collision with exact-difference forcing (eqs. 4, 13-14).
//
// Layout: a workgroup (4 waves, 256 lanes) owns a strip of 256 consecutive columns and a segment
// of H rows, and marches up the segment one row per iteration.  Each iteration
//   A  pulls the populations of the next row (own columns plus two halo columns on each side) and
//      puts rho and the node tag into a 4-row LDS ring; a population arriving across a link is
//      pulled as its bounce-back value, which already gives the node's density at t+1;
//   B  computes psi one row behind (wall nodes: eq. 15 average of their fluid neighbours times
//      phi) into a second 4-row LDS ring;
//   C  two rows behind, applies the link corrections of eqs. 16-18 at boundary nodes, evaluates the
//      force stencil from the psi ring and collides the populations pulled two iterations earlier
//      (kept in registers), then stores them.
// Per node only the populations (read once, written once) and a 4-byte tag reach HBM; rho and psi
// live in LDS.  Halo rows and columns are re-pulled by the neighbouring workgroup and hit in L2 or
// the Infinity Cache.  Node tags are fetched one row ahead, so no load waits on another.
#include "kernels_common.h"

namespace mcb {
namespace {

template <class S, class C>
struct Args2 {
    const S* fa;                 // post-collision populations of time t, SoA [9][N]
    S* fb;                       // post-collision populations of time t+1
    const int32_t* tag;          // >0: (boundary index << 8) | link bits; 0 fluid; -1 solid; -2-w wall w
    const int32_t* bn_link0;     // first link of each boundary node
    const uint32_t* lk_qc;       // q_fixed | class << 30, per link
    C* lk_F;                     // eq. 13 term of the link direction: read at t, rewritten at t+1
    double* dm;                  // eq. 18 correction per boundary node (for the monitor)
    const double* phi;           // wettability factor per wall node
    int32_t* flags;
    uint64_t f_bytes;            // bytes of one population lattice
    uint32_t n_bnodes, n_links, n_wall;
    int nx, ny, H, nsx, nblocks;
    C tau_inv, G, rho_ref;
    Eos<C> eos;
};

// D2Q9 weights
template <class C>
__device__ inline C w9(int i) {
    return i == 0 ? C(4.0 / 9.0) : (i < 5 ? C(1.0 / 9.0) : C(1.0 / 36.0));
}

__device__ constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

struct Res2 {
    __amdgpu_buffer_rsrc_t fa, fb, tag, l0, qc, F, dm, phi;
};

// Issue the loads of the nine populations arriving at (c, r) (eq. 5).  A population whose upstream
// node is solid travelled along a link (x, j) with j its opposite; it is taken as its bounce-back
// value f~_j(x, t), which gives the node's density at t+1 exactly: eq. 18 returns to f_0 whatever the
// curved-boundary value of eqs. 16-17 adds to or takes from that population, and that correction is
// applied just before the collision.  PULL = false reads the node's own populations (the collision
// that starts a run).  Solid nodes read nothing (their loads return 0).
template <class S, class C, bool PULL>
__device__ inline void pull_node(const Res2& R, int nx, int ny, int c, int r, int tg, C f[9]) {
    const uint32_t n = uint32_t(nx) * uint32_t(ny);
    const uint32_t x = uint32_t(r) * nx + c;
    const bool solid = tg < 0;
    constexpr uint32_t s = sizeof(S);
    if (PULL) {
        const uint32_t cm = c == 0 ? nx - 1 : c - 1, cp = c == nx - 1 ? 0 : c + 1;
        const uint32_t o0 = uint32_t(r) * nx;
        const uint32_t om = uint32_t(r == 0 ? ny - 1 : r - 1) * nx;
        const uint32_t op = uint32_t(r == ny - 1 ? 0 : r + 1) * nx;
        const uint32_t src[9] = {o0 + c, o0 + cm, om + c, o0 + cp, op + c, om + cm, om + cp, op + cp, op + cm};
        const uint32_t m = tg > 0 ? uint32_t(tg) & 0xFFu : 0u;  // bit j-1: x + e_j is solid
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const bool bounce = i > 0 && ((m >> (kOpp[i] - 1)) & 1u);
            const uint32_t e = bounce ? uint32_t(kOpp[i]) * n + x : uint32_t(i) * n + src[i];
            f[i] = Buf<S>::ld(R.fa, solid ? OOB : e * s);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = Buf<S>::ld(R.fa, solid ? OOB : (uint32_t(i) * n + x) * s);
    }
}

// Per-workgroup state of the row march.
template <class S, class C>
struct March {
    Args2<S, C> a;
    Res2 R;
    C (*s_rho)[STRIP];
    C (*s_psi)[STRIP];
    int (*s_tag)[STRIP];
    int t, cx, nx, ny, y0, iters;
    uint32_t n;
    bool out_col;
    // pipeline registers: tags and link starts of rows r-2, r-1, r; row r+1 and r+2 in flight
    int tgA, tgB, tgC, l0A, l0B, l0C;
    int rr, rr1, tg_cur, tg_nxt, l0_cur;
    bool bad;
};

// One row of the march (iteration k, row r = y0 - 2 + k).  fC holds the pulled populations of row
// r, fB and fA those of rows r-1 and r-2; the populations of row r+1 are issued into fN.
template <class S, class C, bool PULL>
__device__ __forceinline__ void march_row(March<S, C>& M, int k, C (&fA)[9], C (&fB)[9], C (&fC)[9], C (&fN)[9]) {
    const Args2<S, C>& a = M.a;
    const Res2& R = M.R;
    const int t = M.t, nx = M.nx, ny = M.ny;
    const uint32_t n = M.n;
    constexpr uint32_t s = sizeof(S), sc = sizeof(C);
    const int slot = k & 3;
    M.tgA = M.tgB; M.tgB = M.tgC; M.tgC = M.tg_cur;
    M.l0A = M.l0B; M.l0B = M.l0C; M.l0C = M.l0_cur;
    const int tgA = M.tgA;
    // ---- link data of row r-2 (collided this iteration), in one batch; lanes without the link
    // read nothing, and waves without boundary nodes skip the address arithmetic
    const bool coll = k >= 4 && M.out_col && tgA >= 0;
    const uint32_t mA = (PULL && coll && tgA > 0) ? uint32_t(tgA) & 0xFFu : 0u;
    const int yA = ((M.y0 - 4 + k) % ny + ny) % ny;
    const uint32_t xA = uint32_t(yA) * nx + M.cx;
    const bool wave_links = PULL && __any(mA != 0u);
    uint32_t oq[8], oF[8], oo[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) oq[j] = oF[j] = oo[j] = OOB;
    if (wave_links) {
#pragma unroll
        for (int j = 1; j < 9; ++j) {
            const bool has = (mA >> (j - 1)) & 1u;
            const uint32_t li = uint32_t(M.l0A) + __popc(mA & ((1u << (j - 1)) - 1u));
            oq[j - 1] = has ? li * 4u : OOB;
            oF[j - 1] = has ? li * sc : OOB;
            oo[j - 1] = has ? (uint32_t(kOpp[j]) * n + xA) * s : OOB;
        }
    }
    uint32_t lw[8];
    C lF[8], lo[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        lw[j] = PULL ? uint32_t(ld_i32(R.qc, oq[j])) : 0u;
        lF[j] = PULL ? Buf<C>::ld(R.F, oF[j]) : C(0);
        lo[j] = PULL ? Buf<S>::ld(R.fa, oo[j]) : C(0);
    }
    // wettability factor of a wall node of row r-1 (psi below); other lanes read nothing
    const int tgm = M.s_tag[(k - 1) & 3][t];
    const double phv = Buf<double>::ld(R.phi, (k >= 1 && tgm <= -2) ? uint32_t(-tgm - 2) * 8u : OOB);
    // memory operations retire in issue order: the loads used later in this iteration go out
    // before the prefetch of the next row, so waiting for them leaves the prefetch in flight
    __builtin_amdgcn_sched_barrier(0);
    // ---- row r+1 populations, row r+2 tag, row r+1 link start
    {
        const bool more = k + 1 < M.iters;
        M.rr = M.rr1;
        M.rr1 = M.rr == ny - 1 ? 0 : M.rr + 1;
        M.tg_cur = more ? M.tg_nxt : -1;
        M.l0_cur = ld_i32(R.l0, M.tg_cur > 0 ? uint32_t(M.tg_cur >> 8) * 4u : OOB);
        pull_node<S, C, PULL>(R, nx, ny, M.cx, M.rr, M.tg_cur, fN);
        M.tg_nxt = ld_i32(R.tag, k + 2 < M.iters ? (uint32_t(M.rr1) * nx + M.cx) * 4u : OOB);
    }
    __builtin_amdgcn_sched_barrier(0);
    // ---- A: density of row r
    {
        C sr = C(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) sr += fC[i];
        M.s_rho[slot][t] = sr + a.rho_ref;
        M.s_tag[slot][t] = M.tgC;
    }
    __syncthreads();
    // ---- B: psi of row r - 1
    if (k >= 2 && t >= 1 && t < STRIP - 1) {
        const int s_mid = (k - 1) & 3, s_lo = (k - 2) & 3;
        const int tg = M.s_tag[s_mid][t];
        C rho_n;
        if (tg >= -1) {
            rho_n = M.s_rho[s_mid][t];
        } else {
            // wall node: eq. 15 over the first layer, lattice weights of the fluid neighbours
            C num = C(0), den = C(0);
            const int rows[3] = {s_lo, s_mid, slot};
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    const C w = (dx == 0 || dy == 0) ? C(1.0 / 9.0) : C(1.0 / 36.0);
                    const int sl = rows[dy + 1];
                    if (M.s_tag[sl][t + dx] >= 0) {
                        num += w * M.s_rho[sl][t + dx];
                        den += w;
                    }
                }
            rho_n = C(phv) * num / den;
        }
        M.s_psi[s_mid][t] = tg == -1 ? C(0) : psi_val(rho_n, a.eos, &M.bad);
    }
    __syncthreads();
    // ---- C: boundary links, force and collision of row r - 2; colliding lanes store
    C out[9];
    C Fl[8];
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i] = C(0);
#pragma unroll
    for (int j = 0; j < 8; ++j) Fl[j] = C(0);
    if (k >= 4) {
        if (wave_links) {
            // eqs. 16-17 on each link (x, j), from the bounce-back-pulled values:
            //   f~_j(x, t) = fA[opp j], f~_j(x2, t) = fA[j] (x2 = x - e_j fluid), f~_opp(j)(x, t) = lo;
            // eq. 18: f_0 takes back f~_j(x, t) - f_opp(j)(x, t+1).  Link j rewrites only fA[opp j];
            // fA[j] is read only when x2 is fluid, so (x, opp j) is no link and fA[j] is still the
            // pulled value.
            C dsum = C(0);
#pragma unroll
            for (int j = 1; j < 9; ++j) {
                const bool has = (mA >> (j - 1)) & 1u;
                if (!__any(has)) continue;
                const uint32_t w = lw[j - 1];
                const int cls = int(w >> CLS_SHIFT);
                const C q2 = C(w & QMASK) * C(2.0 / 65536.0);  // 2q
                const C Fj = lF[j - 1];
                const C fj = fA[kOpp[j]];
                const C f16 = q2 * fj + (C(1) - q2) * (fA[j] + Fj);
                const C f17 = (fj + (q2 - C(1)) * (lo[j - 1] + Fj)) * rcp(has && cls == MCB_CLS_EQ17 ? q2 : C(1));
                const C fin = cls == MCB_CLS_EQ16 ? f16 : (cls == MCB_CLS_EQ17 ? f17 : fj);
                fA[kOpp[j]] = has ? fin : fj;
                dsum += has ? fj - fin : C(0);
            }
            fA[0] += dsum;
            Buf<double>::st(R.dm, mA ? uint32_t(tgA >> 8) * 8u : OOB, double(dsum));
        }
        const int sl = (k - 3) & 3, sm = (k - 2) & 3, sh = (k - 1) & 3;
        const int tc = t < 1 ? 1 : (t > STRIP - 2 ? STRIP - 2 : t);
        const C p0 = M.s_psi[sm][tc];
        const C pE = M.s_psi[sm][tc + 1], pW = M.s_psi[sm][tc - 1];
        const C pN = M.s_psi[sh][tc], pS = M.s_psi[sl][tc];
        const C pNE = M.s_psi[sh][tc + 1], pNW = M.s_psi[sh][tc - 1];
        const C pSW = M.s_psi[sl][tc - 1], pSE = M.s_psi[sl][tc + 1];
        // F = -G psi(x) sum_i w^_i psi(x + e_i) e_i, w^ = 1/3 (axes), 1/12 (diagonals)
        const C gp = -a.G * p0;
        const C Fx = gp * (C(1.0 / 3.0) * (pE - pW) + C(1.0 / 12.0) * (pNE - pNW - pSW + pSE));
        const C Fy = gp * (C(1.0 / 3.0) * (pN - pS) + C(1.0 / 12.0) * (pNE + pNW - pSW - pSE));

        C rs = C(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) rs += fA[i];
        const C rho = rs + a.rho_ref;
        const C irho = rcp(coll ? rho : C(1));
        const C ux = (fA[1] - fA[3] + fA[5] - fA[6] - fA[7] + fA[8]) * irho;
        const C uy = (fA[2] - fA[4] + fA[5] + fA[6] - fA[7] - fA[8]) * irho;
        const C dux = Fx * irho, duy = Fy * irho;
        const C ti = a.tau_inv, omc = C(1) - ti;
        // per direction: out_i = f_i (1 - 1/tau) + w_i [rs/tau + rho (sym_i +- anti_i)] with
        //   sym  = (4.5 (e.u)^2 - 1.5 u^2) / tau + 4.5 (e.du)(e.(2u + du)) - 1.5 du.(2u + du)
        //   anti = 3 (e.u / tau + e.du)
        // (eq. 14 equilibrium, eq. 13 forcing term, eq. 4 with S = I / tau)
        const C uu15 = C(1.5) * (ux * ux + uy * uy);
        const C sx2 = C(2) * ux + dux, sy2 = C(2) * uy + duy;
        const C duu15 = C(1.5) * (dux * sx2 + duy * sy2);
        const C c0 = -(ti * uu15 + duu15);
        const C trs = ti * rs;
        // rest
        out[0] = fA[0] * omc + C(4.0 / 9.0) * (trs + rho * c0);
        // a pair of opposite directions with e.u = eu, e.du = ed, e.(2u + du) = es
        auto pair = [&](int ip, int im, C w, C eu, C ed, C es, C& Fp, C& Fm) {
            const C sym = ti * C(4.5) * eu * eu + C(4.5) * ed * es + c0;
            const C anti = C(3) * (ti * eu + ed);
            const C base = w * (trs + rho * sym);
            const C wra = w * rho * anti;
            out[ip] = fA[ip] * omc + base + wra;
            out[im] = fA[im] * omc + base - wra;
            // forcing terms alone, for the link directions
            const C fs = C(4.5) * ed * es - duu15;
            const C fa = C(3) * ed;
            Fp = w * rho * (fs + fa);
            Fm = w * rho * (fs - fa);
        };
        C F1, F3, F2, F4, F5, F7, F6, F8;
        pair(1, 3, C(1.0 / 9.0), ux, dux, sx2, F1, F3);
        pair(2, 4, C(1.0 / 9.0), uy, duy, sy2, F2, F4);
        pair(5, 7, C(1.0 / 36.0), ux + uy, dux + duy, sx2 + sy2, F5, F7);
        pair(6, 8, C(1.0 / 36.0), uy - ux, duy - dux, sy2 - sx2, F6, F8);
        Fl[0] = F1; Fl[1] = F2; Fl[2] = F3; Fl[3] = F4; Fl[4] = F5; Fl[5] = F6; Fl[6] = F7; Fl[7] = F8;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) Buf<S>::st(R.fb, coll ? (uint32_t(i) * n + xA) * s : OOB, out[i]);
    // the link directions keep their forcing term for eqs. 16-17 of the next step
    const uint32_t mk = (coll && tgA > 0) ? uint32_t(tgA) & 0xFFu : 0u;
    uint32_t oS[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) oS[j] = OOB;
    if (__any(mk != 0u)) {
#pragma unroll
        for (int j = 1; j < 9; ++j) {
            const bool has = (mk >> (j - 1)) & 1u;
            oS[j - 1] = has ? (uint32_t(M.l0A) + __popc(mk & ((1u << (j - 1)) - 1u))) * sc : OOB;
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) Buf<C>::st(R.F, oS[j], Fl[j]);
}

template <class S, class C, bool PULL>
__global__ __launch_bounds__(STRIP) void k_step2d(Args2<S, C> a) {
    // XCD-aware order: consecutive logical tiles go to the same XCD (one L2)
    const int bid = blockIdx.x;
    const int per = a.nblocks >> 3, rem = a.nblocks & 7;
    const int xcd = bid & 7, k8 = bid >> 3;
    const int logical = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k8;
    const int sx = logical % a.nsx, sy = logical / a.nsx;
    __shared__ C s_rho[4][STRIP];
    __shared__ C s_psi[4][STRIP];
    __shared__ int s_tag[4][STRIP];

    March<S, C> M;
    M.a = a;
    // lane t covers column x0 - 2 + t; lanes 2 .. 2 + Wv - 1 own the strip's output columns and the
    // two lanes on either side are its halo (psi needs rho two columns out, through the wall nodes)
    const int x0 = sx * STRIP_OUT;
    M.y0 = sy * a.H;
    const int Wv = min(STRIP_OUT, a.nx - x0), Hv = min(a.H, a.ny - M.y0);
    M.t = threadIdx.x;
    M.nx = a.nx;
    M.ny = a.ny;
    M.n = uint32_t(a.nx) * uint32_t(a.ny);
    M.cx = ((x0 - 2 + M.t) % a.nx + a.nx) % a.nx;
    M.out_col = M.t >= 2 && M.t < 2 + Wv;
    M.iters = Hv + 4;
    M.s_rho = s_rho;
    M.s_psi = s_psi;
    M.s_tag = s_tag;
    M.R.fa = make_res(a.fa, a.f_bytes);
    M.R.fb = make_res(a.fb, a.f_bytes);
    M.R.tag = make_res(a.tag, uint64_t(M.n) * 4);
    M.R.l0 = make_res(a.bn_link0, uint64_t(a.n_bnodes) * 4);
    M.R.qc = make_res(a.lk_qc, uint64_t(a.n_links) * 4);
    M.R.F = make_res(a.lk_F, uint64_t(a.n_links) * sizeof(C));
    M.R.dm = make_res(a.dm, uint64_t(a.n_bnodes) * 8);
    M.R.phi = make_res(a.phi, uint64_t(a.n_wall) * 8);
    M.tgA = M.tgB = M.tgC = -1;
    M.l0A = M.l0B = M.l0C = 0;
    M.bad = false;
    // row march: the populations of row r+1 and the tag of row r+2 are in flight while row r is
    // reduced to rho, row r-1 to psi and row r-2 collided; four register sets rotate
    C f0[9], f1[9], f2[9], f3[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f0[i] = f1[i] = f2[i] = C(0);
    M.rr = ((M.y0 - 2) % a.ny + a.ny) % a.ny;
    M.tg_cur = ld_i32(M.R.tag, (uint32_t(M.rr) * a.nx + M.cx) * 4u);
    M.rr1 = M.rr == a.ny - 1 ? 0 : M.rr + 1;
    M.tg_nxt = ld_i32(M.R.tag, (uint32_t(M.rr1) * a.nx + M.cx) * 4u);
    M.l0_cur = ld_i32(M.R.l0, M.tg_cur > 0 ? uint32_t(M.tg_cur >> 8) * 4u : OOB);
    pull_node<S, C, PULL>(M.R, a.nx, a.ny, M.cx, M.rr, M.tg_cur, f3);
    int k = 0;
    for (; k + 4 <= M.iters; k += 4) {
        march_row<S, C, PULL>(M, k + 0, f0, f1, f3, f2);
        march_row<S, C, PULL>(M, k + 1, f1, f3, f2, f0);
        march_row<S, C, PULL>(M, k + 2, f3, f2, f0, f1);
        march_row<S, C, PULL>(M, k + 3, f2, f0, f1, f3);
    }
    const int left = M.iters - k;  // uniform
    if (left > 0) march_row<S, C, PULL>(M, k + 0, f0, f1, f3, f2);
    if (left > 1) march_row<S, C, PULL>(M, k + 1, f1, f3, f2, f0);
    if (left > 2) march_row<S, C, PULL>(M, k + 2, f3, f2, f0, f1);
    if (M.bad) atomicOr(&a.flags[FLAG_DOMAIN], 1);
}

template <class S, class C>
hipError_t launch_step2d(mcb_ctx* c, const void* fcur, void* fnext, bool pull) {
    Args2<S, C> a;
    a.fa = static_cast<const S*>(fcur);
    a.fb = static_cast<S*>(fnext);
    a.tag = reinterpret_cast<const int32_t*>(c->lat + c->L.tag);
    a.bn_link0 = reinterpret_cast<const int32_t*>(c->lk + c->L.bn_link0);
    a.lk_qc = reinterpret_cast<const uint32_t*>(c->lk + c->L.lk_qc);
    a.lk_F = reinterpret_cast<C*>(c->lk + c->L.lk_F);
    a.dm = reinterpret_cast<double*>(c->lk + c->L.dm);
    a.phi = reinterpret_cast<const double*>(c->lk + c->L.wl_phi);
    a.flags = reinterpret_cast<int32_t*>(c->lat + c->L.flags);
    a.f_bytes = uint64_t(c->g.Q) * c->g.N * sizeof(S);
    a.n_bnodes = uint32_t(c->n_bnodes > 0 ? c->n_bnodes : 0);
    a.n_links = uint32_t(c->n_links > 0 ? c->n_links : 0);
    a.n_wall = uint32_t(c->n_wall > 0 ? c->n_wall : 0);
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.nsx = (a.nx + STRIP_OUT - 1) / STRIP_OUT;
    // segment height: long segments amortise the four halo rows; short ones fill the chip
    int H = 64;
    while (H > 8 && int64_t(a.nsx) * ((a.ny + H - 1) / H) < 2048) H >>= 1;
    a.H = H;
    a.nblocks = a.nsx * ((a.ny + H - 1) / H);
    a.tau_inv = C(1.0 / c->p.tau);
    a.G = C(c->p.G);
    a.rho_ref = c->p.precision == MCB_F64 ? C(0) : C(c->p.rho_ref);
    a.eos.RT = C(c->p.eos_R * c->p.eos_T);
    a.eos.a = C(c->p.eos_a);
    a.eos.b4 = C(c->p.eos_b / 4.0);
    a.eos.two_over_G = C(2.0 / c->p.G);
    if (pull)
        hipLaunchKernelGGL((k_step2d<S, C, true>), dim3(a.nblocks), dim3(STRIP), 0, c->stream, a);
    else
        hipLaunchKernelGGL((k_step2d<S, C, false>), dim3(a.nblocks), dim3(STRIP), 0, c->stream, a);
    return hipGetLastError();
}

}  // namespace

hipError_t step2d(mcb_ctx* c, const void* fcur, void* fnext, bool pull) {
    switch (c->p.precision) {
        case MCB_F64: return launch_step2d<double, double>(c, fcur, fnext, pull);
        case MCB_F32S: return launch_step2d<float, float>(c, fcur, fnext, pull);
        default: return launch_step2d<__half, float>(c, fcur, fnext, pull);
    }
}

}  // namespace mcb
