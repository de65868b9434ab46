// Boundary pass of a time step: the multiphase curved boundary condition (eqs. 16-17) on every
// fluid-solid link and the mass modification of eq. 18, one thread per boundary-fluid node, run
// before the fused bulk kernel.
//
// For a link (x, j) (x fluid, x + e_j solid) the population entering x along opp(j) at t+1 is
//   f_in = c1 f~_j(x, t) + c2 (o + F_j(x, t)),
//   eq. 16 (q < 1/2, x2 = x - e_j fluid): c1 = 2q,      c2 = 1 - 2q,       o = f~_j(x2, t)
//   eq. 17 (q >= 1/2):                    c1 = 1/(2q),  c2 = 1 - 1/(2q),   o = f~_opp(j)(x, t)
//   bounce-back (q < 1/2, x2 solid):      c1 = 1,       c2 = 0.
// The bulk kernel pulls population opp(j) of x from x - e_opp(j) = x + e_j, the solid node, whose
// own populations carry nothing; so f_in is written into that slot of the solid node and the
// pull picks it up with no special case.  Each such slot belongs to exactly one link.  Eq. 18 adds
// sum_links (f~_j(x, t) - f_in) to the rest population of x; the bulk kernel takes the corrected
// rest population of a boundary node from f0c.
//
// F_j(x, t) is the exact-difference forcing term (eq. 13) of direction j from the collision of x at
// time t.  It is recomputed here from the node's own post-collision populations and its force
// F(x, t), which the bulk kernel stores for boundary nodes: rho = sum_i f~_i (the collision keeps
// the mass) and rho u = sum_i f~_i e_i - F (the forcing term adds F to the momentum).
#include "kernels_common.h"

namespace mcb {
namespace {

template <class S, class C>
struct BcArgs {
    S* f;                        // post-collision populations of time t (solid slots are written)
    const int32_t* bn_node;      // boundary-fluid nodes
    const uint32_t* bn_mask;     // bit j: x + e_j is solid
    const C* lk_a;               // per slot (node, direction): c1 = |a|; a < 0 marks eq. 17
    const C* Fv;                 // force F(x, t) per boundary node, stride FS
    C* f0c;                      // corrected rest population per boundary node
    double* dm;                  // eq. 18 correction per boundary node
    GridDev g;
    int L, FS;
    int64_t nb;
    C rho_ref;
};

template <class C>
__device__ inline C wq(int L, int i) {
    if (L == 0) return i == 0 ? C(4.0 / 9.0) : (i < 5 ? C(1.0 / 9.0) : C(1.0 / 36.0));
    return i == 0 ? C(1.0 / 3.0) : (i < 7 ? C(1.0 / 18.0) : C(1.0 / 36.0));
}

template <class S, class C, int Q>
__global__ __launch_bounds__(256) void k_bc(BcArgs<S, C> a) {
    constexpr int L = Q == 9 ? 0 : 1;
    const GridDev& g = a.g;
    for (int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; b < a.nb; b += int64_t(gridDim.x) * blockDim.x) {
        const int64_t x = a.bn_node[b];
        const uint32_t mask = a.bn_mask[b];
        const int cx = int(x % g.nx), cy = int((x / g.nx) % g.ny), cz = int(x / (int64_t(g.nx) * g.ny));
        auto node = [&](int i, int sign) {
            return int64_t(wrap1(cx + sign * c_ex[L][i], g.nx)) +
                   int64_t(g.nx) * (wrap1(cy + sign * c_ey[L][i], g.ny) + int64_t(g.ny) * wrap1(cz + sign * c_ez[L][i], g.nz));
        };
        C f[Q];
        C rs = C(0), jx = C(0), jy = C(0), jz = C(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            f[i] = ld<S, C>(a.f, i * g.N + x);
            rs += f[i];
            jx += C(c_ex[L][i]) * f[i];
            jy += C(c_ey[L][i]) * f[i];
            jz += C(c_ez[L][i]) * f[i];
        }
        const C rho = rs + a.rho_ref;
        const C Fx = a.Fv[b * a.FS], Fy = a.Fv[b * a.FS + 1], Fz = Q == 19 ? a.Fv[b * a.FS + 2] : C(0);
        const C irho = C(1) / rho;
        const C ux = (jx - Fx) * irho, uy = (jy - Fy) * irho, uz = (jz - Fz) * irho;
        const C dux = Fx * irho, duy = Fy * irho, duz = Fz * irho;
        const C sx = C(2) * ux + dux, sy = C(2) * uy + duy, sz = C(2) * uz + duz;
        const C duu = C(1.5) * (dux * sx + duy * sy + duz * sz);
        C dsum = C(0);
        for (int j = 1; j < Q; ++j) {
            if (!((mask >> j) & 1u)) continue;
            const C aj = a.lk_a[b * (Q - 1) + (j - 1)];
            const C c1 = aj < C(0) ? -aj : aj, c2 = C(1) - c1;
            // eq. 13 term of direction j: w rho [3 e.du + 4.5 (e.du)(e.(2u + du)) - 1.5 du.(2u + du)]
            const C ed = C(c_ex[L][j]) * dux + C(c_ey[L][j]) * duy + C(c_ez[L][j]) * duz;
            const C es = C(c_ex[L][j]) * sx + C(c_ey[L][j]) * sy + C(c_ez[L][j]) * sz;
            const C Fj = wq<C>(L, j) * rho * (C(3) * ed + C(4.5) * ed * es - duu);
            C o = C(0);
            if (c2 != C(0)) o = aj < C(0) ? f[c_opp[L][j]] : ld<S, C>(a.f, j * g.N + node(j, -1));
            // rounded to the storage format; eq. 18 takes the value as stored
            const C fin = Buf<S>::round(c1 * f[j] + c2 * (o + Fj));
            st<S, C>(a.f, c_opp[L][j] * g.N + node(j, +1), fin);
            dsum += f[j] - fin;
        }
        a.f0c[b] = f[0] + dsum;
        a.dm[b] = double(dsum);
    }
}

template <class S, class C>
hipError_t bc_t(mcb_ctx* c, void* fcur) {
    if (c->n_bnodes <= 0) return hipSuccess;
    BcArgs<S, C> a;
    a.f = static_cast<S*>(fcur);
    a.bn_node = reinterpret_cast<const int32_t*>(c->lk + c->L.bn_node);
    a.bn_mask = reinterpret_cast<const uint32_t*>(c->lk + c->L.bn_mask);
    a.lk_a = reinterpret_cast<const C*>(c->lk + c->L.lk_a);
    a.Fv = reinterpret_cast<const C*>(c->lk + c->L.lk_Fv);
    a.f0c = reinterpret_cast<C*>(c->lk + c->L.lk_f0c);
    a.dm = reinterpret_cast<double*>(c->lk + c->L.dm);
    a.g = c->g;
    a.L = c->g.dim == 2 ? 0 : 1;
    a.FS = c->g.dim == 2 ? 2 : 4;
    a.nb = c->n_bnodes;
    a.rho_ref = c->p.precision == MCB_F64 ? C(0) : C(c->p.rho_ref);
    int64_t blocks = (c->n_bnodes + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    if (c->g.dim == 2)
        hipLaunchKernelGGL((k_bc<S, C, 9>), dim3(unsigned(blocks)), dim3(256), 0, c->stream, a);
    else
        hipLaunchKernelGGL((k_bc<S, C, 19>), dim3(unsigned(blocks)), dim3(256), 0, c->stream, a);
    return hipGetLastError();
}

}  // namespace

hipError_t boundary_pass(mcb_ctx* c, void* fcur) {
    switch (c->p.precision) {
        case MCB_F64: return bc_t<double, double>(c, fcur);
        case MCB_F32S: return bc_t<float, float>(c, fcur);
        default: return bc_t<__half, float>(c, fcur);
    }
}

}  // namespace mcb
