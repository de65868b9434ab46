// Observation and set-up kernels: equilibrium initialisation, the FP64 mass / momentum monitor
// (deterministic two-pass wave64 reduction), the moment output v = u + F / (2 rho), and FP64
// host-format conversions of the stored populations.
#include "kernels_common.h"

namespace mcb {
namespace {

template <class C>
__device__ inline C wgt(int L, int i) {
    if (L == 0) return i == 0 ? C(4.0 / 9.0) : (i < 5 ? C(1.0 / 9.0) : C(1.0 / 36.0));
    return i == 0 ? C(1.0 / 3.0) : (i < 7 ? C(1.0 / 18.0) : C(1.0 / 36.0));
}

// the periodic neighbours x + e_i of node u in every direction, from per-axis offsets formed once
// (32-bit position arithmetic: N < 2^31; the direction tables fold to constants once unrolled)
template <int Q>
__device__ inline void nb_all(const GridDev& g, uint32_t u, uint32_t (&y)[Q]) {
    constexpr int L = Q == 9 ? 0 : 1;
    const uint32_t nx = uint32_t(g.nx), ny = uint32_t(g.ny), nz = uint32_t(g.nz), nxy = nx * ny;
    const uint32_t cz = u / nxy, r = u - cz * nxy, cy = r / nx, cx = r - cy * nx;
    const uint32_t xo[3] = {cx == 0 ? nx - 1 : cx - 1, cx, cx + 1 == nx ? 0 : cx + 1};
    const uint32_t yo[3] = {(cy == 0 ? ny - 1 : cy - 1) * nx, cy * nx, (cy + 1 == ny ? 0 : cy + 1) * nx};
    const uint32_t zo[3] = {(cz == 0 ? nz - 1 : cz - 1) * nxy, cz * nxy, (cz + 1 == nz ? 0 : cz + 1) * nxy};
#pragma unroll
    for (int i = 0; i < Q; ++i) y[i] = xo[c_ex[L][i] + 1] + yo[c_ey[L][i] + 1] + zo[c_ez[L][i] + 1];
}

// f(x, 0) = f^eq(rho, u) - w_i rho_ref on fluid nodes (eq. 14), zero elsewhere
template <class S, class C>
__global__ void k_init_feq(GridDev g, int L, const int32_t* __restrict__ tag, const double* __restrict__ rho,
                           const double* __restrict__ u, C rho_ref, S* __restrict__ f) {
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < g.N; x += int64_t(gridDim.x) * blockDim.x) {
        if (tag[x] < 0) {
            for (int i = 0; i < g.Q; ++i) stp<S, C>(f, i, g.N, x, C(0));
            continue;
        }
        const C r = C(rho[x]);
        C uv[3] = {C(0), C(0), C(0)};
        if (u)
            for (int k = 0; k < g.dim; ++k) uv[k] = C(u[k * g.N + x]);
        const C uu = uv[0] * uv[0] + uv[1] * uv[1] + uv[2] * uv[2];
        for (int i = 0; i < g.Q; ++i) {
            const C eu = C(c_ex[L][i]) * uv[0] + C(c_ey[L][i]) * uv[1] + C(c_ez[L][i]) * uv[2];
            const C w = wgt<C>(L, i);
            const C geq = w * (r - rho_ref) + w * r * (C(3) * eu + C(4.5) * eu * eu - C(1.5) * uu);
            stp<S, C>(f, i, g.N, x, geq);
        }
    }
}

__device__ inline double wave_sum(double v) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// pass 1: fixed grid of MON_BLOCKS workgroups, fixed node assignment -> deterministic partials.
// A lane loads a node's tag and all Q populations together and selects by the tag (solid nodes
// add nothing), so one memory round trip serves the node; the sums keep the direction order.
template <class S, class C, int Q>
__global__ __launch_bounds__(256) void k_mon_partial(GridDev g, const S* __restrict__ f, const int32_t* __restrict__ tag,
                                                     double rho_ref, const C* __restrict__ rec, int rec_stride,
                                                     int64_t nb, double* __restrict__ partials) {
    constexpr int L = Q == 9 ? 0 : 1;
    double acc[MON_FIELDS] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < g.N; x += stride) {
        const bool fl = tag[x] >= 0;
        double v[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = double(ldp<S, C>(f, i, g.N, x));
        double m = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            m += v[i];
            jx += v[i] * c_ex[L][i];
            jy += v[i] * c_ey[L][i];
            jz += v[i] * c_ez[L][i];
        }
        m += rho_ref;
        acc[0] += fl ? m : 0.0;
        acc[1] += fl ? jx : 0.0;
        acc[2] += fl ? jy : 0.0;
        acc[3] += fl ? jz : 0.0;
        if (fl && (!isfinite(m) || !isfinite(jx) || !isfinite(jy) || !isfinite(jz))) acc[5] += 1.0;
    }
    // eq. 18 corrections that the last step applied, from the boundary records of the state
    const int ds = rec_stride - 1;
    for (int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; b < nb; b += stride) acc[4] += double(rec[b * rec_stride + ds]);
    __shared__ double red[MON_FIELDS][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < MON_FIELDS; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) red[k][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < MON_FIELDS) {
        const int k = threadIdx.x;
        partials[blockIdx.x * MON_FIELDS + k] = ((red[k][0] + red[k][1]) + red[k][2]) + red[k][3];
    }
}

// pass 2: one workgroup, fixed order
__global__ __launch_bounds__(256) void k_mon_final(const double* __restrict__ partials, int nparts, double* __restrict__ out) {
    __shared__ double red[MON_FIELDS][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < MON_FIELDS; ++k) {
        double s = 0;
        for (int p = threadIdx.x; p < nparts; p += blockDim.x) s += partials[p * MON_FIELDS + k];
        s = wave_sum(s);
        if (lane == 0) red[k][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < MON_FIELDS) {
        const int k = threadIdx.x;
        out[k] = ((red[k][0] + red[k][1]) + red[k][2]) + red[k][3];
    }
}

// ---- per-node moment arithmetic, shared by the moment output and the one-pass largest speed, so
// that the two give bit-identical velocities
// density of a fluid node from its populations (stored format, shifted by w_i rho_ref)
template <int Q>
__device__ __forceinline__ double node_rho(const double (&v)[Q], double rho_ref) {
    double s = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) s += v[i];
    return s + rho_ref;
}

// eq. 15: the density of a wall node, phi times the weighted mean density of its fluid neighbours
// (neighbour i: tag ty[i], density ry[i])
template <int Q>
__device__ __forceinline__ double wall_rho(const int (&ty)[Q], const double (&ry)[Q], double phi) {
    constexpr int L = Q == 9 ? 0 : 1;
    double num = 0, den = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        num += ty[i] >= 0 ? wgt<double>(L, i) * ry[i] : 0.0;
        den += ty[i] >= 0 ? wgt<double>(L, i) : 0.0;
    }
    return phi * (num / den);
}

// momentum j = sum_i f_i e_i of a node
template <int Q>
__device__ __forceinline__ void node_j(const double (&fv)[Q], double (&j)[3]) {
    constexpr int L = Q == 9 ? 0 : 1;
    j[0] = j[1] = j[2] = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int e[3] = {c_ex[L][i], c_ey[L][i], c_ez[L][i]};
        for (int k = 0; k < 3; ++k) j[k] += fv[i] * e[k];
    }
}

// v = (j - F / 2) / rho, F = -G psi(x) sum_i w^_i psi(x + e_i) e_i + rho g (pv[i] = psi(x + e_i))
template <int Q>
__device__ __forceinline__ void node_v(const double (&j)[3], const double (&pv)[Q], double psi_x, double rho_x, double G,
                                       const double (&gk)[3], int dim, double (&v)[3]) {
    constexpr int L = Q == 9 ? 0 : 1;
    double s[3] = {0, 0, 0};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const double ws = (L == 0) ? (i < 5 ? 1.0 / 3.0 : 1.0 / 12.0) : (i < 7 ? 1.0 / 6.0 : 1.0 / 12.0);
        const int e[3] = {c_ex[L][i], c_ey[L][i], c_ez[L][i]};
        for (int k = 0; k < 3; ++k) s[k] += ws * pv[i] * e[k];
    }
    v[0] = v[1] = v[2] = 0.0;
    const double ir = 1.0 / rho_x;
    for (int k = 0; k < dim; ++k) {
        const double F = -G * psi_x * s[k] + rho_x * gk[k];
        v[k] = (j[k] - 0.5 * F) * ir;
    }
}

// ---- moments: rho, psi (fluid and wall nodes), then v = (j - F / 2) / rho.  Q is a template
// parameter (unrolled direction loops); each lane loads all it needs before using any.
// k_rho_out: the density alone (the chemical-potential model's velocity needs no psi)
template <class S, class C, int Q>
__global__ __launch_bounds__(256) void k_rho_out(GridDev g, const S* __restrict__ f, const int32_t* __restrict__ tag,
                                                 double rho_ref, double* __restrict__ rho) {
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < g.N; x += int64_t(gridDim.x) * blockDim.x) {
        const bool fl = tag[x] >= 0;
        double v[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = double(ldp<S, C>(f, i, g.N, x));
        rho[x] = fl ? node_rho<Q>(v, rho_ref) : 0.0;
    }
}

// rho and psi in one pass: psi(rho) on fluid nodes, zero on solid ones (wall nodes too, until
// k_psi_wall gives them eq. 15's psi once every density is written)
template <class S, class C, int Q>
__global__ __launch_bounds__(256) void k_rho_psi_out(GridDev g, const S* __restrict__ f, const int32_t* __restrict__ tag,
                                                     double rho_ref, Eos<double> eos, int32_t* flags,
                                                     double* __restrict__ rho, double* __restrict__ psi) {
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < g.N; x += int64_t(gridDim.x) * blockDim.x) {
        const bool fl = tag[x] >= 0;
        double v[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = double(ldp<S, C>(f, i, g.N, x));
        const double r = fl ? node_rho<Q>(v, rho_ref) : 0.0;
        rho[x] = r;
        psi[x] = fl ? psi_of(r, eos, flags) : 0.0;
    }
}

// psi of the wall nodes (solid nodes with a fluid neighbour, listed in wl_node): eq. 15's density
// from the neighbours' tags and densities, the solid ones dropped by selection
template <int Q>
__global__ __launch_bounds__(256) void k_psi_wall(GridDev g, int64_t nw, const int32_t* __restrict__ wl_node,
                                                  const int32_t* __restrict__ tag, const double* __restrict__ rho,
                                                  const double* __restrict__ phi, Eos<double> eos, int32_t* flags,
                                                  double* __restrict__ psi) {
    for (int64_t w = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; w < nw; w += int64_t(gridDim.x) * blockDim.x) {
        const int64_t x = wl_node[w];
        uint32_t nb[Q];
        nb_all<Q>(g, uint32_t(x), nb);
        int ty[Q];
        double ry[Q];
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            ty[i] = tag[nb[i]];
            ry[i] = rho[nb[i]];
        }
        psi[x] = psi_of(wall_rho<Q>(ty, ry, phi[w]), eos, flags);
    }
}

// the nodes of a lane in a grid-stride loop.  Workgroups are dealt to the eight XCDs in turn; with
// slabs (a grid of a multiple of 8) each XCD sweeps a contiguous eighth of the lattice instead of
// every eighth row-piece of it, so the rows of neighbours that nodes share are fetched into one L2
// rather than into several
struct Sweep {
    int64_t x0, xe, xs;
};

__device__ inline Sweep sweep(int64_t N, bool slabs) {
    if (!slabs || gridDim.x % 8 != 0)
        return {blockIdx.x * int64_t(blockDim.x) + threadIdx.x, N, int64_t(gridDim.x) * blockDim.x};
    const int64_t slab = (N + 7) / 8, k = blockIdx.x % 8;
    return {k * slab + (blockIdx.x / 8) * int64_t(blockDim.x) + threadIdx.x, min(N, (k + 1) * slab),
            int64_t(gridDim.x / 8) * blockDim.x};
}

// largest |v| over the fluid nodes and the smallest node index attaining it; fixed grid and fixed
// combination order, so the result does not depend on timing
__device__ inline void speed_pick(double& best, double& at, double b, double i) {
    if (b > best || (b == best && i >= 0.0 && (at < 0.0 || i < at))) {
        best = b;
        at = i;
    }
}

__device__ inline void speed_block(double& best, double& at) {
    for (int d = 32; d >= 1; d >>= 1) speed_pick(best, at, __shfl_xor(best, d, 64), __shfl_xor(at, d, 64));
    __shared__ double sb[4], sa[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        sb[wv] = best;
        sa[wv] = at;
    }
    __syncthreads();
    best = sb[0];
    at = sa[0];
    for (int w = 1; w < 4; ++w) speed_pick(best, at, sb[w], sa[w]);
}

// the physical velocity of every node (SPEED = false: into v, zeros on solid nodes), or only the
// largest speed over the fluid nodes and its node (SPEED = true: one (speed, node) pair per
// workgroup into part, for k_speed_final; the same arithmetic, so the same value as the largest
// speed of the stored field, without storing it)
template <class S, class C, int Q, bool SPEED>
__global__ __launch_bounds__(256) void k_vel_out(GridDev g, const S* __restrict__ f, const int32_t* __restrict__ tag,
                                                 const double* __restrict__ rho, const double* __restrict__ psi, double G,
                                                 double gx, double gy, double gz, double* __restrict__ v) {
    double best = -1.0, at = -1.0;
    const Sweep sw = sweep(g.N, SPEED);
    for (int64_t x = sw.x0; x < sw.xe; x += sw.xs) {
        // every load of the node at once, the tag among them (every address is in the lattice);
        // solid nodes evaluate too and are dropped by selection, so one memory round trip per node
        const bool fl = tag[x] >= 0;
        uint32_t nb[Q];
        nb_all<Q>(g, uint32_t(x), nb);
        double fv[Q], pv[Q];
        fv[0] = pv[0] = 0.0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            fv[i] = double(ldp<S, C>(f, i, g.N, x));
            pv[i] = psi[nb[i]];
        }
        double j[3], vv[3];
        node_j<Q>(fv, j);
        const double gk[3] = {gx, gy, gz};
        node_v<Q>(j, pv, psi[x], rho[x], G, gk, g.dim, vv);
        if (SPEED) {
            double s2 = 0.0;
            for (int k = 0; k < g.dim; ++k) s2 += vv[k] * vv[k];
            speed_pick(best, at, fl ? sqrt(s2) : -1.0, fl ? double(x) : -1.0);
        } else {
            for (int k = 0; k < g.dim; ++k) v[k * g.N + x] = fl ? vv[k] : 0.0;
        }
    }
    if (SPEED) {
        speed_block(best, at);
        if (threadIdx.x == 0) {
            v[2 * blockIdx.x] = best;
            v[2 * blockIdx.x + 1] = at;
        }
    }
}

// chemical-potential model: v = (j - F / 2) / rho with F = -rho grad mu + grad(rho) / 3 + rho g from
// the density and chemical-potential fields of the last collision (fourth-order differences);
// SPEED as for k_vel_out.  rho is the density k_rho_out wrote; SPEED forms it itself from the node's
// populations, as k_rho_out does, so the density pass is not needed for the largest speed
template <class S, class C, bool SPEED>
__global__ __launch_bounds__(256) void k_vel_cp(GridDev g, const S* __restrict__ f, const int32_t* __restrict__ tag,
                                                const double* __restrict__ rho, double rho_ref, const C* __restrict__ fr,
                                                const C* __restrict__ fm, double gx, double gy, double* __restrict__ v) {
    double vbest = -1.0, vat = -1.0;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < g.N; x += int64_t(gridDim.x) * blockDim.x) {
        const bool fl = tag[x] >= 0;  // solid nodes evaluate too and are dropped by selection
        double fv[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) fv[i] = (SPEED || i > 0) ? double(ldp<S, C>(f, i, g.N, x)) : 0.0;
        double jx = 0, jy = 0;
        for (int i = 1; i < 9; ++i) {
            jx += fv[i] * c_ex[0][i];
            jy += fv[i] * c_ey[0][i];
        }
        const double rx = SPEED ? node_rho<9>(fv, rho_ref) : rho[x];
        const int cx = int(x % g.nx), cy = int(x / g.nx);
        auto at = [&](const C* a, int dx, int dy) {
            return double(a[int64_t(wrap1(cy + dy, g.ny)) * g.nx + wrap1(cx + dx, g.nx)]);
        };
        auto d1 = [](double m2, double m1, double p1, double p2) { return (8.0 * (p1 - m1) - (p2 - m2)) / 12.0; };
        const double r = double(fr[x]);
        const double Fx = -r * d1(at(fm, -2, 0), at(fm, -1, 0), at(fm, 1, 0), at(fm, 2, 0)) +
                          d1(at(fr, -2, 0), at(fr, -1, 0), at(fr, 1, 0), at(fr, 2, 0)) / 3.0 + r * gx;
        const double Fy = -r * d1(at(fm, 0, -2), at(fm, 0, -1), at(fm, 0, 1), at(fm, 0, 2)) +
                          d1(at(fr, 0, -2), at(fr, 0, -1), at(fr, 0, 1), at(fr, 0, 2)) / 3.0 + r * gy;
        const double vx = (jx - 0.5 * Fx) / rx, vy = (jy - 0.5 * Fy) / rx;
        if (SPEED) {
            double s2 = 0.0;
            s2 += vx * vx;
            s2 += vy * vy;
            speed_pick(vbest, vat, fl ? sqrt(s2) : -1.0, fl ? double(x) : -1.0);
        } else {
            v[x] = fl ? vx : 0.0;
            v[g.N + x] = fl ? vy : 0.0;
        }
    }
    if (SPEED) {
        speed_block(vbest, vat);
        if (threadIdx.x == 0) {
            v[2 * blockIdx.x] = vbest;
            v[2 * blockIdx.x + 1] = vat;
        }
    }
}

template <class S, class C>
__global__ void k_plane_in(int64_t N, const double* __restrict__ src, S* __restrict__ dst, C shift) {
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < N; x += int64_t(gridDim.x) * blockDim.x)
        st<S, C>(dst, x, C(src[x]) - shift);
}

template <class S, class C>
__global__ void k_plane_out(int64_t N, const S* __restrict__ src, const int32_t* __restrict__ tag, double* __restrict__ dst,
                            double shift) {
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < N; x += int64_t(gridDim.x) * blockDim.x)
        dst[x] = tag[x] < 0 ? 0.0 : double(ld<S, C>(src, x)) + shift;
}

inline unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    return unsigned(b < 1 ? 1 : b);
}

inline double w_of(const mcb_ctx* c, int i) {
    if (c->g.dim == 2) return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}

template <class S, class C>
hipError_t init_feq_t(mcb_ctx* c, const double* rho, const double* u, void* fout) {
    const double rr = c->p.precision == MCB_F64 ? 0.0 : c->p.rho_ref;
    hipLaunchKernelGGL((k_init_feq<S, C>), dim3(grid_for(c->g.N)), dim3(256), 0, c->stream, c->g, c->g.dim == 2 ? 0 : 1,
                       reinterpret_cast<const int32_t*>(c->lat + c->L.tag), rho, u, C(rr), static_cast<S*>(fout));
    return hipGetLastError();
}

template <class S, class C>
hipError_t monitor_t(mcb_ctx* c, const void* fcur, const void* rcur, double* partials, double* result) {
    const double rr = c->p.precision == MCB_F64 ? 0.0 : c->p.rho_ref;
    const int32_t* tag = reinterpret_cast<const int32_t*>(c->lat + c->L.tag);
    const int64_t nb = c->n_bnodes > 0 ? c->n_bnodes : 0;
    if (c->g.dim == 2)
        hipLaunchKernelGGL((k_mon_partial<S, C, 9>), dim3(MON_BLOCKS), dim3(256), 0, c->stream, c->g,
                           static_cast<const S*>(fcur), tag, rr, static_cast<const C*>(rcur), int(c->L.rec_stride), nb, partials);
    else
        hipLaunchKernelGGL((k_mon_partial<S, C, 19>), dim3(MON_BLOCKS), dim3(256), 0, c->stream, c->g,
                           static_cast<const S*>(fcur), tag, rr, static_cast<const C*>(rcur), int(c->L.rec_stride), nb, partials);
    hipLaunchKernelGGL(k_mon_final, dim3(1), dim3(256), 0, c->stream, partials, MON_BLOCKS, result);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_speed_final(const double* __restrict__ part, int nparts, double* __restrict__ out) {
    double best = -1.0, at = -1.0;
    for (int p = threadIdx.x; p < nparts; p += blockDim.x) speed_pick(best, at, part[2 * p], part[2 * p + 1]);
    speed_block(best, at);
    if (threadIdx.x == 0) {
        out[0] = best;
        out[1] = at;
    }
}

// ---- the largest speed of a two-dimensional state in one pass.  A workgroup of SW lanes marches
// a strip of SC = NC SW columns (each lane NC columns, SW apart; two halo columns on each side, so
// SC - 4 output columns) along a segment of rows.  Iteration k loads row r = y0 - 2 + k
// (populations and tags; issued one iteration earlier), puts its density and tags in a 3-row LDS
// ring, computes psi of row r - 1 (eq. 15 at wall nodes, from the ring) into a second ring, and
// the velocity of row r - 2 from its own momentum and density (kept in registers) and the psi
// ring.  Each workgroup leaves its largest speed and that node in part.  The loads go through
// buffer resources and every iteration issues them, the rows past the segment included, and the
// eq. 15 factor of a wall node is loaded with its row's densities, one iteration before its psi:
// the compiler counts loads in flight in issue order, so a load that only some iterations issue,
// or one issued just before its use, makes it wait for the next row's loads as well.
constexpr int SW = 256, NC = 1, SC = NC * SW, SO = SC - 4;

template <class S, class C>
__global__ __launch_bounds__(SW) void k_speed2d(GridDev g, const S* __restrict__ f, const int32_t* __restrict__ tag,
                                                double rho_ref, const double* __restrict__ phi, uint32_t n_wall,
                                                Eos<double> eos, double G, double gx, double gy, int Dy, int nbx,
                                                int32_t* flags, double* __restrict__ part) {
    __shared__ double s_rho[3][SC];
    __shared__ int s_tag[3][SC];
    __shared__ double s_psi[3][SC];
    const int t = threadIdx.x;
    const int bx = int(blockIdx.x) % nbx, by = int(blockIdx.x) / nbx;
    const int x0 = bx * SO, y0 = by * Dy;
    const int Dv = min(Dy, g.ny - y0), iters = Dv + 4;
    const double gk[3] = {gx, gy, 0.0};
    int xc[NC];    // the lane's columns (strip positions c = t + h SW)
    bool out[NC];  // output columns
#pragma unroll
    for (int h = 0; h < NC; ++h) {
        const int c = t + h * SW, xr = x0 - 2 + c;
        xc[h] = wrap1(xr < 0 ? xr : xr % g.nx, g.nx);
        out[h] = c >= 2 && c < SO + 2 && xr < g.nx;
    }
    auto rowof = [&](int k) { int r = (y0 - 2 + k) % g.ny; return r < 0 ? r + g.ny : r; };
    constexpr uint32_t s = sizeof(S), P0 = kMixed<S> ? 1 : 0;
    const uint32_t n = uint32_t(g.N);  // the lattice fits the 32-bit buffer offsets
    const __amdgpu_buffer_rsrc_t rf = make_res(f, uint64_t(9 + P0) * n * s);
    const __amdgpu_buffer_rsrc_t rt = make_res(tag, uint64_t(n) * 4);
    const __amdgpu_buffer_rsrc_t rp = make_res(phi, uint64_t(n_wall) * 8);
    // loads of the next row in flight
    C fr[NC][9];
    int tgr[NC];
    auto issue = [&](int k) {
        const uint32_t xrow = uint32_t(rowof(k)) * uint32_t(g.nx);
#pragma unroll
        for (int h = 0; h < NC; ++h) {
            const uint32_t x = xrow + uint32_t(xc[h]);
            tgr[h] = ld_i32(rt, x * 4u);  // first: a copy of it that waits does not wait for the populations
#pragma unroll
            for (int i = 0; i < 9; ++i)
                fr[h][i] = kMixed<S> && i == 0 ? C(Buf<float>::ld(rf, x * 4u))  // FP16 storage: population 0 in FP32
                                               : C(Buf<S>::ld(rf, x * s, uint32_t(i + P0) * n * s));
        }
    };
    issue(0);
    // eq. 15 factors of the wall nodes of rows r - 1 and r in the lane's own column, which is the
    // column whose psi the lane computes (one column per lane)
    static_assert(NC == 1, "psi of the lane's own column");
    double phB[NC] = {}, phC[NC] = {};
    double rA[NC] = {}, rB[NC] = {}, rC[NC] = {};   // density of rows r - 2, r - 1, r (own columns)
    int tA[NC], tB[NC], tC[NC];                     // their tags
    double jA[NC][3] = {}, jB[NC][3] = {}, jC[NC][3] = {};  // their momentum
#pragma unroll
    for (int h = 0; h < NC; ++h) tA[h] = tB[h] = tC[h] = -1;
    double best = -1.0, at = -1.0;
    for (int k = 0; k < iters; ++k) {
        const int s0 = k % 3, s1 = (k + 2) % 3, s2 = (k + 1) % 3;  // ring slots of rows r, r - 1, r - 2
        // ---- row r: density and momentum; its tags and densities to the ring
#pragma unroll
        for (int h = 0; h < NC; ++h) {
            double fv[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) fv[i] = double(fr[h][i]);
            const int tg = tgr[h];
            rA[h] = rB[h];
            rB[h] = rC[h];
            tA[h] = tB[h];
            tB[h] = tC[h];
            for (int q = 0; q < 3; ++q) {
                jA[h][q] = jB[h][q];
                jB[h][q] = jC[h][q];
            }
            rC[h] = tg >= 0 ? node_rho<9>(fv, rho_ref) : 0.0;
            tC[h] = tg;
            node_j<9>(fv, jC[h]);
            s_rho[s0][t + h * SW] = rC[h];
            s_tag[s0][t + h * SW] = tg;
            phB[h] = phC[h];
            phC[h] = Buf<double>::ld(rp, tg < -1 ? uint32_t(-tg - 2) * 8u : OOB);
        }
        issue(k + 1);  // past the segment: a row nothing uses
        __syncthreads();
        // ---- psi of row r - 1 (its neighbours' densities are in the ring from k >= 2)
        if (k >= 2) {
#pragma unroll
            for (int h = 0; h < NC; ++h) {
                const int c = t + h * SW;
                if (c < 1 || c >= SC - 1) continue;
                const int tg = s_tag[s1][c];
                // the density psi is taken of: the node's own (fluid), eq. 15's (wall); other solid
                // nodes have psi = 0
                double re = s_rho[s1][c];
                if (tg < -1) {
                    int ty[9];
                    double ry[9];
                    ty[0] = -1;
                    ry[0] = 0.0;
#pragma unroll
                    for (int i = 1; i < 9; ++i) {
                        const int sl = c_ey[0][i] > 0 ? s0 : (c_ey[0][i] < 0 ? s2 : s1);  // row r - 1 + e_y
                        ty[i] = s_tag[sl][c + c_ex[0][i]];
                        ry[i] = s_rho[sl][c + c_ex[0][i]];
                    }
                    re = wall_rho<9>(ty, ry, phB[h]);  // the lane's own node: c = t (NC = 1)
                }
                s_psi[s1][c] = tg == -1 ? 0.0 : psi_of(re, eos, flags);
            }
        }
        __syncthreads();
        // ---- velocity and speed of row r - 2 (psi of rows r - 3 .. r - 1 in the ring)
        if (k >= 4) {
            const int p0 = s2, pm = s0, pp = s1;  // psi ring slots of rows r - 2, r - 3, r - 1
#pragma unroll
            for (int h = 0; h < NC; ++h) {
                if (!out[h] || tA[h] < 0) continue;
                const int c = t + h * SW;
                double pv[9];
                pv[0] = 0.0;
#pragma unroll
                for (int i = 1; i < 9; ++i) {
                    const int sl = c_ey[0][i] > 0 ? pp : (c_ey[0][i] < 0 ? pm : p0);
                    pv[i] = s_psi[sl][c + c_ex[0][i]];
                }
                double v[3];
                node_v<9>(jA[h], pv, s_psi[p0][c], rA[h], G, gk, 2, v);
                const double sp = sqrt(v[0] * v[0] + v[1] * v[1]);
                speed_pick(best, at, sp, double(int64_t(rowof(k - 2)) * g.nx + xc[h]));
            }
        }
    }
    speed_block(best, at);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = best;
        part[2 * blockIdx.x + 1] = at;
    }
}

// ---- track_dm: the eq. 18 total of the step just taken (the correction slot, last of each
// boundary record), added to a running FP64 sum.  Pass 1: DM_BLOCKS workgroups, each the records
// b = blockIdx.x * 256 + threadIdx.x + k * DM_BLOCKS * 256; pass 2: one workgroup sums the partials
// in a fixed order and adds the total to the running sum.  Deterministic.
template <class C>
__global__ __launch_bounds__(256) void k_dm_partial(const C* __restrict__ rec, int rec_stride, int64_t nb,
                                                    double* __restrict__ part) {
    double acc = 0.0;
    for (int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; b < nb; b += int64_t(gridDim.x) * blockDim.x)
        acc += double(rec[b * rec_stride + rec_stride - 1]);
    __shared__ double red[4];
    const double s = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void k_dm_final(double* __restrict__ part) {
    __shared__ double red[4];
    const double s = wave_sum(threadIdx.x < DM_BLOCKS ? part[threadIdx.x] : 0.0);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[DM_BLOCKS] += ((red[0] + red[1]) + red[2]) + red[3];
}

// workgroups of the velocity kernels in speed mode (a multiple of the eight XCDs): one (speed,
// node) pair each in the partials
constexpr int SPEED_BLOCKS = 2048;
static_assert(SPEED_BLOCKS % 8 == 0 && SPEED_BLOCKS <= MON_BLOCKS * MON_FIELDS / 2, "speed partials");

// rho, psi and the physical velocity of the state into the scratch arena: rho at scratch, psi
// after it, v (dim planes) after that
// part == nullptr: rho, psi and v into the scratch arena; otherwise the velocity kernel leaves
// SPEED_BLOCKS (largest speed, node) pairs in part instead of v
template <class S, class C>
hipError_t moments_dev(mcb_ctx* c, const void* fcur, double* part = nullptr) {
    const double rr = c->p.precision == MCB_F64 ? 0.0 : c->p.rho_ref;
    double* sr = reinterpret_cast<double*>(c->lat + c->L.scratch);
    double* sp = sr + c->g.N;
    double* sv = sp + c->g.N;
    const int32_t* tag = reinterpret_cast<const int32_t*>(c->lat + c->L.tag);
    Eos<double> eos{c->p.eos_R * c->p.eos_T, c->p.eos_a, c->p.eos_b / 4.0, 2.0 / c->p.G};
    const bool d2 = c->g.dim == 2;
    const bool cp = c->p.model == MCB_MODEL_CHEMPOT;
    if (cp) {
        if (!part)  // the chemical-potential speed forms each node's density itself
            hipLaunchKernelGGL((k_rho_out<S, C, 9>), dim3(grid_for(c->g.N)), dim3(256), 0, c->stream, c->g,
                               static_cast<const S*>(fcur), tag, rr, sr);
        const auto vel_cp = part ? k_vel_cp<S, C, true> : k_vel_cp<S, C, false>;
        hipLaunchKernelGGL(vel_cp, dim3(part ? SPEED_BLOCKS : grid_for(c->g.N)), dim3(256), 0, c->stream, c->g,
                           static_cast<const S*>(fcur), tag, sr, rr, reinterpret_cast<const C*>(c->lat + c->L.cp_rho),
                           reinterpret_cast<const C*>(c->lat + c->L.cp_mu), c->p.gravity[0], c->p.gravity[1],
                           part ? part : sv);
        return hipGetLastError();
    }
    int32_t* flags = reinterpret_cast<int32_t*>(c->lat + c->L.flags);
    hipLaunchKernelGGL((d2 ? k_rho_psi_out<S, C, 9> : k_rho_psi_out<S, C, 19>), dim3(grid_for(c->g.N)), dim3(256), 0, c->stream,
                       c->g, static_cast<const S*>(fcur), tag, rr, eos, flags, sr, sp);
    if (c->n_wall > 0)
        hipLaunchKernelGGL(d2 ? k_psi_wall<9> : k_psi_wall<19>, dim3(grid_for(c->n_wall)), dim3(256), 0, c->stream, c->g,
                           c->n_wall, reinterpret_cast<const int32_t*>(c->lk + c->L.wl_node), tag, sr,
                           reinterpret_cast<const double*>(c->lk + c->L.wl_phi), eos, flags, sp);
    const auto vel_out = d2 ? (part ? k_vel_out<S, C, 9, true> : k_vel_out<S, C, 9, false>)
                            : (part ? k_vel_out<S, C, 19, true> : k_vel_out<S, C, 19, false>);
    hipLaunchKernelGGL(vel_out, dim3(part ? SPEED_BLOCKS : grid_for(c->g.N)), dim3(256), 0, c->stream, c->g,
                       static_cast<const S*>(fcur), tag, sr, sp, c->p.G, c->p.gravity[0], c->p.gravity[1], c->p.gravity[2],
                       part ? part : sv);
    return hipGetLastError();
}

template <class S, class C>
hipError_t max_speed_t(mcb_ctx* c, const void* fcur) {
    double* part = reinterpret_cast<double*>(c->lat + c->L.partials);
    if (c->g.dim == 2 && c->p.model != MCB_MODEL_CHEMPOT) {
        // one pass, one resident round of workgroups (at most the partials' capacity)
        const int nbx = (c->g.nx + SO - 1) / SO;
        const int cap = resident_blocks(c, k_speed2d<S, C>, SW, &c->occ[6]);
        const int want = std::max(1, std::min(cap, MON_BLOCKS * MON_FIELDS / 2) / nbx);
        int nseg = std::min(c->g.ny, want);
        const int Dy = (c->g.ny + nseg - 1) / nseg;
        nseg = (c->g.ny + Dy - 1) / Dy;
        const double rr = c->p.precision == MCB_F64 ? 0.0 : c->p.rho_ref;
        Eos<double> eos{c->p.eos_R * c->p.eos_T, c->p.eos_a, c->p.eos_b / 4.0, 2.0 / c->p.G};
        hipLaunchKernelGGL((k_speed2d<S, C>), dim3(nbx * nseg), dim3(SW), 0, c->stream, c->g, static_cast<const S*>(fcur),
                           reinterpret_cast<const int32_t*>(c->lat + c->L.tag), rr,
                           reinterpret_cast<const double*>(c->lk + c->L.wl_phi), uint32_t(c->n_wall > 0 ? c->n_wall : 0),
                           eos, c->p.G, c->p.gravity[0],
                           c->p.gravity[1], Dy, nbx, reinterpret_cast<int32_t*>(c->lat + c->L.flags), part);
        hipLaunchKernelGGL(k_speed_final, dim3(1), dim3(256), 0, c->stream, part, nbx * nseg,
                           reinterpret_cast<double*>(c->lat + c->L.result) + MON_SPEED);
        return hipGetLastError();
    }
    // the moment kernels with the velocity kernel reducing the speed instead of storing v
    hipError_t e = moments_dev<S, C>(c, fcur, part);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_speed_final, dim3(1), dim3(256), 0, c->stream, part, SPEED_BLOCKS,
                       reinterpret_cast<double*>(c->lat + c->L.result) + MON_SPEED);
    return hipGetLastError();
}

template <class S, class C>
hipError_t moments_t(mcb_ctx* c, const void* fcur, double* rho, double* v) {
    double* sr = reinterpret_cast<double*>(c->lat + c->L.scratch);
    double* sv = sr + 2 * c->g.N;
    hipError_t e = moments_dev<S, C>(c, fcur);
    if (e != hipSuccess) return e;
    if (rho) {
        e = hipMemcpyAsync(rho, sr, sizeof(double) * c->g.N, hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) return e;
    }
    if (v) {
        e = hipMemcpyAsync(v, sv, sizeof(double) * c->g.N * c->g.dim, hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) return e;
    }
    return hipStreamSynchronize(c->stream);
}

}  // namespace

hipError_t init_feq(mcb_ctx* c, const double* rho, const double* u, void* fout) {
    switch (c->p.precision) {
        case MCB_F64: return init_feq_t<double, double>(c, rho, u, fout);
        case MCB_F32S: return init_feq_t<float, float>(c, rho, u, fout);
        default: return init_feq_t<__half, float>(c, rho, u, fout);
    }
}

hipError_t monitor(mcb_ctx* c, const void* fcur, const void* rcur, double* partials, double* result) {
    if (!partials) partials = reinterpret_cast<double*>(c->lat + c->L.partials);
    if (!result) result = reinterpret_cast<double*>(c->lat + c->L.result);
    switch (c->p.precision) {
        case MCB_F64: return monitor_t<double, double>(c, fcur, rcur, partials, result);
        case MCB_F32S: return monitor_t<float, float>(c, fcur, rcur, partials, result);
        default: return monitor_t<__half, float>(c, fcur, rcur, partials, result);
    }
}

hipError_t dm_accumulate(mcb_ctx* c, const void* rcur) {
    static_assert(DM_BLOCKS == 256, "one lane per partial in the final pass");
    double* part = reinterpret_cast<double*>(c->lat + c->L.dm);
    const int64_t nb = c->n_bnodes > 0 ? c->n_bnodes : 0;
    const int stride = int(c->L.rec_stride);
    if (c->p.precision == MCB_F64)
        hipLaunchKernelGGL(k_dm_partial<double>, dim3(DM_BLOCKS), dim3(256), 0, c->stream, static_cast<const double*>(rcur),
                           stride, nb, part);
    else
        hipLaunchKernelGGL(k_dm_partial<float>, dim3(DM_BLOCKS), dim3(256), 0, c->stream, static_cast<const float*>(rcur),
                           stride, nb, part);
    hipLaunchKernelGGL(k_dm_final, dim3(1), dim3(256), 0, c->stream, part);
    return hipGetLastError();
}

hipError_t max_speed(mcb_ctx* c, const void* fcur) {
    switch (c->p.precision) {
        case MCB_F64: return max_speed_t<double, double>(c, fcur);
        case MCB_F32S: return max_speed_t<float, float>(c, fcur);
        default: return max_speed_t<__half, float>(c, fcur);
    }
}

hipError_t moments_out(mcb_ctx* c, const void* fcur, double* rho, double* v) {
    switch (c->p.precision) {
        case MCB_F64: return moments_t<double, double>(c, fcur, rho, v);
        case MCB_F32S: return moments_t<float, float>(c, fcur, rho, v);
        default: return moments_t<__half, float>(c, fcur, rho, v);
    }
}

hipError_t convert_plane_in(mcb_ctx* c, const double* src, void* dst_plane, int dir) {
    const double shift = c->p.precision == MCB_F64 ? 0.0 : w_of(c, dir) * c->p.rho_ref;
    switch (c->p.precision) {
        case MCB_F64:
            hipLaunchKernelGGL((k_plane_in<double, double>), dim3(grid_for(c->g.N)), dim3(256), 0, c->stream, c->g.N, src,
                               static_cast<double*>(dst_plane), shift);
            break;
        case MCB_F32S:
            hipLaunchKernelGGL((k_plane_in<float, float>), dim3(grid_for(c->g.N)), dim3(256), 0, c->stream, c->g.N, src,
                               static_cast<float*>(dst_plane), float(shift));
            break;
        default:
            // FP16 storage keeps the rest population in FP32
            if (dir == 0)
                hipLaunchKernelGGL((k_plane_in<float, float>), dim3(grid_for(c->g.N)), dim3(256), 0, c->stream, c->g.N, src,
                                   static_cast<float*>(dst_plane), float(shift));
            else
                hipLaunchKernelGGL((k_plane_in<__half, float>), dim3(grid_for(c->g.N)), dim3(256), 0, c->stream, c->g.N, src,
                                   static_cast<__half*>(dst_plane), float(shift));
    }
    return hipGetLastError();
}

hipError_t convert_plane_out(mcb_ctx* c, const void* src_plane, double* dst, int dir) {
    const double shift = c->p.precision == MCB_F64 ? 0.0 : w_of(c, dir) * c->p.rho_ref;
    const int32_t* tag = reinterpret_cast<const int32_t*>(c->lat + c->L.tag);
    switch (c->p.precision) {
        case MCB_F64:
            hipLaunchKernelGGL((k_plane_out<double, double>), dim3(grid_for(c->g.N)), dim3(256), 0, c->stream, c->g.N,
                               static_cast<const double*>(src_plane), tag, dst, shift);
            break;
        case MCB_F32S:
            hipLaunchKernelGGL((k_plane_out<float, float>), dim3(grid_for(c->g.N)), dim3(256), 0, c->stream, c->g.N,
                               static_cast<const float*>(src_plane), tag, dst, shift);
            break;
        default:
            if (dir == 0)
                hipLaunchKernelGGL((k_plane_out<float, float>), dim3(grid_for(c->g.N)), dim3(256), 0, c->stream, c->g.N,
                                   static_cast<const float*>(src_plane), tag, dst, shift);
            else
                hipLaunchKernelGGL((k_plane_out<__half, float>), dim3(grid_for(c->g.N)), dim3(256), 0, c->stream, c->g.N,
                                   static_cast<const __half*>(src_plane), tag, dst, shift);
    }
    return hipGetLastError();
}

}  // namespace mcb
