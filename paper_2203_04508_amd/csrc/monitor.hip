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

// periodic neighbour x + sign e_i (32-bit position arithmetic: N < 2^31)
__device__ inline int64_t nb_index(const GridDev& g, int L, int64_t x, int i, int sign) {
    const uint32_t u = uint32_t(x), nx = uint32_t(g.nx), nxy = nx * uint32_t(g.ny);
    const uint32_t cz = u / nxy, r = u - cz * nxy, cy = r / nx, cx = r - cy * nx;
    return int64_t(wrap1(int(cx) + sign * c_ex[L][i], g.nx)) +
           int64_t(g.nx) * (wrap1(int(cy) + sign * c_ey[L][i], g.ny) + int64_t(g.ny) * wrap1(int(cz) + sign * c_ez[L][i], g.nz));
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

// ---- moments: rho, psi (fluid and wall nodes), then v = (j - F / 2) / rho.  Q is a template
// parameter (unrolled direction loops); each lane loads all it needs before using any.
template <class S, class C, int Q>
__global__ __launch_bounds__(256) void k_rho_out(GridDev g, const S* __restrict__ f, const int32_t* __restrict__ tag,
                                                 double rho_ref, double* __restrict__ rho) {
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < g.N; x += int64_t(gridDim.x) * blockDim.x) {
        const bool fl = tag[x] >= 0;
        double v[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = double(ldp<S, C>(f, i, g.N, x));
        double s = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) s += v[i];
        rho[x] = fl ? s + rho_ref : 0.0;
    }
}

template <int Q>
__global__ __launch_bounds__(256) void k_psi_out(GridDev g, const int32_t* __restrict__ tag, const double* __restrict__ rho,
                                                 const double* __restrict__ phi, Eos<double> eos, int32_t* flags,
                                                 double* __restrict__ psi) {
    constexpr int L = Q == 9 ? 0 : 1;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < g.N; x += int64_t(gridDim.x) * blockDim.x) {
        const int tg = tag[x];
        if (tg >= 0) { psi[x] = psi_of(rho[x], eos, flags); continue; }
        if (tg == -1) { psi[x] = 0.0; continue; }
        // wall node: every neighbour's tag and density at once, the solid ones dropped by selection
        int ty[Q];
        double ry[Q];
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int64_t y = nb_index(g, L, x, i, +1);
            ty[i] = tag[y];
            ry[i] = rho[y];
        }
        double num = 0, den = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            num += ty[i] >= 0 ? wgt<double>(L, i) * ry[i] : 0.0;
            den += ty[i] >= 0 ? wgt<double>(L, i) : 0.0;
        }
        psi[x] = psi_of(phi[-tg - 2] * (num / den), eos, flags);
    }
}

template <class S, class C, int Q>
__global__ __launch_bounds__(256) void k_vel_out(GridDev g, const S* __restrict__ f, const int32_t* __restrict__ tag,
                                                 const double* __restrict__ rho, const double* __restrict__ psi, double G,
                                                 double gx, double gy, double gz, double* __restrict__ v) {
    constexpr int L = Q == 9 ? 0 : 1;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < g.N; x += int64_t(gridDim.x) * blockDim.x) {
        if (tag[x] < 0) {
            for (int k = 0; k < g.dim; ++k) v[k * g.N + x] = 0.0;
            continue;
        }
        double fv[Q], pv[Q];
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            fv[i] = double(ldp<S, C>(f, i, g.N, x));
            pv[i] = psi[nb_index(g, L, x, i, +1)];
        }
        double j[3] = {0, 0, 0}, s[3] = {0, 0, 0};
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const double ws = (L == 0) ? (i < 5 ? 1.0 / 3.0 : 1.0 / 12.0) : (i < 7 ? 1.0 / 6.0 : 1.0 / 12.0);
            const int e[3] = {c_ex[L][i], c_ey[L][i], c_ez[L][i]};
            for (int k = 0; k < 3; ++k) {
                j[k] += fv[i] * e[k];
                s[k] += ws * pv[i] * e[k];
            }
        }
        const double gk[3] = {gx, gy, gz};
        for (int k = 0; k < g.dim; ++k) {
            const double F = -G * psi[x] * s[k] + rho[x] * gk[k];
            v[k * g.N + x] = (j[k] - 0.5 * F) / rho[x];
        }
    }
}

// chemical-potential model: v = (j - F / 2) / rho with F = -rho grad mu + grad(rho) / 3 + rho g from
// the density and chemical-potential fields of the last collision (fourth-order differences)
template <class S, class C>
__global__ void k_vel_cp(GridDev g, const S* __restrict__ f, const int32_t* __restrict__ tag, const double* __restrict__ rho,
                         const C* __restrict__ fr, const C* __restrict__ fm, double gx, double gy, double* __restrict__ v) {
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < g.N; x += int64_t(gridDim.x) * blockDim.x) {
        if (tag[x] < 0) {
            v[x] = 0.0;
            v[g.N + x] = 0.0;
            continue;
        }
        double jx = 0, jy = 0;
        for (int i = 1; i < 9; ++i) {
            const double fi = double(ldp<S, C>(f, i, g.N, x));
            jx += fi * c_ex[0][i];
            jy += fi * c_ey[0][i];
        }
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
        v[x] = (jx - 0.5 * Fx) / rho[x];
        v[g.N + x] = (jy - 0.5 * Fy) / rho[x];
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

__global__ __launch_bounds__(256) void k_speed_partial(GridDev g, const int32_t* __restrict__ tag, const double* __restrict__ v,
                                                       double* __restrict__ part) {
    double best = -1.0, at = -1.0;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < g.N; x += int64_t(gridDim.x) * blockDim.x) {
        if (tag[x] < 0) continue;
        double s2 = 0.0;
        for (int k = 0; k < g.dim; ++k) s2 += v[k * g.N + x] * v[k * g.N + x];
        speed_pick(best, at, sqrt(s2), double(x));
    }
    speed_block(best, at);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = best;
        part[2 * blockIdx.x + 1] = at;
    }
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

// rho, psi and the physical velocity of the state into the scratch arena: rho at scratch, psi
// after it, v (dim planes) after that
template <class S, class C>
hipError_t moments_dev(mcb_ctx* c, const void* fcur) {
    const double rr = c->p.precision == MCB_F64 ? 0.0 : c->p.rho_ref;
    double* sr = reinterpret_cast<double*>(c->lat + c->L.scratch);
    double* sp = sr + c->g.N;
    double* sv = sp + c->g.N;
    const int32_t* tag = reinterpret_cast<const int32_t*>(c->lat + c->L.tag);
    Eos<double> eos{c->p.eos_R * c->p.eos_T, c->p.eos_a, c->p.eos_b / 4.0, 2.0 / c->p.G};
    const bool d2 = c->g.dim == 2;
    const auto rho_out = d2 ? k_rho_out<S, C, 9> : k_rho_out<S, C, 19>;
    hipLaunchKernelGGL(rho_out, dim3(grid_for(c->g.N)), dim3(256), 0, c->stream, c->g, static_cast<const S*>(fcur), tag, rr, sr);
    if (c->p.model == MCB_MODEL_CHEMPOT) {
        hipLaunchKernelGGL((k_vel_cp<S, C>), dim3(grid_for(c->g.N)), dim3(256), 0, c->stream, c->g, static_cast<const S*>(fcur), tag,
                           sr, reinterpret_cast<const C*>(c->lat + c->L.cp_rho), reinterpret_cast<const C*>(c->lat + c->L.cp_mu),
                           c->p.gravity[0], c->p.gravity[1], sv);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(d2 ? k_psi_out<9> : k_psi_out<19>, dim3(grid_for(c->g.N)), dim3(256), 0, c->stream, c->g, tag, sr,
                       reinterpret_cast<const double*>(c->lk + c->L.wl_phi), eos,
                       reinterpret_cast<int32_t*>(c->lat + c->L.flags), sp);
    const auto vel_out = d2 ? k_vel_out<S, C, 9> : k_vel_out<S, C, 19>;
    hipLaunchKernelGGL(vel_out, dim3(grid_for(c->g.N)), dim3(256), 0, c->stream, c->g, static_cast<const S*>(fcur), tag, sr, sp,
                       c->p.G, c->p.gravity[0], c->p.gravity[1], c->p.gravity[2], sv);
    return hipGetLastError();
}

template <class S, class C>
hipError_t max_speed_t(mcb_ctx* c, const void* fcur) {
    hipError_t e = moments_dev<S, C>(c, fcur);
    if (e != hipSuccess) return e;
    const double* sv = reinterpret_cast<const double*>(c->lat + c->L.scratch) + 2 * c->g.N;
    double* part = reinterpret_cast<double*>(c->lat + c->L.partials);
    hipLaunchKernelGGL(k_speed_partial, dim3(MON_BLOCKS), dim3(256), 0, c->stream, c->g,
                       reinterpret_cast<const int32_t*>(c->lat + c->L.tag), sv, part);
    hipLaunchKernelGGL(k_speed_final, dim3(1), dim3(256), 0, c->stream, part, MON_BLOCKS,
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
