// Exact integer geometry pass on the device: node classification, fluid-solid links with their
// q and class, boundary-fluid nodes and first-layer wall nodes, all in canonical (linear index)
// order.  Units of 2^-16 lattice spacings, periodic minimum image; no floating point.
//
//   solid node          strictly inside some shape
//   link (x1, i)        x1 fluid, x1 + e_i solid (Sec. 3.1 of the paper, Figs. 1-2)
//   q_fixed             first n in [0, 2^16] with x1 + n e_i / 2^16 inside or on some shape
//   class               eq. 16 (q < 1/2, x2 = x1 - e_i fluid), bounce-back (q < 1/2, x2 solid),
//                       eq. 17 (q >= 1/2)
//   wall node           solid node with a fluid neighbour (the first layer of eq. 15)
#include "mcb_internal.h"

namespace mcb {
namespace {

__device__ inline int wrapn(int a, int n) {
    a %= n;
    return a < 0 ? a + n : a;
}

__device__ inline int64_t min_image(int64_t d, int64_t L) {
    d %= L;
    if (d < 0) d += L;
    if (d >= L / 2) d -= L;
    return d;
}

__device__ inline void coords(const GridDev& g, int64_t x, int c[3]) {
    c[0] = int(x % g.nx);
    c[1] = int((x / g.nx) % g.ny);
    c[2] = int(x / (int64_t(g.nx) * g.ny));
}

__device__ inline int64_t lin(const GridDev& g, int x, int y, int z) {
    return x + int64_t(g.nx) * (y + int64_t(g.ny) * z);
}

__device__ inline int64_t neighbour(const GridDev& g, const int c[3], int L, int i, int sign) {
    return lin(g, wrapn(c[0] + sign * c_ex[L][i], g.nx), wrapn(c[1] + sign * c_ey[L][i], g.ny),
               wrapn(c[2] + sign * c_ez[L][i], g.nz));
}

__device__ inline int64_t floor_div(int64_t a, int64_t b) {
    return a >= 0 ? a / b : -((-a + b - 1) / b);
}

struct Bands {
    int n;
    mcb_shape s[MAX_BANDS];
};

// ------------------------------------------------------------------------ classification
__global__ void k_fill_u8(uint8_t* a, int64_t n, uint8_t v) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        a[i] = v;
}

// one workgroup per shape; balls only
__global__ void k_raster_ball(const mcb_shape* __restrict__ shapes, GridDev g, uint8_t* solid) {
    const mcb_shape s = shapes[blockIdx.x];
    if (s.kind != MCB_SHAPE_BALL) return;
    const int64_t C[3] = {s.cx, s.cy, s.cz};
    int lo[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
    for (int k = 0; k < g.dim; ++k) {
        lo[k] = int(floor_div(C[k] - s.radius, ONE));
        ext[k] = int(floor_div(C[k] + s.radius, ONE)) + 1 - lo[k];
    }
    const int64_t total = int64_t(ext[0]) * ext[1] * ext[2];
    const int64_t r2 = s.radius * s.radius;
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int64_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
        int c[3] = {lo[0] + int(idx % ext[0]), lo[1] + int((idx / ext[0]) % ext[1]), lo[2] + int(idx / (int64_t(ext[0]) * ext[1]))};
        int64_t acc = 0;
        for (int k = 0; k < g.dim; ++k) {
            c[k] = wrapn(c[k], n[k]);
            int64_t d = min_image(int64_t(c[k]) * ONE - C[k], int64_t(n[k]) * ONE);
            acc += d * d;
        }
        if (acc < r2) solid[lin(g, c[0], c[1], g.dim == 3 ? c[2] : 0)] = 1;
    }
}

__global__ void k_raster_band(Bands b, GridDev g, uint8_t* solid) {
    const int64_t Ly = int64_t(g.ny) * ONE;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < g.N; x += int64_t(gridDim.x) * blockDim.x) {
        const int64_t Y = ((x / g.nx) % g.ny) * ONE;
        for (int k = 0; k < b.n; ++k) {
            int64_t r = (Y - b.s[k].lo) % Ly;
            if (r < 0) r += Ly;
            if (r < b.s[k].hi - b.s[k].lo) solid[x] = 1;
        }
    }
}

// ------------------------------------------------------------------------ counting and scan
// per-node counts packed in one 64-bit word: links (bits 0-19), boundary node (20-39), wall (40-59)
__device__ inline int64_t node_counts(const GridDev& g, int L, const uint8_t* __restrict__ solid, int64_t x,
                                      uint32_t* mask_out) {
    uint32_t mask = 0;
    int c[3];
    coords(g, x, c);
    const bool fl = solid[x] == 0;
    int nsolid = 0, nfluid = 0;
    for (int i = 1; i < g.Q; ++i) {
        const bool s = solid[neighbour(g, c, L, i, +1)] != 0;
        if (s) { ++nsolid; mask |= 1u << i; } else { ++nfluid; }
    }
    *mask_out = fl ? mask : 0u;
    if (fl) return int64_t(nsolid) | (int64_t(nsolid > 0) << 20);
    return int64_t(nfluid > 0) << 40;
}

__device__ inline int64_t block_excl_scan(int64_t v, int64_t* total) {
    __shared__ int64_t wsum[SCAN_BLOCK / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t s = v;
    for (int d = 1; d < 64; d <<= 1) {
        int64_t o = __shfl_up(s, d, 64);
        if (lane >= d) s += o;
    }
    if (lane == 63) wsum[wid] = s;
    __syncthreads();
    int64_t pre = 0, tot = 0;
    for (int w = 0; w < SCAN_BLOCK / 64; ++w) {
        if (w < wid) pre += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return pre + s - v;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_count(GridDev g, int L, const uint8_t* __restrict__ solid, int64_t* blocksums) {
    const int64_t x = blockIdx.x * int64_t(SCAN_BLOCK) + threadIdx.x;
    uint32_t m;
    const int64_t v = x < g.N ? node_counts(g, L, solid, x, &m) : 0;
    int64_t tot;
    block_excl_scan(v, &tot);
    if (threadIdx.x == 0) {
        blocksums[3 * blockIdx.x + 0] = tot & 0xFFFFF;
        blocksums[3 * blockIdx.x + 1] = (tot >> 20) & 0xFFFFF;
        blocksums[3 * blockIdx.x + 2] = (tot >> 40) & 0xFFFFF;
    }
}

// single workgroup: exclusive scan of the per-block counts, totals stored after the last block
__global__ __launch_bounds__(1024) void k_scan(int64_t* bs, int64_t nblk) {
    __shared__ int64_t part[3][1024];
    const int t = threadIdx.x;
    const int64_t chunk = (nblk + 1023) / 1024;
    const int64_t b0 = t * chunk, b1 = min(nblk, b0 + chunk);
    int64_t loc[3] = {0, 0, 0};
    for (int64_t b = b0; b < b1; ++b)
        for (int k = 0; k < 3; ++k) loc[k] += bs[3 * b + k];
    for (int k = 0; k < 3; ++k) part[k][t] = loc[k];
    __syncthreads();
    if (t < 3) {  // serial exclusive scan of the 1024 partials, one counter per thread
        int64_t run = 0;
        for (int j = 0; j < 1024; ++j) {
            int64_t v = part[t][j];
            part[t][j] = run;
            run += v;
        }
        bs[3 * nblk + t] = run;
    }
    __syncthreads();
    int64_t run[3] = {part[0][t], part[1][t], part[2][t]};
    for (int64_t b = b0; b < b1; ++b)
        for (int k = 0; k < 3; ++k) {
            int64_t v = bs[3 * b + k];
            bs[3 * b + k] = run[k];
            run[k] += v;
        }
}

struct FillOut {
    int32_t* tag;
    uint32_t* nmask;  // 3-D only
    int32_t* bn_node;
    uint32_t* bn_mask;
    int32_t* bn_link0;
    uint32_t* lk_qc;
    int32_t* wl_node;
    double* wl_phi;
};

__global__ __launch_bounds__(SCAN_BLOCK) void k_fill(GridDev g, int L, const uint8_t* __restrict__ solid,
                                                     const int64_t* __restrict__ bs, FillOut o) {
    const int64_t x = blockIdx.x * int64_t(SCAN_BLOCK) + threadIdx.x;
    uint32_t mask = 0;
    const int64_t v = x < g.N ? node_counts(g, L, solid, x, &mask) : 0;
    int64_t tot;
    const int64_t pre = block_excl_scan(v, &tot);
    if (x >= g.N) return;
    const int64_t lpre = (pre & 0xFFFFF) + bs[3 * blockIdx.x + 0];
    const int64_t bpre = ((pre >> 20) & 0xFFFFF) + bs[3 * blockIdx.x + 1];
    const int64_t wpre = ((pre >> 40) & 0xFFFFF) + bs[3 * blockIdx.x + 2];
    if (solid[x] == 0) {
        if (mask) {
            // 2-D: boundary index and the 8 link bits share the tag; 3-D: boundary index + 1
            o.tag[x] = g.dim == 2 ? int32_t((bpre << 8) | (mask >> 1)) : int32_t(bpre + 1);
            if (g.dim == 3) o.nmask[x] = mask >> 1;
            o.bn_node[bpre] = int32_t(x);
            o.bn_mask[bpre] = mask;
            o.bn_link0[bpre] = int32_t(lpre);
            const int nl = __popc(mask);
            for (int k = 0; k < nl; ++k) o.lk_qc[lpre + k] = NOHIT;
        } else {
            o.tag[x] = 0;
            if (g.dim == 3) o.nmask[x] = 0u;
        }
    } else if ((v >> 40) & 1) {
        if (g.dim == 3) o.nmask[x] = 0u;
        o.tag[x] = int32_t(-2 - wpre);
        o.wl_node[wpre] = int32_t(x);
        o.wl_phi[wpre] = 1.0;
    } else {
        if (g.dim == 3) o.nmask[x] = 0u;
        o.tag[x] = -1;
    }
}

// ------------------------------------------------------------------------ q
// First n in [0, 2^16] with f(n) = A n^2 + B n + C <= 0 (the squared distance from the ball
// centre along the link minus r^2); NOHIT if none.  f is convex: decreasing up to its vertex, so
// a bisection on [0, floor(vertex)] finds the first crossing exactly.
__device__ inline uint32_t ball_first_hit(int64_t A, int64_t B, int64_t C) {
    if (C <= 0) return 0;
    if (B >= 0) return NOHIT;
    auto f = [&](int64_t n) { return (A * n + B) * n + C; };
    int64_t m = (-B) / (2 * A);  // floor of the vertex
    if (m > ONE) m = ONE;
    if (f(m) > 0) {
        if (m + 1 <= ONE && f(m + 1) <= 0) return uint32_t(m + 1);
        return NOHIT;
    }
    int64_t lo = 0, hi = m;  // f(lo) > 0, f(hi) <= 0
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (f(mid) <= 0) hi = mid; else lo = mid;
    }
    return uint32_t(hi);
}

__device__ inline void link_hits_ball(const GridDev& g, int L, const mcb_shape& s, int64_t x, const int32_t* __restrict__ tag,
                                      const uint32_t* __restrict__ bn_mask, const int32_t* __restrict__ bn_link0,
                                      uint32_t* lk_qc) {
    const int32_t tg = tag[x];
    if (tg <= 0) return;
    const int b = g.dim == 2 ? (tg >> 8) : tg - 1;
    const uint32_t mask = bn_mask[b];
    int l = bn_link0[b];
    int c[3];
    coords(g, x, c);
    const int64_t C3[3] = {s.cx, s.cy, s.cz};
    const int n[3] = {g.nx, g.ny, g.nz};
    int64_t d[3] = {0, 0, 0};
    for (int k = 0; k < g.dim; ++k) d[k] = min_image(int64_t(c[k]) * ONE - C3[k], int64_t(n[k]) * ONE);
    int64_t C = -s.radius * s.radius;
    for (int k = 0; k < g.dim; ++k) C += d[k] * d[k];
    for (int i = 1; i < g.Q; ++i) {
        if (!((mask >> i) & 1u)) continue;
        const int e[3] = {c_ex[L][i], c_ey[L][i], c_ez[L][i]};
        int64_t A = 0, B = 0;
        for (int k = 0; k < g.dim; ++k) { A += e[k] * e[k]; B += 2 * d[k] * e[k]; }
        const uint32_t h = ball_first_hit(A, B, C);
        if (h != NOHIT) atomicMin(&lk_qc[l], h);
        ++l;
    }
}

__global__ void k_q_ball(const mcb_shape* __restrict__ shapes, GridDev g, int L, const int32_t* __restrict__ tag,
                         const uint32_t* __restrict__ bn_mask, const int32_t* __restrict__ bn_link0, uint32_t* lk_qc) {
    const mcb_shape s = shapes[blockIdx.x];
    if (s.kind != MCB_SHAPE_BALL) return;
    const int64_t C[3] = {s.cx, s.cy, s.cz};
    int lo[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
    for (int k = 0; k < g.dim; ++k) {
        lo[k] = int(floor_div(C[k] - s.radius, ONE)) - 1;
        ext[k] = int(floor_div(C[k] + s.radius, ONE)) + 2 - lo[k];
    }
    const int n[3] = {g.nx, g.ny, g.nz};
    const int64_t total = int64_t(ext[0]) * ext[1] * ext[2];
    for (int64_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
        int c[3] = {lo[0] + int(idx % ext[0]), lo[1] + int((idx / ext[0]) % ext[1]), lo[2] + int(idx / (int64_t(ext[0]) * ext[1]))};
        for (int k = 0; k < 3; ++k) c[k] = wrapn(c[k], n[k]);
        link_hits_ball(g, L, s, lin(g, c[0], c[1], c[2]), tag, bn_mask, bn_link0, lk_qc);
    }
}

__global__ void k_q_band(Bands b, GridDev g, int L, int64_t nb, const int32_t* __restrict__ bn_node,
                         const uint32_t* __restrict__ bn_mask, const int32_t* __restrict__ bn_link0, uint32_t* lk_qc) {
    const int64_t Ly = int64_t(g.ny) * ONE;
    for (int64_t bi = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; bi < nb; bi += int64_t(gridDim.x) * blockDim.x) {
        const int64_t x = bn_node[bi];
        const uint32_t mask = bn_mask[bi];
        const int64_t Y1 = ((x / g.nx) % g.ny) * ONE;
        int l = bn_link0[bi];
        for (int i = 1; i < g.Q; ++i) {
            if (!((mask >> i) & 1u)) continue;
            const int ey = c_ey[L][i];
            uint32_t best = NOHIT;
            for (int k = 0; k < b.n; ++k) {
                const int64_t H = b.s[k].hi - b.s[k].lo;
                int64_t r = (Y1 - b.s[k].lo) % Ly;
                if (r < 0) r += Ly;
                int64_t n = -1;
                if (r <= H) n = 0;
                else if (ey > 0) n = Ly - r;   // climbs into the band's lower face
                else if (ey < 0) n = r - H;    // descends onto its upper face
                if (n >= 0 && n <= ONE && uint32_t(n) < best) best = uint32_t(n);
            }
            if (best != NOHIT) atomicMin(&lk_qc[l], best);
            ++l;
        }
    }
}

// Class from q and the second fluid node, and the link coefficient used by the step: the eq. 16-17
// value is t + a (f~_j(x1) - t) with t = (f~_j(x2) or f~_opp(j)(x1)) + F_j, so the slot holds
// a = 2q (eq. 16), a = 1/(2q) stored negated to mark eq. 17, or a = 1 (bounce-back); slots of
// directions without a link hold NO_LINK.  Flags links no shape was found for.
__global__ void k_class(GridDev g, int L, int64_t nb, const uint8_t* __restrict__ solid, const int32_t* __restrict__ bn_node,
                        const uint32_t* __restrict__ bn_mask, const int32_t* __restrict__ bn_link0, uint32_t* lk_qc,
                        void* rec, int rec_double, int halfway, int32_t* flags) {
    // coefficient a per slot = boundary index * slots per node + direction - 1
    const int64_t QL = g.dim == 2 ? Q2_LINKS : Q3_LINKS;
    for (int64_t bi = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; bi < nb; bi += int64_t(gridDim.x) * blockDim.x) {
        const int64_t x = bn_node[bi];
        const uint32_t mask = bn_mask[bi];
        int c[3];
        coords(g, x, c);
        int l = bn_link0[bi];
        for (int i = 1; i < g.Q; ++i) {
            double a = NO_LINK;
            if ((mask >> i) & 1u) {
                uint32_t q = lk_qc[l] & (NOHIT >> 2);
                if (q > uint32_t(ONE)) {
                    atomicOr(&flags[FLAG_NOHIT], 1);
                    q = uint32_t(ONE / 2);
                }
                int cls;
                if (q >= uint32_t(ONE / 2)) cls = MCB_CLS_EQ17;
                else cls = solid[neighbour(g, c, L, i, -1)] ? MCB_CLS_HBB : MCB_CLS_EQ16;
                lk_qc[l] = q | (uint32_t(cls) << CLS_SHIFT);
                const double q2 = double(q) * (2.0 / 65536.0);
                a = cls == MCB_CLS_EQ16 ? q2 : (cls == MCB_CLS_EQ17 ? -1.0 / q2 : 1.0);
                if (halfway) a = 1.0;  // halfway bounce-back on every link, whatever q
                ++l;
            }
            const int64_t slot = bi * QL + (i - 1);
            if (rec_double) static_cast<double*>(rec)[slot] = a;
            else static_cast<float*>(rec)[slot] = float(a);
        }
        for (int64_t i = g.Q - 1; i < QL; ++i) {
            if (rec_double) static_cast<double*>(rec)[bi * QL + i] = NO_LINK;
            else static_cast<float*>(rec)[bi * QL + i] = float(NO_LINK);
        }
    }
}

// Eq. 15 gives a wall node the lattice-weighted mean density of its fluid neighbours times phi.  The
// weights of the fluid neighbours are fixed by the geometry, so the step takes
// fac = phi / sum_{fluid x + e_i} w_i and multiplies it by sum_i w_i rho(x + e_i), in which solid
// neighbours count with rho = 0.
template <class C>
__global__ void k_wall_fac(GridDev g, int L, int64_t nw, const int32_t* __restrict__ wl_node, const uint8_t* __restrict__ solid,
                           const double* __restrict__ phi, C* __restrict__ fac) {
    for (int64_t w = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; w < nw; w += int64_t(gridDim.x) * blockDim.x) {
        int c[3];
        coords(g, wl_node[w], c);
        double den = 0.0;
        for (int i = 1; i < g.Q; ++i) {
            const double wi = L == 0 ? (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0) : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
            if (!solid[neighbour(g, c, L, i, +1)]) den += wi;
        }
        fac[w] = C(phi[w] / den);
    }
}

inline int lat_index(const mcb_ctx* c) { return c->g.dim == 2 ? 0 : 1; }

inline unsigned grid_for(int64_t n, int block) {
    int64_t b = (n + block - 1) / block;
    if (b > 65535 * 16) b = 65535 * 16;
    return unsigned(b < 1 ? 1 : b);
}

// indices of the second-layer nodes (any order: each is computed on its own)
__global__ void k_cp_l2_list(int64_t N, const int8_t* __restrict__ layer, int32_t* __restrict__ list,
                             unsigned long long* __restrict__ count) {
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < N; x += int64_t(gridDim.x) * blockDim.x)
        if (layer[x] == 2) list[atomicAdd(count, 1ull)] = int32_t(x);
}

// solid layers of eq. 15 for the chemical-potential model: 0 fluid, 1 a wall node (a fluid
// neighbour), 2 a solid node with a wall-node neighbour, 3 deeper
__global__ void k_cp_layers(GridDev g, int L, const int32_t* __restrict__ tag, int8_t* __restrict__ layer) {
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < g.N; x += int64_t(gridDim.x) * blockDim.x) {
        const int32_t tg = tag[x];
        int8_t v = tg >= 0 ? 0 : (tg <= -2 ? 1 : 3);
        if (v == 3) {
            int c[3];
            coords(g, x, c);
            for (int i = 1; i < g.Q; ++i)
                if (tag[neighbour(g, c, L, i, +1)] <= -2) { v = 2; break; }
        }
        layer[x] = v;
    }
}

}  // namespace

hipError_t geom_classify(mcb_ctx* c) {
    uint8_t* solid = reinterpret_cast<uint8_t*>(c->lat + c->L.solid);
    const mcb_shape* shapes = reinterpret_cast<const mcb_shape*>(c->lat + c->L.shapes);
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(c->g.N, 256)), dim3(256), 0, c->stream, solid, c->g.N, uint8_t(0));
    if (c->n_shapes > 0)
        hipLaunchKernelGGL(k_raster_ball, dim3(unsigned(c->n_shapes)), dim3(256), 0, c->stream, shapes, c->g, solid);
    if (c->n_bands > 0) {
        Bands b{};
        b.n = c->n_bands;
        for (int k = 0; k < c->n_bands; ++k) b.s[k] = c->bands[k];
        hipLaunchKernelGGL(k_raster_band, dim3(grid_for(c->g.N, 256)), dim3(256), 0, c->stream, b, c->g, solid);
    }
    return hipGetLastError();
}

hipError_t geom_count(mcb_ctx* c) {
    const uint8_t* solid = reinterpret_cast<const uint8_t*>(c->lat + c->L.solid);
    int64_t* bs = reinterpret_cast<int64_t*>(c->lat + c->L.blocksums);
    const int64_t nblk = (c->g.N + SCAN_BLOCK - 1) / SCAN_BLOCK;
    hipLaunchKernelGGL(k_count, dim3(unsigned(nblk)), dim3(SCAN_BLOCK), 0, c->stream, c->g, lat_index(c), solid, bs);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, c->stream, bs, nblk);
    return hipGetLastError();
}

hipError_t geom_fill(mcb_ctx* c) {
    const uint8_t* solid = reinterpret_cast<const uint8_t*>(c->lat + c->L.solid);
    const int64_t* bs = reinterpret_cast<const int64_t*>(c->lat + c->L.blocksums);
    const int64_t nblk = (c->g.N + SCAN_BLOCK - 1) / SCAN_BLOCK;
    FillOut o;
    o.tag = reinterpret_cast<int32_t*>(c->lat + c->L.tag);
    o.nmask = reinterpret_cast<uint32_t*>(c->lat + c->L.nmask);
    o.bn_node = reinterpret_cast<int32_t*>(c->lk + c->L.bn_node);
    o.bn_mask = reinterpret_cast<uint32_t*>(c->lk + c->L.bn_mask);
    o.bn_link0 = reinterpret_cast<int32_t*>(c->lk + c->L.bn_link0);
    o.lk_qc = reinterpret_cast<uint32_t*>(c->lk + c->L.lk_qc);
    o.wl_node = reinterpret_cast<int32_t*>(c->lk + c->L.wl_node);
    o.wl_phi = reinterpret_cast<double*>(c->lk + c->L.wl_phi);
    const int L = lat_index(c);
    hipLaunchKernelGGL(k_fill, dim3(unsigned(nblk)), dim3(SCAN_BLOCK), 0, c->stream, c->g, L, solid, bs, o);
    const mcb_shape* shapes = reinterpret_cast<const mcb_shape*>(c->lat + c->L.shapes);
    if (c->n_shapes > 0 && c->n_bnodes > 0)
        hipLaunchKernelGGL(k_q_ball, dim3(unsigned(c->n_shapes)), dim3(256), 0, c->stream, shapes, c->g, L, o.tag,
                           o.bn_mask, o.bn_link0, o.lk_qc);
    if (c->n_bands > 0 && c->n_bnodes > 0) {
        Bands b{};
        b.n = c->n_bands;
        for (int k = 0; k < c->n_bands; ++k) b.s[k] = c->bands[k];
        hipLaunchKernelGGL(k_q_band, dim3(grid_for(c->n_bnodes, 256)), dim3(256), 0, c->stream, b, c->g, L, c->n_bnodes,
                           o.bn_node, o.bn_mask, o.bn_link0, o.lk_qc);
    }
    hipError_t e;
    if (c->p.model == MCB_MODEL_CHEMPOT) {
        int8_t* layer = reinterpret_cast<int8_t*>(c->lat + c->L.cp_layer);
        unsigned long long* cnt = reinterpret_cast<unsigned long long*>(c->lat + c->L.cp_l2n);
        hipLaunchKernelGGL(k_cp_layers, dim3(grid_for(c->g.N, 256)), dim3(256), 0, c->stream, c->g, L, o.tag, layer);
        if ((e = hipMemsetAsync(cnt, 0, 8, c->stream)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_cp_l2_list, dim3(grid_for(c->g.N, 256)), dim3(256), 0, c->stream, c->g.N, layer,
                           reinterpret_cast<int32_t*>(c->lat + c->L.cp_l2), cnt);
        // the second-layer count sizes a launch of every step: read it once here
        unsigned long long n = 0;
        if ((e = hipMemcpyAsync(&n, cnt, 8, hipMemcpyDeviceToHost, c->stream)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
        c->n_l2 = int64_t(n);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = wall_factors(c);
    if (e != hipSuccess) return e;
    return geom_reclass(c);
}

hipError_t wall_factors(mcb_ctx* c) {
    // chemical-potential model: the solid layers' chemical potential follows the assigned values
    const hipError_t e = cp_wall_mu(c);
    if (e != hipSuccess || c->n_wall <= 0) return e;
    const uint8_t* solid = reinterpret_cast<const uint8_t*>(c->lat + c->L.solid);
    const int32_t* wn = reinterpret_cast<const int32_t*>(c->lk + c->L.wl_node);
    const double* phi = reinterpret_cast<const double*>(c->lk + c->L.wl_phi);
    if (c->p.precision == MCB_F64)
        hipLaunchKernelGGL(k_wall_fac<double>, dim3(grid_for(c->n_wall, 256)), dim3(256), 0, c->stream, c->g, lat_index(c),
                           c->n_wall, wn, solid, phi, reinterpret_cast<double*>(c->lk + c->L.wl_fac));
    else
        hipLaunchKernelGGL(k_wall_fac<float>, dim3(grid_for(c->n_wall, 256)), dim3(256), 0, c->stream, c->g, lat_index(c),
                           c->n_wall, wn, solid, phi, reinterpret_cast<float*>(c->lk + c->L.wl_fac));
    return hipGetLastError();
}

hipError_t geom_reclass(mcb_ctx* c) {
    if (c->n_bnodes <= 0) return hipSuccess;
    const uint8_t* solid = reinterpret_cast<const uint8_t*>(c->lat + c->L.solid);
    int32_t* flags = reinterpret_cast<int32_t*>(c->lat + c->L.flags);
    hipLaunchKernelGGL(k_class, dim3(grid_for(c->n_bnodes, 256)), dim3(256), 0, c->stream, c->g, lat_index(c), c->n_bnodes,
                       solid, reinterpret_cast<const int32_t*>(c->lk + c->L.bn_node),
                       reinterpret_cast<const uint32_t*>(c->lk + c->L.bn_mask),
                       reinterpret_cast<const int32_t*>(c->lk + c->L.bn_link0),
                       reinterpret_cast<uint32_t*>(c->lk + c->L.lk_qc), static_cast<void*>(c->lk + c->L.lk_a),
                       c->p.precision == MCB_F64 ? 1 : 0, c->p.bc_mode == MCB_BC_HBBC ? 1 : 0, flags);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // both buffers of boundary records start empty (the first collision writes them)
    const size_t rb = size_t(compute_bytes(c->p.precision) * c->L.rec_stride * c->n_bnodes);
    for (int b = 0; b < 2; ++b) {
        const hipError_t e2 = hipMemsetAsync(c->lk + c->L.rec[b], 0, rb, c->stream);
        if (e2 != hipSuccess) return e2;
    }
    return hipSuccess;
}

}  // namespace mcb
