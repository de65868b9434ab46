// Device helpers shared by the step, boundary and monitor kernels.
#pragma once

#include "mcb_internal.h"

#include <type_traits>

namespace mcb {

// ---------------------------------------------------------------- storage conversions
// 64-bit and 32-bit element indices (the 32-bit forms let the compiler address from a scalar base)
template <class S, class C>
__device__ inline C ld(const S* __restrict__ p, int64_t i);
template <>
__device__ inline double ld<double, double>(const double* __restrict__ p, int64_t i) { return p[i]; }
template <>
__device__ inline float ld<float, float>(const float* __restrict__ p, int64_t i) { return p[i]; }
template <>
__device__ inline float ld<__half, float>(const __half* __restrict__ p, int64_t i) { return __half2float(p[i]); }
template <class S, class C>
__device__ inline C ld(const S* __restrict__ p, uint32_t i) { return ld<S, C>(p, int64_t(i)); }

template <class S, class C>
__device__ inline void st(S* __restrict__ p, int64_t i, C v);
template <>
__device__ inline void st<double, double>(double* __restrict__ p, int64_t i, double v) { p[i] = v; }
template <>
__device__ inline void st<float, float>(float* __restrict__ p, int64_t i, float v) { p[i] = v; }
template <>
__device__ inline void st<__half, float>(__half* __restrict__ p, int64_t i, float v) { p[i] = __float2half_rn(v); }
template <class S, class C>
__device__ inline void st(S* __restrict__ p, uint32_t i, C v) { st<S, C>(p, int64_t(i), v); }

// ---------------------------------------------------------------- mass balance of the collision
// The collision gives a node back exactly the mass it pulled: f_0 = (sum of the pulled populations)
// - (the other outputs as stored).  With FP32 storage both sums are formed in FP64 (nine FP32
// values do not add exactly in FP32, and that rounding would stay in the node's mass); FP16 values
// add exactly in FP32, FP64 in FP64.
template <class S, class C>
using MassAcc = typename std::conditional<std::is_same<S, float>::value, double, C>::type;

// The eq. 18 correction of a boundary node is summed in FP64 from its link differences and added to
// the rest population in FP64, then rounded once to the compute type; what that rounding drops (at
// most half an ulp of f_0, carried in the compute type to within 2^-24 of itself) joins the
// collision's mass sum, so the node keeps the mass balance of eq. 18 to within ~2^-48 f_0 whatever
// the storage precision, and the correction never rounds on its own.

// ---------------------------------------------------------------- population planes
// Populations are stored as Q planes of N values (SoA).  With FP16 storage the rest population
// (plane 0) is kept in FP32, in the space of the first two half planes: it holds about 4/9 of the
// mass and takes the rounding of the mass-conserving collision, which in FP16 would bias the mass;
// plane i >= 1 then starts at half plane i + 1.
template <class S>
constexpr bool kMixed = sizeof(S) == 2;
template <class S>
__host__ __device__ inline int64_t plane_off(int i, int64_t N) {  // in elements of S
    return (kMixed<S> && i > 0) ? int64_t(i + 1) * N : int64_t(i) * N;
}
template <class S, class C>
__device__ inline C ldp(const S* __restrict__ f, int i, int64_t N, int64_t x) {
    if (kMixed<S> && i == 0) return C(reinterpret_cast<const float*>(f)[x]);
    return ld<S, C>(f, plane_off<S>(i, N) + x);
}
template <class S, class C>
__device__ inline void stp(S* __restrict__ f, int i, int64_t N, int64_t x, C v) {
    if (kMixed<S> && i == 0) {
        reinterpret_cast<float*>(f)[x] = float(v);
        return;
    }
    st<S, C>(f, plane_off<S>(i, N) + x, v);
}
// the same store, non-temporal (streaming): the lattice being written does not evict from L2 the
// lines other workgroups read next
template <class S, class C>
__device__ inline void stp_nt(S* __restrict__ f, int i, int64_t N, int64_t x, C v) {
    if constexpr (kMixed<S>) {
        if (i == 0) {
            __builtin_nontemporal_store(float(v), reinterpret_cast<float*>(f) + x);
            return;
        }
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, __float2half_rn(float(v))),
                                    reinterpret_cast<unsigned short*>(f) + plane_off<S>(i, N) + x);
    } else {
        __builtin_nontemporal_store(S(v), f + plane_off<S>(i, N) + x);
    }
}

// ---------------------------------------------------------------- bounds-checked buffer access
// Raw buffer instructions address from a scalar 128-bit resource plus a 32-bit per-lane byte
// offset; an offset at or beyond the resource size makes a load return 0 and drops a store.  A
// lane that must not touch memory gets offset OOB, so loads and stores need no divergent branch
// (and the compiler can keep track of how many memory operations are in flight).
constexpr uint32_t OOB = 0xFFFFFF00u;
constexpr uint32_t BUF_MAX = 0xFFFFFE00u;  // largest resource size used

__device__ inline __amdgpu_buffer_rsrc_t make_res(const void* p, uint64_t bytes) {
    const uint32_t n = bytes > BUF_MAX ? BUF_MAX : uint32_t(bytes);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, int(n), 0x00020000);
}

// Loads may also take a wave-uniform part of the offset in soffset (an SGPR).  Only loads do: a
// load whose lane offset is OOB can at worst read a valid word of the same buffer, which the
// caller discards, whereas a store must be dropped for certain.
template <class S>
struct Buf;
// cache policy of a buffer store that streams: non-temporal, so the lattice being written does not
// push out of L2 the lines that neighbouring workgroups are about to read
constexpr int CPOL_NT = 2;
template <>
struct Buf<double> {
    static __device__ inline double ld(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    }
    static __device__ inline double ld(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
    }
    static __device__ inline double round(double v) { return v; }
    static __device__ inline void st(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
    }
    static __device__ inline void st_nt(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, CPOL_NT);
    }
};
template <>
struct Buf<float> {
    static __device__ inline float ld(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
    static __device__ inline float ld(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
    }
    static __device__ inline float round(float v) { return v; }
    static __device__ inline void st(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, 0);
    }
    static __device__ inline void st_nt(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, CPOL_NT);
    }
};
template <>
struct Buf<__half> {
    static __device__ inline float ld(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        return __half2float(__builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0)));
    }
    static __device__ inline float ld(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
        return __half2float(__builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0)));
    }
    static __device__ inline float round(float v) { return __half2float(__float2half_rn(v)); }
    static __device__ inline void st(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, __float2half_rn(v)), r, off, 0, 0);
    }
    static __device__ inline void st_nt(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, __float2half_rn(v)), r, off, 0, CPOL_NT);
    }
};
__device__ inline int32_t ld_i32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return int32_t(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ inline int32_t ld_i32(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return int32_t(__builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}
// unsigned saturating add: an OOB lane offset stays out of bounds for any in-bounds addend
__device__ inline uint32_t sat_add(uint32_t a, uint32_t b) { return __builtin_elementwise_add_sat(a, b); }

// NV consecutive values of type C at byte offset off (a multiple of 16, or OOB) with 16-byte buffer
// loads and stores (8 and 4 bytes for a remainder).  A lane at OOB reads zeros and writes nothing.
template <class C, int NV>
__device__ inline void ld_vec(__amdgpu_buffer_rsrc_t r, uint32_t off, C (&v)[NV]) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    constexpr int B = NV * int(sizeof(C));
    static_assert(B % 4 == 0, "whole words");
    uint32_t w[B / 4];
    int k = 0;
#pragma unroll
    for (; k + 16 <= B; k += 16) {
        const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, off + uint32_t(k), 0, 0);
        w[k / 4] = x[0]; w[k / 4 + 1] = x[1]; w[k / 4 + 2] = x[2]; w[k / 4 + 3] = x[3];
    }
    if (k + 8 <= B) {
        const u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(r, off + uint32_t(k), 0, 0);
        w[k / 4] = x[0]; w[k / 4 + 1] = x[1];
        k += 8;
    }
    if (k + 4 <= B) w[k / 4] = __builtin_amdgcn_raw_buffer_load_b32(r, off + uint32_t(k), 0, 0);
    __builtin_memcpy(v, w, B);
}
template <class C, int NV>
__device__ inline void st_vec(__amdgpu_buffer_rsrc_t r, uint32_t off, const C (&v)[NV]) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    constexpr int B = NV * int(sizeof(C));
    static_assert(B % 4 == 0, "whole words");
    uint32_t w[B / 4];
    __builtin_memcpy(w, v, B);
    int k = 0;
#pragma unroll
    for (; k + 16 <= B; k += 16) {
        const u32x4 x = {w[k / 4], w[k / 4 + 1], w[k / 4 + 2], w[k / 4 + 3]};
        __builtin_amdgcn_raw_buffer_store_b128(x, r, sat_add(off, uint32_t(k)), 0, 0);
    }
    if (k + 8 <= B) {
        const u32x2 x = {w[k / 4], w[k / 4 + 1]};
        __builtin_amdgcn_raw_buffer_store_b64(x, r, sat_add(off, uint32_t(k)), 0, 0);
        k += 8;
    }
    if (k + 4 <= B) __builtin_amdgcn_raw_buffer_store_b32(w[k / 4], r, sat_add(off, uint32_t(k)), 0, 0);
}

// reciprocal: IEEE division in FP64, the hardware reciprocal (1 ulp) in FP32
__device__ inline double rcp(double x) { return 1.0 / x; }
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double fsqrt(double x) { return sqrt(x); }
__device__ inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// ---------------------------------------------------------------- launch shape
// Workgroups of a kernel that the device holds at once (occupancy per compute unit x units).  The
// marching step kernels size their segments so that the whole grid is resident: every workgroup
// starts together, neighbours march in step (their shared halo lines meet in L2), and no partial
// last round leaves units idle.
// occ caches the per-unit occupancy (a property of the kernel alone; 0 = not yet queried).
template <class K>
inline int resident_blocks(const mcb_ctx* c, K kernel, int threads, int* occ) {
    if (*occ < 1) {
        int o = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, kernel, threads, 0) != hipSuccess || o < 1) o = 1;
        *occ = o;
    }
    return *occ * (c->n_cu > 0 ? c->n_cu : 1);
}

// ---------------------------------------------------------------- thermodynamics
template <class C>
struct Eos {
    C RT, a, b4, two_over_G;  // R T, a, b / 4, 2 / G
};

// Effective mass of the EOS-based pseudopotential: rho c_s^2 + G psi^2 / 2 = p_CS(rho), c = 1.
// A non-positive density or a negative square-root argument sets *bad (and gives psi = 0).
template <class C>
__device__ inline C psi_val(C rho, const Eos<C>& e, bool* bad) {
    const C eta = rho * e.b4;
    const C om = C(1) - eta;
    const C p = rho * e.RT * (C(1) + eta + eta * eta - eta * eta * eta) * rcp(om * om * om) - e.a * rho * rho;
    const C arg = (p - rho * C(1.0 / 3.0)) * e.two_over_G;
    const bool ok = (rho > C(0)) && (arg >= C(0));
    *bad = *bad || !ok;
    return ok ? fsqrt(arg) : C(0);
}

// As psi_val, raising the sticky domain flag directly (kernels outside the hot loop).
template <class C>
__device__ inline C psi_of(C rho, const Eos<C>& e, int32_t* flags) {
    const C eta = rho * e.b4;
    const C om = C(1) - eta;
    const C p = rho * e.RT * (C(1) + eta + eta * eta - eta * eta * eta) * rcp(om * om * om) - e.a * rho * rho;
    const C arg = (p - rho * C(1.0 / 3.0)) * e.two_over_G;
    if (!(rho > C(0)) || !(arg >= C(0))) {
        atomicOr(&flags[FLAG_DOMAIN], 1);
        return C(0);
    }
    return fsqrt(arg);
}

__device__ inline int wrap1(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

}  // namespace mcb
