// Bandwidth ceilings of the lattice step's memory pattern on one device: a plain copy of the same
// bytes, and a plain pull (streaming of eq. 5 alone, no collision, no boundary) of D2Q9 and D3Q19
// populations stored as FP32 planes.  Each kernel reads Q planes of N values and writes Q planes,
// which is what one step moves per node; the step kernels are compared against these.
//
//   mcb_ceiling [nx ny [nz]] [reps]     (default 4096 4096 for D2Q9 and 256^3 for D3Q19, 50 reps)
//
// Prints, per kernel, the average time of one launch (HIP events around each launch) and the
// bytes it moves per second.  Standalone: no part of the library.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHK(x)                                                                             \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) {                                                            \
            std::fprintf(stderr, "%s:%d %s: %s\n", __FILE__, __LINE__, #x, hipGetErrorString(e_)); \
            std::exit(1);                                                                  \
        }                                                                                  \
    } while (0)

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// copy of n4 float4 values, one per lane, non-temporal stores
__global__ __launch_bounds__(256) void k_copy_x4(const f4* __restrict__ a, f4* __restrict__ b, uint32_t n4) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < n4) __builtin_nontemporal_store(a[i], b + i);
}

// copy of n float values, one per lane
__global__ __launch_bounds__(256) void k_copy_dw(const float* __restrict__ a, float* __restrict__ b, uint32_t n) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(a[i], b + i);
}

__device__ constexpr int ex2[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int ey2[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// D2Q9 pull, one node per lane: f_i(x) <- f_i(x - e_i), periodic; 256 lanes along a row
__global__ __launch_bounds__(256) void k_pull2d_dw(const float* __restrict__ a, float* __restrict__ b, int nx, int ny) {
    const int nbx = (nx + 255) / 256;
    const int y = blockIdx.x / nbx, x = (blockIdx.x % nbx) * 256 + threadIdx.x;
    if (x >= nx) return;
    const uint32_t N = uint32_t(nx) * uint32_t(ny);
    const int xs[3] = {x == nx - 1 ? 0 : x + 1, x, x == 0 ? nx - 1 : x - 1};
    const int ys[3] = {y == ny - 1 ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
    float f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = a[i * N + uint32_t(ys[ey2[i] + 1]) * nx + xs[ex2[i] + 1]];
    const uint32_t o = uint32_t(y) * nx + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) __builtin_nontemporal_store(f[i], b + i * N + o);
}

// D2Q9 pull, four consecutive nodes of a row per lane (nx a multiple of 4): the unshifted planes
// move as aligned float4, the x-shifted ones as float4 at a 4-byte offset
__global__ __launch_bounds__(256) void k_pull2d_x4(const float* __restrict__ a, float* __restrict__ b, int nx, int ny) {
    const int nq = nx / 4, nbx = (nq + 255) / 256;
    const int y = blockIdx.x / nbx, xq = (blockIdx.x % nbx) * 256 + threadIdx.x;
    if (xq >= nq) return;
    const int x = 4 * xq;
    const uint32_t N = uint32_t(nx) * uint32_t(ny);
    const int ys[3] = {y == ny - 1 ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
    f4 f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const float* row = a + i * N + uint32_t(ys[ey2[i] + 1]) * nx;
        if (ex2[i] == 0) {
            f[i] = *reinterpret_cast<const f4*>(row + x);
        } else if (ex2[i] > 0) {  // from x - 1 .. x + 2
            const float l = row[x == 0 ? nx - 1 : x - 1];
            f[i] = f4{l, row[x], row[x + 1], row[x + 2]};
        } else {  // from x + 1 .. x + 4
            const float r = row[x + 4 == nx ? 0 : x + 4];
            f[i] = f4{row[x + 1], row[x + 2], row[x + 3], r};
        }
    }
    const uint32_t o = uint32_t(y) * nx + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) __builtin_nontemporal_store(f[i], reinterpret_cast<f4*>(b + i * N + o));
}

__device__ constexpr int ex3[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ constexpr int ey3[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int ez3[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

// D3Q19 pull, one node per lane, 256 lanes along a row
__global__ __launch_bounds__(256) void k_pull3d_dw(const float* __restrict__ a, float* __restrict__ b, int nx, int ny, int nz) {
    const int nbx = (nx + 255) / 256;
    const int row = blockIdx.x / nbx, x = (blockIdx.x % nbx) * 256 + threadIdx.x;
    if (x >= nx) return;
    const int y = row % ny, z = row / ny;
    const uint32_t nxy = uint32_t(nx) * uint32_t(ny), N = nxy * uint32_t(nz);
    const int xs[3] = {x == nx - 1 ? 0 : x + 1, x, x == 0 ? nx - 1 : x - 1};
    const int ys[3] = {y == ny - 1 ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
    const int zs[3] = {z == nz - 1 ? 0 : z + 1, z, z == 0 ? nz - 1 : z - 1};
    float f[19];
#pragma unroll
    for (int i = 0; i < 19; ++i)
        f[i] = a[i * N + uint32_t(zs[ez3[i] + 1]) * nxy + uint32_t(ys[ey3[i] + 1]) * nx + xs[ex3[i] + 1]];
    const uint32_t o = uint32_t(z) * nxy + uint32_t(y) * nx + x;
#pragma unroll
    for (int i = 0; i < 19; ++i) __builtin_nontemporal_store(f[i], b + i * N + o);
}

template <class L>
double time_ms(L launch, int reps) {
    hipEvent_t e0, e1;
    CHK(hipEventCreate(&e0));
    CHK(hipEventCreate(&e1));
    for (int w = 0; w < 5; ++w) launch();
    CHK(hipDeviceSynchronize());
    double tot = 0.0;
    for (int r = 0; r < reps; ++r) {
        CHK(hipEventRecord(e0, 0));
        launch();
        CHK(hipEventRecord(e1, 0));
        CHK(hipEventSynchronize(e1));
        float ms = 0.f;
        CHK(hipEventElapsedTime(&ms, e0, e1));
        tot += ms;
    }
    CHK(hipEventDestroy(e0));
    CHK(hipEventDestroy(e1));
    return tot / reps;
}

void report(const char* name, double ms, double bytes) {
    std::printf("%-12s %9.1f us  %8.1f GB/s  (%.1f MB per launch)\n", name, ms * 1e3, bytes / (ms * 1e-3) / 1e9, bytes / 1e6);
    std::fflush(stdout);
}

}  // namespace

int main(int argc, char** argv) {
    int nx = 4096, ny = 4096, nz3 = 256, reps = 50;
    if (argc >= 3) {
        nx = std::atoi(argv[1]);
        ny = std::atoi(argv[2]);
    }
    if (argc >= 4) nz3 = std::atoi(argv[3]);
    if (argc >= 5) reps = std::atoi(argv[4]);
    if (nx < 8 || ny < 3 || nx % 4 || nz3 < 3 || reps < 1) {
        std::fprintf(stderr, "usage: mcb_ceiling [nx ny [nz [reps]]], nx a multiple of 4 and >= 8\n");
        return 2;
    }
    const size_t N2 = size_t(nx) * ny, N3 = size_t(nz3) * nz3 * nz3;
    const size_t elems = std::max(9 * N2, 19 * N3);
    if (elems >= (size_t(1) << 32)) {
        std::fprintf(stderr, "lattice too large for 32-bit indices\n");
        return 2;
    }
    float *a = nullptr, *b = nullptr;
    CHK(hipMalloc(&a, elems * sizeof(float)));
    CHK(hipMalloc(&b, elems * sizeof(float)));
    CHK(hipMemset(a, 0, elems * sizeof(float)));
    CHK(hipMemset(b, 0, elems * sizeof(float)));
    std::printf("D2Q9 %dx%d FP32 (%zu nodes), D3Q19 %d^3 FP32 (%zu nodes), %d launches each\n", nx, ny, N2, nz3, N3, reps);
    {
        const uint32_t n = uint32_t(9 * N2), n4 = n / 4;
        const double bytes = 2.0 * n * 4;
        report("copy_dw_9", time_ms([&] { hipLaunchKernelGGL(k_copy_dw, dim3((n + 255) / 256), dim3(256), 0, 0, a, b, n); }, reps), bytes);
        report("copy_x4_9", time_ms([&] {
                   hipLaunchKernelGGL(k_copy_x4, dim3((n4 + 255) / 256), dim3(256), 0, 0, reinterpret_cast<const f4*>(a),
                                      reinterpret_cast<f4*>(b), n4);
               }, reps), bytes);
        const int nbx = (nx + 255) / 256;
        report("pull2d_dw", time_ms([&] { hipLaunchKernelGGL(k_pull2d_dw, dim3(nbx * ny), dim3(256), 0, 0, a, b, nx, ny); }, reps),
               bytes);
        const int nbq = (nx / 4 + 255) / 256;
        report("pull2d_x4", time_ms([&] { hipLaunchKernelGGL(k_pull2d_x4, dim3(nbq * ny), dim3(256), 0, 0, a, b, nx, ny); }, reps),
               bytes);
    }
    {
        const uint32_t n = uint32_t(19 * N3), n4 = n / 4;
        const double bytes = 2.0 * n * 4;
        report("copy_x4_19", time_ms([&] {
                   hipLaunchKernelGGL(k_copy_x4, dim3((n4 + 255) / 256), dim3(256), 0, 0, reinterpret_cast<const f4*>(a),
                                      reinterpret_cast<f4*>(b), n4);
               }, reps), bytes);
        const int nbx = (nz3 + 255) / 256;
        report("pull3d_dw", time_ms([&] {
                   hipLaunchKernelGGL(k_pull3d_dw, dim3(nbx * nz3 * nz3), dim3(256), 0, 0, a, b, nz3, nz3, nz3);
               }, reps), bytes);
    }
    CHK(hipFree(a));
    CHK(hipFree(b));
    return 0;
}
