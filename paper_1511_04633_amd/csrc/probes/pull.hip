// pull.hip -- the lattice Boltzmann step's access pattern without arithmetic:
// 26 population streams of a 256^3 FP32 lattice in the slab layout of
// kernels.hpp (2048 nodes per slab), each node reading its 26 values from
// the upstream neighbours (x-shifted streams unaligned) and writing them at
// itself with non-temporal stores, with 1, 2 or 4 consecutive nodes per
// thread (4-, 8- and 16-byte accesses).  Indices are clamped into the
// lattice, so the pattern is the step's and every access is in bounds.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>

#define CK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e), __LINE__); exit(1);} } while (0)

typedef float f1a;
typedef float f2a __attribute__((ext_vector_type(2), aligned(4)));
typedef float f4a __attribute__((ext_vector_type(4), aligned(4)));
typedef float f2n __attribute__((ext_vector_type(2)));
typedef float f4n __attribute__((ext_vector_type(4)));

__constant__ int EX[26] = {0,1,-1,0,0,0,0,1,-1,1,-1,1,-1,1,-1,0,0,0,0, 0,1,-1,0,0,0,0};
__constant__ int EY[26] = {0,0,0,1,-1,0,0,1,1,-1,-1,0,0,0,0,1,-1,1,-1, 0,0,0,1,-1,0,0};
__constant__ int EZ[26] = {0,0,0,0,0,1,-1,0,0,0,0,1,1,-1,-1,1,1,-1,-1, 0,0,0,0,0,1,-1};

constexpr int L = 11;
constexpr unsigned SEG = 4u << L, SLAB = 26u * SEG;

__device__ __forceinline__ unsigned off(unsigned c, int i) { return c * 4u + (c >> L) * (SLAB - SEG) + unsigned(i) * SEG; }

template <int NPT>
__global__ __launch_bounds__(256) void k_pull(const char *__restrict__ src, char *__restrict__ dst, int n, unsigned maxoff)
{
    const int x0 = (blockIdx.x * blockDim.x + threadIdx.x) * NPT;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x0 >= n) return;
    const unsigned c = unsigned(x0) + unsigned(n) * (unsigned(y) + unsigned(n) * unsigned(z));
    using V = typename std::conditional<NPT == 1, f1a, typename std::conditional<NPT == 2, f2a, f4a>::type>::type;
    using W = typename std::conditional<NPT == 1, float, typename std::conditional<NPT == 2, f2n, f4n>::type>::type;
    V v[26];
#pragma unroll
    for (int i = 0; i < 26; ++i) {
        const int up = int(c) - EX[i] - EY[i] * n - EZ[i] * n * n;
        unsigned o = off(unsigned(min(max(up, 0), n * n * n - NPT)), i);
        o = min(o, maxoff);
        v[i] = *(const V *)(src + o);
    }
#pragma unroll
    for (int i = 0; i < 26; ++i)
        __builtin_nontemporal_store((W)v[i], (W *)(dst + off(c, i)));
}

int main()
{
    const int n = 256;
    const size_t cells = size_t(n) * n * n;
    const size_t bytes = cells * 104;
    char *a, *b;
    CK(hipMalloc(&a, bytes));
    CK(hipMalloc(&b, bytes));
    CK(hipMemset(a, 0, bytes));
    CK(hipMemset(b, 0, bytes));
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    auto timeit = [&](const char *name, auto launch) {
        for (int w = 0; w < 3; ++w) launch();
        CK(hipDeviceSynchronize());
        const int reps = 20;
        CK(hipEventRecord(e0, 0));
        for (int r = 0; r < reps; ++r) launch();
        CK(hipEventRecord(e1, 0));
        CK(hipEventSynchronize(e1));
        float ms = 0;
        CK(hipEventElapsedTime(&ms, e0, e1));
        const double us = 1e3 * ms / reps;
        printf("%-34s %8.1f us %7.1f GB/s\n", name, us, 2.0 * bytes / (us * 1e-6) / 1e9);
        fflush(stdout);
    };
    const unsigned maxoff1 = unsigned(bytes - 4), maxoff2 = unsigned(bytes - 8), maxoff4 = unsigned(bytes - 16);
    timeit("pull26 1 node/thread (dword)", [&] { hipLaunchKernelGGL(k_pull<1>, dim3(1, n, n), dim3(256), 0, 0, a, b, n, maxoff1); });
    timeit("pull26 2 nodes/thread (dwordx2)", [&] { hipLaunchKernelGGL(k_pull<2>, dim3(1, n, n), dim3(128), 0, 0, a, b, n, maxoff2); });
    timeit("pull26 4 nodes/thread (dwordx4)", [&] { hipLaunchKernelGGL(k_pull<4>, dim3(1, n, n), dim3(64), 0, 0, a, b, n, maxoff4); });
    CK(hipFree(a)); CK(hipFree(b));
    printf("done\n");
    return 0;
}
