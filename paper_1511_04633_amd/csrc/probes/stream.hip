// stream.hip -- HBM streaming probes for MI355X: read-only, write-only and
// copy kernels over buffers the size of one FP32 256^3 lattice (1.745 GB),
// with 4- and 16-byte accesses, plain and non-temporal stores, one element
// per thread or grid-stride loops of 4..32 blocks per CU, and the 26-plane
// copy shape of the lattice Boltzmann step.  Prints one line per variant:
// time per launch (HIP events, 10 launches after 3 warm-up) and GB/s moved.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <vector>

typedef float f4v __attribute__((ext_vector_type(4)));
#define CK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e), __LINE__); exit(1);} } while (0)

// grid-stride read of f4v, sum kept; writes only if the sum is a magic value
__global__ void k_read4(const f4v *__restrict__ a, size_t n, float *out)
{
    float s = 0.f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        f4v v = a[i];
        s += v.x + v.y + v.z + v.w;
    }
    if (s == 1234.5678f) out[0] = s;
}
// read of f4v, UNR independent loads per thread per iteration
template <int UNR>
__global__ void k_read4u(const f4v *__restrict__ a, size_t n, float *out)
{
    float s = 0.f;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    for (; i + (UNR - 1) * stride < n; i += UNR * stride) {
        f4v v[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) v[u] = a[i + u * stride];
#pragma unroll
        for (int u = 0; u < UNR; ++u) s += v[u].x + v[u].y + v[u].z + v[u].w;
    }
    for (; i < n; i += stride) { f4v v = a[i]; s += v.x + v.y + v.z + v.w; }
    if (s == 1234.5678f) out[0] = s;
}
__global__ void k_read1(const float *__restrict__ a, size_t n, float *out)
{
    float s = 0.f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        s += a[i];
    if (s == 1234.5678f) out[0] = s;
}
template <bool NT>
__global__ void k_write4(f4v *__restrict__ a, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        f4v v = f4v{float(i), 1.f, 2.f, 3.f};
        if (NT) __builtin_nontemporal_store(v, a + i); else a[i] = v;
    }
}
template <bool NT>
__global__ void k_write1(float *__restrict__ a, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        if (NT) __builtin_nontemporal_store(float(i), a + i); else a[i] = float(i);
    }
}
template <bool NT>
__global__ void k_copy4(const f4v *__restrict__ a, f4v *__restrict__ b, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        f4v v = a[i];
        if (NT) __builtin_nontemporal_store(v, b + i); else b[i] = v;
    }
}
template <bool NT>
__global__ void k_copy1(const float *__restrict__ a, float *__restrict__ b, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float v = a[i];
        if (NT) __builtin_nontemporal_store(v, b + i); else b[i] = v;
    }
}
// 26 streams of one-element-per-thread (the LBM step's shape without arithmetic,
// plain SoA planes) : read 26 floats at c from 26 planes, write 26 at c
__global__ void k_copy26(const float *__restrict__ a, float *__restrict__ b, size_t cells)
{
    size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (c >= cells) return;
    float v[26];
#pragma unroll
    for (int i = 0; i < 26; ++i) v[i] = a[i * cells + c];
#pragma unroll
    for (int i = 0; i < 26; ++i) __builtin_nontemporal_store(v[i], b + i * cells + c);
}

int main(int argc, char **argv)
{
    const size_t bytes = size_t(256) * 256 * 256 * 104;  // one FP32 lattice, 1.745 GB
    const size_t n4 = bytes / 16, n1 = bytes / 4;
    float *a, *b, *o;
    CK(hipMalloc(&a, bytes));
    CK(hipMalloc(&b, bytes));
    CK(hipMalloc(&o, 256));
    CK(hipMemset(a, 0, bytes));
    CK(hipMemset(b, 0, bytes));
    hipDeviceProp_t prop;
    CK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    printf("device %s, %d CUs, buffer %.3f GB\n", prop.gcnArchName, cus, bytes / 1e9);
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    auto timeit = [&](const char *name, double moved, auto launch) {
        for (int w = 0; w < 3; ++w) launch();
        CK(hipDeviceSynchronize());
        const int reps = 10;
        CK(hipEventRecord(e0, 0));
        for (int r = 0; r < reps; ++r) launch();
        CK(hipEventRecord(e1, 0));
        CK(hipEventSynchronize(e1));
        float ms = 0;
        CK(hipEventElapsedTime(&ms, e0, e1));
        const double us = 1e3 * ms / reps;
        printf("%-44s %9.1f us  %7.1f GB/s\n", name, us, moved / (us * 1e-6) / 1e9);
        fflush(stdout);
    };
    char name[128];
    for (int block : {256, 512, 1024}) {
        for (int gmul : {0, 4, 8, 16, 32}) {
            // gmul 0: one element per thread (grid covers the data)
            const unsigned g4 = gmul ? unsigned(gmul * cus) : unsigned((n4 + block - 1) / block);
            const unsigned g1 = gmul ? unsigned(gmul * cus) : unsigned((n1 + block - 1) / block);
            snprintf(name, sizeof name, "read  f4  b%4d g%s%d", block, gmul ? "CUx" : "full", gmul);
            timeit(name, bytes, [&] { hipLaunchKernelGGL(k_read4, dim3(g4), dim3(block), 0, 0, (const f4v *)a, n4, o); });
            snprintf(name, sizeof name, "read  f1  b%4d g%s%d", block, gmul ? "CUx" : "full", gmul);
            timeit(name, bytes, [&] { hipLaunchKernelGGL(k_read1, dim3(g1), dim3(block), 0, 0, a, n1, o); });
            snprintf(name, sizeof name, "write f4 nt b%4d g%s%d", block, gmul ? "CUx" : "full", gmul);
            timeit(name, bytes, [&] { hipLaunchKernelGGL(k_write4<true>, dim3(g4), dim3(block), 0, 0, (f4v *)b, n4); });
            snprintf(name, sizeof name, "write f4    b%4d g%s%d", block, gmul ? "CUx" : "full", gmul);
            timeit(name, bytes, [&] { hipLaunchKernelGGL(k_write4<false>, dim3(g4), dim3(block), 0, 0, (f4v *)b, n4); });
            snprintf(name, sizeof name, "write f1 nt b%4d g%s%d", block, gmul ? "CUx" : "full", gmul);
            timeit(name, bytes, [&] { hipLaunchKernelGGL(k_write1<true>, dim3(g1), dim3(block), 0, 0, b, n1); });
            snprintf(name, sizeof name, "copy  f4 nt b%4d g%s%d", block, gmul ? "CUx" : "full", gmul);
            timeit(name, 2.0 * bytes, [&] { hipLaunchKernelGGL(k_copy4<true>, dim3(g4), dim3(block), 0, 0, (const f4v *)a, (f4v *)b, n4); });
            snprintf(name, sizeof name, "copy  f4    b%4d g%s%d", block, gmul ? "CUx" : "full", gmul);
            timeit(name, 2.0 * bytes, [&] { hipLaunchKernelGGL(k_copy4<false>, dim3(g4), dim3(block), 0, 0, (const f4v *)a, (f4v *)b, n4); });
            snprintf(name, sizeof name, "copy  f1 nt b%4d g%s%d", block, gmul ? "CUx" : "full", gmul);
            timeit(name, 2.0 * bytes, [&] { hipLaunchKernelGGL(k_copy1<true>, dim3(g1), dim3(block), 0, 0, a, b, n1); });
        }
    }
    for (int gmul : {4, 8, 16}) {
        const unsigned g = unsigned(gmul * cus);
        snprintf(name, sizeof name, "read  f4 x4unroll b256 gCUx%d", gmul);
        timeit(name, bytes, [&] { hipLaunchKernelGGL(k_read4u<4>, dim3(g), dim3(256), 0, 0, (const f4v *)a, n4, o); });
        snprintf(name, sizeof name, "read  f4 x8unroll b256 gCUx%d", gmul);
        timeit(name, bytes, [&] { hipLaunchKernelGGL(k_read4u<8>, dim3(g), dim3(256), 0, 0, (const f4v *)a, n4, o); });
    }
    const size_t cells = size_t(256) * 256 * 256;
    for (int block : {64, 128, 256, 512})
        { snprintf(name, sizeof name, "copy26 planes nt b%d", block);
          timeit(name, 2.0 * bytes, [&] { hipLaunchKernelGGL(k_copy26, dim3(unsigned((cells + block - 1) / block)), dim3(block), 0, 0, a, b, cells); }); }
    CK(hipMemcpy(b, a, 256, hipMemcpyDeviceToDevice));
    timeit("hipMemcpyDtoD", 2.0 * bytes, [&] { (void)hipMemcpyAsync(b, a, bytes, hipMemcpyDeviceToDevice, 0); });
    CK(hipFree(a)); CK(hipFree(b)); CK(hipFree(o));
    printf("done\n");
    return 0;
}
