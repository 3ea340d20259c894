// Read+write streaming ceiling of the GPU, for the roofline of the fused
// iteration (which reads one state array and writes another of the same
// size). Copies one float32 state array of the 128 x 128 x 64, Q = 1600
// workload (6,710,886,400 bytes) with several cache policies and launch
// shapes (grid-stride loops, and one element per thread) and reports the
// best of 5 timed launches each. Stand-alone executable, not part of
// libssmap.
#include <hip/hip_runtime.h>

#include <cstdio>

typedef float v4f __attribute__((ext_vector_type(4)));

template <int V>
__global__ void __launch_bounds__(256) copy_kernel(const v4f *__restrict__ a, v4f *__restrict__ b,
                                                   size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        if constexpr (V == 0) b[i] = a[i];
        if constexpr (V == 1) __builtin_nontemporal_store(a[i], &b[i]);
        if constexpr (V == 2) __builtin_nontemporal_store(__builtin_nontemporal_load(&a[i]), &b[i]);
    }
}

// One 16-byte element per thread, one block per 256 elements (no loop): the
// access pattern the memory system streams fastest here.
template <int V>
__global__ void __launch_bounds__(256) copy_once(const v4f *__restrict__ a, v4f *__restrict__ b) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if constexpr (V == 0) b[i] = a[i];
    if constexpr (V == 2) __builtin_nontemporal_store(__builtin_nontemporal_load(&a[i]), &b[i]);
}

template <int V>
static double run_once(const v4f *a, v4f *b, size_t n) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
    const dim3 grid((unsigned)(n / 256));
    hipLaunchKernelGGL(copy_once<V>, grid, dim3(256), 0, nullptr, a, b);
    float best = 1e30f;
    for (int k = 0; k < 5; ++k) {
        (void)hipEventRecord(e0);
        hipLaunchKernelGGL(copy_once<V>, grid, dim3(256), 0, nullptr, a, b);
        (void)hipEventRecord(e1);
        (void)hipEventSynchronize(e1);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

template <int V>
static double run(const v4f *a, v4f *b, size_t n, int grid) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
    hipLaunchKernelGGL(copy_kernel<V>, dim3(grid), dim3(256), 0, nullptr, a, b, n);
    float best = 1e30f;
    for (int k = 0; k < 5; ++k) {
        (void)hipEventRecord(e0);
        hipLaunchKernelGGL(copy_kernel<V>, dim3(grid), dim3(256), 0, nullptr, a, b, n);
        (void)hipEventRecord(e1);
        (void)hipEventSynchronize(e1);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

int main() {
    const size_t bytes = (size_t)6710886400;
    const size_t n = bytes / sizeof(v4f);
    v4f *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
        std::printf("allocation failed\n");
        return 1;
    }
    if (hipMemset(a, 0, bytes) != hipSuccess) return 1;
    const char *names[3] = {"default", "non-temporal store", "non-temporal load+store"};
    for (int grid : {4096, 16384}) {
        const double ms[3] = {run<0>(a, b, n, grid), run<1>(a, b, n, grid), run<2>(a, b, n, grid)};
        for (int v = 0; v < 3; ++v)
            std::printf("copy grid %5d x 256, %-24s %.3f ms  %.0f GB/s (read + write)\n", grid,
                        names[v], ms[v], 2.0 * bytes / ms[v] / 1e6);
    }
    // n = 419,430,400 elements: a whole number of 256-element blocks
    const double once[2] = {run_once<0>(a, b, n), run_once<2>(a, b, n)};
    std::printf("copy one element per thread, default             %.3f ms  %.0f GB/s (read + write)\n",
                once[0], 2.0 * bytes / once[0] / 1e6);
    std::printf("copy one element per thread, non-temporal        %.3f ms  %.0f GB/s (read + write)\n",
                once[1], 2.0 * bytes / once[1] / 1e6);
    const hipError_t e = hipDeviceSynchronize();
    std::printf("status %s\n", hipGetErrorString(e));
    (void)hipFree(a);
    (void)hipFree(b);
    return e == hipSuccess ? 0 : 1;
}
