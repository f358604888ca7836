// fma_issue_rate -- the fused multiply-add rate this GPU sustains in a loop
// with nothing else in it: every lane runs NACC independent accumulator
// chains of a * acc + b, entirely in registers, over a grid of 4096
// workgroups of 256 threads.  It is the practical ceiling against which the
// arithmetic-bound kernels of this library (the FP64 near field and M2L)
// are read: the published vector peaks count every issue slot as an FMA.
// Packed FP32 instructions are disabled in this build, so the FP32 figure
// is the single-issue rate.
#include <hip/hip_runtime.h>

#include <cstdio>

template <typename T, int NACC>
__global__ void __launch_bounds__(256) k_fma(T* out, T a, T b, int iters)
{
    T acc[NACC];
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = T(threadIdx.x + i);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < NACC; ++i) acc[i] = fma(acc[i], a, b);
    }
    T s = 0;
#pragma unroll
    for (int i = 0; i < NACC; ++i) s += acc[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;   // one value per thread: the grid's own slot
}

template <typename T, int NACC>
int run(const char* name, int iters)
{
    constexpr int kBlocks = 4096;
    T* out = nullptr;
    if (hipMalloc(&out, sizeof(T) * kBlocks * 256) != hipSuccess) return 1;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
    hipLaunchKernelGGL((k_fma<T, NACC>), dim3(kBlocks), dim3(256), 0, 0, out, T(0.999), T(0.001), iters);
    constexpr int kReps = 5;
    if (hipEventRecord(e0) != hipSuccess) return 1;
    for (int r = 0; r < kReps; ++r)
        hipLaunchKernelGGL((k_fma<T, NACC>), dim3(kBlocks), dim3(256), 0, 0, out, T(0.999), T(0.001), iters);
    if (hipEventRecord(e1) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1;
    const double flops = 2.0 * NACC * double(iters) * kBlocks * 256 * kReps;
    std::printf("%s, %d independent chains per lane: %.1f TFLOP/s\n", name, NACC, flops / (ms * 1e-3) / 1e12);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return hipFree(out) == hipSuccess ? 0 : 1;
}

int main()
{
    int rc = 0;
    rc |= run<double, 8>("FP64 FMA", 4096);
    rc |= run<double, 16>("FP64 FMA", 4096);
    rc |= run<double, 32>("FP64 FMA", 2048);
    rc |= run<float, 16>("FP32 FMA", 4096);
    rc |= run<float, 32>("FP32 FMA", 2048);
    return rc;
}
