// fmm_eval_file -- one FMM evaluation through the C ABI alone (include/fmm.h):
// no Python, no PyTorch.  Reads n particles from a binary file, evaluates the
// velocity of eq. 9 on the GPU and writes it to another file.
//
//   fmm_eval_file IN OUT SIGMA P DEPTH
//
// IN:  int64 n, then n doubles x, n doubles y, n doubles gamma
// OUT: n doubles u, then n doubles v (input order)
// The domain is the unit square [0, 1]^2.  Exit status 0 on success; on an
// error the failing call and its status text go to stderr.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/fmm.h"

namespace {

int fail(const char* what, int status)
{
    std::fprintf(stderr, "%s: %s (%d)\n", what, fmm_status_string(fmm_status(status)), status);
    return 1;
}

bool read_all(std::FILE* f, void* dst, size_t bytes) { return std::fread(dst, 1, bytes, f) == bytes; }

}  // namespace

int main(int argc, char** argv)
{
    if (argc != 6) {
        std::fprintf(stderr, "usage: %s IN OUT SIGMA P DEPTH\n", argv[0]);
        return 2;
    }
    std::FILE* in = std::fopen(argv[1], "rb");
    if (!in) {
        std::perror(argv[1]);
        return 1;
    }
    int64_t n = 0;
    if (!read_all(in, &n, sizeof n) || n < 0 || n > (int64_t(1) << 31) - 1) {
        std::fprintf(stderr, "bad header in %s\n", argv[1]);
        return 1;
    }
    std::vector<double> host(size_t(3 * n));
    if (!read_all(in, host.data(), host.size() * sizeof(double))) {
        std::fprintf(stderr, "short read from %s\n", argv[1]);
        return 1;
    }
    std::fclose(in);

    fmm_params prm{};
    prm.n_max = n;
    prm.sigma = std::atof(argv[3]);
    prm.p = std::atoi(argv[4]);
    prm.depth = std::atoi(argv[5]);
    prm.x0 = 0.0;
    prm.y0 = 0.0;
    prm.width = 1.0;
    prm.precision = FMM_PREC_FP64;
    prm.kernel = FMM_KERNEL_GAUSSIAN;

    size_t bytes = 0;
    int s = fmm_workspace_size(&prm, &bytes);
    if (s != FMM_OK) return fail("fmm_workspace_size", s);

    // device memory: the caller owns all of it, the workspace included
    double* d_in = nullptr;
    double* d_out = nullptr;
    void* d_ws = nullptr;
    const size_t nb = size_t(n) * sizeof(double);
    if (hipMalloc(&d_in, 3 * nb + 8) != hipSuccess || hipMalloc(&d_out, 2 * nb + 8) != hipSuccess ||
        hipMalloc(&d_ws, bytes) != hipSuccess)
        return fail("hipMalloc", FMM_E_DEVICE);
    hipStream_t st = nullptr;
    if (hipStreamCreate(&st) != hipSuccess) return fail("hipStreamCreate", FMM_E_DEVICE);
    if (hipMemcpyAsync(d_in, host.data(), 3 * nb, hipMemcpyHostToDevice, st) != hipSuccess)
        return fail("hipMemcpyAsync", FMM_E_DEVICE);

    fmm_plan_t plan = nullptr;
    s = fmm_plan(&prm, d_ws, bytes, st, &plan);
    if (s != FMM_OK) return fail("fmm_plan", s);
    s = fmm_evaluate(plan, n, d_in, d_in + n, d_in + 2 * n, d_out, d_out + n, st);
    if (s != FMM_OK) return fail("fmm_evaluate", s);
    int64_t n_bad = 0;
    s = fmm_get_status(plan, st, &n_bad);       // synchronises the stream
    if (s != FMM_OK) return fail("fmm_get_status", s);

    std::vector<double> out(size_t(2 * n));
    if (hipMemcpy(out.data(), d_out, 2 * nb, hipMemcpyDeviceToHost) != hipSuccess)
        return fail("hipMemcpy", FMM_E_DEVICE);
    fmm_destroy(plan);
    (void)hipStreamDestroy(st);
    (void)hipFree(d_ws);
    (void)hipFree(d_out);
    (void)hipFree(d_in);

    std::FILE* f = std::fopen(argv[2], "wb");
    if (!f || std::fwrite(out.data(), sizeof(double), out.size(), f) != out.size()) {
        std::perror(argv[2]);
        return 1;
    }
    std::fclose(f);
    return 0;
}
