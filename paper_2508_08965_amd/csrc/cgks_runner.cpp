// Native runner of the CGKS-5 library: loads a state file, advances it on the GPU and reports
// the time per step.  It makes no use of PyTorch, so hardware-counter profilers see only the
// library's kernels (plus one plain copy kernel of known size, the reference for byte counters).
//
// usage: cgks_runner STATE_FILE STEPS [COPY_MIB [RECON_PREC FLUX_PREC]]
//
// State file (little endian): 8-byte magic "CGKSST01"; int32 nx, ny, nz, size of cgks_params;
// the cgks_params struct; nodes (nx+1)(ny+1)(nz+1)*3 doubles; Q[5][N], G[5][3][N], L[5][12][N]
// doubles (the layouts of cgks.h).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "cgks.h"

namespace {

__global__ void __launch_bounds__(256) k_copy(const double *__restrict__ a, double *__restrict__ b, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) b[i] = a[i];
}

bool read_exact(FILE *f, void *p, size_t bytes) { return std::fread(p, 1, bytes, f) == bytes; }

#define CHECK_HIP(call)                                                                 \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            std::fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));      \
            return 3;                                                                   \
        }                                                                               \
    } while (0)

}  // namespace

int main(int argc, char **argv) {
    if (argc < 3) {
        std::fprintf(stderr, "usage: %s STATE_FILE STEPS [COPY_MIB [RECON_PREC FLUX_PREC]]\n", argv[0]);
        return 2;
    }
    const int steps = std::atoi(argv[2]);
    const long copy_mib = argc > 3 ? std::atol(argv[3]) : 0;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) {
        std::fprintf(stderr, "cannot open %s\n", argv[1]);
        return 2;
    }
    char magic[8];
    int hdr[4];
    cgks_params p;
    if (!read_exact(f, magic, 8) || std::memcmp(magic, "CGKSST01", 8) || !read_exact(f, hdr, sizeof hdr) ||
        hdr[3] != (int)sizeof(cgks_params) || !read_exact(f, &p, sizeof p)) {
        std::fprintf(stderr, "bad state file header\n");
        return 2;
    }
    if (argc > 5) {  // precision variant of the same workload
        p.recon_prec = std::atoi(argv[4]);
        p.flux_prec = std::atoi(argv[5]);
    }
    const int dims[3] = {hdr[0], hdr[1], hdr[2]};
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || steps < 0) {
        std::fprintf(stderr, "bad sizes\n");
        return 2;
    }
    const long N = (long)dims[0] * dims[1] * dims[2];
    const size_t nn = (size_t)(dims[0] + 1) * (dims[1] + 1) * (dims[2] + 1) * 3;
    std::vector<double> nodes(nn), state((size_t)80 * N);
    if (!read_exact(f, nodes.data(), nn * 8) || !read_exact(f, state.data(), state.size() * 8)) {
        std::fprintf(stderr, "state file too short\n");
        return 2;
    }
    std::fclose(f);

    double *Q = nullptr, *dt = nullptr;
    CHECK_HIP(hipMalloc((void **)&Q, sizeof(double) * 80 * N));
    CHECK_HIP(hipMalloc((void **)&dt, sizeof(double)));
    CHECK_HIP(hipMemcpy(Q, state.data(), sizeof(double) * 80 * N, hipMemcpyHostToDevice));
    double *G = Q + 5 * N, *L = Q + 20 * N;
    const double *np = nodes.data();
    cgks_ctx *ctx = nullptr;
    if (cgks_ctx_create(&ctx, 1, dims, &np, &p, nullptr) != CGKS_OK) {
        std::fprintf(stderr, "cgks_ctx_create: %s\n", cgks_last_error());
        return 3;
    }
    if (copy_mib > 0) {
        const long n = copy_mib * (1L << 20) / 8;
        double *a = nullptr, *b = nullptr;
        CHECK_HIP(hipMalloc((void **)&a, n * 8));
        CHECK_HIP(hipMalloc((void **)&b, n * 8));
        CHECK_HIP(hipMemset(a, 0, n * 8));
        hipLaunchKernelGGL(k_copy, dim3(8192), dim3(256), 0, 0, a, b, n);
        CHECK_HIP(hipGetLastError());
        CHECK_HIP(hipDeviceSynchronize());
        std::printf("copy kernel: %ld MiB read, %ld MiB written\n", copy_mib, copy_mib);
        CHECK_HIP(hipFree(a));
        CHECK_HIP(hipFree(b));
    }
    for (int s = 0; s < steps; ++s) {
        const auto t0 = std::chrono::steady_clock::now();
        if (cgks_step(ctx, Q, G, L, dt, 1, nullptr) != CGKS_OK) {
            std::fprintf(stderr, "cgks_step: %s\n", cgks_last_error());
            return 3;
        }
        CHECK_HIP(hipDeviceSynchronize());
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        int flags = 0;
        const int st = cgks_check(ctx, &flags);
        double dth = 0.0;
        CHECK_HIP(hipMemcpy(&dth, dt, sizeof dth, hipMemcpyDeviceToHost));
        std::printf("step %d: %.3f ms, dt %.6e, flags %d\n", s, ms, dth, flags);
        std::fflush(stdout);
        if (st != CGKS_OK) return 4;
    }
    cgks_ctx_destroy(ctx);
    CHECK_HIP(hipFree(Q));
    CHECK_HIP(hipFree(dt));
    std::printf("done\n");
    return 0;
}
