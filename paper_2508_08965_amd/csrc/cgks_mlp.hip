// Learned blend weights: jump indicator, BF16 inference on the matrix cores, and FP32 training
// (forward and backward pass, gradient reduction, Adam) of the MLP described in cgks_mlp.h.
#include <hip/hip_runtime.h>

#include <cstring>

#include "cgks_device.h"
#include "cgks_mlp.h"

namespace cgks {

// ---- host packing ------------------------------------------------------------------------
static unsigned short bf16_bits(float f) {
    unsigned int u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);  // nearest, ties to even
    return (unsigned short)(u >> 16);
}

void mlp_pack(const float *w, unsigned char *packed) {
    unsigned short *blk = (unsigned short *)packed;
    for (int lane = 0; lane < 64; ++lane) {
        const int row = lane & 15, g = lane >> 4;
        for (int j = 0; j < 8; ++j) {
            const int f = mlp_slot_feature(g, j);
            for (int t = 0; t < 2; ++t)
                blk[(t * 64 + lane) * 8 + j] = bf16_bits(f >= 0 ? w[(16 * t + row) * kMlpIn + f] : 0.0f);
            const int h = mlp_slot_hidden(g, j);
            blk[(2 * 64 + lane) * 8 + j] = bf16_bits(row < kMlpOut ? w[kMlpOffW2 + row * kMlpHidden + h] : 0.0f);
        }
    }
    float *bias = (float *)(packed + kMlpPackBf16 * 2);
    for (int i = 0; i < kMlpHidden; ++i) bias[i] = w[kMlpOffB1 + i];
    for (int i = 0; i < 8; ++i) bias[kMlpHidden + i] = i < kMlpOut ? w[kMlpOffB2 + i] : 0.0f;
}

// ---- jump indicator ----------------------------------------------------------------------
__device__ inline double pressure(const double *Q, long Ntot, long c, double gm1) {
    const double r = Q[c], mu = Q[Ntot + c], mv = Q[2 * Ntot + c], mw = Q[3 * Ntot + c], E = Q[4 * Ntot + c];
    return gm1 * (E - 0.5 * (mu * mu + mv * mv + mw * mw) / r);
}

// flag[c] = max over the six face neighbours of |p_m - p_0| / (p_m + p_0) > thresh; count[0]
// accumulates the number of flagged cells.  Behind a symmetry plane or no-slip wall the
// neighbour is the mirror image of the cell itself (same pressure); behind a far-field side it
// is the far-field state (pressure pfar).
__global__ void __launch_bounds__(256) k_jump(WorkList W, long Ntot, const double *__restrict__ Q, double gm1,
                                              double thresh, double pfar, unsigned char *__restrict__ flag,
                                              unsigned long long *__restrict__ count) {
    __shared__ int nflag;
    if (threadIdx.x == 0) nflag = 0;
    __syncthreads();
    const long u = blockIdx.x;
    const Tile tile = W.tiles[u];
    int mine = 0;
    if ((int)threadIdx.x < tile.count) {
        const BlockView b = W.blocks[tile.blk];
        const long cl = tile.start + threadIdx.x;
        const int i = (int)(cl % b.nx);
        const long t = cl / b.nx;
        const int j = (int)(t % b.ny), k = (int)(t / b.ny);
        const long c = b.off + cl;
        const double p0 = pressure(Q, Ntot, c, gm1);
        double ind = 0.0;
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            int o[3] = {0, 0, 0};
            o[m >> 1] = (m & 1) ? 1 : -1;
            int ii = i + o[0], jj = j + o[1], kk = k + o[2];
            ii = ii < 0 ? ii + b.nx : (ii >= b.nx ? ii - b.nx : ii);
            jj = jj < 0 ? jj + b.ny : (jj >= b.ny ? jj - b.ny : jj);
            kk = kk < 0 ? kk + b.nz : (kk >= b.nz ? kk - b.nz : kk);
            const int iq = (m < 2) ? i : (m < 4) ? j : k, nq = (m < 2) ? b.nx : (m < 4) ? b.ny : b.nz;
            const bool at_wall = ((b.wall >> m) & 1) && iq == ((m & 1) ? nq - 1 : 0);
            const double pm = !at_wall ? pressure(Q, Ntot, b.off + ii + (long)b.nx * (jj + (long)b.ny * kk), gm1)
                                       : (((b.wall >> (16 + m)) & 1) ? pfar : p0);
            const double r = fabs(pm - p0) / (pm + p0);
            ind = r > ind ? r : ind;
        }
        mine = ind > thresh;
        flag[c] = (unsigned char)mine;
    }
    if (mine) atomicAdd(&nflag, 1);
    __syncthreads();
    if (threadIdx.x == 0 && nflag) atomicAdd(count, (unsigned long long)nflag);
}

hipError_t launch_jump(const WorkList &W, long Ntot, const double *Q, const DevParams &P, unsigned char *flag,
                       unsigned long long *count, hipStream_t s) {
    if (W.ntiles <= 0) return hipSuccess;
    const double pfar = (P.far[0] > 0.0)
                            ? (P.gamma - 1.0) * (P.far[4] - 0.5 * (P.far[1] * P.far[1] + P.far[2] * P.far[2] +
                                                                   P.far[3] * P.far[3]) / P.far[0])
                            : 0.0;
    hipLaunchKernelGGL(k_jump, dim3((unsigned)W.ntiles), dim3(kUpdateTile), 0, s, W, Ntot, Q, P.gamma - 1.0,
                       P.jump_thresh, pfar, flag, count);
    return hipGetLastError();
}

// ---- inference on given features (test and diagnostics path) -----------------------------
// X [n][18] FP32 features, Y [n][7] outputs (chi, omega_1..6); a wave takes 16 samples.
__global__ void __launch_bounds__(256) k_mlp_infer(const float *__restrict__ X, long n,
                                                   const unsigned char *__restrict__ packed, double *__restrict__ Y) {
    __shared__ v8bf_t wl[3 * 64];
    __shared__ float bias[kMlpHidden + 8];
    const v8bf_t *src = (const v8bf_t *)packed;
    for (int i = threadIdx.x; i < 3 * 64; i += blockDim.x) wl[i] = src[i];
    const float *bsrc = (const float *)(packed + kMlpPackBf16 * 2);
    for (int i = threadIdx.x; i < kMlpHidden + 8; i += blockDim.x) bias[i] = bsrc[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
    const long base = ((long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 16;
    if (base >= n) return;  // whole waves leave together
    const long s = base + col < n ? base + col : n - 1;
    v8bf_t x;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int f = mlp_slot_feature(g, j);
        x[j] = (__bf16)(f >= 0 ? X[s * kMlpIn + f] : 0.0f);
    }
    float z[7];
    mlp_eval(wl + lane, bias, bias + kMlpHidden, x, g, col, z);
    double chi, om[6];
    mlp_weights(z, chi, om);
    if (g == 0 && base + col < n) {
        Y[s * 7] = chi;
#pragma unroll
        for (int m = 0; m < 6; ++m) Y[s * 7 + 1 + m] = om[m];
    }
}

hipError_t launch_mlp_infer(const float *X, long n, const unsigned char *packed, double *Y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const long waves = (n + 15) / 16;
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, X, n, packed, Y);
    return hipGetLastError();
}

// ---- training (FP32) -----------------------------------------------------------------------
// Per sample s of the batch (dataset index (first + s) mod n): forward pass, squared error of
// (sigmoid(z0), softmax(z1..6)) against the target, and the backward pass to the output and
// hidden pre-activations.  S[s] = [dz (7), dh (32), h (32), loss (1)].
constexpr int kMlpScratch = 72;

__global__ void __launch_bounds__(256) k_mlp_fwd_bwd(const float *__restrict__ w, const float *__restrict__ X,
                                                     const float *__restrict__ T, long n, long first, int B,
                                                     float *__restrict__ S) {
    __shared__ float ws[kMlpParams];
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) ws[i] = w[i];
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    const long idx = (first + s) % n;
    const float *x = X + idx * kMlpIn, *t = T + idx * kMlpOut;
    float xv[kMlpIn], h[kMlpHidden], z[kMlpOut], y[kMlpOut];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) xv[i] = x[i];
#pragma unroll
    for (int j = 0; j < kMlpHidden; ++j) {
        float a = ws[kMlpOffB1 + j];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) a = fmaf(ws[j * kMlpIn + i], xv[i], a);
        h[j] = a > 0.f ? a : 0.f;
    }
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) {
        float a = ws[kMlpOffB2 + o];
#pragma unroll
        for (int j = 0; j < kMlpHidden; ++j) a = fmaf(ws[kMlpOffW2 + o * kMlpHidden + j], h[j], a);
        z[o] = a;
    }
    y[0] = 1.f / (1.f + expf(-z[0]));
    float zmax = z[1];
#pragma unroll
    for (int o = 2; o < kMlpOut; ++o) zmax = fmaxf(zmax, z[o]);
    float den = 0.f;
#pragma unroll
    for (int o = 1; o < kMlpOut; ++o) {
        y[o] = expf(z[o] - zmax);
        den += y[o];
    }
#pragma unroll
    for (int o = 1; o < kMlpOut; ++o) y[o] /= den;
    float loss = 0.f, dy[kMlpOut], dz[kMlpOut];
    const float sc = 2.f / (float)B;
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) {
        const float e = y[o] - t[o];
        loss = fmaf(e, e, loss);
        dy[o] = sc * e;
    }
    dz[0] = dy[0] * y[0] * (1.f - y[0]);
    float sdot = 0.f;
#pragma unroll
    for (int o = 1; o < kMlpOut; ++o) sdot = fmaf(dy[o], y[o], sdot);
#pragma unroll
    for (int o = 1; o < kMlpOut; ++o) dz[o] = y[o] * (dy[o] - sdot);
    float *out = S + (long)s * kMlpScratch;
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) out[o] = dz[o];
#pragma unroll
    for (int j = 0; j < kMlpHidden; ++j) {
        float a = 0.f;
#pragma unroll
        for (int o = 0; o < kMlpOut; ++o) a = fmaf(ws[kMlpOffW2 + o * kMlpHidden + j], dz[o], a);
        out[7 + j] = h[j] > 0.f ? a : 0.f;
        out[39 + j] = h[j];
    }
    out[71] = loss;
}

// Gradient of the batch loss and the loss itself.  Block r < 32: hidden unit r (dW1[r][*],
// db1[r]); block 32 + o: output o (dW2[o][*], db2[o]); block 39: the mean loss into *loss.
// Each thread sums a fixed strided subset of the batch, then a fixed-shape tree: the result
// does not depend on timing.
__global__ void __launch_bounds__(256) k_mlp_reduce(const float *__restrict__ X, long n, long first, int B,
                                                    const float *__restrict__ S, float *__restrict__ grad,
                                                    float *__restrict__ loss) {
    __shared__ float red[256][34];
    const int r = blockIdx.x, tid = threadIdx.x;
    float acc[33];
#pragma unroll
    for (int i = 0; i < 33; ++i) acc[i] = 0.f;
    for (int s = tid; s < B; s += blockDim.x) {
        const float *row = S + (long)s * kMlpScratch;
        if (r < kMlpHidden) {
            const float d = row[7 + r];
            const float *x = X + ((first + s) % n) * kMlpIn;
#pragma unroll
            for (int i = 0; i < kMlpIn; ++i) acc[i] = fmaf(d, x[i], acc[i]);
            acc[kMlpIn] += d;
        } else if (r < kMlpHidden + kMlpOut) {
            const float d = row[r - kMlpHidden];
#pragma unroll
            for (int j = 0; j < kMlpHidden; ++j) acc[j] = fmaf(d, row[39 + j], acc[j]);
            acc[kMlpHidden] += d;
        } else {
            acc[0] += row[71];
        }
    }
#pragma unroll
    for (int i = 0; i < 33; ++i) red[tid][i] = acc[i];
    __syncthreads();
    for (int half = 128; half > 0; half >>= 1) {
        if (tid < half)
            for (int i = 0; i < 33; ++i) red[tid][i] += red[tid + half][i];
        __syncthreads();
    }
    if (r < kMlpHidden) {
        if (tid < kMlpIn) grad[r * kMlpIn + tid] = red[0][tid];
        if (tid == kMlpIn) grad[kMlpOffB1 + r] = red[0][kMlpIn];
    } else if (r < kMlpHidden + kMlpOut) {
        const int o = r - kMlpHidden;
        if (tid < kMlpHidden) grad[kMlpOffW2 + o * kMlpHidden + tid] = red[0][tid];
        if (tid == kMlpHidden) grad[kMlpOffB2 + o] = red[0][kMlpHidden];
    } else if (tid == 0) {
        *loss = red[0][0] / (float)B;
    }
}

// Adam (Kingma & Ba 2015) at step t: bias-corrected first and second moments.
__global__ void __launch_bounds__(256) k_mlp_adam(float *__restrict__ w, float *__restrict__ m,
                                                  float *__restrict__ v, const float *__restrict__ g, float lr,
                                                  float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kMlpParams) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_mlp_grad(const float *w, const float *X, const float *T, long n, long first, int B, float *S,
                           float *grad, float *loss, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, w, X, T, n, first, B, S);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_reduce, dim3(kMlpHidden + kMlpOut + 1), dim3(256), 0, s, X, n, first, B, S, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *w, float *m, float *v, const float *g, float lr, float b1, float b2, float eps,
                           int t, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, w, m, v, g, lr, b1, b2, eps, c1,
                       c2);
    return hipGetLastError();
}

int mlp_scratch_floats(int B) { return B * kMlpScratch; }

}  // namespace cgks
