// Learned blend weights: an MLP 18 -> 32 -> 7 that stands in for the nonlinear weights of the
// reconstruction (Sec. 3.3: chi of the path function and the weights omega_m of the six linear
// sub-polynomials).  Output 0 gives chi through a logistic sigmoid, outputs 1..6 give omega_m
// through a softmax.  Inputs per cell and conserved variable: the six face-neighbour
// differences Q_{1,m} - Q_0 (m = 2q + s) and the twelve line derivatives L_s, divided by
// (max of their magnitudes + 1e-12).  Hidden layer: 32 ReLU units.
//
// Parameter vector (FP32 master copy, 839 values): W1[32][18], b1[32], W2[7][32], b2[7].
//
// Inference runs on the 16x16x32 BF16 matrix cores, 16 (cell, variable) columns per wave:
// lane l = 16 g + col supplies input slots 8g..8g+7 of column col.  Slot j of lane group g
// holds, for j < 3, the line derivative 4j + g (feature 6 + 4j + g); for j = 3, 4 and g < 3 the
// face difference 2g + j - 3 (feature 2g + j - 3); the other slots are zero.  Every lane thus
// reads only the line derivatives it already holds in the reconstruction.  The first layer's
// two output tiles put hidden unit 16t + 4g + v in register v of lane group g (tile t); the
// second layer reads slot j of lane group g as hidden unit 16(j/4) + 4g + (j%4).
#pragma once

#include <hip/hip_runtime.h>

namespace cgks {

constexpr int kMlpIn = 18, kMlpHidden = 32, kMlpOut = 7;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpOut * kMlpHidden + kMlpOut;  // 839
constexpr int kMlpOffB1 = kMlpHidden * kMlpIn, kMlpOffW2 = kMlpOffB1 + kMlpHidden,
              kMlpOffB2 = kMlpOffW2 + kMlpOut * kMlpHidden;
// packed inference blocks: 3 x 64 lanes x 8 BF16 (layer-1 tiles 0, 1; layer 2), then b1[32]
// and b2[8] as FP32
constexpr int kMlpPackBf16 = 3 * 64 * 8;
constexpr int kMlpPackBytes = kMlpPackBf16 * 2 + (kMlpHidden + 8) * 4;

// feature index held in slot j of lane group g (-1: zero slot)
inline __host__ __device__ int mlp_slot_feature(int g, int j) {
    if (j < 3) return 6 + 4 * j + g;
    if (j < 5 && g < 3) return 2 * g + j - 3;
    return -1;
}
// hidden unit read from slot j of lane group g by the second layer
inline __host__ __device__ int mlp_slot_hidden(int g, int j) { return 16 * (j >> 2) + 4 * g + (j & 3); }

// Pack the FP32 parameters into the inference blocks (BF16, round to nearest even).
void mlp_pack(const float *w, unsigned char *packed);

#ifdef __HIPCC__
typedef __bf16 v8bf_t __attribute__((ext_vector_type(8)));
typedef float v4f_t __attribute__((ext_vector_type(4)));

// z[0..6] (pre-activation outputs) of column col of the wave, in every lane of the column.
// Wl: the three packed blocks, already offset by the lane (stride 64 v8bf per block);
// b1, b2: biases (FP32).  x: this lane's input slots.
__device__ inline void mlp_eval(const v8bf_t *Wl, const float *b1, const float *b2, const v8bf_t &x, int g,
                                int col, float z[7]) {
    const v4f_t zero = {0.f, 0.f, 0.f, 0.f};
    const v4f_t h0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wl[0], x, zero, 0, 0, 0);
    const v4f_t h1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wl[64], x, zero, 0, 0, 0);
    v8bf_t hb;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const float a = h0[v] + b1[4 * g + v], c = h1[v] + b1[16 + 4 * g + v];
        hb[v] = (__bf16)(a > 0.f ? a : 0.f);
        hb[4 + v] = (__bf16)(c > 0.f ? c : 0.f);
    }
    const v4f_t zz = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wl[128], hb, zero, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) z[v] = __shfl(zz[v], col, 64) + b2[v];
#pragma unroll
    for (int v = 0; v < 3; ++v) z[4 + v] = __shfl(zz[v], col + 16, 64) + b2[4 + v];
}

// chi (sigmoid) and omega_1..6 (softmax) from the outputs, in FP32 like the outputs themselves
__device__ inline void mlp_weights(const float z[7], double &chi, double om[6]) {
    chi = (double)(1.0f / (1.0f + __expf(-z[0])));
    float zmax = z[1];
#pragma unroll
    for (int m = 2; m < 7; ++m) zmax = fmaxf(zmax, z[m]);
    float e[6], den = 0.0f;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        e[m] = __expf(z[1 + m] - zmax);
        den += e[m];
    }
    const float id = 1.0f / den;
#pragma unroll
    for (int m = 0; m < 6; ++m) om[m] = (double)(e[m] * id);
}
#endif

}  // namespace cgks
