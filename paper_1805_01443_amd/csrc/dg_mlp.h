// The learned troubled-cell indicator's network (64 -> 32 -> 32 -> 1, ReLU,
// bf16 operands, FP32 accumulation on v_mfma_f32_16x16x16bf16_1k), shared by
// the flag kernel and the order-4 adiabatic stage kernel that forms the flags
// of the rows it has just written.  Sixteen samples per wavefront: the sample
// of lane l is column l mod 16 of every MFMA tile, and lane group gq = l / 16
// holds rows 4 gq .. 4 gq + 3 of the B fragments, i.e. modes (a = gq, b = 0..3)
// of one variable per K step.
#pragma once

#include <hip/hip_runtime.h>

namespace dgk {

constexpr int kIn = 64, kH = 32;
constexpr int kW1 = 0, kB1 = kW1 + kH * kIn, kW2 = kB1 + kH, kB2 = kW2 + kH * kH, kW3 = kB2 + kH, kB3 = kW3 + kH;
constexpr int kNParam = kB3 + 1;  // 3169

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float x) {
    // round to nearest even (finite inputs)
    unsigned int b = __float_as_uint(x);
    if ((b & 0x7f800000u) == 0x7f800000u) return (unsigned short)(b >> 16);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (unsigned short)(b >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

// The weights of one lane in fragment form: a1[t][s] = W1 rows 16 t + (l mod
// 16), columns 16 s + 4 gq .. + 3 (bf16); a2 likewise for W2; the biases and
// output weights of rows 16 t + 4 gq + k.
struct MlpLane {
    bf16x4 a1[2][4], a2[2][2];
    float b1v[2][4], b2v[2][4], w3v[2][4];
    float b3;
};

// Packed per-lane form written once per step from the FP32 parameters
// (k_mlp_pack): 12 fragments of 8 bytes per lane, [fragment][lane], then 24
// floats per lane, [value][lane], then b3.
constexpr int kPackFrag = 12, kPackVec = 24;
constexpr int kPackBytes = kPackFrag * 64 * 8 + kPackVec * 64 * 4 + 16;

__device__ __forceinline__ void mlp_lane_from_params(const float* __restrict__ par, int lane, MlpLane& w) {
    const int i = lane & 15, gq = lane >> 4;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int k = 0; k < 4; ++k) w.a1[t][s][k] = (short)f2bf(par[kW1 + (16 * t + i) * kIn + 16 * s + 4 * gq + k]);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int k = 0; k < 4; ++k) w.a2[t][s][k] = (short)f2bf(par[kW2 + (16 * t + i) * kH + 16 * s + 4 * gq + k]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int row = 16 * t + 4 * gq + k;
            w.b1v[t][k] = par[kB1 + row];
            w.b2v[t][k] = par[kB2 + row];
            w.w3v[t][k] = bf2f(f2bf(par[kW3 + row]));
        }
    }
    w.b3 = par[kB3];
}

__device__ __forceinline__ void mlp_lane_from_pack(const void* __restrict__ pack, int lane, MlpLane& w) {
    const unsigned long long* fr = (const unsigned long long*)pack;
    const float* fv = (const float*)(fr + kPackFrag * 64);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
        for (int s = 0; s < 4; ++s) w.a1[t][s] = __builtin_bit_cast(bf16x4, fr[(t * 4 + s) * 64 + lane]);
#pragma unroll
        for (int s = 0; s < 2; ++s) w.a2[t][s] = __builtin_bit_cast(bf16x4, fr[(8 + t * 2 + s) * 64 + lane]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            w.b1v[t][k] = fv[(t * 4 + k) * 64 + lane];
            w.b2v[t][k] = fv[(8 + t * 4 + k) * 64 + lane];
            w.w3v[t][k] = fv[(16 + t * 4 + k) * 64 + lane];
        }
    }
    w.b3 = fv[kPackVec * 64];
}

// The logit of this lane's sample from its four B fragments (K step s =
// variable s); every lane of the sample's column gets it.
__device__ __forceinline__ float mlp_logit(const MlpLane& w, const bf16x4 (&b)[4]) {
    f32x4 c1[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) c1[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < 2; ++t) c1[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w.a1[t][s], b[s], c1[t], 0, 0, 0);
    // bias, ReLU, round to bf16: these are the B fragments of layer 2
    bf16x4 hb[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float zz = c1[t][k] + w.b1v[t][k];
            hb[t][k] = (short)f2bf(zz > 0.f ? zz : 0.f);
        }
    f32x4 c2[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) c2[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 2; ++t) c2[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w.a2[t][s], hb[s], c2[t], 0, 0, 0);
    float part = 0.f;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float zz = c2[t][k] + w.b2v[t][k];
            part += w.w3v[t][k] * bf2f(f2bf(zz > 0.f ? zz : 0.f));
        }
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    return part + w.b3;
}

}  // namespace dgk
