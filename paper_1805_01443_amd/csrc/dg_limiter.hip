// Troubled-cell treatment on gfx950: the modal-decay indicator, the minmod
// slope limiter of the Cockburn-Shu RKDG scheme the paper builds on (Sec. 2.2),
// and the small learned indicator (64 -> 32 -> 32 -> 1 MLP) with its BF16
// MFMA forward pass, FP32 backward pass and Adam update.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "dg_basis.h"
#include "dg_internal.h"
#include "dg_mlp.h"
#include "dg_pp.h"

namespace dgk {

// ------------------------------------------------------------------ indicator + minmod
__device__ __forceinline__ double minmod3(double a, double b, double c) {
    if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
    if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
    return 0.0;
}

// mean of variable v of the neighbour across edge f (0 W, 1 E, 2 S, 3 N);
// at a fixed box edge the exterior mean is the element's own initial mean, at
// a gradient-free edge its own current mean
template <int N, int NV>
__device__ __forceinline__ double nb_mean(const Geo& g, const double* __restrict__ u, const double* __restrict__ u0,
                                          int i, int j, int v, int f) {
    int in = i + (f == 1) - (f == 0), jn = j + (f == 3) - (f == 2);
    const bool outside = in < 0 || in >= g.nx || jn < 0 || jn >= g.ny;
    if (outside && g.bc == 1) return u0[tiled_base<N, NV>(g, i, j) + mode_off<N>(v, 0, 0)];
    if (outside && g.bc == 2) return u[tiled_base<N, NV>(g, i, j) + mode_off<N>(v, 0, 0)];
    in = (in + g.nx) % g.nx;
    jn = (jn + g.ny) % g.ny;
    return u[tiled_base<N, NV>(g, in, jn) + mode_off<N>(v, 0, 0)];
}

// ------------------------------------------------------------------ positivity
// Positivity scaling (Sec. 2.4) with N lanes per element (lane (s, k) = lane
// k * EW + s, EW = 64 / N elements per wavefront, one wavefront per block): lane k loads mode
// row k of every variable; the factors come from pp_factors (dg_pp.h); each
// lane of a changed element scales and stores its row.
template <int N, int NV>
__global__ void __launch_bounds__(64) k_pp_c(const Geo g, double* u, double e0, unsigned char* changed_out,
                                             double* theta_out, const unsigned char* __restrict__ pp_ok) {
    constexpr int EW = 64 / N;
    constexpr int SLOT = pp_slot<N, NV>() | 1;  // odd: the slots of one k on distinct banks
    __shared__ double lds[EW * SLOT];
    const int lane = threadIdx.x;
    // lane k * EW + s: index k of element slot s (rows contiguous in lane
    // order); lanes beyond N * EW shadow slot 0's element
    const bool own = lane < N * EW;
    const int k = own ? lane / EW : lane - N * EW;
    const int sl = own ? lane - k * EW : EW;
    const int tile = blockIdx.x;
    // a tile that the stage kernel found admissible and the troubled-cell
    // limiter left alone needs no scaling: the whole block leaves at once
    if (pp_ok && pp_ok[tile]) return;
    const int j = tile / g.tiles_x;
    const int i0 = (tile - j * g.tiles_x) * EW;
    const bool active = sl < EW && i0 + sl < g.nx;
    const int i = active ? i0 + sl : i0;
    double* S = lds + (own ? sl : 0) * SLOT;
    const unsigned base = tiled_base<N, NV>(g, i, j);
    double Ua[NV][N];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int b = 0; b < N; ++b) Ua[v][b] = u[base + mode_off<N>(v, k, b)];
    double th1, th2;
    pp_factors<N, NV>(g, S, k, Ua, e0, th1, th2);
    const bool changed = th1 < 1.0 || th2 < 1.0;
    if (active && changed) {
        // the row again (from L2: fewer live registers), scaled
        double Ub[NV][N];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int b = 0; b < N; ++b) Ub[v][b] = u[base + mode_off<N>(v, k, b)];
        pp_scale_row<N, NV>(k, th1, th2, Ub);
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int b = 0; b < N; ++b) u[base + mode_off<N>(v, k, b)] = Ub[v][b];
    }
    if (active && k == 0) {
        const long long e = (long long)j * g.nx + i;
        if (changed_out) changed_out[e] = changed ? 1 : 0;
        if (theta_out) {
            theta_out[2 * e] = th1;
            theta_out[2 * e + 1] = th2;
        }
    }
}

// mode: 0 = flags from the modal-decay sensor (s > s0), 1 = flags given,
// 2 = no flags (the positivity scaling alone).  apply = 1: limit the flagged
// elements in place; 0: only report.  PP (with apply): then the positivity
// scaling on every element.  Outputs (each may be NULL): flag[e],
// changed[e] (a mode changed), sensor[e] (log10 of the top-degree density
// energy share), theta[2e], theta[2e+1] (the positivity factors).
template <int N, int NV>
__global__ void __launch_bounds__(256) k_troubled(const Geo g, double* u, const double* __restrict__ u0, double s0,
                                                  int mode, int apply, const unsigned char* __restrict__ flag_in,
                                                  unsigned char* flag_out, unsigned char* changed_out,
                                                  float* sensor_out, double* theta_out, unsigned char* pp_ok) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= g.E) return;
    const int i = (int)(e % g.nx), j = (int)(e / g.nx);
    const unsigned base = tiled_base<N, NV>(g, i, j);
    bool flag = false;
    if (mode == 0) {
        double top = 0.0, all = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
            for (int b = 0; b < N; ++b) {
                const double v = u[base + mode_off<N>(0, a, b)];
                all += v * v;
                if (a == N - 1 || b == N - 1) top += v * v;
            }
        const double s = (all > 0.0 && top > 0.0) ? log10(top / all) : -300.0;
        flag = s > s0;
        if (sensor_out) sensor_out[e] = (float)s;
    } else if (mode == 1) {
        flag = flag_in[e] != 0;
    }
    if (flag_out) flag_out[e] = flag ? 1 : 0;
    bool changed = false;
    if (flag) {
        const double r3 = sqrt(3.0);
        double sx[NV], sy[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double m = u[base + mode_off<N>(v, 0, 0)];
            const double ax = r3 * u[base + mode_off<N>(v, 1, 0)];
            const double ay = r3 * u[base + mode_off<N>(v, 0, 1)];
            const double lx = minmod3(ax, nb_mean<N, NV>(g, u, u0, i, j, v, 1) - m, m - nb_mean<N, NV>(g, u, u0, i, j, v, 0));
            const double ly = minmod3(ay, nb_mean<N, NV>(g, u, u0, i, j, v, 3) - m, m - nb_mean<N, NV>(g, u, u0, i, j, v, 2));
            sx[v] = lx;
            sy[v] = ly;
            if (lx != ax || ly != ay) changed = true;
        }
        if (changed && apply) {
            // means are never modified, so the neighbours read above are
            // unaffected by other threads' updates
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int a = 0; a < N; ++a)
#pragma unroll
                    for (int b = 0; b < N; ++b) {
                        if (a == 0 && b == 0) continue;
                        u[base + mode_off<N>(v, a, b)] = (a == 1 && b == 0) ? sx[v] / r3 : (a == 0 && b == 1) ? sy[v] / r3 : 0.0;
                    }
        }
    }
    if (changed_out) changed_out[e] = changed ? 1 : 0;
    // an element changed here needs the positivity check again
    if (pp_ok && changed && apply) pp_ok[j * g.tiles_x + i / (64 / N)] = 0;
}

// ------------------------------------------------------------------ learned indicator

// features of every element: f[e][v*16 + m] = u_vm / (|u_v00| + scale_v), bf16
template <int N, int NV>
__global__ void __launch_bounds__(256) k_features(const Geo g, const double* __restrict__ u,
                                                  const double* __restrict__ scale, unsigned short* __restrict__ f) {
    constexpr int NN = N * N;
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= g.E) return;
    const unsigned base = tiled_base<N, NV>(g, (int)(e % g.nx), (int)(e / g.nx));
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double d = fabs(u[base + mode_off<N>(v, 0, 0)]) + scale[v];
#pragma unroll
        for (int m = 0; m < NN; ++m)
            f[e * (NV * NN) + v * NN + m] = f2bf((float)(u[base + mode_off<N>(v, m / N, m % N)] / d));
    }
}

// Forward pass on bf16 MFMA 16x16x16 tiles; one wavefront handles 16 samples
// per iteration.  Fragment layouts (lane l, i = l % 16, g = l / 16):
//   A (16 x 16): A[i][4g + k], k = 0..3     B (16 x 16): B[4g + k][i]
//   C (16 x 16): C[4g + k][i]
// Layer 1: H1 (32 x 16) = W1 (32 x 64) X^T, two row tiles, four K steps.
// Layer 2: the C fragments of the two H1 row tiles are exactly the B
// fragments of the two K steps of W2 H1, so no data moves between lanes.
// The 32 -> 1 output is a lane dot product plus a reduction over g.
// Optional outputs for training: z (logits), h1/h2 (bf16 activations fed on,
// sample-major [n][32]) and the pre-activation signs.
__global__ void __launch_bounds__(256) k_mlp_forward(const unsigned short* __restrict__ x, long long n,
                                                     const float* __restrict__ par, float* __restrict__ z_out,
                                                     float* __restrict__ h1_out, float* __restrict__ h2_out,
                                                     unsigned char* __restrict__ flag_out, float zthr) {
    __shared__ unsigned short sW1[kH * kIn], sW2[kH * kH];
    for (int k = threadIdx.x; k < kH * kIn; k += 256) sW1[k] = f2bf(par[kW1 + k]);
    for (int k = threadIdx.x; k < kH * kH; k += 256) sW2[k] = f2bf(par[kW2 + k]);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, gq = lane >> 4;
    // weight fragments (A operands), held for all tiles
    bf16x4 a1[2][4], a2[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int k = 0; k < 4; ++k) a1[t][s][k] = (short)sW1[(16 * t + i) * kIn + 16 * s + 4 * gq + k];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int k = 0; k < 4; ++k) a2[t][s][k] = (short)sW2[(16 * t + i) * kH + 16 * s + 4 * gq + k];
    }
    float b1v[2][4], b2v[2][4], w3v[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int row = 16 * t + 4 * gq + k;
            b1v[t][k] = par[kB1 + row];
            b2v[t][k] = par[kB2 + row];
            w3v[t][k] = bf2f(f2bf(par[kW3 + row]));
        }
    const float b3 = par[kB3];
    const long long ntile = (n + 15) / 16;
    for (long long tile = (long long)blockIdx.x * 4 + wave; tile < ntile; tile += (long long)gridDim.x * 4) {
        const long long sidx = tile * 16 + i;  // this lane's sample (column)
        const bool valid = sidx < n;
        const long long sl = valid ? sidx : n - 1;  // loads stay in bounds on a ragged last tile
        // layer 1
        f32x4 c1[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) c1[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            bf16x4 b;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const short xv = (short)x[sl * kIn + 16 * s + 4 * gq + k];
                b[k] = valid ? xv : (short)0;
            }
#pragma unroll
            for (int t = 0; t < 2; ++t) c1[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[t][s], b, c1[t], 0, 0, 0);
        }
        // bias, ReLU, round to bf16: these are the B fragments of layer 2
        bf16x4 hb[2];
        float h1f[2][4];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float zz = c1[t][k] + b1v[t][k];
                const unsigned short hv = f2bf(zz > 0.f ? zz : 0.f);
                hb[t][k] = (short)hv;
                h1f[t][k] = bf2f(hv);
            }
        f32x4 c2[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) c2[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int t = 0; t < 2; ++t) c2[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2[t][s], hb[s], c2[t], 0, 0, 0);
        float part = 0.f;
        float h2f[2][4];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float zz = c2[t][k] + b2v[t][k];
                h2f[t][k] = bf2f(f2bf(zz > 0.f ? zz : 0.f));
                part += w3v[t][k] * h2f[t][k];
            }
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        const float zl = part + b3;
        if (valid) {
            if (gq == 0) {
                if (z_out) z_out[sidx] = zl;
                if (flag_out) flag_out[sidx] = zl > zthr ? 1 : 0;
            }
            if (h1_out) {
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        h1_out[sidx * kH + 16 * t + 4 * gq + k] = h1f[t][k];
                        h2_out[sidx * kH + 16 * t + 4 * gq + k] = h2f[t][k];
                    }
            }
        }
    }
}

// The network's weights in the per-lane fragment form of dg_mlp.h, from the
// FP32 parameters (one wavefront), for the stage kernel that forms the flags
// of the rows it writes.
__global__ void __launch_bounds__(64) k_mlp_pack(const float* __restrict__ par, void* __restrict__ pack) {
    const int lane = threadIdx.x;
    MlpLane w;
    mlp_lane_from_params(par, lane, w);
    unsigned long long* fr = (unsigned long long*)pack;
    float* fv = (float*)(fr + kPackFrag * 64);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
        for (int s = 0; s < 4; ++s) fr[(t * 4 + s) * 64 + lane] = __builtin_bit_cast(unsigned long long, w.a1[t][s]);
#pragma unroll
        for (int s = 0; s < 2; ++s) fr[(8 + t * 2 + s) * 64 + lane] = __builtin_bit_cast(unsigned long long, w.a2[t][s]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            fv[(t * 4 + k) * 64 + lane] = w.b1v[t][k];
            fv[(8 + t * 4 + k) * 64 + lane] = w.b2v[t][k];
            fv[(16 + t * 4 + k) * 64 + lane] = w.w3v[t][k];
        }
    }
    if (lane == 0) fv[kPackVec * 64] = w.b3;
}

// Backward pass of the BCE-with-logits loss (mean over n, positives weighted
// by pos_weight) through the forward values saved by k_mlp_forward (bf16
// rounding treated as identity), FP32.  k_mlp_delta: one thread per sample,
// the output and hidden-layer deltas; k_mlp_grad: one thread per parameter,
// the sum over samples in sample order (FP64 accumulation), so the gradient is
// deterministic.
__global__ void __launch_bounds__(256) k_mlp_delta(const float* __restrict__ y, long long n, float pos_weight,
                                                   const float* __restrict__ par, const float* __restrict__ z,
                                                   const float* __restrict__ h1, const float* __restrict__ h2,
                                                   float* __restrict__ dz_out, float* __restrict__ d1_out,
                                                   float* __restrict__ d2_out, float* __restrict__ loss_part) {
    __shared__ float red[256];
    const long long sidx = (long long)blockIdx.x * 256 + threadIdx.x;
    float loss = 0.f;
    if (sidx < n) {
        const float zz = z[sidx], yy = y[sidx];
        const float sg = 1.f / (1.f + expf(-zz));
        const float lsp = zz >= 0.f ? -log1pf(expf(-zz)) : zz - log1pf(expf(zz));
        const float lsn = zz >= 0.f ? -zz - log1pf(expf(-zz)) : -log1pf(expf(zz));
        loss = -(pos_weight * yy * lsp + (1.f - yy) * lsn) / (float)n;
        const float dz = (pos_weight * yy * (sg - 1.f) + (1.f - yy) * sg) / (float)n;
        dz_out[sidx] = dz;
        float d2[kH];
#pragma unroll
        for (int k = 0; k < kH; ++k) {
            d2[k] = h2[sidx * kH + k] > 0.f ? dz * bf2f(f2bf(par[kW3 + k])) : 0.f;
            d2_out[sidx * kH + k] = d2[k];
        }
#pragma unroll
        for (int k = 0; k < kH; ++k) {
            float s = 0.f;
#pragma unroll
            for (int o = 0; o < kH; ++o) s += d2[o] * bf2f(f2bf(par[kW2 + o * kH + k]));
            d1_out[sidx * kH + k] = h1[sidx * kH + k] > 0.f ? s : 0.f;
        }
    }
    red[threadIdx.x] = loss;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_mlp_grad(const unsigned short* __restrict__ x, long long n,
                                                  const float* __restrict__ dz, const float* __restrict__ d1,
                                                  const float* __restrict__ d2, const float* __restrict__ h1,
                                                  const float* __restrict__ h2, float* __restrict__ grad) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kNParam) return;
    double s = 0.0;
    if (p < kB1) {
        const int o = p / kIn, k = p % kIn;
        for (long long i = 0; i < n; ++i) s += (double)(d1[i * kH + o] * bf2f(x[i * kIn + k]));
    } else if (p < kW2) {
        const int o = p - kB1;
        for (long long i = 0; i < n; ++i) s += (double)d1[i * kH + o];
    } else if (p < kB2) {
        const int o = (p - kW2) / kH, k = (p - kW2) % kH;
        for (long long i = 0; i < n; ++i) s += (double)(d2[i * kH + o] * h1[i * kH + k]);
    } else if (p < kW3) {
        const int o = p - kB2;
        for (long long i = 0; i < n; ++i) s += (double)d2[i * kH + o];
    } else if (p < kB3) {
        const int k = p - kW3;
        for (long long i = 0; i < n; ++i) s += (double)(dz[i] * h2[i * kH + k]);
    } else {
        for (long long i = 0; i < n; ++i) s += (double)dz[i];
    }
    grad[p] = (float)s;
}

// Adam (Kingma & Ba 2015) on the FP32 master parameters; the loss partials
// are summed in block order into loss_out
__global__ void __launch_bounds__(256) k_mlp_adam(const float* __restrict__ grad, const float* __restrict__ loss_part,
                                                  int nblk, float* __restrict__ par, float* __restrict__ m,
                                                  float* __restrict__ v, long long t, float lr, float b1, float b2,
                                                  float eps, float* __restrict__ loss_out) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p == 0 && loss_out) {
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += loss_part[b];
        *loss_out = s;
    }
    if (p >= kNParam || lr <= 0.f) return;
    const float gs = grad[p];
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    const float mm = b1 * m[p] + (1.f - b1) * gs;
    const float vv = b2 * v[p] + (1.f - b2) * gs * gs;
    m[p] = mm;
    v[p] = vv;
    par[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// ------------------------------------------------------------------ launchers
#define DGL_DISPATCH(n, nv, BODY)                                                    \
    if (n == 2 && nv == 3) { constexpr int NT = 2, VT = 3; BODY; }                   \
    else if (n == 3 && nv == 3) { constexpr int NT = 3, VT = 3; BODY; }              \
    else if (n == 4 && nv == 3) { constexpr int NT = 4, VT = 3; BODY; }              \
    else if (n == 5 && nv == 3) { constexpr int NT = 5, VT = 3; BODY; }              \
    else if (n == 2 && nv == 4) { constexpr int NT = 2, VT = 4; BODY; }              \
    else if (n == 3 && nv == 4) { constexpr int NT = 3, VT = 4; BODY; }              \
    else if (n == 4 && nv == 4) { constexpr int NT = 4, VT = 4; BODY; }              \
    else if (n == 5 && nv == 4) { constexpr int NT = 5, VT = 4; BODY; }              \
    else return hipErrorInvalidValue;

hipError_t launch_troubled(int n, int nvar, const Geo& g, double* u, const double* u0, double s0, int mode, int apply,
                           const unsigned char* flag_in, unsigned char* flag_out, unsigned char* changed_out,
                           float* sensor_out, int pp, double* theta_out, hipStream_t s, unsigned char* pp_ok) {
    // the tile marks are only used where no per-element output is asked for
    if (changed_out || theta_out || !pp) pp_ok = nullptr;
    const int blocks = (int)((g.E + 255) / 256);
    // flags and minmod (skipped when there are no flags), then the positivity
    // scaling with N lanes per element
    if (mode != 2 || !pp) {
        DGL_DISPATCH(n, nvar, hipLaunchKernelGGL((k_troubled<NT, VT>), dim3(blocks), dim3(256), 0, s, g, u, u0,
                                                 s0, mode, apply, flag_in, flag_out, pp ? nullptr : changed_out,
                                                 sensor_out, nullptr, pp_ok));
    }
    if (pp && apply) {
        const int tiles = g.tiles_x * g.ny;
        DGL_DISPATCH(n, nvar, hipLaunchKernelGGL((k_pp_c<NT, VT>), dim3(tiles), dim3(64), 0, s, g, u, g.pp_eps,
                                                 changed_out, theta_out, pp_ok));
    }
    return hipGetLastError();
}

hipError_t launch_features(int n, int nvar, const Geo& g, const double* u, const double* scale, unsigned short* f,
                           hipStream_t s) {
    const int blocks = (int)((g.E + 255) / 256);
    DGL_DISPATCH(n, nvar, hipLaunchKernelGGL((k_features<NT, VT>), dim3(blocks), dim3(256), 0, s, g, u, scale, f));
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const unsigned short* x, long long n, const float* par, float* z, float* h1, float* h2,
                              unsigned char* flags, float zthr, hipStream_t s) {
    const long long ntile = (n + 15) / 16;
    long long blocks = (ntile + 3) / 4;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(256), 0, s, x, n, par, z, h1, h2, flags, zthr);
    return hipGetLastError();
}

hipError_t launch_mlp_pack(const float* par, void* pack, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_pack, dim3(1), dim3(64), 0, s, par, pack);
    return hipGetLastError();
}

int mlp_pack_bytes() { return kPackBytes; }

int mlp_delta_blocks(long long n) { return (int)((n + 255) / 256); }
int mlp_nparam() { return kNParam; }

hipError_t launch_mlp_backward(const unsigned short* x, const float* y, long long n, float pos_weight,
                               const float* par, const float* z, const float* h1, const float* h2, float* dz,
                               float* d1, float* d2, float* loss_part, float* grad, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_delta, dim3(mlp_delta_blocks(n)), dim3(256), 0, s, y, n, pos_weight, par, z, h1, h2, dz,
                       d1, d2, loss_part);
    hipLaunchKernelGGL(k_mlp_grad, dim3((kNParam + 255) / 256), dim3(256), 0, s, x, n, dz, d1, d2, h1, h2, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(const float* grad, const float* loss_part, int nblk, float* par, float* m, float* v,
                           long long t, float lr, float b1, float b2, float eps, float* loss_out, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((kNParam + 255) / 256), dim3(256), 0, s, grad, loss_part, nblk, par, m, v, t,
                       lr, b1, b2, eps, loss_out);
    return hipGetLastError();
}

}  // namespace dgk
