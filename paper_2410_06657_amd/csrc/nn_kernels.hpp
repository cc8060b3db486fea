// Kernels of the learned warm start of the potential: a six-layer network of dilated 3x3
// convolutions (3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1 channels, dilations 1, 2, 4, 8, 4, 1,
// tanh between layers) that maps coarse maps of the phase field and of the conductivity and
// permittivity ratios to the coarse deviation of the potential from the linear electrode
// ramp.  FP16 weights and activations, FP32 accumulation on the matrix cores
// (v_mfma_f32_32x32x8_f16), FP32 master weights and Adam moments.
//
// Layout: activations NHWC (channels fastest) so that the four consecutive channels an MFMA
// lane supplies are one 8-byte load; layer weights [tap][out][in] with tap = 3 ky + kx and
// offset ((kx - 1) d, (ky - 1) d) for dilation d; zero padding outside the image.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nn {

constexpr int NL = 6;        // layers
constexpr int CH = 32;       // hidden channels (and the padded output width of every layer)
constexpr int CIN0 = 8;      // input channels as stored (3 used, padded to one MFMA k-block)
constexpr int NIN = 3;       // input maps: psi, ln(sigma/sigma_gas), ln(eps/eps_gas)
constexpr int WGT = 256;     // threads per workgroup of the conv kernels (4 waves)

__host__ __device__ constexpr int dil(int l) { return l == 0 ? 1 : l == 1 ? 2 : l == 2 ? 4 : l == 3 ? 8 : l == 4 ? 4 : 1; }
__host__ __device__ constexpr int cin(int l) { return l == 0 ? CIN0 : CH; }
// stored weights of layer l: 9 taps x 32 outputs x cin(l) inputs
__host__ __device__ constexpr int wcount(int l) { return 9 * CH * cin(l); }
__host__ __device__ constexpr int woff(int l) {
    int o = 0;
    for (int k = 0; k < l; k++) o += wcount(k);
    return o;
}
constexpr int WTOTAL = woff(NL);          // all stored weights
constexpr int BTOTAL = NL * CH;           // all stored biases
constexpr int PTOTAL = WTOTAL + BTOTAL;   // stored parameters (master copy: weights then biases)

// Real (trainable) entries: layer 0 reads 3 input maps, layer 5 writes 1 output map; the
// padding entries stay exactly zero.
__host__ __device__ inline bool w_real(int l, int o, int i) {
    if (l == 0 && i >= NIN) return false;
    if (l == NL - 1 && o >= 1) return false;
    return true;
}
__host__ __device__ inline bool b_real(int l, int o) { return !(l == NL - 1 && o >= 1); }

typedef _Float16 half;
typedef half half4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ half4 load4(const half* p) { return *reinterpret_cast<const half4*>(p); }

// ---------------------------------------------------------------------------
// Input conversion: x (N, H, W, 3) FP32 -> FP16 with 8 channels (zeros beyond 3).
__global__ void k_pack_input(const float* __restrict__ x, half* __restrict__ xh, int npix) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    half4 a, b;
    a[0] = (half)x[3 * (int64_t)p];
    a[1] = (half)x[3 * (int64_t)p + 1];
    a[2] = (half)x[3 * (int64_t)p + 2];
    a[3] = (half)0.f;
    b[0] = b[1] = b[2] = b[3] = (half)0.f;
    *reinterpret_cast<half4*>(xh + (int64_t)p * CIN0) = a;
    *reinterpret_cast<half4*>(xh + (int64_t)p * CIN0 + 4) = b;
}

// ---------------------------------------------------------------------------
// Convolution as an implicit GEMM: out[p][o] = sum_t sum_k in[p + off_t][k] * w[t][o][k].
// Each wave computes 32 consecutive pixels of one row x all 32 outputs with one 32x32
// accumulator; the K loop runs over 9 taps x (KIN / 8) k-blocks.  The weights of the layer
// (9 x 32 x KIN halves) are staged in LDS once per workgroup.
//
// Epilogues:
//   EPI_TANH   out_h[p][o] = tanh(acc + b[o])                     (hidden layers)
//   EPI_LINEAR out_f[p]    = acc(o = 0) + b[0]                    (last layer, FP32)
//   EPI_DTANH  out_h[p][o] = acc * (1 - a[p][o]^2) * scale         (backward: dZ of the layer below)
enum { EPI_TANH = 0, EPI_LINEAR = 1, EPI_DTANH = 2 };

template <int KIN, int EPI>
__global__ void __launch_bounds__(WGT) k_conv(const half* __restrict__ in, const half* __restrict__ w,
                                              const float* __restrict__ bias, const half* __restrict__ act,
                                              half* __restrict__ out_h, float* __restrict__ out_f, int n, int H,
                                              int W, int d, float scale) {
    __shared__ __align__(16) half ws[9 * CH * KIN];
    for (int k = threadIdx.x; k < 9 * CH * KIN / 4; k += WGT)
        reinterpret_cast<half4*>(ws)[k] = reinterpret_cast<const half4*>(w)[k];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int segs = (W + 31) / 32;
    const int64_t seg = (int64_t)blockIdx.x * (WGT / 64) + wave;  // (image, row, segment)
    if (seg >= (int64_t)n * H * segs) return;
    const int sx = (int)(seg % segs);
    const int64_t r = seg / segs;
    const int y = (int)(r % H), img = (int)(r / H);
    const int x0 = sx * 32;
    const int m = lane & 31, kg = lane >> 5;
    floatx16 acc;
#pragma unroll
    for (int i = 0; i < 16; i++) acc[i] = 0.f;
    const int x = x0 + m;
#pragma unroll
    for (int t = 0; t < 9; t++) {
        const int yy = y + (t / 3 - 1) * d, xx = x + (t % 3 - 1) * d;
        const bool inside = yy >= 0 && yy < H && xx >= 0 && xx < W && x < W;
        const half* src = in + (((int64_t)img * H + (inside ? yy : 0)) * W + (inside ? xx : 0)) * KIN;
#pragma unroll
        for (int kb = 0; kb < KIN / 8; kb++) {
            half4 a;
            if (inside) {
                a = load4(src + kb * 8 + 4 * kg);
            } else {
                a[0] = a[1] = a[2] = a[3] = (half)0.f;
            }
            half4 b = load4(ws + (t * CH + m) * KIN + kb * 8 + 4 * kg);
            acc = __builtin_amdgcn_mfma_f32_32x32x8f16(a, b, acc, 0, 0, 0);
        }
    }
    // acc[q] holds pixel row 8 (q / 4) + 4 kg + (q % 4) of the tile, output channel m
    const int o = m;
#pragma unroll
    for (int q = 0; q < 16; q++) {
        const int pm = 8 * (q >> 2) + 4 * kg + (q & 3);
        const int px = x0 + pm;
        if (px >= W) continue;
        const int64_t p = ((int64_t)img * H + y) * W + px;
        if (EPI == EPI_TANH) {
            out_h[p * CH + o] = (half)tanhf(acc[q] + bias[o]);
        } else if (EPI == EPI_LINEAR) {
            if (o == 0) out_f[p] = acc[q] + bias[0];
        } else {
            const float av = (float)act[p * CH + o];
            out_h[p * CH + o] = (half)(acc[q] * (1.f - av * av) * scale);
        }
    }
}

// Weights of the transposed convolution that propagates dZ of layer l to its input:
// wt[8 - t][i][o] = w[t][o][i] (offsets negated, in and out swapped); KIN of the result is
// CH (the outputs of layer l), its outputs the cin(l) inputs (padded to CH).
__global__ void k_flip(const half* __restrict__ w, half* __restrict__ wt, int kin) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 9 * CH * CH) return;
    int t = e / (CH * CH), i = (e / CH) % CH, o = e % CH;  // destination [t][i][o]
    half v = (half)0.f;
    if (i < kin) v = w[((8 - t) * CH + o) * kin + i];
    wt[e] = v;
}

// ---------------------------------------------------------------------------
// Loss: y (FP32) against the target; L = sum (y - t)^2 over all pixels; dZ of the last layer
// (32 channels, channel 0 used) = 2 (y - t) * scale in FP16; per-workgroup FP64 partials.
__global__ void __launch_bounds__(WGT) k_loss(const float* __restrict__ y, const float* __restrict__ tgt,
                                              half* __restrict__ dz, double* __restrict__ part, int npix,
                                              float scale) {
    __shared__ double sh[WGT / 64];
    int p = blockIdx.x * WGT + threadIdx.x;
    double l = 0.0;
    if (p < npix) {
        float e = y[p] - tgt[p];
        l = (double)e * (double)e;
        half4 z;
        z[0] = (half)(2.f * e * scale);
        z[1] = z[2] = z[3] = (half)0.f;
        half4 zero;
        zero[0] = zero[1] = zero[2] = zero[3] = (half)0.f;
        half4* q = reinterpret_cast<half4*>(dz + (int64_t)p * CH);
        q[0] = z;
#pragma unroll
        for (int k = 1; k < CH / 4; k++) q[k] = zero;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) l += __shfl_down(l, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < WGT / 64; k++) s += sh[k];
        part[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// Weight gradient of one layer: dW[t][o][i] = sum_p dZ[p][o] * X[p + off_t][i] and
// db[o] = sum_p dZ[p][o], as an MFMA GEMM with M = o, N = i, K = pixels (8 per block).  Each
// wave walks row segments of 32 pixels with a grid stride; the four waves of a workgroup are
// summed through LDS and every workgroup writes one partial (9 x 32 x 32 + 32 floats).
template <int KIN>
__global__ void __launch_bounds__(WGT) k_dw(const half* __restrict__ dz, const half* __restrict__ x,
                                            float* __restrict__ part, int n, int H, int W, int d) {
    constexpr int PW = 9 * CH * CH + CH;  // partial floats per workgroup (dW padded to 32 inputs)
    __shared__ float red[PW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 31, kg = lane >> 5;
    const int segs = (W + 31) / 32;
    const int64_t nseg = (int64_t)n * H * segs;
    floatx16 acc[9];
#pragma unroll
    for (int t = 0; t < 9; t++)
#pragma unroll
        for (int i = 0; i < 16; i++) acc[t][i] = 0.f;
    float bsum = 0.f;
    for (int64_t seg = (int64_t)blockIdx.x * (WGT / 64) + wave; seg < nseg; seg += (int64_t)gridDim.x * (WGT / 64)) {
        const int sx = (int)(seg % segs);
        const int64_t r = seg / segs;
        const int y = (int)(r % H), img = (int)(r / H);
        const int x0 = sx * 32;
#pragma unroll
        for (int pb = 0; pb < 4; pb++) {
            // the 8 pixels x0 + 8 pb + 4 kg + j (j = 0..3) of this k-block
            half4 a;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int px = x0 + 8 * pb + 4 * kg + j;
                a[j] = px < W ? dz[(((int64_t)img * H + y) * W + px) * CH + m] : (half)0.f;
                bsum += (float)a[j];
            }
#pragma unroll
            for (int t = 0; t < 9; t++) {
                const int yy = y + (t / 3 - 1) * d;
                half4 b;
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int px = x0 + 8 * pb + 4 * kg + j;
                    const int xx = px + (t % 3 - 1) * d;
                    const bool inside = px < W && yy >= 0 && yy < H && xx >= 0 && xx < W && m < KIN;
                    b[j] = inside ? x[(((int64_t)img * H + yy) * W + xx) * KIN + m] : (half)0.f;
                }
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x8f16(a, b, acc[t], 0, 0, 0);
            }
        }
    }
    // acc[t][q] = dW[t][o = 8 (q / 4) + 4 kg + (q % 4)][i = m]; bsum holds dZ[.][m] of this lane
    bsum += __shfl_down(bsum, 32, 64);
    for (int k = threadIdx.x; k < PW; k += WGT) red[k] = 0.f;
    __syncthreads();
    for (int wv = 0; wv < WGT / 64; wv++) {
        if (wave == wv) {
#pragma unroll
            for (int t = 0; t < 9; t++)
#pragma unroll
                for (int q = 0; q < 16; q++) {
                    const int o = 8 * (q >> 2) + 4 * kg + (q & 3);
                    red[(t * CH + o) * CH + m] += acc[t][q];
                }
            if (kg == 0) red[9 * CH * CH + m] += bsum;
        }
        __syncthreads();
    }
    float* dst = part + (int64_t)blockIdx.x * PW;
    for (int k = threadIdx.x; k < PW; k += WGT) dst[k] = red[k];
}

// ---------------------------------------------------------------------------
// Sum the workgroup partials of one layer into the FP32 gradient (stored layout [t][o][i]
// with cin(l) inputs, then 32 biases), divided by `scale`; entries that are padding get 0.
__global__ void k_dw_reduce(const float* __restrict__ part, int nparts, float* __restrict__ gw,
                            float* __restrict__ gb, int layer, int kin, float inv_scale) {
    constexpr int PW = 9 * CH * CH + CH;
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    int nw = 9 * CH * kin;
    if (e >= nw + CH) return;
    int src;
    bool real;
    if (e < nw) {
        int t = e / (CH * kin), o = (e / kin) % CH, i = e % kin;
        src = (t * CH + o) * CH + i;
        real = w_real(layer, o, i);
    } else {
        int o = e - nw;
        src = 9 * CH * CH + o;
        real = b_real(layer, o);
    }
    double s = 0.0;
    for (int k = 0; k < nparts; k++) s += part[(int64_t)k * PW + src];
    float v = real ? (float)(s * inv_scale) : 0.f;
    if (e < nw) gw[e] = v; else gb[e - nw] = v;
}

// ---------------------------------------------------------------------------
// Adam on the FP32 master parameters (weights then biases), then the FP16 weight copy.
__global__ void k_adam(float* __restrict__ p, float* __restrict__ mo, float* __restrict__ ve,
                       const float* __restrict__ g, half* __restrict__ wh, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= PTOTAL) return;
    float gg = g[e];
    float m1 = b1 * mo[e] + (1.f - b1) * gg;
    float v1 = b2 * ve[e] + (1.f - b2) * gg * gg;
    mo[e] = m1;
    ve[e] = v1;
    float step = lr * (m1 * c1) / (sqrtf(v1 * c2) + eps);
    float np = p[e] - step;
    p[e] = np;
    if (e < WTOTAL) wh[e] = (half)np;
}

// FP16 copy of the master weights (after a host write of the parameters).
__global__ void k_to_half(const float* __restrict__ p, half* __restrict__ wh) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < WTOTAL) wh[e] = (half)p[e];
}

}  // namespace nn
