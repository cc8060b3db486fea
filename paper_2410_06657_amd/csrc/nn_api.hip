// C ABI of the warm-start network: workspace carving, parameter I/O, forward pass, gradient
// and one Adam training step.  Every operation runs in the kernels of nn_kernels.hpp on the
// network's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lbm.h"
#include "nn_kernels.hpp"
#include "nn_state.hpp"

static_assert(NN_HIDDEN == nn::NL - 1, "one hidden buffer per layer but the last");

using nn::half;

namespace {

constexpr size_t ALIGN = 256;
size_t rup(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct NnLayout {
    size_t p, mo, ve, g, wh, wflip, xh, act[nn::NL - 1], dz[2], x, y, lpart, lsum, dwpart, total;
};

int64_t loss_blocks(int64_t cap) { return (cap + nn::WGT - 1) / nn::WGT; }

NnLayout nn_layout(int64_t cap) {
    NnLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t r = off; off = rup(off + bytes); return r; };
    L.p = take(sizeof(float) * nn::PTOTAL);
    L.mo = take(sizeof(float) * nn::PTOTAL);
    L.ve = take(sizeof(float) * nn::PTOTAL);
    L.g = take(sizeof(float) * nn::PTOTAL);
    L.wh = take(sizeof(half) * nn::WTOTAL);
    L.wflip = take(sizeof(half) * 9 * nn::CH * nn::CH);
    L.xh = take(sizeof(half) * cap * nn::CIN0);
    for (int l = 0; l < nn::NL - 1; l++) L.act[l] = take(sizeof(half) * cap * nn::CH);
    L.dz[0] = take(sizeof(half) * cap * nn::CH);
    L.dz[1] = take(sizeof(half) * cap * nn::CH);
    L.x = take(sizeof(float) * cap * nn::NIN);
    L.y = take(sizeof(float) * cap);
    L.lpart = take(sizeof(double) * loss_blocks(cap));
    L.lsum = take(sizeof(double));
    L.dwpart = take(sizeof(float) * nnapi::DW_PARTS * (9 * nn::CH * nn::CH + nn::CH));
    L.total = off;
    return L;
}

#define NNCHK(nnh, x)                                                    \
    do {                                                                 \
        hipError_t e_ = (x);                                             \
        if (e_ != hipSuccess) {                                          \
            (nnh)->err = std::string(#x) + ": " + hipGetErrorString(e_); \
            return LBM_EHIP;                                             \
        }                                                                \
    } while (0)

uint64_t splitmix(uint64_t& s) {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Glorot-uniform weights on the real entries (fan in 9 cin, fan out 9 cout), the last layer
// scaled by 0.1 so the untrained output starts near zero; biases zero.
std::vector<float> initial_params(unsigned long long seed) {
    std::vector<float> v(nn::PTOTAL, 0.f);
    uint64_t s = seed;
    for (int l = 0; l < nn::NL; l++) {
        int ci = l == 0 ? nn::NIN : nn::CH, co = l == nn::NL - 1 ? 1 : nn::CH;
        double a = std::sqrt(6.0 / (9.0 * (ci + co))) * (l == nn::NL - 1 ? 0.1 : 1.0);
        int kin = nn::cin(l);
        for (int t = 0; t < 9; t++)
            for (int o = 0; o < nn::CH; o++)
                for (int i = 0; i < kin; i++) {
                    double u = (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
                    if (nn::w_real(l, o, i)) v[nn::woff(l) + (t * nn::CH + o) * kin + i] = (float)((2.0 * u - 1.0) * a);
                }
    }
    return v;
}

bool shape_ok(const lbm_nn* nn, int n, int h, int w) {
    return n >= 1 && h >= 1 && w >= 1 && (int64_t)n * h * w <= nn->cap;
}

// Forward pass into the packed-input buffer xh and the hidden buffers act[0..NL-2] (layer l
// reads act[l-1] and writes act[l]: consecutive entries must differ).  The handle's own
// buffers keep the activations for a following backward pass.
int run_forward_into(lbm_nn* nn, const float* x, float* y, int n, int h, int w, hipStream_t st, half* xh,
                     half* const* act) {
    const int npix = n * h * w;
    nn::k_pack_input<<<(npix + 255) / 256, 256, 0, st>>>(x, xh, npix);
    const int segs = (w + 31) / 32;
    const int64_t waves = (int64_t)n * h * segs;
    const int blocks = (int)((waves + 3) / 4);
    const half* in = xh;
    for (int l = 0; l < nn::NL; l++) {
        const half* wl = nn->wh + nn::woff(l);
        const float* bl = nn->p + nn::WTOTAL + l * nn::CH;
        if (l == 0)
            nn::k_conv<nn::CIN0, nn::EPI_TANH><<<blocks, nn::WGT, 0, st>>>(in, wl, bl, nullptr, act[0], nullptr, n, h,
                                                                            w, nn::dil(l), 1.f);
        else if (l < nn::NL - 1)
            nn::k_conv<nn::CH, nn::EPI_TANH><<<blocks, nn::WGT, 0, st>>>(in, wl, bl, nullptr, act[l], nullptr, n, h,
                                                                          w, nn::dil(l), 1.f);
        else
            nn::k_conv<nn::CH, nn::EPI_LINEAR><<<blocks, nn::WGT, 0, st>>>(in, wl, bl, nullptr, nullptr, y, n, h, w,
                                                                            nn::dil(l), 1.f);
        if (l < nn::NL - 1) in = act[l];
    }
    NNCHK(nn, hipGetLastError());
    return LBM_OK;
}

int run_forward(lbm_nn* nn, const float* x, float* y, int n, int h, int w, hipStream_t st) {
    return run_forward_into(nn, x, y, n, h, w, st, nn->xh, nn->act);
}

// Scratch of the allocation-free forward pass (lbm_nn_forward_noalloc): the packed input
// (CIN0 channels) and two hidden buffers used in turn (CH channels each), FP16, for up to
// LBM_NN_NOALLOC_MAX_PIXELS pixels: 2.25 MiB per device, held until the process ends.  In
// host code this name stands for the array, not its device address: kernels get the address
// from noalloc_scratch().
constexpr int64_t NOALLOC_HALVES = (int64_t)LBM_NN_NOALLOC_MAX_PIXELS * (nn::CIN0 + 2 * nn::CH);
static __device__ __align__(256) half scratch[NOALLOC_HALVES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
half* scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`, looked up on the first call on
// that device.
int noalloc_scratch(lbm_nn* nn, half** out) {
    int dev = 0;
    NNCHK(nn, hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) {
        nn->err = "device index beyond the scratch table";
        return LBM_EINVAL;
    }
    std::lock_guard<std::mutex> g(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        NNCHK(nn, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        scratch_ptr[dev] = (half*)p;
    }
    *out = scratch_ptr[dev];
    return LBM_OK;
}

__global__ void k_sum_parts(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double sh[4];
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) s += part[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = sh[0] + sh[1] + sh[2] + sh[3];
}

// Loss and gradient of L = sum (y - t)^2 into nn->g (FP32, parameter order).
constexpr float GSCALE = 256.f;  // FP16 gradient scale (undone in the FP32 reduction)

int run_backward(lbm_nn* nn, const float* t, int n, int h, int w, hipStream_t st) {
    const int npix = n * h * w;
    const int lb = (int)loss_blocks(npix);
    nn::k_loss<<<lb, nn::WGT, 0, st>>>(nn->y, t, nn->dz[0], nn->lpart, npix, GSCALE);
    k_sum_parts<<<1, 256, 0, st>>>(nn->lpart, lb, nn->lsum);
    const int segs = (w + 31) / 32;
    const int64_t waves = (int64_t)n * h * segs;
    const int blocks = (int)((waves + 3) / 4);
    int cur = 0;
    for (int l = nn::NL - 1; l >= 0; l--) {
        const half* input = l == 0 ? nn->xh : nn->act[l - 1];
        const int kin = nn::cin(l);
        if (l == 0)
            nn::k_dw<nn::CIN0><<<nnapi::DW_PARTS, nn::WGT, 0, st>>>(nn->dz[cur], input, nn->dwpart, n, h, w, nn::dil(l));
        else
            nn::k_dw<nn::CH><<<nnapi::DW_PARTS, nn::WGT, 0, st>>>(nn->dz[cur], input, nn->dwpart, n, h, w, nn::dil(l));
        const int ne = 9 * nn::CH * kin + nn::CH;
        nn::k_dw_reduce<<<(ne + 255) / 256, 256, 0, st>>>(nn->dwpart, nnapi::DW_PARTS, nn->g + nn::woff(l),
                                                          nn->g + nn::WTOTAL + l * nn::CH, l, kin, 1.f / GSCALE);
        if (l > 0) {
            nn::k_flip<<<(9 * nn::CH * nn::CH + 255) / 256, 256, 0, st>>>(nn->wh + nn::woff(l), nn->wflip, kin);
            nn::k_conv<nn::CH, nn::EPI_DTANH><<<blocks, nn::WGT, 0, st>>>(nn->dz[cur], nn->wflip, nullptr, nn->act[l - 1],
                                                                           nn->dz[cur ^ 1], nullptr, n, h, w, nn::dil(l),
                                                                           1.f);
            cur ^= 1;
        }
    }
    NNCHK(nn, hipGetLastError());
    return LBM_OK;
}

int fetch_loss(lbm_nn* nn, double* loss) {
    if (!loss) return LBM_OK;
    NNCHK(nn, hipMemcpyAsync(nn->hloss, nn->lsum, sizeof(double), hipMemcpyDeviceToHost, nn->stream));
    NNCHK(nn, hipStreamSynchronize(nn->stream));
    *loss = *nn->hloss;
    return LBM_OK;
}

}  // namespace

namespace nnapi {
int forward(lbm_nn* nn, const float* x, float* y, int n, int h, int w, hipStream_t stream) {
    if (!shape_ok(nn, n, h, w)) return LBM_EINVAL;
    return run_forward(nn, x ? x : nn->x, y ? y : nn->y, n, h, w, stream);
}
}  // namespace nnapi

extern "C" {

int lbm_nn_param_count(int* count) {
    if (!count) return LBM_EINVAL;
    *count = nn::PTOTAL;
    return LBM_OK;
}

int lbm_nn_workspace_bytes(long long max_pixels, size_t* bytes) {
    if (max_pixels < 1 || !bytes) return LBM_EINVAL;
    *bytes = nn_layout(max_pixels).total;
    return LBM_OK;
}

int lbm_nn_init(void* workspace, size_t bytes, long long max_pixels, unsigned long long seed, void* stream,
                lbm_nn** out) {
    if (!workspace || !out || max_pixels < 1 || ((uintptr_t)workspace % ALIGN) != 0) return LBM_EINVAL;
    NnLayout L = nn_layout(max_pixels);
    if (bytes < L.total) return LBM_ESPACE;
    lbm_nn* nnh = new (std::nothrow) lbm_nn();
    if (!nnh) return LBM_EINVAL;
    char* ws = (char*)workspace;
    nnh->cap = max_pixels;
    nnh->stream = (hipStream_t)stream;
    nnh->p = (float*)(ws + L.p);
    nnh->mo = (float*)(ws + L.mo);
    nnh->ve = (float*)(ws + L.ve);
    nnh->g = (float*)(ws + L.g);
    nnh->wh = (half*)(ws + L.wh);
    nnh->wflip = (half*)(ws + L.wflip);
    nnh->xh = (half*)(ws + L.xh);
    for (int l = 0; l < nn::NL - 1; l++) nnh->act[l] = (half*)(ws + L.act[l]);
    nnh->dz[0] = (half*)(ws + L.dz[0]);
    nnh->dz[1] = (half*)(ws + L.dz[1]);
    nnh->x = (float*)(ws + L.x);
    nnh->y = (float*)(ws + L.y);
    nnh->lpart = (double*)(ws + L.lpart);
    nnh->lsum = (double*)(ws + L.lsum);
    nnh->dwpart = (float*)(ws + L.dwpart);
    if (hipHostMalloc((void**)&nnh->hloss, sizeof(double), hipHostMallocDefault) != hipSuccess) {
        delete nnh;
        return LBM_EHIP;
    }
    std::vector<float> p0 = initial_params(seed);
    int rc = lbm_nn_set_params(nnh, p0.data());
    if (rc) {
        lbm_nn_destroy(nnh);
        return rc;
    }
    *out = nnh;
    return LBM_OK;
}

int lbm_nn_set_params(lbm_nn* nnh, const float* host) {
    if (!nnh) return LBM_ESTATE;
    if (!host) return LBM_EINVAL;
    // padding entries are forced to zero whatever the caller passes
    std::vector<float> v(host, host + nn::PTOTAL);
    for (int l = 0; l < nn::NL; l++) {
        int kin = nn::cin(l);
        for (int t = 0; t < 9; t++)
            for (int o = 0; o < nn::CH; o++)
                for (int i = 0; i < kin; i++)
                    if (!nn::w_real(l, o, i)) v[nn::woff(l) + (t * nn::CH + o) * kin + i] = 0.f;
        for (int o = 0; o < nn::CH; o++)
            if (!nn::b_real(l, o)) v[nn::WTOTAL + l * nn::CH + o] = 0.f;
    }
    // pageable source that ends with this call: drain the stream, then a blocking copy
    NNCHK(nnh, hipStreamSynchronize(nnh->stream));
    NNCHK(nnh, hipMemcpy(nnh->p, v.data(), sizeof(float) * nn::PTOTAL, hipMemcpyHostToDevice));
    NNCHK(nnh, hipMemsetAsync(nnh->mo, 0, sizeof(float) * nn::PTOTAL, nnh->stream));
    NNCHK(nnh, hipMemsetAsync(nnh->ve, 0, sizeof(float) * nn::PTOTAL, nnh->stream));
    nn::k_to_half<<<(nn::WTOTAL + 255) / 256, 256, 0, nnh->stream>>>(nnh->p, nnh->wh);
    NNCHK(nnh, hipGetLastError());
    NNCHK(nnh, hipStreamSynchronize(nnh->stream));
    nnh->t = 0;
    return LBM_OK;
}

int lbm_nn_get_params(lbm_nn* nnh, float* host) {
    if (!nnh) return LBM_ESTATE;
    if (!host) return LBM_EINVAL;
    // pageable destination: drain the stream, then a blocking copy
    NNCHK(nnh, hipStreamSynchronize(nnh->stream));
    NNCHK(nnh, hipMemcpy(host, nnh->p, sizeof(float) * nn::PTOTAL, hipMemcpyDeviceToHost));
    return LBM_OK;
}

int lbm_nn_forward(lbm_nn* nnh, const float* x, float* y, int n, int h, int w) {
    if (!nnh) return LBM_ESTATE;
    if (!x || !y) return LBM_EINVAL;
    return nnapi::forward(nnh, x, y, n, h, w, nnh->stream);
}

int lbm_nn_forward_noalloc(lbm_nn* nnh, const float* x, float* y, int n, int h, int w) {
    if (!nnh) return LBM_ESTATE;
    if (!x || !y || n < 1 || h < 1 || w < 1 || (int64_t)n * h * w > LBM_NN_NOALLOC_MAX_PIXELS) return LBM_EINVAL;
    half* base = nullptr;
    int rc = noalloc_scratch(nnh, &base);
    if (rc) return rc;
    half* xh = base;
    half* a0 = xh + (int64_t)LBM_NN_NOALLOC_MAX_PIXELS * nn::CIN0;
    half* a1 = a0 + (int64_t)LBM_NN_NOALLOC_MAX_PIXELS * nn::CH;
    half* act[nn::NL - 1];
    for (int l = 0; l < nn::NL - 1; l++) act[l] = (l & 1) ? a1 : a0;
    return run_forward_into(nnh, x, y, n, h, w, nnh->stream, xh, act);
}

int lbm_nn_gradient(lbm_nn* nnh, const float* x, const float* t, int n, int h, int w, float* grad, double* loss) {
    if (!nnh) return LBM_ESTATE;
    if (!x || !t || !grad || !shape_ok(nnh, n, h, w)) return LBM_EINVAL;
    int rc = run_forward(nnh, x, nnh->y, n, h, w, nnh->stream);
    if (!rc) rc = run_backward(nnh, t, n, h, w, nnh->stream);
    if (rc) return rc;
    NNCHK(nnh, hipStreamSynchronize(nnh->stream));
    NNCHK(nnh, hipMemcpy(grad, nnh->g, sizeof(float) * nn::PTOTAL, hipMemcpyDeviceToHost));
    return fetch_loss(nnh, loss ? loss : nnh->hloss);
}

int lbm_nn_train_step(lbm_nn* nnh, const float* x, const float* t, int n, int h, int w, float lr, double* loss) {
    if (!nnh) return LBM_ESTATE;
    if (!x || !t || !shape_ok(nnh, n, h, w) || !(lr > 0.f)) return LBM_EINVAL;
    int rc = run_forward(nnh, x, nnh->y, n, h, w, nnh->stream);
    if (!rc) rc = run_backward(nnh, t, n, h, w, nnh->stream);
    if (rc) return rc;
    nnh->t++;
    const float b1 = 0.9f, b2 = 0.999f;
    float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)nnh->t)));
    float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)nnh->t)));
    nn::k_adam<<<(nn::PTOTAL + 255) / 256, 256, 0, nnh->stream>>>(nnh->p, nnh->mo, nnh->ve, nnh->g, nnh->wh, lr, b1,
                                                                   b2, c1, c2, 1e-8f);
    NNCHK(nnh, hipGetLastError());
    return fetch_loss(nnh, loss);
}

int lbm_nn_destroy(lbm_nn* nnh) {
    if (!nnh) return LBM_OK;
    (void)hipStreamSynchronize(nnh->stream);
    if (nnh->hloss) (void)hipHostFree(nnh->hloss);
    delete nnh;
    return LBM_OK;
}

const char* lbm_nn_last_error(const lbm_nn* nnh) { return nnh ? nnh->err.c_str() : ""; }

}  // extern "C"
