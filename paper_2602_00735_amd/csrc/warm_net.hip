// Learned warm start: the network object, its forward and backward passes
// and Adam (kernels in k_warm.hip).
//
// Five levels on a grid x grid map (grid divisible by 16), level widths
// c0..c4 (c3 == c4, each at most 64):
//   e0 = relu(conv(x)), e_l = relu(conv(pool(e_{l-1}))) for l = 1..4,
//   d3 = relu(conv(up(e4) + e3)), d2 = relu(conv(up(d3) + e2)),
//   d1 = relu(conv(up(d2) + e1)), d0 = relu(conv(up(d1) + e0)),
//   y = conv(d0) (two channels, fp32).
// The backward pass runs the same steps in reverse; the weight gradients
// are fp32, the activations and their gradients bfloat16.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "warm.h"

#define RCHK(x)                   \
    do {                          \
        const int rc_ = (x);      \
        if (rc_ != RAS_OK) return rc_; \
    } while (0)

namespace raspml {

void warm_conv(const void *X, const void *Wp, void *Y, const void *gate, int B, int H, int W,
               int CPin, int CPout, bool relu, bool acc, bool out_f32, int creal, bool in2, hipStream_t s);
int warm_wgrad_strip_blocks_max(int B, int W, int CPin, int CPout);
int warm_wgrad(const void *X, const void *dZ, float *part, int B, int H, int W, int CPin, int CPout,
               bool x2, bool z2, hipStream_t s);
void warm_sum_layers(int nl, const float *const *part, const int *nblk, const int *n, float *const *tmp,
                     float *const *g, hipStream_t s);
void warm_pool(const void *X, void *Y, int B, int H, int W, int C, hipStream_t s);
void warm_pool_bwd(const void *dY, const void *add, const void *gate, void *dX, int B, int H,
                   int W, int C, hipStream_t s);
void warm_up_add(const void *Yc, const void *E, void *S, int B, int H, int W, int C, hipStream_t s);
void warm_up_bwd(const void *dS, const void *gate, void *dYc, int B, int H, int W, int C,
                 hipStream_t s);
void warm_mse(const float *y, const float *t, long long npix, double *partial, int nblk, void *dY,
              double *loss, hipStream_t s);
void warm_adam_pack(int nl, float *const *w, float *const *m, float *const *v, float *const *g,
                    void *const *fwd, void *const *bwd, const int *cin, const int *cout, const int *cip,
                    const int *cop, float lr, float b1, float b2, float c1, float c2, float eps,
                    hipStream_t s);
void warm_pack_weights(const float *w, int cin, int cout, int cip, int cop, void *fwd, void *bwd,
                       hipStream_t s);

}  // namespace raspml

using namespace raspml;

namespace {

constexpr int kLayers = 10;            // e0 e1 e2 e3 e4 d3 d2 d1 d0 head
constexpr int kMseBlocks = 1024;
// Channels padded to what the kernels are instantiated for: one, two or
// four blocks of 16.
int cpad(int c) { return c <= 16 ? 16 : c <= 32 ? 32 : 64; }

}  // namespace

struct ras_pml_wsnet {
    int grid = 0, bmax = 0;
    int ch[5] = {};
    int cin[kLayers] = {}, cout[kLayers] = {}, lvl[kLayers] = {};
    float *w[kLayers] = {}, *m[kLayers] = {}, *v[kLayers] = {}, *g[kLayers] = {};
    void *wf[kLayers] = {}, *wb[kLayers] = {};
    void *e[5] = {}, *p[5] = {}, *s[4] = {}, *d[4] = {};
    void *gp[5] = {}, *gs[4] = {};
    float *gy = nullptr;                // the loss gradient: two fp32 channels per pixel
    void *dz = nullptr;                 // the current layer's output gradient, ReLU-masked
    float *y = nullptr, *stage = nullptr;
    // each layer's weight-gradient partials and slice sums, added for all
    // layers at once at the end of the backward pass
    float *part[kLayers] = {}, *psum[kLayers] = {};
    double *lpart = nullptr, *loss = nullptr;
    long long step = 0;
    std::vector<void *> allocs;
    std::string err;

    int cip(int L) const { return cpad(cin[L]); }
    int cop(int L) const { return cpad(cout[L]); }
    int side(int l) const { return grid >> l; }
    ~ras_pml_wsnet() {
        for (void *a : allocs) (void)hipFree(a);
    }
    template <typename T>
    bool alloc(T **ptr, size_t bytes) {
        void *q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) return false;
        if (hipMemset(q, 0, bytes) != hipSuccess) return false;
        allocs.push_back(q);
        *ptr = static_cast<T *>(q);
        return true;
    }
};

namespace raspml {

// forward pass on B samples; x: (B, grid, grid, 2) fp32, out: same shape
int wsnet_forward(ras_pml_wsnet *N, const float *x, int B, float *out, hipStream_t st) {
    const int G = N->grid;
    const int C[5] = {cpad(N->ch[0]), cpad(N->ch[1]), cpad(N->ch[2]), cpad(N->ch[3]), cpad(N->ch[4])};
    // the first layer reads the two fp32 input channels itself
    warm_conv(x, N->wf[0], N->e[0], nullptr, B, G, G, 16, C[0], true, false, false, 0, true, st);
    for (int l = 1; l <= 4; ++l) {
        const int S = N->side(l);
        warm_pool(N->e[l - 1], N->p[l], B, 2 * S, 2 * S, C[l - 1], st);
        warm_conv(N->p[l], N->wf[l], N->e[l], nullptr, B, S, S, C[l - 1], C[l], true, false, false, 0,
                  false, st);
    }
    // decoder: layer index 5 + (3 - l) for level l = 3..0
    const int din[4] = {C[0], C[1], C[2], C[3]};    // channels of s_l
    const int dout[4] = {C[0], C[0], C[1], C[2]};   // channels of d_l
    const void *prev = N->e[4];
    for (int l = 3; l >= 0; --l) {
        const int S = N->side(l), L = 5 + (3 - l);
        warm_up_add(prev, N->e[l], N->s[l], B, S, S, din[l], st);
        warm_conv(N->s[l], N->wf[L], N->d[l], nullptr, B, S, S, din[l], dout[l], true, false, false, 0,
                  false, st);
        prev = N->d[l];
    }
    warm_conv(N->d[0], N->wf[9], out, nullptr, B, G, G, C[0], 16, false, false, true, 2, false, st);
    return hipGetLastError() == hipSuccess ? RAS_OK : RAS_EHIP;
}

// forward, squared error against t, backward; the weight gradients are left
// in N->g (padded layout), the loss in N->loss (device)
int wsnet_gradient(ras_pml_wsnet *N, const float *x, const float *t, int B, hipStream_t st) {
    const int G = N->grid;
    const int C[5] = {cpad(N->ch[0]), cpad(N->ch[1]), cpad(N->ch[2]), cpad(N->ch[3]), cpad(N->ch[4])};
    RCHK(wsnet_forward(N, x, B, N->y, st));
    warm_mse(N->y, t, static_cast<long long>(B) * G * G, N->lpart, kMseBlocks, N->gy, N->loss, st);
    // Every gradient is written already multiplied by the ReLU mask of the
    // tensor it belongs to, into dz, which the next layer's weight gradient
    // and input gradient then read.
    // head (no ReLU): gradient of d0
    int nblk[kLayers], npar[kLayers];
    nblk[9] = warm_wgrad(N->d[0], N->gy, N->part[9], B, G, G, C[0], 16, false, true, st);
    warm_conv(N->gy, N->wb[9], N->dz, N->d[0], B, G, G, 16, C[0], false, false, false, 0, true, st);
    // decoder, level 0 up to 3
    const int din[4] = {C[0], C[1], C[2], C[3]};
    const int dout[4] = {C[0], C[0], C[1], C[2]};
    for (int l = 0; l <= 3; ++l) {
        const int S = N->side(l), L = 5 + (3 - l);
        nblk[L] = warm_wgrad(N->s[l], N->dz, N->part[L], B, S, S, din[l], dout[l], false, false, st);
        warm_conv(N->dz, N->wb[L], N->gs[l], nullptr, B, S, S, dout[l], din[l], false, false, false, 0,
                  false, st);
        const void *below = l < 3 ? N->d[l + 1] : N->e[4];   // the tensor one level down
        warm_up_bwd(N->gs[l], below, N->dz, B, S, S, din[l], st);
    }
    // encoder, level 4 down to 1; the skip gradient of s_{l-1} joins e_{l-1}
    for (int l = 4; l >= 1; --l) {
        const int S = N->side(l);
        nblk[l] = warm_wgrad(N->p[l], N->dz, N->part[l], B, S, S, C[l - 1], C[l], false, false, st);
        warm_conv(N->dz, N->wb[l], N->gp[l], nullptr, B, S, S, C[l], C[l - 1], false, false, false, 0,
                  false, st);
        warm_pool_bwd(N->gp[l], N->gs[l - 1], N->e[l - 1], N->dz, B, 2 * S, 2 * S, C[l - 1], st);
    }
    nblk[0] = warm_wgrad(x, N->dz, N->part[0], B, G, G, 16, C[0], true, false, st);
    // every layer's partials added in a fixed order: two launches
    for (int L = 0; L < kLayers; ++L) npar[L] = 9 * N->cip(L) * N->cop(L);
    warm_sum_layers(kLayers, N->part, nblk, npar, N->psum, N->g, st);
    return hipGetLastError() == hipSuccess ? RAS_OK : RAS_EHIP;
}

int wsnet_adam(ras_pml_wsnet *N, float lr, hipStream_t st) {
    constexpr float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    N->step += 1;
    const float c1 = static_cast<float>(1.0 - std::pow(0.9, static_cast<double>(N->step)));
    const float c2 = static_cast<float>(1.0 - std::pow(0.999, static_cast<double>(N->step)));
    // every layer's Adam step and the packing of its updated weights: one launch
    int cip[kLayers], cop[kLayers];
    for (int L = 0; L < kLayers; ++L) {
        cip[L] = N->cip(L);
        cop[L] = N->cop(L);
    }
    warm_adam_pack(kLayers, N->w, N->m, N->v, N->g, N->wf, N->wb, N->cin, N->cout, cip, cop, lr, b1, b2,
                   c1, c2, eps, st);
    return hipGetLastError() == hipSuccess ? RAS_OK : RAS_EHIP;
}

int wsnet_grid(const ras_pml_wsnet *N) { return N->grid; }
float *wsnet_stage(ras_pml_wsnet *N) { return N->stage; }
float *wsnet_out(ras_pml_wsnet *N) { return N->y; }

}  // namespace raspml

namespace {

int set_error(ras_pml_wsnet *N, const char *msg, int rc) {
    if (N) N->err = msg;
    return rc;
}

int check_batch(ras_pml_wsnet *N, const void *x, int B) {
    if (!x || B < 1 || B > N->bmax) return set_error(N, "invalid input or batch size", RAS_EINVAL);
    return RAS_OK;
}

}  // namespace

extern "C" {

int ras_pml_wsnet_create(int grid, const int channels[5], int batch_max, ras_pml_wsnet_t *out) {
    if (!out) return RAS_EINVAL;
    *out = nullptr;
    if (!channels || grid < 16 || grid % 16 != 0 || grid > 8192 || batch_max < 1) return RAS_EINVAL;
    for (int l = 0; l < 5; ++l)
        if (channels[l] < 1 || channels[l] > 64) return RAS_EINVAL;
    if (channels[3] != channels[4]) return RAS_EINVAL;
    if (static_cast<long long>(batch_max) * grid * grid >= (1LL << 31) / 64) return RAS_EINVAL;
    std::unique_ptr<ras_pml_wsnet> N(new (std::nothrow) ras_pml_wsnet());
    if (!N) return RAS_ENOMEM;
    N->grid = grid;
    N->bmax = batch_max;
    for (int l = 0; l < 5; ++l) N->ch[l] = channels[l];
    const int *c = channels;
    const int cin[kLayers] = {2, c[0], c[1], c[2], c[3], c[4], c[2], c[1], c[0], c[0]};
    const int cout[kLayers] = {c[0], c[1], c[2], c[3], c[4], c[2], c[1], c[0], c[0], 2};
    const int lvl[kLayers] = {0, 1, 2, 3, 4, 3, 2, 1, 0, 0};
    for (int L = 0; L < kLayers; ++L) {
        N->cin[L] = cin[L];
        N->cout[L] = cout[L];
        N->lvl[L] = lvl[L];
        const size_t nw = 9 * static_cast<size_t>(cin[L]) * cout[L];
        const size_t np = 9 * static_cast<size_t>(N->cip(L)) * N->cop(L);
        if (!N->alloc(&N->w[L], nw * 4) || !N->alloc(&N->m[L], nw * 4) || !N->alloc(&N->v[L], nw * 4) ||
            !N->alloc(&N->g[L], np * 4) || !N->alloc(&N->wf[L], np * 2) || !N->alloc(&N->wb[L], np * 2))
            return RAS_ENOMEM;
        // the layer's weight-gradient partial blocks for any batch up to
        // batch_max, and its slice sums
        const int S = grid >> lvl[L];
        const size_t nbmax = warm_wgrad_strip_blocks_max(batch_max, S, N->cip(L), N->cop(L));
        if (!N->alloc(&N->part[L], nbmax * np * 4) || !N->alloc(&N->psum[L], 32 * np * 4)) return RAS_ENOMEM;
    }
    auto act = [&](void **ptr, int l, int C) {
        const size_t S = static_cast<size_t>(grid >> l);
        return N->alloc(ptr, static_cast<size_t>(batch_max) * S * S * cpad(C) * 2);
    };
    bool ok = true;
    for (int l = 0; l < 5 && ok; ++l) ok = act(&N->e[l], l, c[l]);
    for (int l = 1; l < 5 && ok; ++l) ok = act(&N->p[l], l, c[l - 1]) && act(&N->gp[l], l, c[l - 1]);
    const int dch[4] = {c[0], c[0], c[1], c[2]};
    for (int l = 0; l < 4 && ok; ++l)
        ok = act(&N->s[l], l, c[l]) && act(&N->gs[l], l, c[l]) && act(&N->d[l], l, dch[l]);
    // the masked gradient: the largest of the tensors it stands for (e_l, d_l)
    size_t dz_max = 0;
    for (int l = 0; l < 5; ++l) {
        const size_t S = static_cast<size_t>(grid >> l);
        dz_max = std::max(dz_max, S * S * cpad(c[l]));
        if (l < 4) dz_max = std::max(dz_max, S * S * cpad(dch[l]));
    }
    ok = ok && N->alloc(&N->dz, static_cast<size_t>(batch_max) * dz_max * 2);
    const size_t npix = static_cast<size_t>(batch_max) * grid * grid;
    ok = ok && N->alloc(&N->y, npix * 2 * 4) && N->alloc(&N->stage, npix * 2 * 4) &&
         N->alloc(&N->gy, npix * 2 * 4) &&

         N->alloc(&N->lpart, kMseBlocks * 8) &&
         N->alloc(&N->loss, 8);
    if (!ok) return RAS_ENOMEM;
    *out = N.release();
    return RAS_OK;
}

void ras_pml_wsnet_destroy(ras_pml_wsnet_t N) { delete N; }

int ras_pml_wsnet_num_weights(ras_pml_wsnet_t N, long long *n) {
    if (!N || !n) return RAS_EINVAL;
    long long t = 0;
    for (int L = 0; L < kLayers; ++L) t += 9LL * N->cin[L] * N->cout[L];
    *n = t;
    return RAS_OK;
}

int ras_pml_wsnet_set_weights(ras_pml_wsnet_t N, const float *host, long long n) {
    long long want = 0;
    if (!N || !host || ras_pml_wsnet_num_weights(N, &want) != RAS_OK || n != want)
        return set_error(N, "weight count does not match the network", RAS_EINVAL);
    long long off = 0;
    for (int L = 0; L < kLayers; ++L) {
        const size_t nw = 9 * static_cast<size_t>(N->cin[L]) * N->cout[L];
        if (hipMemcpy(N->w[L], host + off, nw * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(N->m[L], 0, nw * 4) != hipSuccess || hipMemset(N->v[L], 0, nw * 4) != hipSuccess)
            return set_error(N, "copy to the device failed", RAS_EHIP);
        warm_pack_weights(N->w[L], N->cin[L], N->cout[L], N->cip(L), N->cop(L), N->wf[L], N->wb[L],
                          nullptr);
        off += static_cast<long long>(nw);
    }
    N->step = 0;
    return hipDeviceSynchronize() == hipSuccess ? RAS_OK : set_error(N, "packing failed", RAS_EHIP);
}

int ras_pml_wsnet_get_weights(ras_pml_wsnet_t N, float *host, long long n) {
    long long want = 0;
    if (!N || !host || ras_pml_wsnet_num_weights(N, &want) != RAS_OK || n != want)
        return set_error(N, "weight count does not match the network", RAS_EINVAL);
    if (hipDeviceSynchronize() != hipSuccess) return set_error(N, "device error", RAS_EHIP);
    long long off = 0;
    for (int L = 0; L < kLayers; ++L) {
        const size_t nw = 9 * static_cast<size_t>(N->cin[L]) * N->cout[L];
        if (hipMemcpy(host + off, N->w[L], nw * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return set_error(N, "copy from the device failed", RAS_EHIP);
        off += static_cast<long long>(nw);
    }
    return RAS_OK;
}

int ras_pml_wsnet_forward(ras_pml_wsnet_t N, const float *x, int batch, float *y, void *stream) {
    if (!N || !y) return RAS_EINVAL;
    RCHK(check_batch(N, x, batch));
    return wsnet_forward(N, x, batch, y, static_cast<hipStream_t>(stream));
}

int ras_pml_wsnet_gradient(ras_pml_wsnet_t N, const float *x, const float *target, int batch,
                           double *loss, float *grad_host, void *stream) {
    if (!N || !target) return RAS_EINVAL;
    RCHK(check_batch(N, x, batch));
    hipStream_t st = static_cast<hipStream_t>(stream);
    RCHK(wsnet_gradient(N, x, target, batch, st));
    if (loss) {
        if (hipMemcpyAsync(loss, N->loss, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return set_error(N, "reading the loss failed", RAS_EHIP);
    }
    if (grad_host) {       // real channels only, in the order of the weights
        if (hipStreamSynchronize(st) != hipSuccess) return set_error(N, "device error", RAS_EHIP);
        long long off = 0;
        std::vector<float> pad;
        for (int L = 0; L < kLayers; ++L) {
            const int ci = N->cin[L], co = N->cout[L], cip = N->cip(L), cop = N->cop(L);
            pad.resize(9 * static_cast<size_t>(cip) * cop);
            if (hipMemcpy(pad.data(), N->g[L], pad.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
                return set_error(N, "copy from the device failed", RAS_EHIP);
            for (int tap = 0; tap < 9; ++tap)
                for (int i = 0; i < ci; ++i)
                    for (int o = 0; o < co; ++o)
                        grad_host[off + (static_cast<long long>(tap) * ci + i) * co + o] =
                            pad[(static_cast<size_t>(tap) * cip + i) * cop + o];
            off += 9LL * ci * co;
        }
    }
    return RAS_OK;
}

int ras_pml_wsnet_adam(ras_pml_wsnet_t N, float lr, void *stream) {
    if (!N || !(lr > 0.f)) return RAS_EINVAL;
    return wsnet_adam(N, lr, static_cast<hipStream_t>(stream));
}

int ras_pml_wsnet_train_step(ras_pml_wsnet_t N, const float *x, const float *target, int batch,
                             float lr, double *loss, void *stream) {
    RCHK(ras_pml_wsnet_gradient(N, x, target, batch, nullptr, nullptr, stream));
    RCHK(ras_pml_wsnet_adam(N, lr, stream));
    if (loss) {
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (hipMemcpyAsync(loss, N->loss, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return set_error(N, "reading the loss failed", RAS_EHIP);
    }
    return RAS_OK;
}

const char *ras_pml_wsnet_last_error(ras_pml_wsnet_t N) { return N ? N->err.c_str() : ""; }

}  // extern "C"
