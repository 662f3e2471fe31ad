// Learned warm start: the convolutional encoder-decoder's kernels.
//
// Tensors are NHWC bfloat16 with the channel count padded to a multiple of
// 16 (padding channels hold zeros); accumulation is fp32.  Every 3 x 3
// convolution (zero padding, no bias) is an implicit GEMM on the matrix
// cores, v_mfma_f32_16x16x16_bf16:
//   forward / input gradient: rows = 16 output pixels per wave, columns =
//     output channels (NT tiles of 16), K = 9 taps x input channels; the
//     A operand is gathered straight from the input tensor (4 channels of
//     one pixel per lane, one 8-byte load), the B operand from weights
//     packed per (tap, channel block, column tile) as 16 x 16 blocks;
//     the input gradient is the same kernel on the output gradient with
//     the taps flipped and the channel roles swapped (every gradient is
//     written already multiplied by the ReLU mask of its tensor, by the
//     kernel that produces it);
//   weight gradient: rows = (tap, input channel), columns = output
//     channels, K = pixels, split over workgroups in fixed chunks; every
//     workgroup writes its partial sums and a second kernel adds them in a
//     fixed order (deterministic).
// Pooling (2 x 2 mean), nearest upsampling with the additive skip, the
// squared-error loss and Adam are plain elementwise kernels.
#include "device.h"

namespace raspml {

namespace {

typedef unsigned short bf16;
typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float(static_cast<unsigned>(h) << 16); }
__device__ __forceinline__ bf16 f2bf(float f) {          // round to nearest even
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<bf16>(u >> 16);
}
// out[p][co] (+)= sum_{tap, ci} X[p + off(tap)][ci] W[tap][ci][co].
// NT: output channel tiles.  OUT_F32: write the first `creal` channels as
// fp32 (the network's head).  gate (nullable, shaped as the output): values
// are kept only where the gate is positive (the ReLU mask of the tensor
// whose gradient this is; a post-ReLU value is positive exactly when its
// bits are non-zero).
template <int NT, bool OUT_F32>
__global__ __launch_bounds__(256) void k_conv3x3(const bf16 *__restrict__ X,
                                                 const bf16 *__restrict__ Wp, void *__restrict__ Y,
                                                 const bf16 *__restrict__ gate, int B, int H, int W,
                                                 int CPin, int relu, int acc, int creal) {
    constexpr int CPout = 16 * NT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int M = B * H * W;                // M * 64 < 2^31 (checked at creation)
    const int p0 = (blockIdx.x * 4 + wave) * 16;
    if (p0 >= M) return;                    // no barrier in this kernel
    const int i = lane & 15, kq = lane >> 4;
    const int p = p0 + i;
    const bool pin = p < M;
    const int pc = pin ? p : M - 1;
    const int x = pc % W, y = (pc / W) % H;
    // border flags of the pixel, then each tap is a uniform offset from it
    const bool xlo = x > 0, xhi = x < W - 1, ylo = y > 0, yhi = y < H - 1;
    const bf16 *xc = X + pc * CPin + 4 * kq;
    v4f c[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) c[t] = v4f{0.f, 0.f, 0.f, 0.f};
    const int KC = CPin >> 4;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const bool ok = pin && (dy < 0 ? ylo : (dy > 0 ? yhi : true)) &&
                        (dx < 0 ? xlo : (dx > 0 ? xhi : true));
        const bf16 *xr = xc + (ok ? (dy * W + dx) * CPin : 0);
        const bf16 *wb = Wp + tap * KC * NT * 256 + i * 16 + 4 * kq;
        for (int kc = 0; kc < KC; ++kc) {
            v4s a = *reinterpret_cast<const v4s *>(xr + 16 * kc);
            if (!ok) a = v4s{0, 0, 0, 0};
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const v4s bb = *reinterpret_cast<const v4s *>(wb + (kc * NT + t) * 256);
                c[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, c[t], 0, 0, 0);
            }
        }
    }
    // lane holds D[4 kq + r][i] of every tile: pixel p0 + 4 kq + r, channel 16 t + i
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int po = p0 + 4 * kq + r;
            if (po >= M) continue;
            float v = c[t][r];
            if (relu) v = fmaxf(v, 0.f);
            const int ch = 16 * t + i;
            if (OUT_F32) {
                if (ch < creal) static_cast<float *>(Y)[po * creal + ch] = v;
            } else {
                bf16 *yb = static_cast<bf16 *>(Y) + po * CPout + ch;
                if (acc) v += bf2f(*yb);
                if (gate != nullptr && gate[po * CPout + ch] == 0) v = 0.f;
                *yb = f2bf(v);
            }
        }
}

// Partial weight gradient of one pixel chunk:
//   part[blk][tap][ci][co] = sum_{p in chunk} X[p + off(tap)][ci] dZ[p][co]
// (dZ: the output gradient, already multiplied by the ReLU mask).
// Each wave owns the (tap, channel block) row tiles w, w + 4, ...: at most
// MAXT = ceil(9 KC / 4) of them (KC = input channel blocks).  The lane's four
// pixels advance by 16 per step; their coordinates are stepped, not divided.
template <int NT, int KC>
__global__ __launch_bounds__(256) void k_conv3x3_wgrad(const bf16 *__restrict__ X,
                                                       const bf16 *__restrict__ dZ,
                                                       float *__restrict__ part, int B, int H,
                                                       int W, int chunk) {
    constexpr int CPin = 16 * KC, CPout = 16 * NT;
    constexpr int ntile = 9 * KC, MAXT = (ntile + 3) / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const int M = B * H * W;
    const int c0 = blockIdx.x * chunk;
    const int c1 = min(c0 + chunk, M);
    v4f c[MAXT][NT];
#pragma unroll
    for (int s = 0; s < MAXT; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t) c[s][t] = v4f{0.f, 0.f, 0.f, 0.f};
    int px[4], py[4], pb[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int q = min(c0 + 4 * kq + e, M - 1);
        px[e] = q % W;
        py[e] = (q / W) % H;
        pb[e] = q / (W * H);
    }
    for (int p = c0; p < c1; p += 16) {
        bool pv[4];
        int q[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            pv[e] = p + 4 * kq + e < c1;
            q[e] = (pb[e] * H + py[e]) * W + px[e];
        }
        v4s bz[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const short v = static_cast<short>(dZ[static_cast<long long>(pv[e] ? q[e] : 0) * CPout + 16 * t + i]);
                bz[t][e] = pv[e] ? v : short(0);
            }
#pragma unroll
        for (int s = 0; s < MAXT; ++s) {
            const int T = wave + 4 * s;
            if (T >= ntile) continue;
            const int tap = T / KC, kc = T % KC;
            const int dy = tap / 3 - 1, dx = tap % 3 - 1;
            v4s a;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int yy = py[e] + dy, xx = px[e] + dx;
                const bool ok = pv[e] && yy >= 0 && yy < H && xx >= 0 && xx < W;
                const int qq = ok ? q[e] + dy * W + dx : 0;
                const short v = static_cast<short>(X[static_cast<long long>(qq) * CPin + 16 * kc + i]);
                a[e] = ok ? v : short(0);
            }
#pragma unroll
            for (int t = 0; t < NT; ++t)
                c[s][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bz[t], c[s][t], 0, 0, 0);
        }
        // advance the four pixels by 16
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            px[e] += 16;
            while (px[e] >= W) {
                px[e] -= W;
                if (++py[e] == H) {
                    py[e] = 0;
                    ++pb[e];
                }
            }
        }
    }
    float *pw = part + static_cast<long long>(blockIdx.x) * 9 * CPin * CPout;
#pragma unroll
    for (int s = 0; s < MAXT; ++s) {
        const int T = wave + 4 * s;
        if (T >= ntile) continue;
        const int tap = T / KC, kc = T % KC;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ci = 16 * kc + 4 * kq + r, co = 16 * t + i;
                pw[(tap * CPin + ci) * CPout + co] = c[s][t][r];
            }
    }
}

// The weight gradient for 16 input channels and W divisible by 4: a lane's
// four pixels then lie in one image row, so for each kernel row the six
// input values x-1 .. x+4 serve the three horizontal taps (6 loads instead
// of 12), and each wave takes all nine taps for its own pixels (no output
// gradient is loaded twice).  Every wave writes its own partial sums:
//   part[4 blk + wave][tap][ci][co].
template <int NT>
__global__ __launch_bounds__(256) void k_conv3x3_wgrad_k16(const bf16 *__restrict__ X,
                                                           const bf16 *__restrict__ dZ,
                                                           float *__restrict__ part, int B, int H,
                                                           int W, int chunk) {
    constexpr int CPin = 16, CPout = 16 * NT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const int M = B * H * W;                   // a multiple of 4, as is every chunk bound
    const int c0 = blockIdx.x * chunk;
    const int c1 = min(c0 + chunk, M);
    v4f c[9][NT];
#pragma unroll
    for (int s = 0; s < 9; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t) c[s][t] = v4f{0.f, 0.f, 0.f, 0.f};
    int p = c0 + 16 * wave + 4 * kq;           // first of the lane's four pixels
    const int q0 = min(p, M - 4);
    int x = q0 % W, y = (q0 / W) % H, b = q0 / (W * H);
    for (; p - 4 * kq < c1; p += 64) {
        const bool pv = p < c1;                // then p + 3 < c1 too
        v4s bz[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e)
            {
                const short z = static_cast<short>(dZ[static_cast<long long>(pv ? p + e : 0) * CPout + 16 * t + i]);
                bz[t][e] = pv ? z : short(0);
            }
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = y + dy;
            const bool rok = pv && yy >= 0 && yy < H;
            const int row = (b * H + (rok ? yy : 0)) * W;
            short v[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const int xx = x - 1 + k;
                const bool ok = rok && xx >= 0 && xx < W;
                const short u = static_cast<short>(X[static_cast<long long>(ok ? row + xx : 0) * CPin + i]);
                v[k] = ok ? u : short(0);
            }
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const v4s a = v4s{v[dx], v[dx + 1], v[dx + 2], v[dx + 3]};
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    c[3 * (dy + 1) + dx][t] =
                        __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bz[t], c[3 * (dy + 1) + dx][t], 0, 0, 0);
            }
        }
        x += 64;                               // next step: 64 pixels on
        while (x >= W) {
            x -= W;
            if (++y == H) {
                y = 0;
                ++b;
            }
        }
    }
    float *pw = part + (static_cast<long long>(blockIdx.x) * 4 + wave) * 9 * CPin * CPout;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                pw[(tap * CPin + 4 * kq + r) * CPout + 16 * t + i] = c[tap][t][r];
}

// g[idx] = sum over blocks of part[blk][idx]: 32 slices of the blocks are
// summed in order by 32 threads, then the slice sums in slice order
// (the same order at every launch: deterministic).
__global__ __launch_bounds__(256) void k_sum_partials(const float *__restrict__ part, int nblk,
                                                      int n, float *__restrict__ g) {
    __shared__ float red[8][33];
    const int sl = threadIdx.x & 31, o = threadIdx.x >> 5;     // slice, output in block
    const int idx = blockIdx.x * 8 + o;
    float s = 0.f;
    if (idx < n)
        for (int k = sl; k < nblk; k += 32) s += part[static_cast<long long>(k) * n + idx];
    red[o][sl] = s;
    __syncthreads();
    if (sl == 0 && idx < n) {
        float t = 0.f;
        for (int j = 0; j < 32; ++j) t += red[o][j];
        g[idx] = t;
    }
}

// 2 x 2 mean: Y (B, H/2, W/2, C) from X (B, H, W, C).
__global__ void k_pool2(const bf16 *__restrict__ X, bf16 *__restrict__ Y, int B, int H, int W,
                        int C) {
    const long long n = static_cast<long long>(B) * (H / 2) * (W / 2) * C;
    const long long o = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const int c = static_cast<int>(o % C);
    const long long pix = o / C;
    const int x = static_cast<int>(pix % (W / 2)), y = static_cast<int>((pix / (W / 2)) % (H / 2));
    const long long b = pix / (static_cast<long long>(W / 2) * (H / 2));
    const long long base = ((b * H + 2 * y) * W + 2 * x) * C + c;
    const float s = bf2f(X[base]) + bf2f(X[base + C]) + bf2f(X[base + static_cast<long long>(W) * C]) +
                    bf2f(X[base + static_cast<long long>(W) * C + C]);
    Y[o] = f2bf(0.25f * s);
}

// dX (B, H, W, C) = dY (B, H/2, W/2, C) / 4 spread over each block, plus
// `add`, kept where `gate` (nullable) is positive.
__global__ void k_pool2_bwd(const bf16 *__restrict__ dY, const bf16 *__restrict__ add,
                            const bf16 *__restrict__ gate, bf16 *__restrict__ dX, int B, int H,
                            int W, int C) {
    const long long n = static_cast<long long>(B) * H * W * C;
    const long long o = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const int c = static_cast<int>(o % C);
    const long long pix = o / C;
    const int x = static_cast<int>(pix % W), y = static_cast<int>((pix / W) % H);
    const long long b = pix / (static_cast<long long>(W) * H);
    float v = 0.25f * bf2f(dY[((b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c]);
    if (add != nullptr) v += bf2f(add[o]);
    if (gate != nullptr && gate[o] == 0) v = 0.f;
    dX[o] = f2bf(v);
}

// S (B, H, W, C) = nearest upsampling of Yc (B, H/2, W/2, C) + E.
__global__ void k_up2_add(const bf16 *__restrict__ Yc, const bf16 *__restrict__ E,
                          bf16 *__restrict__ S, int B, int H, int W, int C) {
    const long long n = static_cast<long long>(B) * H * W * C;
    const long long o = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const int c = static_cast<int>(o % C);
    const long long pix = o / C;
    const int x = static_cast<int>(pix % W), y = static_cast<int>((pix / W) % H);
    const long long b = pix / (static_cast<long long>(W) * H);
    const float v = bf2f(Yc[((b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c]) + bf2f(E[o]);
    S[o] = f2bf(v);
}

// dYc (B, H/2, W/2, C) = sum of dS over each 2 x 2 block, kept where `gate`
// (nullable, shaped as dYc) is positive.
__global__ void k_up2_bwd(const bf16 *__restrict__ dS, const bf16 *__restrict__ gate,
                          bf16 *__restrict__ dYc, int B, int H, int W, int C) {
    const long long n = static_cast<long long>(B) * (H / 2) * (W / 2) * C;
    const long long o = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const int c = static_cast<int>(o % C);
    const long long pix = o / C;
    const int x = static_cast<int>(pix % (W / 2)), y = static_cast<int>((pix / (W / 2)) % (H / 2));
    const long long b = pix / (static_cast<long long>(W / 2) * (H / 2));
    const long long base = ((b * H + 2 * y) * W + 2 * x) * C + c;
    float s = bf2f(dS[base]) + bf2f(dS[base + C]) + bf2f(dS[base + static_cast<long long>(W) * C]) +
              bf2f(dS[base + static_cast<long long>(W) * C + C]);
    if (gate != nullptr && gate[o] == 0) s = 0.f;
    dYc[o] = f2bf(s);
}

// Two-channel fp32 grid (B, G, G, 2) -> bf16 input with 16 channels.
__global__ void k_pack_input(const float *__restrict__ x, bf16 *__restrict__ X, long long npix) {
    const long long o = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= npix * 16) return;
    const long long p = o >> 4;
    const int c = static_cast<int>(o & 15);
    X[o] = c < 2 ? f2bf(x[2 * p + c]) : bf16(0);
}

// Squared error: per-block partial sums (double) and the gradient of the
// mean, 2 (y - t) / n, into the 16-channel bf16 tensor dY (channels >= 2
// stay zero).
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ y,
                                             const float *__restrict__ t, long long npix,
                                             double *__restrict__ partial,
                                             bf16 *__restrict__ dY, float scale) {
    __shared__ double red[256];
    double s = 0.0;
    for (long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; p < npix;
         p += static_cast<long long>(gridDim.x) * blockDim.x) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const float d = y[2 * p + c] - t[2 * p + c];
            s += static_cast<double>(d) * d;
            dY[16 * p + c] = f2bf(scale * d);
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_sum_double(const double *__restrict__ partial, int n, double scale,
                             double *__restrict__ out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += partial[k];
    *out = s * scale;
}

// Adam on the fp32 master weights W[tap][ci][co] (real channel counts) with
// the gradient in the padded layout g[tap][cip][cop].
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int cin, int cout, int cip, int cop, float lr,
                       float b1, float b2, float c1, float c2, float eps) {
    const int n = 9 * cin * cout;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int co = idx % cout, ci = (idx / cout) % cin, tap = idx / (cout * cin);
    const float gr = g[(tap * cip + ci) * cop + co];
    const float mm = b1 * m[idx] + (1.f - b1) * gr;
    const float vv = b2 * v[idx] + (1.f - b2) * gr * gr;
    m[idx] = mm;
    v[idx] = vv;
    w[idx] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// Packs the master weights into the two B-operand layouts:
//   forward:  block (tap, kc, t) = 16 x 16 with [j][k] = W[tap][16 kc + k][16 t + j];
//   input gradient: taps flipped and channel roles swapped,
//             [j][k] = W[8 - tap][16 t + j][16 kc + k].
__global__ void k_pack_weights(const float *__restrict__ w, int cin, int cout, int cip, int cop,
                               bf16 *__restrict__ fwd, bf16 *__restrict__ bwd) {
    const int n = 9 * cip * cop;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int k = idx & 15, j = (idx >> 4) & 15, blk = idx >> 8;
    {   // forward: blocks ordered (tap, kc in cip/16, t in cop/16)
        const int NT = cop >> 4, KC = cip >> 4;
        const int t = blk % NT, kc = (blk / NT) % KC, tap = blk / (NT * KC);
        const int ci = 16 * kc + k, co = 16 * t + j;
        fwd[idx] = (ci < cin && co < cout) ? f2bf(w[(tap * cin + ci) * cout + co]) : bf16(0);
    }
    {   // input gradient: input channels are the forward outputs
        const int NT = cip >> 4, KC = cop >> 4;
        const int t = blk % NT, kc = (blk / NT) % KC, tap = blk / (NT * KC);
        const int o = 16 * kc + k, ci = 16 * t + j;
        bwd[idx] = (ci < cin && o < cout) ? f2bf(w[((8 - tap) * cin + ci) * cout + o]) : bf16(0);
    }
}

// Grid of the interior box <-> unknowns of one problem: grid point (gx, gy)
// is node (G + gx, G + gy); out[(gy * grid + gx) * 2 + c] = scale * part c.
__global__ void k_grid_sample(const double2 *__restrict__ vec, int n1, int G, int grid,
                              double scale, float *__restrict__ out) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= grid * grid) return;
    const int gx = o % grid, gy = o / grid;
    const double2 z = vec[static_cast<long long>(G + gy - 1) * n1 + (G + gx - 1)];
    out[2 * o] = static_cast<float>(scale * z.x);
    out[2 * o + 1] = static_cast<float>(scale * z.y);
}

// vec (all unknowns, zero outside the grid) = scale * grid values.
__global__ void k_grid_scatter(const float *__restrict__ in, int n1, int G, int grid, double scale,
                               double2 *__restrict__ vec, long long ndof) {
    const long long o = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= ndof) return;
    const int i = static_cast<int>(o % n1) + 1, j = static_cast<int>(o / n1) + 1;
    const int gx = i - G, gy = j - G;
    double2 z = make_double2(0.0, 0.0);
    if (gx >= 0 && gx < grid && gy >= 0 && gy < grid) {
        const long long q = static_cast<long long>(gy) * grid + gx;
        z = make_double2(scale * in[2 * q], scale * in[2 * q + 1]);
    }
    vec[o] = z;
}

unsigned blocks(long long n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

}  // namespace

// ---------------------------------------------------------------- launchers
// B * H * W < 2^31 (the network object checks it at creation).
void warm_conv(const void *X, const void *Wp, void *Y, const void *gate, int B, int H, int W,
               int CPin, int CPout, bool relu, bool acc, bool out_f32, int creal, hipStream_t s) {
    const long long M = static_cast<long long>(B) * H * W;
    const dim3 grid(blocks(M, 64)), blk(256);
    const bf16 *x = static_cast<const bf16 *>(X), *w = static_cast<const bf16 *>(Wp),
               *g = static_cast<const bf16 *>(gate);
#define RAS_CONV(NT, F32)                                                                        \
    hipLaunchKernelGGL((k_conv3x3<NT, F32>), grid, blk, 0, s, x, w, Y, g, B, H, W, CPin,        \
                       relu ? 1 : 0, acc ? 1 : 0, creal)
    if (out_f32) {
        RAS_CONV(1, true);
    } else if (CPout == 16) {
        RAS_CONV(1, false);
    } else if (CPout == 32) {
        RAS_CONV(2, false);
    } else {
        RAS_CONV(4, false);
    }
#undef RAS_CONV
}

int warm_wgrad_blocks(long long M, int *chunk) {
    long long c = (M + 1023) / 1024;
    c = (c + 15) / 16 * 16;
    if (c < 256) c = 256;
    *chunk = static_cast<int>(c);
    return static_cast<int>((M + c - 1) / c);
}

void warm_wgrad(const void *X, const void *dZ, float *part, float *g, int B, int H, int W,
                int CPin, int CPout, hipStream_t s) {
    const long long M = static_cast<long long>(B) * H * W;
    int chunk = 0;
    const int nblk = warm_wgrad_blocks(M, &chunk);
    const bf16 *x = static_cast<const bf16 *>(X), *dz = static_cast<const bf16 *>(dZ);
    const int n = 9 * CPin * CPout;
    if (CPin == 16 && CPout <= 32 && W % 4 == 0) {     // per-wave partials: 4 per block
        if (CPout == 16)
            hipLaunchKernelGGL(k_conv3x3_wgrad_k16<1>, dim3(nblk), dim3(256), 0, s, x, dz, part, B, H,
                               W, chunk);
        else
            hipLaunchKernelGGL(k_conv3x3_wgrad_k16<2>, dim3(nblk), dim3(256), 0, s, x, dz, part, B, H,
                               W, chunk);
        hipLaunchKernelGGL(k_sum_partials, dim3(blocks(n, 8)), dim3(256), 0, s, part, 4 * nblk, n, g);
        return;
    }
#define RAS_WG(NT, KC)                                                                           \
    hipLaunchKernelGGL((k_conv3x3_wgrad<NT, KC>), dim3(nblk), dim3(256), 0, s, x, dz, part, B, H, \
                       W, chunk)
#define RAS_WG_KC(NT)                                                                            \
    do {                                                                                         \
        if (CPin == 16) RAS_WG(NT, 1);                                                           \
        else if (CPin == 32) RAS_WG(NT, 2);                                                      \
        else RAS_WG(NT, 4);                                                                      \
    } while (0)
    if (CPout == 16)
        RAS_WG_KC(1);
    else if (CPout == 32)
        RAS_WG_KC(2);
    else
        RAS_WG_KC(4);
#undef RAS_WG_KC
#undef RAS_WG
    hipLaunchKernelGGL(k_sum_partials, dim3(blocks(n, 8)), dim3(256), 0, s, part, nblk, n, g);
}


void warm_pool(const void *X, void *Y, int B, int H, int W, int C, hipStream_t s) {
    const long long n = static_cast<long long>(B) * (H / 2) * (W / 2) * C;
    hipLaunchKernelGGL(k_pool2, dim3(blocks(n, 256)), dim3(256), 0, s, static_cast<const bf16 *>(X),
                       static_cast<bf16 *>(Y), B, H, W, C);
}
void warm_pool_bwd(const void *dY, const void *add, const void *gate, void *dX, int B, int H,
                   int W, int C, hipStream_t s) {
    const long long n = static_cast<long long>(B) * H * W * C;
    hipLaunchKernelGGL(k_pool2_bwd, dim3(blocks(n, 256)), dim3(256), 0, s,
                       static_cast<const bf16 *>(dY), static_cast<const bf16 *>(add),
                       static_cast<const bf16 *>(gate), static_cast<bf16 *>(dX), B, H, W, C);
}
void warm_up_add(const void *Yc, const void *E, void *S, int B, int H, int W, int C, hipStream_t s) {
    const long long n = static_cast<long long>(B) * H * W * C;
    hipLaunchKernelGGL(k_up2_add, dim3(blocks(n, 256)), dim3(256), 0, s, static_cast<const bf16 *>(Yc),
                       static_cast<const bf16 *>(E), static_cast<bf16 *>(S), B, H, W, C);
}
void warm_up_bwd(const void *dS, const void *gate, void *dYc, int B, int H, int W, int C,
                 hipStream_t s) {
    const long long n = static_cast<long long>(B) * (H / 2) * (W / 2) * C;
    hipLaunchKernelGGL(k_up2_bwd, dim3(blocks(n, 256)), dim3(256), 0, s, static_cast<const bf16 *>(dS),
                       static_cast<const bf16 *>(gate), static_cast<bf16 *>(dYc), B, H, W, C);
}
void warm_pack_input(const float *x, void *X, long long npix, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_input, dim3(blocks(npix * 16, 256)), dim3(256), 0, s, x,
                       static_cast<bf16 *>(X), npix);
}
void warm_mse(const float *y, const float *t, long long npix, double *partial, int nblk, void *dY,
              double *loss, hipStream_t s) {
    const float scale = static_cast<float>(2.0 / (2.0 * npix));
    hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, s, y, t, npix, partial,
                       static_cast<bf16 *>(dY), scale);
    hipLaunchKernelGGL(k_sum_double, dim3(1), dim3(64), 0, s, partial, nblk, 1.0 / (2.0 * npix),
                       loss);
}
void warm_adam(float *w, float *m, float *v, const float *g, int cin, int cout, int cip, int cop,
               float lr, float b1, float b2, float c1, float c2, float eps, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(blocks(9 * cin * cout, 256)), dim3(256), 0, s, w, m, v, g, cin,
                       cout, cip, cop, lr, b1, b2, c1, c2, eps);
}
void warm_pack_weights(const float *w, int cin, int cout, int cip, int cop, void *fwd, void *bwd,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_pack_weights, dim3(blocks(9 * cip * cop, 256)), dim3(256), 0, s, w, cin,
                       cout, cip, cop, static_cast<bf16 *>(fwd), static_cast<bf16 *>(bwd));
}
void warm_grid_sample(const double2 *vec, int n1, int G, int grid, double scale, float *out,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_grid_sample, dim3(blocks(static_cast<long long>(grid) * grid, 256)),
                       dim3(256), 0, s, vec, n1, G, grid, scale, out);
}
void warm_grid_scatter(const float *in, int n1, int G, int grid, double scale, double2 *vec,
                       long long ndof, hipStream_t s) {
    hipLaunchKernelGGL(k_grid_scatter, dim3(blocks(ndof, 256)), dim3(256), 0, s, in, n1, G, grid,
                       scale, vec, ndof);
}

}  // namespace raspml
