// Learned warm start: the convolutional encoder-decoder's kernels.
//
// Tensors are NHWC bfloat16 with the channel count padded to 16, 32 or 64
// (padding channels hold zeros), except the network's two-channel ends (its
// input, its output and the loss gradient), which are fp32 pairs;
// accumulation is fp32.  Every 3 x 3
// convolution (zero padding, no bias) is an implicit GEMM on the matrix
// cores, v_mfma_f32_16x16x16_bf16:
//   forward / input gradient: rows = output channels (NT tiles of 16),
//     columns = 16 output pixels, K = 9 taps x input channels; the weights
//     are packed per (tap, channel block, column tile) as 16 x 16 blocks,
//     the input is staged in LDS per tile of 4 x 64 pixels;
//     the input gradient is the same kernel on the output gradient with
//     the taps flipped and the channel roles swapped (every gradient is
//     written already multiplied by the ReLU mask of its tensor, by the
//     kernel that produces it);
//   weight gradient: rows = (tap, input channel), columns = output
//     channels, K = pixels, split over waves by 64-column strips and row
//     chunks; every workgroup writes its partial sums and two more kernels
//     add them in a fixed order (deterministic).
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
// Block i runs on XCD i mod 8 (the dispatcher deals blocks out round
// robin); the tile it takes: XCD x gets the x-th contiguous run of the n
// tiles, in order, so that a tile row and the next one (which share two
// input rows) are staged through the same L2.  A bijection of 0 .. n - 1.
__device__ __forceinline__ int xcd_run(int i, int n) {
    const int x = i & 7, l = i >> 3, q = n >> 3, r = n & 7;
    return x * q + min(x, r) + l;
}

// out[p][co] (+)= sum_{tap, ci} X[p + off(tap)][ci] W[tap][ci][co].
// A block computes a tile of 4 rows x 64 pixels (wave w: row w, four tiles
// of 16 pixels; rows past the image's edge are skipped, pixels past it are
// computed on the staged zeros and not written) and first loads the 6 x 66
// input pixels that tile reads (zeros outside the image) into LDS with
// 16-byte loads, channels of a pixel contiguous.  The matrix-core product is
// D[co][p] = W^T X^T: A is the weight block (lane: output channel
// lane & 15, input channels 4 (lane >> 4) .. + 3), B the input (lane: pixel
// lane & 15, the same four input channels, one 8-byte LDS read), so a tap's
// weights serve the wave's 64 pixels and each lane ends with four
// consecutive output channels of one pixel, written with one 8-byte store.
// With 32 or 64 input channels the LDS pixel pitch is padded by eight
// channels: a wave's read of 16 pixels x 16 channels then spreads over all
// LDS banks (unpadded, 64 channels put all of it on 8 of the 32 banks).
// NT: output channel tiles of the block (tiles NT blockIdx.y .. of the
// ntot), KC: input channel blocks.  IN2: the input is two fp32 channels per
// pixel (the network's input, or the loss gradient at its head), rounded to
// bf16 as it is staged, channels 2 .. 15 zero (KC = 1).  OUT_F32: write the
// first `creal` (<= 4) channels as fp32 (the network's head).  gate
// (nullable, shaped as the output): values are kept only where the gate is
// positive (the ReLU mask of the tensor whose gradient this is; a post-ReLU
// value is positive exactly when its bits are non-zero).
template <int NT, int KC, bool OUT_F32, bool IN2 = false>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(NT == 4 ? 1 : KC == 1 ? (NT == 1 ? 8 : 6) : KC == 2 ? 5 : 2))) void
k_conv3x3_tile(const bf16 *__restrict__ X, const bf16 *__restrict__ Wp, void *__restrict__ Y,
               const bf16 *__restrict__ gate, int B, int H, int W, int relu, int acc, int creal, int ntot) {
    constexpr int CPin = 16 * KC;
    constexpr int PP = KC == 1 ? CPin : CPin + 8;          // LDS pixel pitch
    const int CPout = 16 * ntot, t0 = blockIdx.y * NT;     // this block's column tiles
    constexpr int TW = 64, TH = 4, SW = TW + 2, SH = TH + 2;
    __shared__ __align__(16) bf16 S[SH * SW * PP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const int tx = (W + TW - 1) / TW, ty = (H + TH - 1) / TH;
    int blk = xcd_run(blockIdx.x, gridDim.x);
    const int bx = blk % tx;
    blk /= tx;
    const int by = blk % ty;
    const int b = blk / ty;
    const int x0 = bx * TW, y0 = by * TH;
    // with at most two (channel block, column tile) pairs the wave's weights
    // (9 KC NT operands) are loaded before the input tile, so that their
    // latency overlaps the staging instead of the multiplies
    constexpr bool PRE = KC * NT <= 2;
    v4s wpre[PRE ? 9 * KC * NT : 1];
    if constexpr (PRE) {
#pragma unroll
        for (int q = 0; q < 9 * KC; ++q)
#pragma unroll
            for (int t = 0; t < NT; ++t)
                wpre[q * NT + t] = *reinterpret_cast<const v4s *>(Wp + (q * ntot + t0 + t) * 256 + i * 16 + 4 * kq);
    }
    if constexpr (IN2) {   // two fp32 channels per pixel, one 8-byte load each
        static_assert(KC == 1, "two-channel input: one channel block");
        constexpr int items = SH * SW, NIT = (items + 255) / 256;
        const float *Xf = reinterpret_cast<const float *>(X);
        float2 v[NIT];
#pragma unroll
        for (int k = 0; k < NIT; ++k) {
            const int pix = tid + 256 * k;
            const int sx = pix % SW, sy = pix / SW;
            const int gx = x0 + sx - 1, gy = y0 + sy - 1;
            const bool ok = pix < items && gx >= 0 && gx < W && gy >= 0 && gy < H;
            const long long off = ok ? ((static_cast<long long>(b) * H + gy) * W + gx) * 2 : 0;
            unsigned m = ok ? 0xFFFFFFFFu : 0u;
            asm volatile("" : "+v"(m));
            const float2 t = *reinterpret_cast<const float2 *>(Xf + off);
            v[k] = float2{__uint_as_float(__float_as_uint(t.x) & m), __uint_as_float(__float_as_uint(t.y) & m)};
        }
#pragma unroll
        for (int k = 0; k < NIT; ++k) {
            const int pix = tid + 256 * k;
            if (pix < items) {
                const unsigned u = static_cast<unsigned>(f2bf(v[k].x)) | (static_cast<unsigned>(f2bf(v[k].y)) << 16);
                *reinterpret_cast<uint4 *>(S + pix * PP) = uint4{u, 0u, 0u, 0u};
                *reinterpret_cast<uint4 *>(S + pix * PP + 8) = uint4{0u, 0u, 0u, 0u};
            }
        }
    } else {   // stage the input tile: pixel (sy, sx) of the tile is input pixel
        // (y0 + sy - 1, x0 + sx - 1); every load of the thread is issued
        // before the first LDS write, so that their latencies overlap
        constexpr int C8 = CPin / 8, items = SH * SW * C8, NIT = (items + 255) / 256;
        uint4 v[NIT];
#pragma unroll
        for (int k = 0; k < NIT; ++k) {
            const int it = tid + 256 * k;
            const int c = (it % C8) * 8, pix = it / C8;
            const int sx = pix % SW, sy = pix / SW;
            const int gx = x0 + sx - 1, gy = y0 + sy - 1;
            // branch-free: outside the image the load reads element 0 and
            // the value is masked to zeros (the mask is opaque to the
            // compiler, which would otherwise move the load into a branch)
            const bool ok = it < items && gx >= 0 && gx < W && gy >= 0 && gy < H;
            const long long off = ok ? ((static_cast<long long>(b) * H + gy) * W + gx) * CPin + c : 0;
            unsigned m = ok ? 0xFFFFFFFFu : 0u;
            asm volatile("" : "+v"(m));
            const uint4 t = *reinterpret_cast<const uint4 *>(X + off);
            v[k] = uint4{t.x & m, t.y & m, t.z & m, t.w & m};
        }
#pragma unroll
        for (int k = 0; k < NIT; ++k) {
            const int it = tid + 256 * k;
            if (it < items) *reinterpret_cast<uint4 *>(S + (it / C8) * PP + (it % C8) * 8) = v[k];
        }
    }
    __syncthreads();
    const int y = y0 + wave;
    if (y >= H) return;
    v4f c[4][NT];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < NT; ++t) c[u][t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const bf16 *wb = Wp + (tap * KC * ntot + t0) * 256 + i * 16 + 4 * kq;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            v4s wt[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if constexpr (PRE)
                    wt[t] = wpre[(tap * KC + kc) * NT + t];
                else
                    wt[t] = *reinterpret_cast<const v4s *>(wb + (kc * ntot + t) * 256);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {        // pixels past the edge are zeros: no branch
                const int sp = (wave + dy + 1) * SW + 16 * u + i + dx + 1;
                const v4s a = *reinterpret_cast<const v4s *>(S + sp * PP + 16 * kc + 4 * kq);
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    c[u][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wt[t], a, c[u][t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (x0 + 16 * u + i >= W) continue;
        const long long po = (static_cast<long long>(b) * H + y) * W + x0 + 16 * u + i;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = relu ? fmaxf(c[u][t][r], 0.f) : c[u][t][r];
            const int ch = 16 * (t0 + t) + 4 * kq;
            if (OUT_F32) {
                float *yf = static_cast<float *>(Y) + po * creal;
                if (t == 0 && kq == 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (r < creal) yf[r] = v[r];
                }
            } else {
                bf16 *yb = static_cast<bf16 *>(Y) + po * CPout + ch;
                if (acc) {
                    const uint2 q = *reinterpret_cast<const uint2 *>(yb);
                    v[0] += __uint_as_float(q.x << 16);
                    v[1] += __uint_as_float(q.x & 0xFFFF0000u);
                    v[2] += __uint_as_float(q.y << 16);
                    v[3] += __uint_as_float(q.y & 0xFFFF0000u);
                }
                if (gate != nullptr) {
                    const uint2 q = *reinterpret_cast<const uint2 *>(gate + po * CPout + ch);
                    if ((q.x & 0xFFFFu) == 0) v[0] = 0.f;
                    if ((q.x >> 16) == 0) v[1] = 0.f;
                    if ((q.y & 0xFFFFu) == 0) v[2] = 0.f;
                    if ((q.y >> 16) == 0) v[3] = 0.f;
                }
                *reinterpret_cast<uint2 *>(yb) =
                    uint2{static_cast<unsigned>(f2bf(v[0])) | (static_cast<unsigned>(f2bf(v[1])) << 16),
                          static_cast<unsigned>(f2bf(v[2])) | (static_cast<unsigned>(f2bf(v[3])) << 16)};
            }
        }
    }
}

// Weight gradient, one wave per strip: part[blk][tap][ci][co] = sum over
// the block's pixels of X[y + dy][x + dx][ci] dZ[y][x][co], for the input
// channel block kc = blockIdx.y (channels 16 kc .. 16 kc + 15 of the CPin)
// and the output tiles t0 .. t0 + NT - 1, t0 = NT blockIdx.z (of CPout / 16).
// A wave takes a strip of 64 columns and rows y0 .. y1 - 1 of one image;
// its own LDS holds the input rows y - 1 .. y + 1 of the strip (its channel
// block) with the two halo columns as a ring of three rows, transposed to
// [ci][x - x0 + 1], and the output-gradient row of the strip as [co][x - x0];
// rows and columns outside the image are zero, so a strip that overhangs
// the image's right edge computes on zeros without a branch.  Each step
// writes the rows that the registers hold (input row y + 1, output gradient
// row y), issues the 16-byte loads of the next step's rows into the
// registers, and then runs the 36 NT multiplies of row y: for every group of
// 16 pixels and kernel row, one 8-byte and one 4-byte LDS read give the six
// values x - 1 .. x + 4 that serve the three horizontal taps.  No wave waits
// for another until the four waves' sums are added in LDS, in wave order, so
// that the block writes one partial (its channel block's rows of it).
// X2 / Z2: the input / the output gradient is two fp32 channels per pixel
// (the network's input; the loss gradient at its head), rounded to bf16 as
// it is staged, the other 14 channel rows of the LDS buffers zero.
template <int NT, bool X2 = false, bool Z2 = false>
__global__ __launch_bounds__(256) void k_wgrad_strip(const bf16 *__restrict__ X,
                                                     const bf16 *__restrict__ dZ,
                                                     float *__restrict__ part, int B, int H, int W,
                                                     int CPin, int CPout, int rows_per_wave, int nchunk) {
    constexpr int ZR = (32 * NT + 63) / 64;
    constexpr int XP = 68;                         // columns x0 - 1 .. x0 + 64 at 0 .. 65
    constexpr int XS = 3 * 16 * XP, ZS = 16 * NT * 64;
    constexpr int RED = 3 * 36 * 64;               // floats of the wave-sum exchange
    constexpr int LDS_EL = 4 * (XS + ZS) > 2 * RED ? 4 * (XS + ZS) : 2 * RED;
    __shared__ __align__(16) bf16 lds[LDS_EL];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    bf16 *Xs = lds + wave * (XS + ZS);
    bf16 *Zs = Xs + XS;
    const int nstrip = (W + 63) >> 6, kc = blockIdx.y, t0 = NT * blockIdx.z;
    const int item = blockIdx.x * 4 + wave;
    v4f c[9][NT];
#pragma unroll
    for (int s = 0; s < 9; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t) c[s][t] = v4f{0.f, 0.f, 0.f, 0.f};
    if (item < B * nchunk * nstrip) {
        const int x0 = (item % nstrip) << 6;
        const int chunk = (item / nstrip) % nchunk, b = item / (nstrip * nchunk);
        const int y0 = chunk * rows_per_wave, y1 = min(H, y0 + rows_per_wave);
        const bf16 *img = X + static_cast<long long>(b) * H * W * CPin + 16 * kc;
        const bf16 *zimg = dZ + static_cast<long long>(b) * H * W * CPout + 16 * t0;
        const float *imgf = reinterpret_cast<const float *>(X) + static_cast<long long>(b) * H * W * 2;
        const float *zimgf = reinterpret_cast<const float *>(dZ) + static_cast<long long>(b) * H * W * 2;
        if constexpr (X2 || Z2) {   // the channel rows that two-channel tensors leave zero
            for (int e = lane; e < (XS + ZS) / 8; e += 64)
                reinterpret_cast<uint4 *>(Xs)[e] = uint4{0u, 0u, 0u, 0u};
        }
        // input row yy: item it < 132 is column x0 - 1 + (it >> 1), channels 8 (it & 1) ..
        auto load_x = [&](int yy, uint4 (&xr)[3]) {
            const bool in = yy >= 0 && yy < H;
            if constexpr (X2) {   // item it < 66: column x0 - 1 + it, two fp32 channels
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int it = lane + 64 * r;
                    const int gx = x0 - 1 + it;
                    xr[r] = uint4{0u, 0u, 0u, 0u};
                    if (it < 66 && in && gx >= 0 && gx < W) {
                        const float2 v = *reinterpret_cast<const float2 *>(imgf + (static_cast<long long>(yy) * W + gx) * 2);
                        xr[r].x = __float_as_uint(v.x);
                        xr[r].y = __float_as_uint(v.y);
                    }
                }
                return;
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int it = lane + 64 * r;
                const int gx = x0 - 1 + (it >> 1);
                xr[r] = uint4{0u, 0u, 0u, 0u};
                if (it < 132 && in && gx >= 0 && gx < W)
                    xr[r] = *reinterpret_cast<const uint4 *>(img + (static_cast<long long>(yy) * W + gx) * CPin +
                                                             8 * (it & 1));
            }
        };
        auto store_x = [&](int yy, const uint4 (&xr)[3]) {
            bf16 *dst = Xs + ((yy + 3) % 3) * 16 * XP;
            if constexpr (X2) {
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int it = lane + 64 * r;
                    if (it < 66) {
                        dst[it] = f2bf(__uint_as_float(xr[r].x));
                        dst[XP + it] = f2bf(__uint_as_float(xr[r].y));
                    }
                }
                return;
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int it = lane + 64 * r;
                if (it < 132) {
                    const int col = it >> 1, c8 = 8 * (it & 1);
                    const unsigned u[4] = {xr[r].x, xr[r].y, xr[r].z, xr[r].w};
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        dst[(c8 + 2 * k) * XP + col] = static_cast<bf16>(u[k] & 0xFFFFu);
                        dst[(c8 + 2 * k + 1) * XP + col] = static_cast<bf16>(u[k] >> 16);
                    }
                }
            }
        };
        // output-gradient row y: item it < 32 NT is pixels x0 + 4 (it & 15) .. + 3,
        // channels 8 (it >> 4) .. (zeros past the image's edge)
        auto load_z = [&](int y, uint4 (&zr)[ZR][4]) {
            if constexpr (Z2) {   // lane: pixel x0 + lane, two fp32 channels
                const int px = x0 + lane;
                zr[0][0] = uint4{0u, 0u, 0u, 0u};
                if (px < W) {
                    const float2 v = *reinterpret_cast<const float2 *>(zimgf + (static_cast<long long>(y) * W + px) * 2);
                    zr[0][0].x = __float_as_uint(v.x);
                    zr[0][0].y = __float_as_uint(v.y);
                }
                return;
            }
#pragma unroll
            for (int r = 0; r < ZR; ++r) {
                const int it = lane + 64 * r;
                if (it < 32 * NT) {
                    const int px = x0 + 4 * (it & 15);
                    const bf16 *src = zimg + (static_cast<long long>(y) * W + px) * CPout + 8 * (it >> 4);
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        zr[r][e] = px + e < W ? *reinterpret_cast<const uint4 *>(src + e * CPout)
                                              : uint4{0u, 0u, 0u, 0u};
                }
            }
        };
        auto store_z = [&](const uint4 (&zr)[ZR][4]) {
            if constexpr (Z2) {
                Zs[lane] = f2bf(__uint_as_float(zr[0][0].x));
                Zs[64 + lane] = f2bf(__uint_as_float(zr[0][0].y));
                return;
            }
#pragma unroll
            for (int r = 0; r < ZR; ++r) {
                const int it = lane + 64 * r;
                if (it < 32 * NT) {
                    const int q = it & 15, c8 = 8 * (it >> 4);
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        unsigned h[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const unsigned w = (k >> 1) == 0 ? zr[r][e].x : (k >> 1) == 1 ? zr[r][e].y
                                             : (k >> 1) == 2 ? zr[r][e].z : zr[r][e].w;
                            h[e] = (k & 1) ? (w >> 16) : (w & 0xFFFFu);
                        }
                        *reinterpret_cast<uint2 *>(Zs + (c8 + k) * 64 + 4 * q) =
                            uint2{h[0] | (h[1] << 16), h[2] | (h[3] << 16)};
                    }
                }
            }
        };
        uint4 xr[3], zr[ZR][4];
        load_x(y0 - 1, xr);
        store_x(y0 - 1, xr);
        load_x(y0, xr);
        store_x(y0, xr);
        load_x(y0 + 1, xr);
        load_z(y0, zr);
        for (int y = y0; y < y1; ++y) {
            // the previous step's reads of the slot and of Zs are done: a
            // wave's LDS accesses complete in order
            __builtin_amdgcn_wave_barrier();
            store_x(y + 1, xr);
            store_z(zr);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (y + 1 < y1) {
                load_x(y + 2, xr);
                load_z(y + 1, zr);
            }
#pragma unroll
            for (int xg = 0; xg < 64; xg += 16) {
                v4s bz[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    bz[t] = *reinterpret_cast<const v4s *>(Zs + (16 * t + i) * 64 + xg + 4 * kq);
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) {
                    const bf16 *rowl = Xs + ((y + dy + 2) % 3) * 16 * XP + i * XP + xg + 4 * kq;
                    const unsigned long long lo = *reinterpret_cast<const unsigned long long *>(rowl);
                    const unsigned hi = *reinterpret_cast<const unsigned *>(rowl + 4);
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx) {
                        const unsigned long long w =
                            dx == 0 ? lo : (lo >> (16 * dx)) | (static_cast<unsigned long long>(hi) << (64 - 16 * dx));
                        v4s a;
                        a[0] = static_cast<short>(w & 0xFFFFu);
                        a[1] = static_cast<short>((w >> 16) & 0xFFFFu);
                        a[2] = static_cast<short>((w >> 32) & 0xFFFFu);
                        a[3] = static_cast<short>((w >> 48) & 0xFFFFu);
#pragma unroll
                        for (int t = 0; t < NT; ++t)
                            c[3 * dy + dx][t] =
                                __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bz[t], c[3 * dy + dx][t], 0, 0, 0);
                    }
                }
            }
        }
    }
    // waves 1..3 leave their sums in LDS (one output tile column t at a
    // time), wave 0 adds them in wave order and writes the block's partial
    float *red = reinterpret_cast<float *>(lds);
    float *pw = part + static_cast<long long>(blockIdx.x) * 9 * CPin * CPout;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        __syncthreads();
        if (wave > 0) {
#pragma unroll
            for (int tap = 0; tap < 9; ++tap)
#pragma unroll
                for (int r = 0; r < 4; ++r) red[((wave - 1) * 36 + tap * 4 + r) * 64 + lane] = c[tap][t][r];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int tap = 0; tap < 9; ++tap)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int q = tap * 4 + r;
                    const float w = ((c[tap][t][r] + red[q * 64 + lane]) + red[(36 + q) * 64 + lane]) +
                                    red[(72 + q) * 64 + lane];
                    pw[(tap * CPin + 16 * kc + 4 * kq + r) * CPout + 16 * (t0 + t) + i] = w;
                }
        }
    }
}

// g[idx] = sum over blocks of part[blk][idx] for every layer of a table, in
// two stages with a fixed order (deterministic): slice s of a layer's
// blocks, [s per, (s + 1) per), is summed in block order into tmp[s][idx];
// then the slices in slice order.  One thread per (layer, idx) of the flat
// list, layer L holding off[L] .. off[L + 1] - 1; consecutive threads take
// consecutive idx, so every load is coalesced.
constexpr int kSumSlices = 32;
constexpr int kSumLayers = 10;
struct SumLayers {
    const float *part[kSumLayers];
    float *tmp[kSumLayers], *g[kSumLayers];
    int n[kSumLayers], nblk[kSumLayers], per[kSumLayers];
    int off[kSumLayers + 1];
    int nl;
};
__device__ __forceinline__ int sum_layer(const SumLayers &P, int f) {
    int L = 0;
    while (f >= P.off[L + 1]) ++L;
    return L;
}
__global__ __launch_bounds__(256) void k_sum_slices(const SumLayers P) {
    const int f = blockIdx.x * 256 + threadIdx.x;
    if (f >= P.off[P.nl]) return;
    const int L = sum_layer(P, f), idx = f - P.off[L], n = P.n[L];
    const int k0 = blockIdx.y * P.per[L], k1 = min(k0 + P.per[L], P.nblk[L]);
    const float *part = P.part[L];
    // eight loads in flight, then their sum in block order
    float s = 0.f;
    int k = k0;
    for (; k + 8 <= k1; k += 8) {
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = part[static_cast<long long>(k + e) * n + idx];
#pragma unroll
        for (int e = 0; e < 8; ++e) s += v[e];
    }
    for (; k < k1; ++k) s += part[static_cast<long long>(k) * n + idx];
    P.tmp[L][static_cast<long long>(blockIdx.y) * n + idx] = s;
}
__global__ __launch_bounds__(256) void k_sum_tmp(const SumLayers P) {
    const int f = blockIdx.x * 256 + threadIdx.x;
    if (f >= P.off[P.nl]) return;
    const int L = sum_layer(P, f), idx = f - P.off[L], n = P.n[L];
    const float *tmp = P.tmp[L];
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kSumSlices; ++k) s += tmp[static_cast<long long>(k) * n + idx];
    P.g[L][idx] = s;
}

// Eight bfloat16 values (16 bytes) <-> floats, for the elementwise kernels:
// every thread moves 16 bytes per tensor (channels are a multiple of 16).
struct bf8 {
    float f[8];
};
__device__ __forceinline__ bf8 ld8(const bf16 *p) {
    const uint4 q = *reinterpret_cast<const uint4 *>(p);
    const unsigned u[4] = {q.x, q.y, q.z, q.w};
    bf8 r;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        r.f[2 * k] = __uint_as_float(u[k] << 16);
        r.f[2 * k + 1] = __uint_as_float(u[k] & 0xFFFF0000u);
    }
    return r;
}
__device__ __forceinline__ void st8(bf16 *p, const bf8 &v) {
    unsigned u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        u[k] = static_cast<unsigned>(f2bf(v.f[2 * k])) |
               (static_cast<unsigned>(f2bf(v.f[2 * k + 1])) << 16);
    *reinterpret_cast<uint4 *>(p) = uint4{u[0], u[1], u[2], u[3]};
}
// Zero the values whose gate bits are zero (a post-ReLU value is positive
// exactly when its bits are non-zero).
__device__ __forceinline__ void gate8(bf8 &v, const bf16 *g) {
    const uint4 q = *reinterpret_cast<const uint4 *>(g);
    const unsigned u[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if ((u[k] & 0xFFFFu) == 0) v.f[2 * k] = 0.f;
        if ((u[k] >> 16) == 0) v.f[2 * k + 1] = 0.f;
    }
}

// 2 x 2 mean: Y (B, H/2, W/2, C) from X (B, H, W, C); eight channels per
// thread.
__global__ void k_pool2(const bf16 *__restrict__ X, bf16 *__restrict__ Y, int B, int H, int W,
                        int C) {
    const int C8 = C >> 3;
    const long long n = static_cast<long long>(B) * (H / 2) * (W / 2) * C8;
    const long long o = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const int c = static_cast<int>(o % C8) * 8;
    const long long pix = o / C8;
    const int x = static_cast<int>(pix % (W / 2)), y = static_cast<int>((pix / (W / 2)) % (H / 2));
    const long long b = pix / (static_cast<long long>(W / 2) * (H / 2));
    const long long base = ((b * H + 2 * y) * W + 2 * x) * C + c;
    const bf8 a0 = ld8(X + base), a1 = ld8(X + base + C), a2 = ld8(X + base + static_cast<long long>(W) * C),
              a3 = ld8(X + base + static_cast<long long>(W) * C + C);
    bf8 r;
#pragma unroll
    for (int k = 0; k < 8; ++k) r.f[k] = 0.25f * (a0.f[k] + a1.f[k] + a2.f[k] + a3.f[k]);
    st8(Y + pix * C + c, r);
}

// dX (B, H, W, C) = dY (B, H/2, W/2, C) / 4 spread over each block, plus
// `add`, kept where `gate` (nullable) is positive; eight channels per thread.
__global__ void k_pool2_bwd(const bf16 *__restrict__ dY, const bf16 *__restrict__ add,
                            const bf16 *__restrict__ gate, bf16 *__restrict__ dX, int B, int H,
                            int W, int C) {
    const int C8 = C >> 3;
    const long long n = static_cast<long long>(B) * H * W * C8;
    const long long o = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const int c = static_cast<int>(o % C8) * 8;
    const long long pix = o / C8;
    const int x = static_cast<int>(pix % W), y = static_cast<int>((pix / W) % H);
    const long long b = pix / (static_cast<long long>(W) * H);
    const long long e = pix * C + c;
    bf8 v = ld8(dY + ((b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c);
#pragma unroll
    for (int k = 0; k < 8; ++k) v.f[k] *= 0.25f;
    if (add != nullptr) {
        const bf8 a = ld8(add + e);
#pragma unroll
        for (int k = 0; k < 8; ++k) v.f[k] += a.f[k];
    }
    if (gate != nullptr) gate8(v, gate + e);
    st8(dX + e, v);
}

// S (B, H, W, C) = nearest upsampling of Yc (B, H/2, W/2, C) + E; eight
// channels per thread.
__global__ void k_up2_add(const bf16 *__restrict__ Yc, const bf16 *__restrict__ E,
                          bf16 *__restrict__ S, int B, int H, int W, int C) {
    const int C8 = C >> 3;
    const long long n = static_cast<long long>(B) * H * W * C8;
    const long long o = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const int c = static_cast<int>(o % C8) * 8;
    const long long pix = o / C8;
    const int x = static_cast<int>(pix % W), y = static_cast<int>((pix / W) % H);
    const long long b = pix / (static_cast<long long>(W) * H);
    const long long e = pix * C + c;
    bf8 v = ld8(Yc + ((b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c);
    const bf8 a = ld8(E + e);
#pragma unroll
    for (int k = 0; k < 8; ++k) v.f[k] += a.f[k];
    st8(S + e, v);
}

// dYc (B, H/2, W/2, C) = sum of dS over each 2 x 2 block, kept where `gate`
// (nullable, shaped as dYc) is positive; eight channels per thread.
__global__ void k_up2_bwd(const bf16 *__restrict__ dS, const bf16 *__restrict__ gate,
                          bf16 *__restrict__ dYc, int B, int H, int W, int C) {
    const int C8 = C >> 3;
    const long long n = static_cast<long long>(B) * (H / 2) * (W / 2) * C8;
    const long long o = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const int c = static_cast<int>(o % C8) * 8;
    const long long pix = o / C8;
    const int x = static_cast<int>(pix % (W / 2)), y = static_cast<int>((pix / (W / 2)) % (H / 2));
    const long long b = pix / (static_cast<long long>(W / 2) * (H / 2));
    const long long base = ((b * H + 2 * y) * W + 2 * x) * C + c;
    const bf8 a0 = ld8(dS + base), a1 = ld8(dS + base + C), a2 = ld8(dS + base + static_cast<long long>(W) * C),
              a3 = ld8(dS + base + static_cast<long long>(W) * C + C);
    bf8 r;
#pragma unroll
    for (int k = 0; k < 8; ++k) r.f[k] = a0.f[k] + a1.f[k] + a2.f[k] + a3.f[k];
    if (gate != nullptr) gate8(r, gate + pix * C + c);
    st8(dYc + pix * C + c, r);
}

// Squared error: per-block partial sums (double) and the gradient of the
// mean, 2 (y - t) / n, into dY: two fp32 channels per pixel (the kernels
// that read it round it to bf16 as they stage it).
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ y,
                                             const float *__restrict__ t, long long npix,
                                             double *__restrict__ partial,
                                             float *__restrict__ dY, float scale) {
    __shared__ double red[256];
    double s = 0.0;
    for (long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; p < npix;
         p += static_cast<long long>(gridDim.x) * blockDim.x) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const float d = y[2 * p + c] - t[2 * p + c];
            s += static_cast<double>(d) * d;
            dY[2 * p + c] = scale * d;
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

// out = scale * sum of the n partials: one block, each thread a strided
// subset in order, then a tree in LDS (fixed order: deterministic).
__global__ __launch_bounds__(256) void k_sum_double(const double *__restrict__ partial, int n,
                                                    double scale, double *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) s += partial[k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// Adam on every layer's master weights at once, each updated weight also
// written into the two packed bf16 layouts below (its forward and its
// input-gradient entry; the padding entries stay zero from creation).  One
// thread per real weight of the flat list, layer L holding off[L] ..
// off[L + 1] - 1: W[tap][ci][co] (real channel counts), the gradient in the
// padded layout g[tap][cip][cop]; the packing is k_pack_weights'.
constexpr int kMaxLayers = 10;
struct AdamLayers {
    float *w[kMaxLayers], *m[kMaxLayers], *v[kMaxLayers];
    const float *g[kMaxLayers];
    bf16 *fwd[kMaxLayers], *bwd[kMaxLayers];
    int cin[kMaxLayers], cout[kMaxLayers], cip[kMaxLayers], cop[kMaxLayers];
    int off[kMaxLayers + 1];
    int nl;
};
__global__ void k_adam_pack(const AdamLayers P, float lr, float b1, float b2, float c1, float c2,
                            float eps) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= P.off[P.nl]) return;
    int L = 0;
    while (f >= P.off[L + 1]) ++L;
    const int idx = f - P.off[L];
    const int cin = P.cin[L], cout = P.cout[L], cip = P.cip[L], cop = P.cop[L];
    const int co = idx % cout, ci = (idx / cout) % cin, tap = idx / (cout * cin);
    const float gr = P.g[L][(tap * cip + ci) * cop + co];
    const float mm = b1 * P.m[L][idx] + (1.f - b1) * gr;
    const float vv = b2 * P.v[L][idx] + (1.f - b2) * gr * gr;
    P.m[L][idx] = mm;
    P.v[L][idx] = vv;
    const float w = P.w[L][idx] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    P.w[L][idx] = w;
    const bf16 h = f2bf(w);
    {   // forward block (tap, kc, t), entry [co mod 16][ci mod 16]
        const int KC = cip >> 4, NT = cop >> 4;
        P.fwd[L][((tap * KC + (ci >> 4)) * NT + (co >> 4)) * 256 + (co & 15) * 16 + (ci & 15)] = h;
    }
    {   // input-gradient block (8 - tap, co / 16, ci / 16), entry [ci mod 16][co mod 16]
        const int KC = cop >> 4, NT = cip >> 4;
        P.bwd[L][(((8 - tap) * KC + (co >> 4)) * NT + (ci >> 4)) * 256 + (ci & 15) * 16 + (co & 15)] = h;
    }
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
// B * H * W < 2^31 (the network object checks it at creation); channels
// padded to 16, 32 or 64.
void warm_conv(const void *X, const void *Wp, void *Y, const void *gate, int B, int H, int W,
               int CPin, int CPout, bool relu, bool acc, bool out_f32, int creal, bool in2, hipStream_t s) {
    const long long tiles = static_cast<long long>(B) * ((H + 3) / 4) * ((W + 63) / 64);
    // fewer than 1024 pixel tiles: the output channel tiles are split over
    // blocks (each stages the same input) so that more CUs take part
    const int ntot = CPout / 16;
    int split = 1;
    while (split < ntot && tiles * split < 1024) split *= 2;
    const int nt = ntot / split;
    const dim3 grid(static_cast<unsigned>(tiles), split), blk(256);
    const bf16 *x = static_cast<const bf16 *>(X), *w = static_cast<const bf16 *>(Wp),
               *g = static_cast<const bf16 *>(gate);
#define RAS_TILE(NT, KC, F32)                                                                    \
    hipLaunchKernelGGL((k_conv3x3_tile<NT, KC, F32>), grid, blk, 0, s, x, w, Y, g, B, H, W,      \
                       relu ? 1 : 0, acc ? 1 : 0, creal, ntot)
#define RAS_TILE_KC(NT, F32)                  \
    do {                                      \
        if (CPin == 16) RAS_TILE(NT, 1, F32); \
        else if (CPin == 32) RAS_TILE(NT, 2, F32); \
        else RAS_TILE(NT, 4, F32);            \
    } while (0)
    if (in2) {                                 // two fp32 input channels (16 once staged)
        if (nt == 1) hipLaunchKernelGGL((k_conv3x3_tile<1, 1, false, true>), grid, blk, 0, s, x, w, Y, g, B, H,
                                        W, relu ? 1 : 0, acc ? 1 : 0, creal, ntot);
        else if (nt == 2) hipLaunchKernelGGL((k_conv3x3_tile<2, 1, false, true>), grid, blk, 0, s, x, w, Y, g,
                                             B, H, W, relu ? 1 : 0, acc ? 1 : 0, creal, ntot);
        else hipLaunchKernelGGL((k_conv3x3_tile<4, 1, false, true>), grid, blk, 0, s, x, w, Y, g, B, H, W,
                                relu ? 1 : 0, acc ? 1 : 0, creal, ntot);
    } else if (out_f32) RAS_TILE_KC(1, true);  // one column tile: the head
    else if (nt == 1) RAS_TILE_KC(1, false);
    else if (nt == 2) RAS_TILE_KC(2, false);
    else RAS_TILE_KC(4, false);
#undef RAS_TILE_KC
#undef RAS_TILE
}

// g[L] = sum of layer L's nblk[L] partial gradients (n[L] values each) for
// the nl layers (nl <= 10), tmp[L]: kSumSlices * n[L]; two launches in all.
void warm_sum_layers(int nl, const float *const *part, const int *nblk, const int *n, float *const *tmp,
                     float *const *g, hipStream_t s) {
    SumLayers P{};
    P.nl = nl;
    P.off[0] = 0;
    for (int L = 0; L < nl; ++L) {
        P.part[L] = part[L];
        P.tmp[L] = tmp[L];
        P.g[L] = g[L];
        P.n[L] = n[L];
        P.nblk[L] = nblk[L];
        P.per[L] = (nblk[L] + kSumSlices - 1) / kSumSlices;
        P.off[L + 1] = P.off[L] + n[L];
    }
    hipLaunchKernelGGL(k_sum_slices, dim3(blocks(P.off[nl], 256), kSumSlices), dim3(256), 0, s, P);
    hipLaunchKernelGGL(k_sum_tmp, dim3(blocks(P.off[nl], 256)), dim3(256), 0, s, P);
}

// Strips and row chunks of k_wgrad_strip: about 4096 waves over the input
// channel blocks and output tile groups (2048 with two output tiles a wave,
// whose registers leave two waves per SIMD), at least one row per wave.
// Returns the blocks in x.
int warm_wgrad_strip_blocks(int B, int H, int W, int KC, int NT, int NZ, int *rows_per_wave,
                            int *nchunk) {
    const int nstrip = (W + 63) / 64;
    const int target = std::max(1, (NT == 2 ? 2048 : 4096) / (KC * NZ));
    const int want = std::max(1, std::min(H, target / std::max(1, B * nstrip)));
    const int rpw = (H + want - 1) / want;
    *rows_per_wave = rpw;
    *nchunk = (H + rpw - 1) / rpw;
    return (B * *nchunk * nstrip + 3) / 4;
}
// The most blocks (in x) it gives for any batch up to B, for a layer of
// CPin -> CPout channels (B nchunk nstrip items never exceed the larger of
// the wave target and B nstrip).
int warm_wgrad_strip_blocks_max(int B, int W, int CPin, int CPout) {
    const int KC = CPin / 16, NT = CPout == 16 ? 1 : 2, NZ = CPout / (16 * NT);
    const int target = std::max(1, (NT == 2 ? 2048 : 4096) / (KC * NZ));
    return (std::max(target, B * ((W + 63) / 64)) + 3) / 4 + 1;
}

// The partial weight gradients of one layer into part; returns their count
// (the blocks), which warm_sum_layers adds.
int warm_wgrad(const void *X, const void *dZ, float *part, int B, int H, int W, int CPin, int CPout,
               bool x2, bool z2, hipStream_t s) {
    const bf16 *x = static_cast<const bf16 *>(X), *dz = static_cast<const bf16 *>(dZ);
    // one wave per strip, at most two output tiles a wave
    const int KC = CPin / 16, NT = CPout == 16 ? 1 : 2, NZ = CPout / (16 * NT);
    int rpw = 0, nch = 0;
    const int nb = warm_wgrad_strip_blocks(B, H, W, KC, NT, NZ, &rpw, &nch);
    const dim3 grid(nb, KC, NZ);
    // two fp32 channels: the input (16 channels once staged) or, with 16
    // output channels, the output gradient
    if (x2 && z2)
        hipLaunchKernelGGL((k_wgrad_strip<1, true, true>), grid, dim3(256), 0, s, x, dz, part, B, H, W, CPin,
                           CPout, rpw, nch);
    else if (x2 && NT == 1)
        hipLaunchKernelGGL((k_wgrad_strip<1, true, false>), grid, dim3(256), 0, s, x, dz, part, B, H, W, CPin,
                           CPout, rpw, nch);
    else if (x2)
        hipLaunchKernelGGL((k_wgrad_strip<2, true, false>), grid, dim3(256), 0, s, x, dz, part, B, H, W, CPin,
                           CPout, rpw, nch);
    else if (z2)
        hipLaunchKernelGGL((k_wgrad_strip<1, false, true>), grid, dim3(256), 0, s, x, dz, part, B, H, W, CPin,
                           CPout, rpw, nch);
    else if (NT == 1)
        hipLaunchKernelGGL(k_wgrad_strip<1>, grid, dim3(256), 0, s, x, dz, part, B, H, W, CPin, CPout, rpw,
                           nch);
    else
        hipLaunchKernelGGL(k_wgrad_strip<2>, grid, dim3(256), 0, s, x, dz, part, B, H, W, CPin, CPout, rpw,
                           nch);
    return nb;
}

void warm_pool(const void *X, void *Y, int B, int H, int W, int C, hipStream_t s) {
    const long long n = static_cast<long long>(B) * (H / 2) * (W / 2) * (C / 8);
    hipLaunchKernelGGL(k_pool2, dim3(blocks(n, 256)), dim3(256), 0, s, static_cast<const bf16 *>(X),
                       static_cast<bf16 *>(Y), B, H, W, C);
}
void warm_pool_bwd(const void *dY, const void *add, const void *gate, void *dX, int B, int H,
                   int W, int C, hipStream_t s) {
    const long long n = static_cast<long long>(B) * H * W * (C / 8);
    hipLaunchKernelGGL(k_pool2_bwd, dim3(blocks(n, 256)), dim3(256), 0, s,
                       static_cast<const bf16 *>(dY), static_cast<const bf16 *>(add),
                       static_cast<const bf16 *>(gate), static_cast<bf16 *>(dX), B, H, W, C);
}
void warm_up_add(const void *Yc, const void *E, void *S, int B, int H, int W, int C, hipStream_t s) {
    const long long n = static_cast<long long>(B) * H * W * (C / 8);
    hipLaunchKernelGGL(k_up2_add, dim3(blocks(n, 256)), dim3(256), 0, s, static_cast<const bf16 *>(Yc),
                       static_cast<const bf16 *>(E), static_cast<bf16 *>(S), B, H, W, C);
}
void warm_up_bwd(const void *dS, const void *gate, void *dYc, int B, int H, int W, int C,
                 hipStream_t s) {
    const long long n = static_cast<long long>(B) * (H / 2) * (W / 2) * (C / 8);
    hipLaunchKernelGGL(k_up2_bwd, dim3(blocks(n, 256)), dim3(256), 0, s, static_cast<const bf16 *>(dS),
                       static_cast<const bf16 *>(gate), static_cast<bf16 *>(dYc), B, H, W, C);
}
void warm_mse(const float *y, const float *t, long long npix, double *partial, int nblk, void *dY,
              double *loss, hipStream_t s) {
    const float scale = static_cast<float>(2.0 / (2.0 * npix));
    hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, s, y, t, npix, partial,
                       static_cast<float *>(dY), scale);
    hipLaunchKernelGGL(k_sum_double, dim3(1), dim3(256), 0, s, partial, nblk, 1.0 / (2.0 * npix),
                       loss);
}
// Adam and the packing of the nl layers in one launch (nl <= 10).
void warm_adam_pack(int nl, float *const *w, float *const *m, float *const *v, float *const *g,
                    void *const *fwd, void *const *bwd, const int *cin, const int *cout, const int *cip,
                    const int *cop, float lr, float b1, float b2, float c1, float c2, float eps,
                    hipStream_t s) {
    AdamLayers P{};
    P.nl = nl;
    P.off[0] = 0;
    for (int L = 0; L < nl; ++L) {
        P.w[L] = w[L];
        P.m[L] = m[L];
        P.v[L] = v[L];
        P.g[L] = g[L];
        P.fwd[L] = static_cast<bf16 *>(fwd[L]);
        P.bwd[L] = static_cast<bf16 *>(bwd[L]);
        P.cin[L] = cin[L];
        P.cout[L] = cout[L];
        P.cip[L] = cip[L];
        P.cop[L] = cop[L];
        P.off[L + 1] = P.off[L] + 9 * cin[L] * cout[L];
    }
    hipLaunchKernelGGL(k_adam_pack, dim3(blocks(P.off[nl], 256)), dim3(256), 0, s, P, lr, b1, b2, c1, c2,
                       eps);
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
