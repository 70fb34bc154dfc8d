// Device code of the surrogate network: a U-Net of periodic 3x3
// convolutions on NHWC FP32 activations, evaluated on the gfx950 matrix
// cores in bfloat16 with FP32 accumulation.
//
// Convolutions are implicit GEMMs: output[pixel][cout] = sum over (tap,
// cin) of input[pixel + tap][cin] W[tap][cin][cout].  The MFMA used is
// v_mfma_f32_16x16x32_bf16: A (16 x 32) holds, in lane l, row l % 16 and
// k = 8 (l / 16) + j for its 8 values j; B (32 x 16) holds k = 8 (l / 16) + j
// and column l % 16; the 16 x 16 result holds, in lane l, rows 4 (l / 16) + i
// and column l % 16 for its 4 values i.
#pragma once
#include <hip/hip_runtime.h>

namespace sur {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float floatx4;

constexpr int NT = 256;  // threads per block of every kernel here

// An NHWC activation: element (b, y, x, c) at p[((b H + y) W + x) C + off + c].
struct View {
  float *p;
  int C, off;
};

// Work folded into a convolution launch on the inference path, in place of
// separate elementwise launches (all off when zero-initialised):
//  * up: input channels [0, up_split) come from this half-resolution NHWC
//    activation (up_C channels per pixel, from channel up_off), repeated over
//    2 x 2 pixels (the nearest-neighbour upsampling of the decoder);
//  * scale_in: input channel k < 3 is multiplied by in_scale[k] (the
//    normalisation of the state);
//  * pool: the 2 x 2 mean of the output (after bias and ReLU) is written at
//    half resolution as well (the encoder's pooling), summed in the order
//    of the separate pooling kernel;
//  * resid: out = (resid * in_scale[n] + v) * out_scale[n] with resid of N
//    channels per pixel: the residual output x + head in normalised units,
//    scaled back, with the roundings of the separate kernels.
struct ConvFuse {
  const float *up;
  int up_C, up_off, up_split;
  int scale_in;
  float in_scale[3];
  View pool;
  const float *resid;
  float out_scale[3];
};

__device__ __forceinline__ int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }  // round to nearest even

// ------------------------------------------------------------ weight packing
// Fragments of B for the convolution kernel: frag[tap][kc][ct][lane][8] =
// Wsrc(tap, k = 32 kc + 8 (lane / 16) + j, n = 16 ct + lane % 16), zero
// outside K x N.  Forward: Wsrc(tap, k, n) = W[tap][k][n] (K = cin, N = cout).
// Input gradient: Wsrc(tap, k, n) = W[taps - 1 - tap][n][k] (K = cout,
// N = cin): the adjoint of a periodic correlation is the correlation with
// the flipped, transposed kernel.
__global__ void __launch_bounds__(NT) k_pack(const float *__restrict__ w, int taps, int cin, int cout, int transpose,
                                             __bf16 *__restrict__ frag, int nkc, int nct) {
  const int total = taps * nkc * nct * 64 * 8;
  for (int i = blockIdx.x * NT + threadIdx.x; i < total; i += gridDim.x * NT) {
    const int j = i % 8, lane = (i / 8) % 64, ct = (i / 512) % nct, kc = (i / (512 * nct)) % nkc,
              tap = i / (512 * nct * nkc);
    const int k = 32 * kc + 8 * (lane / 16) + j, n = 16 * ct + lane % 16;
    float v = 0.f;
    if (!transpose) {
      if (k < cin && n < cout) v = w[((size_t)tap * cin + k) * cout + n];
    } else {
      if (k < cout && n < cin) v = w[((size_t)(taps - 1 - tap) * cin + n) * cout + k];
    }
    frag[i] = to_bf16(v);
  }
}

// ---------------------------------------------------------------- convolution
// out[b][y][x][n] = epilogue(sum_{tap, k} in[b][y + dy][x + dx][k] Wsrc(tap, k, n))
// over a TX x TY pixel tile and NCT x 16 output channels per block
// (blockIdx.y picks the group of channels).  The input tile (with a halo of
// 1 for 3x3) is staged in LDS as bfloat16, 32 channels at a time.  Wave w
// owns pixel tiles 2w and 2w + 1 (16 consecutive pixels of the tile each).
// Epilogue: + bias (may be null), ReLU if relu, times (mask > 0) if mask.p.
template <int TAPS, int NCT>
__global__ void __launch_bounds__(NT) k_conv(int H, int W, View in, int K, const bf16x8 *__restrict__ frag, int nkc,
                                             int nct_total, const float *__restrict__ bias, View out, int N, int relu,
                                             View mask, ConvFuse fu) {
  constexpr int TX = 16, TY = 8;
  constexpr int HALO = TAPS == 9 ? 1 : 0;
  constexpr int SX = TX + 2 * HALO, SY = TY + 2 * HALO;
  constexpr int PITCH = 40;  // 32 channels + 8 of padding (bf16), 80 bytes per pixel
  __shared__ __attribute__((aligned(16))) __bf16 tile[SY * SX * PITCH];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int tiles_x = (W + TX - 1) / TX, tiles_y = (H + TY - 1) / TY;
  const int bimg = blockIdx.x / (tiles_x * tiles_y);
  const int t = blockIdx.x % (tiles_x * tiles_y);
  const int x0 = (t % tiles_x) * TX, y0 = (t / tiles_x) * TY;
  const int ct0 = blockIdx.y * NCT;  // first 16-channel tile of this block
  floatx4 acc[2][NCT];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int c = 0; c < NCT; c++) acc[a][c] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int kc = 0; kc < nkc; kc++) {
    // stage the input tile: SY x SX pixels x 32 channels, FP32 -> bf16
    for (int i = threadIdx.x; i < SY * SX * 8; i += NT) {
      const int q = i % 8, pix = i / 8;  // 4 channels q*4 .. q*4+3 of pixel pix
      const int sx = pix % SX, sy = pix / SX;
      const int gx = wrapi(x0 + sx - HALO, W), gy = wrapi(y0 + sy - HALO, H);
      const int k = 32 * kc + 4 * q;
      // the channels of this group come from the input or, below up_split,
      // from the half-resolution activation (up_split is a multiple of 4)
      const bool from_up = fu.up && k < fu.up_split;
      const float *src = from_up ? fu.up + ((size_t)(bimg * (H / 2) + gy / 2) * (W / 2) + gx / 2) * fu.up_C + fu.up_off
                                 : in.p + ((size_t)(bimg * H + gy) * W + gx) * in.C + in.off;
      const int sC = from_up ? fu.up_C : in.C, soff = from_up ? fu.up_off : in.off;
      float v[4];
      if (k + 3 < K && ((sC | soff) & 3) == 0) {
        const float4 f = *reinterpret_cast<const float4 *>(src + k);
        v[0] = f.x;
        v[1] = f.y;
        v[2] = f.z;
        v[3] = f.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; e++) v[e] = k + e < K ? src[k + e] : 0.f;
      }
      if (fu.scale_in) {
#pragma unroll
        for (int e = 0; e < 4; e++)
          if (k + e < 3) v[e] *= fu.in_scale[k + e];
      }
      __bf16 *d = tile + pix * PITCH + 4 * q;
#pragma unroll
      for (int e = 0; e < 4; e++) d[e] = to_bf16(v[e]);
    }
    __syncthreads();
#pragma unroll
    for (int tap = 0; tap < TAPS; tap++) {
      const int dy = TAPS == 9 ? tap / 3 - 1 : 0, dx = TAPS == 9 ? tap % 3 - 1 : 0;
      bf16x8 a[2];
#pragma unroll
      for (int pt = 0; pt < 2; pt++) {
        const int p = 16 * (2 * wave + pt) + lane % 16;  // pixel of the tile
        const int px = p % TX, py = p / TX;
        const int s = (py + HALO + dy) * SX + (px + HALO + dx);
        a[pt] = *reinterpret_cast<const bf16x8 *>(tile + s * PITCH + 8 * (lane / 16));
      }
#pragma unroll
      for (int c = 0; c < NCT; c++) {
        if (ct0 + c >= nct_total) continue;  // last group of channels may be partial
        const bf16x8 bfr = frag[((size_t)(tap * nkc + kc) * nct_total + ct0 + c) * 64 + lane];
#pragma unroll
        for (int pt = 0; pt < 2; pt++)
          acc[pt][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[pt], bfr, acc[pt][c], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // epilogue: lane holds pixels 4 (lane / 16) + i of each pixel tile, channel
  // lane % 16; pixel tile pt of wave w is image row y0 + 2 w + pt
#pragma unroll
  for (int pt = 0; pt < 2; pt++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int p = 16 * (2 * wave + pt) + 4 * (lane / 16) + i;
      const int gx = x0 + p % TX, gy = y0 + p / TX;
      if (gx >= W || gy >= H) continue;
      const size_t pix = (size_t)(bimg * H + gy) * W + gx;
#pragma unroll
      for (int c = 0; c < NCT; c++) {
        const int n = 16 * (ct0 + c) + lane % 16;
        if (ct0 + c >= nct_total || n >= N) continue;
        float v = acc[pt][c][i];
        if (bias) v += bias[n];
        if (relu) v = fmaxf(v, 0.f);
        if (mask.p && !(mask.p[pix * mask.C + mask.off + n] > 0.f)) v = 0.f;
        acc[pt][c][i] = v;  // kept for the pooled output
        if (fu.resid) {
#pragma clang fp contract(off)  // each product and sum rounded on its own, as in separate kernels
          const float xn = fu.resid[pix * N + n] * fu.in_scale[n];
          v = (xn + v) * fu.out_scale[n];
        }
        out.p[pix * out.C + out.off + n] = v;
      }
    }
  if (fu.pool.p) {
    // the 2 x 2 block of pixels (x, x + 1) x (rows 2 w, 2 w + 1 of the tile)
    // is in this lane: pixels i, i + 1 of both pixel tiles.  H and W are even
    // and x0, y0 too, so a block lies wholly inside or wholly outside.
#pragma unroll
    for (int i = 0; i < 4; i += 2) {
      const int gx = x0 + 4 * (lane / 16) + i, gy = y0 + 2 * wave;
      if (gx >= W || gy >= H) continue;
      const size_t po = (size_t)(bimg * (H / 2) + gy / 2) * (W / 2) + gx / 2;
#pragma unroll
      for (int c = 0; c < NCT; c++) {
        const int n = 16 * (ct0 + c) + lane % 16;
        if (ct0 + c >= nct_total || n >= N) continue;
        const float s = (acc[0][c][i] + acc[0][c][i + 1]) + (acc[1][c][i] + acc[1][c][i + 1]);
        fu.pool.p[po * fu.pool.C + fu.pool.off + n] = 0.25f * s;
      }
    }
  }
}

// --------------------------------------------------------- weight gradient
// part[pc][tap][k][n] = sum over the pixels of chunk pc of
// in[pixel + tap][k] dz[pixel][n], for k in a 32-channel chunk (blockIdx.y)
// and n in a 64-channel group (blockIdx.z); blockIdx.x = tap + taps pc.  A
// chunk is `rows` image rows of one image.  Pixels are staged 64 at a time,
// transposed in LDS ([channel][pixel], bf16) so an MFMA fragment (8
// consecutive pixels of one channel) is one 16-byte read.  Wave w owns
// output columns 16w .. 16w + 15 and both 16-row halves of the k chunk.
template <int TAPS>
__global__ void __launch_bounds__(NT) k_wgrad(int H, int W, View in, int K, View dz, int N, int rows,
                                              float *__restrict__ part, int KP, int NP) {
  constexpr int PX = 64, PP = PX + 8;  // pixels per stage, padded pitch
  __shared__ __attribute__((aligned(16))) __bf16 sx[32 * PP];
  __shared__ __attribute__((aligned(16))) __bf16 sd[64 * PP];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int tap = blockIdx.x % TAPS, pc = blockIdx.x / TAPS;
  const int dy = TAPS == 9 ? tap / 3 - 1 : 0, dx = TAPS == 9 ? tap % 3 - 1 : 0;
  const int k0 = 32 * blockIdx.y, n0 = 64 * blockIdx.z;
  const int chunks_per_img = H / rows;
  const int bimg = pc / chunks_per_img, r0 = (pc % chunks_per_img) * rows;
  const int npix = rows * W;
  floatx4 acc[2] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
  for (int p0 = 0; p0 < npix; p0 += PX) {
    // stage in[p + tap][k0 .. k0 + 31] and dz[p][n0 .. n0 + 63] for 64 pixels, transposed
    for (int i = threadIdx.x; i < PX * 8; i += NT) {
      const int q = i % 8, pl = i / 8;  // channels 4q .. 4q+3
      const int p = p0 + pl;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (p < npix) {
        const int y = r0 + p / W, x = p % W;
        const int gy = wrapi(y + dy, H), gx = wrapi(x + dx, W);
        const float *src = in.p + ((size_t)(bimg * H + gy) * W + gx) * in.C + in.off;
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int k = k0 + 4 * q + e;
          v[e] = k < K ? src[k] : 0.f;
        }
      }
#pragma unroll
      for (int e = 0; e < 4; e++) sx[(4 * q + e) * PP + pl] = to_bf16(v[e]);
    }
    for (int i = threadIdx.x; i < PX * 16; i += NT) {
      const int q = i % 16, pl = i / 16;  // channels 4q .. 4q+3
      const int p = p0 + pl;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (p < npix) {
        const int y = r0 + p / W, x = p % W;
        const float *src = dz.p + ((size_t)(bimg * H + y) * W + x) * dz.C + dz.off;
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int n = n0 + 4 * q + e;
          v[e] = n < N ? src[n] : 0.f;
        }
      }
#pragma unroll
      for (int e = 0; e < 4; e++) sd[(4 * q + e) * PP + pl] = to_bf16(v[e]);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < PX / 32; ks++) {
      const int kp = 32 * ks + 8 * (lane / 16);  // pixel offset of this lane's fragment
      const bf16x8 b = *reinterpret_cast<const bf16x8 *>(sd + (16 * wave + lane % 16) * PP + kp);
#pragma unroll
      for (int h = 0; h < 2; h++) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(sx + (16 * h + lane % 16) * PP + kp);
        acc[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[h], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // result rows k (4 (lane / 16) + i of half h), column n = 16 wave + lane % 16
  float *dst = part + ((size_t)pc * TAPS + tap) * KP * NP;
#pragma unroll
  for (int h = 0; h < 2; h++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int k = k0 + 16 * h + 4 * (lane / 16) + i, n = n0 + 16 * wave + lane % 16;
      dst[(size_t)k * NP + n] = acc[h][i];
    }
}

// dW[tap][k][n] = sum over pc of part[pc][tap][k][n] (fixed order), k < K, n < N.
__global__ void __launch_bounds__(NT) k_wgrad_reduce(const float *__restrict__ part, int npc, int taps, int KP, int NP,
                                                     int K, int N, float *__restrict__ dw) {
  const int total = taps * K * N;
  for (int i = blockIdx.x * NT + threadIdx.x; i < total; i += gridDim.x * NT) {
    const int n = i % N, k = (i / N) % K, tap = i / (N * K);
    const size_t stride = (size_t)taps * KP * NP, off = ((size_t)tap * KP + k) * NP + n;
    float s = 0.f;
    for (int pc = 0; pc < npc; pc++) s += part[pc * stride + off];
    dw[i] = s;
  }
}

// Bias gradient, stage 1: part[blk][n] = sum of dz[p][n] over the pixel
// range of block blk (`per` pixels); stage 2 sums the blocks in order.
__global__ void __launch_bounds__(NT) k_bgrad(View dz, int N, long long npix, int per, float *__restrict__ part) {
  const long long p0 = (long long)blockIdx.x * per;
  for (int n = threadIdx.x; n < N; n += NT) {
    float s = 0.f;
    for (int p = 0; p < per && p0 + p < npix; p++) s += dz.p[(size_t)(p0 + p) * dz.C + dz.off + n];
    part[(size_t)blockIdx.x * N + n] = s;
  }
}

__global__ void __launch_bounds__(NT) k_bgrad_reduce(const float *__restrict__ part, int nblk, int N,
                                                     float *__restrict__ db) {
  for (int n = blockIdx.x * NT + threadIdx.x; n < N; n += gridDim.x * NT) {
    float s = 0.f;
    for (int b = 0; b < nblk; b++) s += part[(size_t)b * N + n];
    db[n] = s;
  }
}

// ------------------------------------------------------------- elementwise
// The elementwise kernels below index with 32-bit integers: every tensor of
// the network holds fewer than 2^31 elements (the host checks it).

// Adjoint of the 2x2 mean: din[y][x] (+)= dout[y/2][x/2] / 4 (H, W of din).
__global__ void __launch_bounds__(NT) k_pool_back(int B, int H, int W, View dout, View din, int C, int accumulate) {
  const int total = B * H * W * C;
  for (int i = blockIdx.x * NT + threadIdx.x; i < total; i += gridDim.x * NT) {
    const int c = i % C, pix = i / C;
    const int x = pix % W, y = (pix / W) % H, b = pix / (W * H);
    const float g = 0.25f * dout.p[((b * (H / 2) + y / 2) * (W / 2) + x / 2) * dout.C + dout.off + c];
    float &d = din.p[pix * din.C + din.off + c];
    d = accumulate ? d + g : g;
  }
}

// Nearest 2x upsampling: out (H x W) from in (H/2 x W/2).
__global__ void __launch_bounds__(NT) k_up(int B, int H, int W, View in, View out, int C) {
  const int total = B * H * W * C;
  for (int i = blockIdx.x * NT + threadIdx.x; i < total; i += gridDim.x * NT) {
    const int c = i % C, pix = i / C;
    const int x = pix % W, y = (pix / W) % H, b = pix / (W * H);
    out.p[pix * out.C + out.off + c] = in.p[((b * (H / 2) + y / 2) * (W / 2) + x / 2) * in.C + in.off + c];
  }
}

// Adjoint of the upsampling: din[y][x] = sum of the 2x2 block of dout (H, W of din).
__global__ void __launch_bounds__(NT) k_up_back(int B, int H, int W, View dout, View din, int C) {
  const int total = B * H * W * C;
  for (int i = blockIdx.x * NT + threadIdx.x; i < total; i += gridDim.x * NT) {
    const int c = i % C, pix = i / C;
    const int x = pix % W, y = (pix / W) % H, b = pix / (W * H);
    const float *r0 = dout.p + ((b * 2 * H + 2 * y) * (2 * W) + 2 * x) * dout.C + dout.off + c;
    const float *r1 = r0 + 2 * W * dout.C;
    din.p[pix * din.C + din.off + c] = (r0[0] + r0[dout.C]) + (r1[0] + r1[dout.C]);
  }
}

// d *= (a > 0), elementwise over npix pixels and C channels.
__global__ void __launch_bounds__(NT) k_relu_mask(int npix, View d, View a, int C) {
  const int total = npix * C;
  for (int i = blockIdx.x * NT + threadIdx.x; i < total; i += gridDim.x * NT) {
    const int c = i % C, pix = i / C;
    if (!(a.p[pix * a.C + a.off + c] > 0.f)) d.p[pix * d.C + d.off + c] = 0.f;
  }
}

// Normalisation of the network's input and output: out = in * s[c] (3 channels).
__global__ void __launch_bounds__(NT) k_scale3(long long n, const float *__restrict__ in, float *__restrict__ out,
                                               float s0, float s1, float s2) {
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n * 3; i += (long long)gridDim.x * NT) {
    const int c = i % 3;
    out[i] = in[i] * (c == 0 ? s0 : (c == 1 ? s1 : s2));
  }
}

// y = x + h (the residual output), elementwise.
__global__ void __launch_bounds__(NT) k_add(long long n, const float *__restrict__ x, const float *__restrict__ h,
                                            float *__restrict__ y) {
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) y[i] = x[i] + h[i];
}

// Mean squared error: g = 2 (y - t) / n and per-block partial sums of (y - t)^2 in FP64.
__global__ void __launch_bounds__(NT) k_mse(long long n, const float *__restrict__ y, const float *__restrict__ t,
                                            float *__restrict__ g, double *__restrict__ part) {
  __shared__ double red[NT];
  double s = 0.0;
  const float inv = 2.0f / (float)n;
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const float d = y[i] - t[i];
    g[i] = inv * d;
    s += (double)d * (double)d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = NT / 2; w > 0; w /= 2) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Adam (Kingma and Ba, Algorithm 1), with the bias corrections c1 = 1/(1 -
// beta1^t) and c2 = 1/(1 - beta2^t) computed on the host.
__global__ void __launch_bounds__(NT) k_adam(long long n, float *__restrict__ p, float *__restrict__ m,
                                             float *__restrict__ v, const float *__restrict__ g, float lr, float b1,
                                             float b2, float eps, float c1, float c2) {
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

}  // namespace sur
