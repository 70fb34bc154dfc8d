// Host side of the surrogate network (include/sur.h): workspace layout,
// layer sequencing of the forward and backward passes, Adam, timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "sur.h"
#include "sur_kernels.hpp"

using sur::View;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

enum Layer { E0A, E0B, E1A, E1B, B2A, B2B, D1A, D1B, D0A, D0B, HEAD, NLAYER };

struct LayerSpec {
  int cin, cout, taps, relu, level;  // level: 0 full, 1 half, 2 quarter resolution
};

void specs(const sur_config &c, LayerSpec s[NLAYER]) {
  s[E0A] = {3, c.c0, 9, 1, 0};
  s[E0B] = {c.c0, c.c0, 9, 1, 0};
  s[E1A] = {c.c0, c.c1, 9, 1, 1};
  s[E1B] = {c.c1, c.c1, 9, 1, 1};
  s[B2A] = {c.c1, c.c2, 9, 1, 2};
  s[B2B] = {c.c2, c.c2, 9, 1, 2};
  s[D1A] = {c.c2 + c.c1, c.c1, 9, 1, 1};
  s[D1B] = {c.c1, c.c1, 9, 1, 1};
  s[D0A] = {c.c1 + c.c0, c.c0, 9, 1, 0};
  s[D0B] = {c.c0, c.c0, 9, 1, 0};
  s[HEAD] = {c.c0, 3, 1, 0, 0};
}

bool config_ok(const sur_config *c) {
  if (!(c && c->batch >= 1 && c->height >= 4 && c->width >= 4 && c->height % 4 == 0 && c->width % 4 == 0 &&
        c->c0 >= 1 && c->c1 >= 1 && c->c2 >= 1 && c->scale[0] > 0 && c->scale[1] > 0 && c->scale[2] > 0))
    return false;
  // the largest activation (full resolution, c1 + c0 channels) is indexed with 32-bit integers
  return (long long)c->batch * c->height * c->width * (c->c0 + c->c1 + c->c2 + 3) < (1LL << 31);
}

// Activation and gradient buffers (float counts per image at their level).
enum Buf {
  XN, TN, A_E0A, U0, P0, A_E1A, U1, P1, A_B2A, A_B2B, A_D1A, A_D1B, A_D0A, A_D0B, HD, YN,  // activations
  G_HD, G_D0B, G_D0A, G_U0, G_D1B, G_D1A, G_U1, G_B2B, G_B2A, G_P1, G_E1A, G_P0, G_E0A,  // gradients
  NBUF
};

struct BufSpec {
  int level, channels;
};

void buf_specs(const sur_config &c, BufSpec b[NBUF]) {
  const int c0 = c.c0, c1 = c.c1, c2 = c.c2;
  b[XN] = {0, 3};
  b[TN] = {0, 3};
  b[A_E0A] = {0, c0};
  b[U0] = {0, c1 + c0};  // [up(d1b) | e0b]
  b[P0] = {1, c0};
  b[A_E1A] = {1, c1};
  b[U1] = {1, c2 + c1};  // [up(b2b) | e1b]
  b[P1] = {2, c1};
  b[A_B2A] = {2, c2};
  b[A_B2B] = {2, c2};
  b[A_D1A] = {1, c1};
  b[A_D1B] = {1, c1};
  b[A_D0A] = {0, c0};
  b[A_D0B] = {0, c0};
  b[HD] = {0, 3};
  b[YN] = {0, 3};
  b[G_HD] = {0, 3};
  b[G_D0B] = {0, c0};
  b[G_D0A] = {0, c0};
  b[G_U0] = {0, c1 + c0};
  b[G_D1B] = {1, c1};
  b[G_D1A] = {1, c1};
  b[G_U1] = {1, c2 + c1};
  b[G_B2B] = {2, c2};
  b[G_B2A] = {2, c2};
  b[G_P1] = {2, c1};
  b[G_E1A] = {1, c1};
  b[G_P0] = {1, c0};
  b[G_E0A] = {0, c0};
}

int level_h(const sur_config &c, int level) { return c.height >> level; }
int level_w(const sur_config &c, int level) { return c.width >> level; }

// Rows of a weight-gradient pixel chunk: the largest divisor of H with
// rows * W <= 4096 (at least 1).
int wgrad_rows(int H, int W) {
  int best = 1;
  for (int r = 1; r <= H; r++)
    if (H % r == 0 && (long long)r * W <= 4096) best = r;
  return best;
}

struct Layout {
  size_t buf[NBUF];
  size_t params, grads, m, v;
  size_t frag_f[NLAYER], frag_t[NLAYER];
  size_t wpart, bpart, lpart, total;
  size_t nparam;
  size_t w_off[NLAYER], b_off[NLAYER];  // offsets in the parameter vector (floats)
  int nkc_f[NLAYER], nct_f[NLAYER], nkc_t[NLAYER], nct_t[NLAYER];
  int nblk_loss, nblk_bias;
};

constexpr int kLossBlocks = 1024;

Layout make_layout(const sur_config &c) {
  Layout L{};
  LayerSpec s[NLAYER];
  specs(c, s);
  BufSpec bs[NBUF];
  buf_specs(c, bs);
  size_t off = 0;
  for (int i = 0; i < NBUF; i++) {
    L.buf[i] = off;
    const size_t n = (size_t)c.batch * level_h(c, bs[i].level) * level_w(c, bs[i].level) * bs[i].channels;
    off = align_up(off + 4 * n);
  }
  size_t np = 0;
  for (int l = 0; l < NLAYER; l++) {
    L.w_off[l] = np;
    np += (size_t)s[l].taps * s[l].cin * s[l].cout;
    L.b_off[l] = np;
    np += s[l].cout;
  }
  L.nparam = np;
  L.params = off;
  off = align_up(off + 4 * np);
  L.grads = off;
  off = align_up(off + 4 * np);
  L.m = off;
  off = align_up(off + 4 * np);
  L.v = off;
  off = align_up(off + 4 * np);
  size_t wpart = 0;
  long long max_pix = 0;
  for (int l = 0; l < NLAYER; l++) {
    L.nkc_f[l] = cdiv(s[l].cin, 32);
    L.nct_f[l] = cdiv(s[l].cout, 16);
    L.nkc_t[l] = cdiv(s[l].cout, 32);
    L.nct_t[l] = cdiv(s[l].cin, 16);
    L.frag_f[l] = off;
    off = align_up(off + 2 * (size_t)s[l].taps * L.nkc_f[l] * L.nct_f[l] * 512);
    L.frag_t[l] = off;
    off = align_up(off + 2 * (size_t)s[l].taps * L.nkc_t[l] * L.nct_t[l] * 512);
    const int H = level_h(c, s[l].level), W = level_w(c, s[l].level);
    const int npc = c.batch * (H / wgrad_rows(H, W));
    wpart = std::max(wpart, (size_t)npc * s[l].taps * (32 * L.nkc_f[l]) * (64 * (size_t)cdiv(s[l].cout, 64)));
    max_pix = std::max(max_pix, (long long)c.batch * H * W);
  }
  L.wpart = off;
  off = align_up(off + 4 * wpart);
  L.nblk_bias = cdiv(max_pix, 1024);
  L.bpart = off;
  off = align_up(off + 4 * (size_t)L.nblk_bias * std::max({c.c0, c.c1, c.c2, c.c1 + c.c2}));
  L.nblk_loss = kLossBlocks;
  L.lpart = off;
  off = align_up(off + 8 * (size_t)kLossBlocks);
  L.total = off;
  return L;
}

}  // namespace

struct sur_net {
  sur_config cfg;
  LayerSpec spec[NLAYER];
  Layout lay;
  hipStream_t stream;
  char *ws;
  long long adam_t;
  bool have_grad;
  std::string err;
};

namespace {

thread_local std::string g_sur_error;

hlb_status sfail(sur_net *n, hlb_status s, const std::string &msg) {
  if (n) n->err = msg;
  else g_sur_error = msg;
  return s;
}

hlb_status shf(sur_net *n, hipError_t e, const char *what) {
  return sfail(n, HLB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
T *at(sur_net *n, size_t off) {
  return reinterpret_cast<T *>(n->ws + off);
}

View view(sur_net *n, Buf b, int off = 0) {
  BufSpec bs[NBUF];
  buf_specs(n->cfg, bs);
  return View{at<float>(n, n->lay.buf[b]), bs[b].channels, off};
}

const View kNoView{nullptr, 0, 0};

unsigned grid_for(long long work) { return (unsigned)std::min<long long>(std::max<long long>(cdiv(work, 256), 1), 8192); }

void pack_layer(sur_net *n, int l) {
  const LayerSpec &s = n->spec[l];
  const Layout &L = n->lay;
  const float *w = at<float>(n, L.params) + L.w_off[l];
  const int tf = s.taps * L.nkc_f[l] * L.nct_f[l] * 512, tt = s.taps * L.nkc_t[l] * L.nct_t[l] * 512;
  hipLaunchKernelGGL(sur::k_pack, dim3(grid_for(tf)), dim3(256), 0, n->stream, w, s.taps, s.cin, s.cout, 0,
                     at<__bf16>(n, L.frag_f[l]), L.nkc_f[l], L.nct_f[l]);
  hipLaunchKernelGGL(sur::k_pack, dim3(grid_for(tt)), dim3(256), 0, n->stream, w, s.taps, s.cin, s.cout, 1,
                     at<__bf16>(n, L.frag_t[l]), L.nkc_t[l], L.nct_t[l]);
}

void pack_all(sur_net *n) {
  for (int l = 0; l < NLAYER; l++) pack_layer(n, l);
}

// out = conv(in) of layer l at its level: forward (bias, ReLU) or input
// gradient (transposed weights, optional mask).
void conv(sur_net *n, int l, int batch, View in, View out, bool transpose, View mask,
          const sur::ConvFuse &fu = sur::ConvFuse{}) {
  const LayerSpec &s = n->spec[l];
  const Layout &L = n->lay;
  const int H = level_h(n->cfg, s.level), W = level_w(n->cfg, s.level);
  const int K = transpose ? s.cout : s.cin, N = transpose ? s.cin : s.cout;
  const int nkc = transpose ? L.nkc_t[l] : L.nkc_f[l], nct = transpose ? L.nct_t[l] : L.nct_f[l];
  const auto *frag = reinterpret_cast<const sur::bf16x8 *>(at<__bf16>(n, transpose ? L.frag_t[l] : L.frag_f[l]));
  const float *bias = transpose ? nullptr : at<float>(n, L.params) + L.b_off[l];
  const int relu = transpose ? 0 : s.relu;
  // 16-channel tiles per block: 4 where that still gives two blocks per CU,
  // fewer on the coarse levels of a small batch (more blocks, each staging
  // the same input tile for fewer output channels)
  const long long ptiles = (long long)batch * cdiv(W, 16) * cdiv(H, 8);
  int ncg = nct >= 4 ? 4 : nct;
  while (ncg > 1 && ptiles * cdiv(nct, ncg) < 512) ncg = ncg == 4 ? 2 : 1;
  const dim3 grid((unsigned)ptiles, cdiv(nct, ncg));
#define SUR_CONV(TAPS, NCT)                                                                                        \
  hipLaunchKernelGGL((sur::k_conv<TAPS, NCT>), grid, dim3(256), 0, n->stream, H, W, in, K, frag, nkc, nct, bias, \
                     out, N, relu, mask, fu)
  if (s.taps == 9) {
    if (ncg == 4) SUR_CONV(9, 4);
    else if (ncg == 2) SUR_CONV(9, 2);
    else if (ncg == 3) SUR_CONV(9, 3);
    else SUR_CONV(9, 1);
  } else {
    if (ncg == 4) SUR_CONV(1, 4);
    else if (ncg == 2) SUR_CONV(1, 2);
    else if (ncg == 3) SUR_CONV(1, 3);
    else SUR_CONV(1, 1);
  }
#undef SUR_CONV
}

// Weight and bias gradients of layer l from its input and the gradient of
// its pre-activation output.
void wgrad(sur_net *n, int l, int batch, View in, View dz) {
  const LayerSpec &s = n->spec[l];
  const Layout &L = n->lay;
  const int H = level_h(n->cfg, s.level), W = level_w(n->cfg, s.level);
  const int rows = wgrad_rows(H, W);
  const int npc = batch * (H / rows);
  const int KP = 32 * L.nkc_f[l], NP = 64 * cdiv(s.cout, 64);
  float *part = at<float>(n, L.wpart);
  float *g = at<float>(n, L.grads);
  const dim3 grid(s.taps * npc, KP / 32, NP / 64);
  if (s.taps == 9)
    hipLaunchKernelGGL(sur::k_wgrad<9>, grid, dim3(256), 0, n->stream, H, W, in, s.cin, dz, s.cout, rows, part, KP, NP);
  else
    hipLaunchKernelGGL(sur::k_wgrad<1>, grid, dim3(256), 0, n->stream, H, W, in, s.cin, dz, s.cout, rows, part, KP, NP);
  const long long nw = (long long)s.taps * s.cin * s.cout;
  hipLaunchKernelGGL(sur::k_wgrad_reduce, dim3(grid_for(nw)), dim3(256), 0, n->stream, part, npc, s.taps, KP, NP,
                     s.cin, s.cout, g + L.w_off[l]);
  const long long npix = (long long)batch * H * W;
  const int per = 1024, nblk = cdiv(npix, per);
  float *bp = at<float>(n, L.bpart);
  hipLaunchKernelGGL(sur::k_bgrad, dim3(nblk), dim3(256), 0, n->stream, dz, s.cout, npix, per, bp);
  hipLaunchKernelGGL(sur::k_bgrad_reduce, dim3(1), dim3(256), 0, n->stream, bp, nblk, s.cout, g + L.b_off[l]);
}

long long npix_at(sur_net *n, int batch, int level) {
  return (long long)batch * level_h(n->cfg, level) * level_w(n->cfg, level);
}

void up(sur_net *n, int batch, int level, View in, View out, int C) {  // level of the output
  const int H = level_h(n->cfg, level), W = level_w(n->cfg, level);
  hipLaunchKernelGGL(sur::k_up, dim3(grid_for(npix_at(n, batch, level) * C)), dim3(256), 0, n->stream, batch, H, W,
                     in, out, C);
}

// The forward pass.  Training (x == nullptr): from the normalised input XN
// to YN = XN + head, keeping every activation the backward pass reads.
// Inference (x, y device arrays of the caller): y = x + scale * head(x /
// scale), with the normalisation, the upsampling and the residual folded into
// the convolutions (ConvFuse) instead of separate launches; the results are
// the same floats.  Both fold the pooling into the encoder convolutions.
void forward_normalised(sur_net *n, int batch, hipEvent_t *ev, const float *x = nullptr, float *y = nullptr) {
  const int c1 = n->cfg.c1, c2 = n->cfg.c2;
  const bool fused = x != nullptr;
  const double *sc = n->cfg.scale;
  // events around each convolution when timing (ev: 2 per layer)
  auto cv = [&](int l, View in, View out, const sur::ConvFuse &fu = sur::ConvFuse{}) {
    if (ev) (void)hipEventRecord(ev[2 * l], n->stream);
    conv(n, l, batch, in, out, false, kNoView, fu);
    if (ev) (void)hipEventRecord(ev[2 * l + 1], n->stream);
  };
  auto pooled = [&](Buf b) {
    sur::ConvFuse fu{};
    fu.pool = view(n, b);
    return fu;
  };
  // upsampling folded into the decoder's first convolution, when the
  // upsampled channels end on a 4-channel group
  auto up_into = [&](int level, Buf src, int C, Buf dst) {
    sur::ConvFuse fu{};
    if (fused && C % 4 == 0) {
      fu.up = at<float>(n, n->lay.buf[src]);
      fu.up_C = C;
      fu.up_off = 0;
      fu.up_split = C;
    } else {
      up(n, batch, level, view(n, src), view(n, dst, 0), C);
    }
    return fu;
  };
  if (fused) {
    sur::ConvFuse fu{};
    fu.scale_in = 1;
    for (int c = 0; c < 3; c++) fu.in_scale[c] = (float)(1.0 / sc[c]);
    cv(E0A, View{const_cast<float *>(x), 3, 0}, view(n, A_E0A), fu);
  } else {
    cv(E0A, view(n, XN), view(n, A_E0A));
  }
  cv(E0B, view(n, A_E0A), view(n, U0, c1), pooled(P0));
  cv(E1A, view(n, P0), view(n, A_E1A));
  cv(E1B, view(n, A_E1A), view(n, U1, c2), pooled(P1));
  cv(B2A, view(n, P1), view(n, A_B2A));
  cv(B2B, view(n, A_B2A), view(n, A_B2B));
  cv(D1A, view(n, U1), view(n, A_D1A), up_into(1, A_B2B, c2, U1));
  cv(D1B, view(n, A_D1A), view(n, A_D1B));
  cv(D0A, view(n, U0), view(n, A_D0A), up_into(0, A_D1B, c1, U0));
  cv(D0B, view(n, A_D0A), view(n, A_D0B));
  if (fused) {
    sur::ConvFuse fu{};
    fu.resid = x;
    for (int c = 0; c < 3; c++) {
      fu.in_scale[c] = (float)(1.0 / sc[c]);
      fu.out_scale[c] = (float)sc[c];
    }
    cv(HEAD, view(n, A_D0B), View{y, 3, 0}, fu);
    return;
  }
  cv(HEAD, view(n, A_D0B), view(n, HD));
  const long long ne = npix_at(n, batch, 0) * 3;
  hipLaunchKernelGGL(sur::k_add, dim3(grid_for(ne)), dim3(256), 0, n->stream, ne, at<float>(n, n->lay.buf[XN]),
                     at<float>(n, n->lay.buf[HD]), at<float>(n, n->lay.buf[YN]));
}

void backward(sur_net *n, int batch) {
  const int c0 = n->cfg.c0, c1 = n->cfg.c1, c2 = n->cfg.c2;
  // head: dz = d(head output) = G_HD
  wgrad(n, HEAD, batch, view(n, A_D0B), view(n, G_HD));
  conv(n, HEAD, batch, view(n, G_HD), view(n, G_D0B), true, view(n, A_D0B));  // masked: dz of d0b
  wgrad(n, D0B, batch, view(n, A_D0A), view(n, G_D0B));
  conv(n, D0B, batch, view(n, G_D0B), view(n, G_D0A), true, view(n, A_D0A));
  wgrad(n, D0A, batch, view(n, U0), view(n, G_D0A));
  conv(n, D0A, batch, view(n, G_D0A), view(n, G_U0), true, kNoView);
  // u0 = [up(d1b) | e0b]
  {
    const int H = level_h(n->cfg, 1), W = level_w(n->cfg, 1);
    hipLaunchKernelGGL(sur::k_up_back, dim3(grid_for(npix_at(n, batch, 1) * c1)), dim3(256), 0, n->stream, batch, H,
                       W, view(n, G_U0, 0), view(n, G_D1B), c1);
    hipLaunchKernelGGL(sur::k_relu_mask, dim3(grid_for(npix_at(n, batch, 1) * c1)), dim3(256), 0, n->stream,
                       (int)npix_at(n, batch, 1), view(n, G_D1B), view(n, A_D1B), c1);
  }
  wgrad(n, D1B, batch, view(n, A_D1A), view(n, G_D1B));
  conv(n, D1B, batch, view(n, G_D1B), view(n, G_D1A), true, view(n, A_D1A));
  wgrad(n, D1A, batch, view(n, U1), view(n, G_D1A));
  conv(n, D1A, batch, view(n, G_D1A), view(n, G_U1), true, kNoView);
  // u1 = [up(b2b) | e1b]
  {
    const int H = level_h(n->cfg, 2), W = level_w(n->cfg, 2);
    hipLaunchKernelGGL(sur::k_up_back, dim3(grid_for(npix_at(n, batch, 2) * c2)), dim3(256), 0, n->stream, batch, H,
                       W, view(n, G_U1, 0), view(n, G_B2B), c2);
    hipLaunchKernelGGL(sur::k_relu_mask, dim3(grid_for(npix_at(n, batch, 2) * c2)), dim3(256), 0, n->stream,
                       (int)npix_at(n, batch, 2), view(n, G_B2B), view(n, A_B2B), c2);
  }
  wgrad(n, B2B, batch, view(n, A_B2A), view(n, G_B2B));
  conv(n, B2B, batch, view(n, G_B2B), view(n, G_B2A), true, view(n, A_B2A));
  wgrad(n, B2A, batch, view(n, P1), view(n, G_B2A));
  conv(n, B2A, batch, view(n, G_B2A), view(n, G_P1), true, kNoView);
  // d e1b = d(skip slice of u1) + pool adjoint of d p1, then the ReLU of e1b
  {
    const int H = level_h(n->cfg, 1), W = level_w(n->cfg, 1);
    hipLaunchKernelGGL(sur::k_pool_back, dim3(grid_for(npix_at(n, batch, 1) * c1)), dim3(256), 0, n->stream, batch,
                       H, W, view(n, G_P1), view(n, G_U1, c2), c1, 1);
    hipLaunchKernelGGL(sur::k_relu_mask, dim3(grid_for(npix_at(n, batch, 1) * c1)), dim3(256), 0, n->stream,
                       (int)npix_at(n, batch, 1), view(n, G_U1, c2), view(n, U1, c2), c1);
  }
  wgrad(n, E1B, batch, view(n, A_E1A), view(n, G_U1, c2));
  conv(n, E1B, batch, view(n, G_U1, c2), view(n, G_E1A), true, view(n, A_E1A));
  wgrad(n, E1A, batch, view(n, P0), view(n, G_E1A));
  conv(n, E1A, batch, view(n, G_E1A), view(n, G_P0), true, kNoView);
  {
    const int H = level_h(n->cfg, 0), W = level_w(n->cfg, 0);
    hipLaunchKernelGGL(sur::k_pool_back, dim3(grid_for(npix_at(n, batch, 0) * c0)), dim3(256), 0, n->stream, batch,
                       H, W, view(n, G_P0), view(n, G_U0, c1), c0, 1);
    hipLaunchKernelGGL(sur::k_relu_mask, dim3(grid_for(npix_at(n, batch, 0) * c0)), dim3(256), 0, n->stream,
                       (int)npix_at(n, batch, 0), view(n, G_U0, c1), view(n, U0, c1), c0);
  }
  wgrad(n, E0B, batch, view(n, A_E0A), view(n, G_U0, c1));
  conv(n, E0B, batch, view(n, G_U0, c1), view(n, G_E0A), true, view(n, A_E0A));
  wgrad(n, E0A, batch, view(n, XN), view(n, G_E0A));
}

hlb_status batch_ok(sur_net *n, int batch) {
  if (batch < 1 || batch > n->cfg.batch) return sfail(n, HLB_EINVAL, "batch must be in 1..cfg.batch");
  return HLB_OK;
}

hlb_status ssync(sur_net *n) {
  hipError_t e = hipStreamSynchronize(n->stream);
  if (e != hipSuccess) return shf(n, e, "hipStreamSynchronize");
  return HLB_OK;
}

hlb_status scheck(sur_net *n, const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return shf(n, e, what);
  return HLB_OK;
}

void normalise_in(sur_net *n, const float *x, Buf dst, int batch) {
  const long long np = npix_at(n, batch, 0);
  const double *s = n->cfg.scale;
  hipLaunchKernelGGL(sur::k_scale3, dim3(grid_for(np * 3)), dim3(256), 0, n->stream, np, x,
                     at<float>(n, n->lay.buf[dst]), (float)(1.0 / s[0]), (float)(1.0 / s[1]), (float)(1.0 / s[2]));
}

double conv_flops(const sur_net *n, int batch) {
  double f = 0;
  for (int l = 0; l < NLAYER; l++) {
    const LayerSpec &s = n->spec[l];
    f += 2.0 * batch * level_h(n->cfg, s.level) * level_w(n->cfg, s.level) * s.taps * s.cin * s.cout;
  }
  return f;
}

}  // namespace

extern "C" {

hlb_status sur_config_default(sur_config *c) {
  if (!c) return HLB_EINVAL;
  c->batch = 1;
  c->height = c->width = 256;
  c->c0 = 32;
  c->c1 = 64;
  c->c2 = 128;
  c->scale[0] = 1.0;
  c->scale[1] = c->scale[2] = 0.05;
  return HLB_OK;
}

hlb_status sur_param_count(const sur_config *c, size_t *n) {
  if (!n || !config_ok(c)) return sfail(nullptr, HLB_EINVAL, "invalid configuration");
  *n = make_layout(*c).nparam;
  return HLB_OK;
}

hlb_status sur_workspace_size(const sur_config *c, size_t *bytes) {
  if (!bytes || !config_ok(c)) return sfail(nullptr, HLB_EINVAL, "invalid configuration");
  *bytes = make_layout(*c).total;
  return HLB_OK;
}

hlb_status sur_create(sur_net **out, const sur_config *c, void *workspace, size_t bytes, void *stream) {
  if (!out) return sfail(nullptr, HLB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!config_ok(c)) return sfail(nullptr, HLB_EINVAL, "invalid configuration");
  const Layout L = make_layout(*c);
  if (!workspace || bytes < L.total) return sfail(nullptr, HLB_ESHAPE, "workspace missing or too small");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return sfail(nullptr, HLB_EINVAL, "workspace must be 256-byte aligned");
  sur_net *n = new (std::nothrow) sur_net();
  if (!n) return sfail(nullptr, HLB_EINVAL, "out of host memory");
  n->cfg = *c;
  specs(*c, n->spec);
  n->lay = L;
  n->stream = reinterpret_cast<hipStream_t>(stream);
  n->ws = reinterpret_cast<char *>(workspace);
  n->adam_t = 0;
  n->have_grad = false;
  hipError_t e = hipMemsetAsync(n->ws + L.params, 0, L.v + 4 * L.nparam - L.params, n->stream);  // params .. v
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (e != hipSuccess) {
    delete n;
    return sfail(nullptr, HLB_EHIP, std::string("sur_create: ") + hipGetErrorString(e));
  }
  pack_all(n);
  hlb_status s = scheck(n, "pack kernels");
  if (s == HLB_OK) s = ssync(n);
  if (s != HLB_OK) {
    g_sur_error = n->err;
    delete n;
    return s;
  }
  *out = n;
  return HLB_OK;
}

hlb_status sur_set_params(sur_net *n, const float *host) {
  if (!n || !host) return HLB_EINVAL;
  const Layout &L = n->lay;
  hipError_t e = hipMemcpyAsync(n->ws + L.params, host, 4 * L.nparam, hipMemcpyHostToDevice, n->stream);
  if (e == hipSuccess) e = hipMemsetAsync(n->ws + L.m, 0, 4 * L.nparam, n->stream);
  if (e == hipSuccess) e = hipMemsetAsync(n->ws + L.v, 0, 4 * L.nparam, n->stream);
  if (e != hipSuccess) return shf(n, e, "sur_set_params");
  n->adam_t = 0;
  pack_all(n);
  hlb_status s = scheck(n, "pack kernels");
  if (s != HLB_OK) return s;
  return ssync(n);
}

hlb_status sur_get_params(sur_net *n, float *host) {
  if (!n || !host) return HLB_EINVAL;
  hipError_t e = hipMemcpyAsync(host, n->ws + n->lay.params, 4 * n->lay.nparam, hipMemcpyDeviceToHost, n->stream);
  if (e != hipSuccess) return shf(n, e, "sur_get_params");
  return ssync(n);
}

hlb_status sur_forward(sur_net *n, const float *x, float *y, int batch) {
  if (!n || !x || !y) return HLB_EINVAL;
  hlb_status s = batch_ok(n, batch);
  if (s != HLB_OK) return s;
  forward_normalised(n, batch, nullptr, x, y);
  return scheck(n, "forward kernels");
}

hlb_status sur_loss_grad(sur_net *n, const float *x, const float *target, int batch, double *loss,
                         float *host_grads) {
  if (!n || !x || !target) return HLB_EINVAL;
  hlb_status s = batch_ok(n, batch);
  if (s != HLB_OK) return s;
  normalise_in(n, x, XN, batch);
  normalise_in(n, target, TN, batch);
  forward_normalised(n, batch, nullptr);
  const long long ne = npix_at(n, batch, 0) * 3;
  double *lp = at<double>(n, n->lay.lpart);
  hipLaunchKernelGGL(sur::k_mse, dim3(n->lay.nblk_loss), dim3(256), 0, n->stream, ne, at<float>(n, n->lay.buf[YN]),
                     at<float>(n, n->lay.buf[TN]), at<float>(n, n->lay.buf[G_HD]), lp);
  backward(n, batch);
  s = scheck(n, "training kernels");
  if (s != HLB_OK) return s;
  n->have_grad = true;
  if (loss) {
    std::vector<double> part(n->lay.nblk_loss);
    hipError_t e = hipMemcpyAsync(part.data(), lp, 8 * part.size(), hipMemcpyDeviceToHost, n->stream);
    if (e != hipSuccess) return shf(n, e, "hipMemcpyAsync");
    s = ssync(n);
    if (s != HLB_OK) return s;
    double acc = 0;
    for (double v : part) acc += v;
    *loss = acc / (double)ne;
  }
  if (host_grads) {
    hipError_t e = hipMemcpyAsync(host_grads, n->ws + n->lay.grads, 4 * n->lay.nparam, hipMemcpyDeviceToHost,
                                  n->stream);
    if (e != hipSuccess) return shf(n, e, "hipMemcpyAsync");
    s = ssync(n);
    if (s != HLB_OK) return s;
  }
  return HLB_OK;
}

hlb_status sur_adam_step(sur_net *n, double lr, double beta1, double beta2, double eps) {
  if (!n) return HLB_EINVAL;
  if (!n->have_grad) return sfail(n, HLB_ESTATE, "no gradient: call sur_loss_grad first");
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return sfail(n, HLB_EINVAL, "Adam needs lr > 0, 0 <= beta < 1, eps > 0");
  n->adam_t++;
  const double c1 = 1.0 / (1.0 - std::pow(beta1, (double)n->adam_t));
  const double c2 = 1.0 / (1.0 - std::pow(beta2, (double)n->adam_t));
  const Layout &L = n->lay;
  const long long np = (long long)L.nparam;
  hipLaunchKernelGGL(sur::k_adam, dim3(grid_for(np)), dim3(256), 0, n->stream, np, at<float>(n, L.params),
                     at<float>(n, L.m), at<float>(n, L.v), at<float>(n, L.grads), (float)lr, (float)beta1,
                     (float)beta2, (float)eps, (float)c1, (float)c2);
  pack_all(n);
  return scheck(n, "Adam kernels");
}

hlb_status sur_forward_timed(sur_net *n, const float *x, float *y, int batch, int reps, double ms[2],
                             double *flops) {
  if (!n || !x || !y || !ms || reps < 1) return HLB_EINVAL;
  hlb_status s = batch_ok(n, batch);
  if (s != HLB_OK) return s;
  std::vector<hipEvent_t> ev(2 * NLAYER + 2);
  for (auto &e : ev)
    if (hipEventCreate(&e) != hipSuccess) return sfail(n, HLB_EHIP, "hipEventCreate");
  ms[0] = ms[1] = 0;
  for (int r = 0; r < reps && s == HLB_OK; r++) {
    (void)hipEventRecord(ev[2 * NLAYER], n->stream);
    forward_normalised(n, batch, ev.data(), x, y);
    (void)hipEventRecord(ev[2 * NLAYER + 1], n->stream);
    s = scheck(n, "forward kernels");
    if (s == HLB_OK) s = ssync(n);
    if (s != HLB_OK) break;
    float t = 0;
    for (int l = 0; l < NLAYER; l++) {
      (void)hipEventElapsedTime(&t, ev[2 * l], ev[2 * l + 1]);
      ms[0] += t;
    }
    (void)hipEventElapsedTime(&t, ev[2 * NLAYER], ev[2 * NLAYER + 1]);
    ms[1] += t;
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  ms[0] /= reps;
  ms[1] /= reps;
  if (flops) *flops = conv_flops(n, batch);
  return s;
}

const char *sur_last_error(const sur_net *n) { return n ? n->err.c_str() : g_sur_error.c_str(); }

hlb_status sur_destroy(sur_net *n) {
  delete n;
  return HLB_OK;
}

}  // extern "C"
