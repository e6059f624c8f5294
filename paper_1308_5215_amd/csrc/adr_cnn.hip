// Warm-start network for the solver (include/adr_cnn.h): 3x3 convolutions
// on CDNA4 matrix cores (v_mfma_f32_16x16x32_bf16), exact GELU, the MSE
// loss, weight gradients, Adam, and the kernels that build the network's
// input fields from an assembled problem and widen its output into an FP64
// initial guess.
//
// Convolution as a product per tap: for output tile T (16 x 16 nodes),
//   Z[co][p] += sum_ci Wt[co][ci] * In[ci][p + delta_tap]
// with the weights as the MFMA A operand (rows = output channels, 32 input
// channels per tap as K) and the LDS-staged input tile as the B operand
// (columns = 16 nodes of one tile row).  The same kernel computes the input
// gradient of a layer (flipped taps, transposed channel roles).  Weight
// gradients use K = nodes: both operands are staged transposed in LDS
// (channel-major) so that one lane reads 8 consecutive nodes of one channel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/adr_cnn.h"
#include "adr_internal.h"

using namespace adr;

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

namespace {

constexpr int CH = 32;        // channels of every stored activation tensor
constexpr int TS = 16;        // output tile edge (nodes)
constexpr int HALO = TS + 2;  // staged input tile edge
constexpr int NLAYER = 6;
constexpr int NFIELD = 10;   // input fields per node
constexpr int CIN[NLAYER] = {NFIELD, 32, 32, 32, 32, 32};
constexpr int COUT[NLAYER] = {32, 32, 32, 32, 32, 1};
constexpr int WGRAD_MAX_WG = 512;


constexpr int64_t layer_size(int l) { return 9LL * CIN[l] * COUT[l] + COUT[l]; }
constexpr int64_t param_count() {
  int64_t s = 0;
  for (int l = 0; l < NLAYER; ++l) s += layer_size(l);
  return s;
}
constexpr int cout_pad(int l) { return COUT[l] <= 16 ? 16 : 32; }

// ---- bfloat16 (bits in uint16_t), round to nearest even ----
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }
// two values rounded to nearest even by the hardware conversion
// (v_cvt_pk_bf16_f32): the same bits as f2bf for every finite value
__device__ __forceinline__ uint32_t pack2(float a, float b) {
  typedef float v2f __attribute__((ext_vector_type(2)));
  typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f){a, b}, v2bf));
}

// GELU z Phi(z) of the forward pass, erf by Abramowitz & Stegun, Handbook of
// Mathematical Functions, formula 7.1.26 (|error| <= 1.5e-7, far below the
// bfloat16 step the activations are rounded to; one reciprocal, one
// exponential, a degree-5 polynomial), written for Phi directly: with
// a = |z| / sqrt(2), t = 1 / (1 + p a) and h =
// (q(t) / 2) exp(-z^2 / 2), Phi(z) = 1 - h for z >= 0 and h for z < 0 (the
// halves folded into the coefficients), so z Phi(z) = max(z, 0) - |z| h
__device__ __forceinline__ float gelu(float z) {
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, fabsf(z), 1.0f));
  float q = fmaf(0.5f * 1.061405429f, t, 0.5f * -1.453152027f);
  q = fmaf(q, t, 0.5f * 1.421413741f);
  q = fmaf(q, t, 0.5f * -0.284496736f);
  q = fmaf(q, t, 0.5f * 0.254829592f);
  q *= t;
  const float h = q * __builtin_amdgcn_exp2f((z * (-0.5f * 1.4426950408889634f)) * z);
  // z Phi(z) = max(z, 0) - |z| h for either sign of z
  return fmaf(-fabsf(z), h, fmaxf(z, 0.0f));
}
__device__ __forceinline__ float gelu_d(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * (z * z));
  return cdf + z * pdf;
}

__device__ __forceinline__ v8bf as_bf(u32x4 v) { return __builtin_bit_cast(v8bf, v); }

__device__ __forceinline__ v4f mfma(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// FWD_GELU_Z: FWD_GELU that also stores the FP32 pre-activations (training)
enum { FWD_GELU = 0, FWD_OUT = 1, BWD_GELU = 2, FWD_GELU_Z = 3 };

struct ConvArgs {
  const uint16_t *in;    // [B][H][W][32]
  const uint16_t *w;     // [9][COUT][32]: tap, output channel, input channel
  const float *bias;     // [COUT] (forward modes)
  float *z;              // FWD_GELU_Z: pre-activations [B][H][W][32]
  uint16_t *h;           // FWD_GELU(_Z): activations; BWD_GELU: input gradient
  const float *zprev;    // BWD_GELU: pre-activations of the layer below
  float *u;              // FWD_OUT: [B][H][W]
  int H, W, tx, ty, nb;
};

// 16 x 16 output tiles; wave w computes tile rows 4w..4w+3.  Persistent: a
// workgroup loads the layer's weights into registers once and takes tiles
// in turn (dealt per XCD, below); the next tile's input is loaded
// into registers while the current one's products run and is written to the
// other half of a double-buffered LDS tile afterwards.
template <int NOUT, int MODE>
__global__ __launch_bounds__(256, 2) void k_conv(ConvArgs a) {
  constexpr int PS = 40;  // LDS node stride in bf16 (80 B: rows of 16 B reads do not collide)
  constexpr int MB = NOUT / 16;
  constexpr int NLD = (HALO * HALO * 4 + 255) / 256;   // 16-byte staging loads per thread
  __shared__ __attribute__((aligned(16))) uint16_t s_in[2][HALO * HALO * PS];
  // each wave's 4 x 16 output nodes (32 bf16 channels), stored from here with
  // whole-node 16-byte writes instead of four 8-byte pieces per node
  constexpr int OPS = CH + 8;   // node stride in bf16 (80 B)
  __shared__ __attribute__((aligned(16))) uint16_t s_out[4][4 * TS * OPS];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int px = lane & 15, q = lane >> 4;
  const int ntiles = a.nb * a.tx * a.ty;
  // Tiles are dealt per XCD: workgroup b runs on XCD b mod 8 and takes the
  // tiles of that XCD's contiguous eighth of the tile list in turn, so the
  // tiles in flight on one XCD are neighbours and find much of their halo in
  // its L2 (a mapping that only placement depends on, not correctness).
  const int G = gridDim.x;
  const bool by_xcd = (G & 7) == 0 && ntiles >= G;
  const int per = by_xcd ? (ntiles + 7) / 8 : ntiles;   // tiles per XCD
  const int stride = by_xcd ? G / 8 : G;                 // workgroups per XCD
  const int t_lo = by_xcd ? (int)(blockIdx.x & 7) * per : 0;
  const int t_hi = by_xcd ? min(t_lo + per, ntiles) : ntiles;
  int t = t_lo + (by_xcd ? (int)(blockIdx.x >> 3) : (int)blockIdx.x);
  if (t >= t_hi) return;
  auto origin = [&](int tile, int &b, int &y0, int &x0) {
    const int tpx = tile % a.tx, rest = tile / a.tx;
    const int tpy = rest % a.ty;
    b = rest / a.ty;
    y0 = tpy * TS;
    x0 = tpx * TS;
  };
  u32x4 pre[NLD];
  // byte offset of each staging load from the halo tile's first node, the
  // same for every tile
  unsigned hoff[NLD];
#pragma unroll
  for (int k = 0; k < NLD; ++k) {
    const int i = tid + k * 256, node = i >> 2, r = node / HALO;
    hoff[k] = (unsigned)(((r * a.W + (node - r * HALO)) * CH + (i & 3) * 8) * 2);
  }
  auto fetch = [&](int tile, u32x4 (&pre)[NLD]) {
    int b, y0, x0;
    origin(tile, b, y0, x0);
    if (y0 >= 1 && x0 >= 1 && y0 + HALO - 1 <= a.H && x0 + HALO - 1 <= a.W) {
      // the whole halo lies in the grid: no bounds tests
      const char *tb = (const char *)(a.in + (((size_t)b * a.H + (y0 - 1)) * a.W + (x0 - 1)) * CH);
#pragma unroll
      for (int k = 0; k < NLD; ++k) {
        pre[k] = u32x4{0u, 0u, 0u, 0u};
        if (tid + k * 256 < HALO * HALO * 4) pre[k] = *(const u32x4 *)(tb + hoff[k]);
      }
      return;
    }
    const uint16_t *inb = a.in + (size_t)b * a.H * a.W * CH;
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int i = tid + k * 256;
      const int c8 = i & 3, node = i >> 2;
      const int r = node / HALO, c = node - r * HALO;
      const int gy = y0 + r - 1, gx = x0 + c - 1;
      pre[k] = u32x4{0u, 0u, 0u, 0u};
      if (i < HALO * HALO * 4 && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
        pre[k] = *(const u32x4 *)(inb + ((size_t)gy * a.W + gx) * CH + c8 * 8);
    }
  };
  auto put = [&](int buf, const u32x4 (&pre)[NLD]) {
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int i = tid + k * 256;
      if (i < HALO * HALO * 4) *(u32x4 *)(&s_in[buf][0] + (i >> 2) * PS + (i & 3) * 8) = pre[k];
    }
  };
  v8bf wa[9][MB];
#pragma unroll
  for (int tp = 0; tp < 9; ++tp)
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      wa[tp][mb] = as_bf(*(const u32x4 *)(a.w + ((size_t)(tp * NOUT + mb * 16 + px)) * CH + q * 8));
  v4f acc0[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const int co = mb * 16 + 4 * q;
    acc0[mb] = MODE == BWD_GELU ? v4f{0.f, 0.f, 0.f, 0.f}
                                : (MODE == FWD_OUT ? v4f{a.bias[0], 0.f, 0.f, 0.f}
                                                   : v4f{a.bias[co], a.bias[co + 1], a.bias[co + 2], a.bias[co + 3]});
  }
  fetch(t, pre);
  put(0, pre);
  // step for tile t from LDS half `buf`: the workgroup's next tile (t +
  // stride) is fetched into registers while it runs and put into the other
  // half afterwards
  auto step = [&](int buf) {
    const int tn = t + stride;
    if (tn < t_hi) fetch(tn, pre);
    __syncthreads();              // this tile staged; the other half no longer read
    int b, y0, x0;
    origin(t, b, y0, x0);
    const uint16_t *sb = &s_in[buf][0];
    // forward: the accumulators start at the bias
    v4f acc[4][MB];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) acc[r][mb] = acc0[mb];
    // taps outside, rows inside: 4 MB independent accumulations in flight.
    // The products run at raised issue priority, so that a wave in this
    // phase gets its matrix instructions issued while the other workgroup's
    // wave on the SIMD is in its VALU-bound epilogue.
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int tp = 0; tp < 9; ++tp) {
      const int dy = tp / 3, dx = tp % 3;
      v8bf bv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
        bv[r] = as_bf(*(const u32x4 *)(sb + ((wv * 4 + r + dy) * HALO + px + dx) * PS + q * 8));
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[r][mb] = mfma(wa[tp][mb], bv[r], acc[r][mb]);
    }
    __builtin_amdgcn_s_setprio(0);
    // lane holds channels mb*16 + 4q + i of node (row, px)
    uint16_t *so = &s_out[wv][0];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gy = y0 + wv * 4 + r, gx = x0 + px;
      const size_t node = ((size_t)b * a.H + min(gy, a.H - 1)) * a.W + min(gx, a.W - 1);
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int co = mb * 16 + 4 * q;
        const v4f s = acc[r][mb];
        u32x2 hv = u32x2{0u, 0u};
        if (MODE == FWD_GELU || MODE == FWD_GELU_Z) {
          if (MODE == FWD_GELU_Z && gy < a.H && gx < a.W) *(v4f *)(a.z + node * CH + co) = s;
          hv = u32x2{pack2(gelu(s[0]), gelu(s[1])), pack2(gelu(s[2]), gelu(s[3]))};
        } else if (MODE == FWD_OUT) {
          if (mb == 0 && q == 0 && gy < a.H && gx < a.W) a.u[node] = s[0];
        } else {
          const v4f zp = *(const v4f *)(a.zprev + node * CH + co);
          const float g0 = s[0] * gelu_d(zp[0]), g1 = s[1] * gelu_d(zp[1]);
          const float g2 = s[2] * gelu_d(zp[2]), g3 = s[3] * gelu_d(zp[3]);
          hv = u32x2{pack2(g0, g1), pack2(g2, g3)};
        }
        if (MODE != FWD_OUT) *(u32x2 *)(so + (r * TS + px) * OPS + co) = hv;
      }
    }
    if (MODE != FWD_OUT) {
      // the wave reads back what its own lanes wrote: no workgroup barrier
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
      const int nl = lane >> 2, c8 = lane & 3;   // node of the row, 16-byte chunk
      if (y0 + TS <= a.H && x0 + TS <= a.W) {
        // every node of the tile is in the grid
        char *ob = (char *)(a.h + (((size_t)b * a.H + y0 + wv * 4) * a.W + x0) * CH);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          *(u32x4 *)(ob + ((unsigned)((r * a.W + nl) * CH + c8 * 8) * 2u)) =
              *(const u32x4 *)(so + (r * TS + nl) * OPS + c8 * 8);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gy = y0 + wv * 4 + r, gx = x0 + nl;
          const u32x4 v = *(const u32x4 *)(so + (r * TS + nl) * OPS + c8 * 8);
          if (gy < a.H && gx < a.W) *(u32x4 *)(a.h + (((size_t)b * a.H + gy) * a.W + gx) * CH + c8 * 8) = v;
        }
      }
    }
    if (tn < t_hi) put(buf ^ 1, pre);
  };
  for (int buf = 0; t < t_hi; t += stride, buf ^= 1) step(buf);
}

struct WgArgs {
  const uint16_t *h;     // layer input [B][H][W][32]
  const uint16_t *g;     // gradient of the layer's pre-activation [B][H][W][32]
  float *part;           // [gridDim.x][9*NOUT*32 + NOUT]
  int H, W, tx, ty, ntiles;
};

// Weight and bias gradient partials: workgroup k accumulates the tiles
// k, k + gridDim.x, ... ; wave w takes the taps of kernel row w.
template <int NOUT>
__global__ __launch_bounds__(192) void k_wgrad(WgArgs a) {
  constexpr int MB = NOUT / 16;
  constexpr int GP = TS * TS + 8;     // per-channel pitch of the gradient tile (bf16)
  constexpr int HP = HALO * TS + 8;   // per-channel pitch of each shifted input copy (bf16)
  constexpr int NG = NOUT / 8;        // 16 B chunks per node of the gradient
  __shared__ __attribute__((aligned(16))) uint16_t s_g[NOUT * GP];
  __shared__ __attribute__((aligned(16))) uint16_t s_h[3 * CH * HP];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int px = lane & 15, q = lane >> 4;
  v4f acc[3][MB][2];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) acc[d][mb][nb] = v4f{0.f, 0.f, 0.f, 0.f};
  float bsum[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) bsum[e] = 0.f;
  const int per = a.tx * a.ty;
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const int b = t / per, rem = t - b * per;
    const int tpy = rem / a.tx, tpx = rem - tpy * a.tx;
    const int y0 = tpy * TS, x0 = tpx * TS;
    const size_t base = (size_t)b * a.H * a.W;
    __syncthreads();
    for (int i = tid; i < TS * TS * NG; i += 192) {
      const int cg = i % NG, node = i / NG;
      const int r = node / TS, c = node - r * TS;
      const int gy = y0 + r, gx = x0 + c;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (gy < a.H && gx < a.W) v = *(const u32x4 *)(a.g + (base + (size_t)gy * a.W + gx) * CH + cg * 8);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t hv = (v[e >> 1] >> (16 * (e & 1))) & 0xffffu;
        s_g[(cg * 8 + e) * GP + r * TS + c] = (uint16_t)hv;
        bsum[e] += bf2f(hv);
      }
    }
    for (int i = tid; i < HALO * HALO * 4; i += 192) {
      const int cg = i & 3, node = i >> 2;
      const int r = node / HALO, c = node - r * HALO;
      const int gy = y0 + r - 1, gx = x0 + c - 1;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
        v = *(const u32x4 *)(a.h + (base + (size_t)gy * a.W + gx) * CH + cg * 8);
      // copy d holds column c - d: the input that tap column d reads at tile column c - d
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int col = c - d;
        if (col < 0 || col >= TS) continue;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          s_h[(d * CH + cg * 8 + e) * HP + r * TS + col] = (uint16_t)((v[e >> 1] >> (16 * (e & 1))) & 0xffffu);
      }
    }
    __syncthreads();
    // K = 32 nodes: tile rows 2kb and 2kb + 1; lane group q takes 8 nodes
#pragma unroll 2
    for (int kb = 0; kb < TS / 2; ++kb) {
      const int r = 2 * kb + (q >> 1), c0 = (q & 1) * 8;
      v8bf ga[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) ga[mb] = as_bf(*(const u32x4 *)(s_g + (mb * 16 + px) * GP + r * TS + c0));
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const v8bf hb = as_bf(*(const u32x4 *)(s_h + (d * CH + nb * 16 + px) * HP + (r + wv) * TS + c0));
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) acc[d][mb][nb] = mfma(ga[mb], hb, acc[d][mb][nb]);
        }
    }
  }
  float *pb = a.part + (size_t)blockIdx.x * (9 * NOUT * CH + NOUT);
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          pb[((wv * 3 + d) * NOUT + mb * 16 + 4 * q + i) * CH + nb * 16 + px] = acc[d][mb][nb][i];
  // bias: thread tid always staged channel group tid % NG (192 is a multiple of NG)
  __syncthreads();
  float *s_b = (float *)s_h;
#pragma unroll
  for (int e = 0; e < 8; ++e) s_b[tid * 8 + e] = bsum[e];
  __syncthreads();
  if (tid < NOUT) {
    const int cg = tid / 8, e = tid % 8;
    float s = 0.f;
    for (int t2 = cg; t2 < 192; t2 += NG) s += s_b[t2 * 8 + e];
    pb[9 * NOUT * CH + tid] = s;
  }
}

// Sum the workgroup partials in FP64 in workgroup order and scatter into the
// packed gradient of one layer.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *part, int nwg, int nout, int cin, int cout,
                                                      float *grad) {
  const int per = 9 * nout * CH + nout;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= per) return;
  double s = 0.0;
  for (int w = 0; w < nwg; ++w) s += (double)part[(size_t)w * per + e];
  if (e < 9 * nout * CH) {
    const int t = e / (nout * CH), rem = e - t * nout * CH;
    const int co = rem / CH, ci = rem - co * CH;
    if (co < cout && ci < cin) grad[((size_t)t * cin + ci) * cout + co] = (float)s;
  } else {
    const int co = e - 9 * nout * CH;
    if (co < cout) grad[(size_t)9 * cin * cout + co] = (float)s;
  }
}

// Loss gradient of the output (channel 0 of a 32-channel tensor) and the
// per-block partial sums of the squared error.
__global__ __launch_bounds__(256) void k_loss(const float *u, const float *target, uint16_t *g, int nb, int H,
                                              int W, float scale, double *part) {
  const int64_t total = (int64_t)nb * H * W;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double e2 = 0.0;
  if (k < total) {
    const int col = (int)(k % W);
    const int64_t t2 = k / W;
    const int row = (int)(t2 % H), b = (int)(t2 / H);
    float gv = 0.f;
    if (row >= 1 && row <= H - 2 && col >= 1 && col <= W - 2) {
      const float d = u[k] - target[((int64_t)b * (H - 2) + (row - 1)) * (W - 2) + (col - 1)];
      gv = (2.0f * d) * scale;
      e2 = (double)d * (double)d;
    }
    u32x4 *gp = (u32x4 *)(g + k * CH);
    gp[0] = u32x4{(uint32_t)f2bf(gv), 0u, 0u, 0u};
    gp[1] = u32x4{0u, 0u, 0u, 0u};
    gp[2] = u32x4{0u, 0u, 0u, 0u};
    gp[3] = u32x4{0u, 0u, 0u, 0u};
  }
  __shared__ double s[256];
  s[threadIdx.x] = e2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}
__global__ __launch_bounds__(256) void k_loss_fin(const double *part, int n, double scale, double *out) {
  __shared__ double s[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += part[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0] * scale;
}

struct LayerDev {
  int64_t off;          // offset in the packed parameters
  int cin, cout, nout;  // real channels, padded output channels
  uint16_t *wf;         // forward weights [9][nout][32]
  uint16_t *wd;         // input-gradient weights [9][32][32] (null for the first layer)
  float *bias;          // [nout]
};
struct NetDev {
  LayerDev L[NLAYER];
};

// Adam on the packed FP32 parameters (update = 0: only republish), then the
// bfloat16 copies the convolutions read.
__global__ __launch_bounds__(256) void k_adam(NetDev nd, float *param, const float *grad, float *m, float *v,
                                              int64_t n, int update, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float p = param[i];
  if (update) {
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * (g * g);
    m[i] = mi;
    v[i] = vi;
    p = p - lr * ((mi * c1) / (sqrtf(vi * c2) + eps));
    param[i] = p;
  }
  int l = 0;
  while (l + 1 < NLAYER && i >= nd.L[l + 1].off) ++l;
  const LayerDev &L = nd.L[l];
  const int64_t li = i - L.off;
  const int64_t nw = 9LL * L.cin * L.cout;
  if (li < nw) {
    const int t = (int)(li / (L.cin * L.cout));
    const int rem = (int)(li - (int64_t)t * L.cin * L.cout);
    const int ci = rem / L.cout, co = rem - ci * L.cout;
    const uint16_t hb = f2bf(p);
    L.wf[((size_t)t * L.nout + co) * CH + ci] = hb;
    if (L.wd) L.wd[((size_t)(8 - t) * CH + ci) * CH + co] = hb;
  } else {
    L.bias[li - nw] = p;
  }
}

// ---- input fields and the FP64 guess ----
__global__ __launch_bounds__(256) void k_features(const FeatInst *fi, int count, int H, int W, const double *F,
                                                  uint16_t *out) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= (int64_t)count * H * W) return;
  const int I = (int)(k % W);
  const int64_t t2 = k / W;
  const int J = (int)(t2 % H), b = (int)(t2 / H);
  const FeatInst P = fi[b];
  const int nx = P.nx, ny = P.ny;
  const double dx = P.X / (double)(nx + 1), dy = P.Y / (double)(ny + 1);
  const double x = (double)I * dx, y = (double)J * dy;
  const double av = 1.0 + x * x, bv = P.X * exp(-y);
  double fv, mask;
  const bool interior = I >= 1 && I <= nx && J >= 1 && J <= ny;
  if (interior) {
    fv = F[P.off + (int64_t)(J - 1) * nx + (I - 1)] / 10.0;
    mask = 0.0;
  } else {
    const bool neu_x = P.bc == 1 && I == nx + 1 && J >= 1;
    const bool neu_y = P.bc == 1 && J == ny + 1 && I >= 1;
    if (neu_x && neu_y) {
      fv = 0.0;
      mask = -1.0;
    } else if (neu_x) {  // du/dx on x = X
      fv = (-1.0 / P.X) * exp(-1.0) * (1.0 - exp(-y / P.Y)) * y;
      mask = -1.0;
    } else if (neu_y) {  // du/dy on y = Y
      fv = exp(-x / P.X);
      mask = -1.0;
    } else {
      fv = exp(-x / P.X) * (1.0 - exp(-y / P.Y)) * y;
      mask = 1.0;
    }
  }
  u32x4 *o = (u32x4 *)(out + k * CH);
  o[0] = u32x4{pack2((float)(av / 5.0), (float)(bv / 2.0)), pack2((float)fv, (float)(log10(P.eps) / 3.0)),
               pack2((float)mask, (float)(x / P.X)), pack2((float)(y / P.Y), (float)(P.X / 2.0))};
  o[1] = u32x4{pack2((float)(P.Y / 2.0), (float)P.scheme), 0u, 0u, 0u};
  o[2] = u32x4{0u, 0u, 0u, 0u};
  o[3] = u32x4{0u, 0u, 0u, 0u};
}

__global__ __launch_bounds__(256) void k_extract(const FeatInst *fi, int count, int H, int W, const float *u,
                                                 double *x) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int nx = W - 2, ny = H - 2;
  if (k >= (int64_t)count * nx * ny) return;
  const int i = (int)(k % nx);
  const int64_t t2 = k / nx;
  const int j = (int)(t2 % ny), b = (int)(t2 / ny);
  x[fi[b].off + (int64_t)j * nx + i] = (double)u[((int64_t)b * H + (j + 1)) * W + (i + 1)];
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

namespace adr {
hipError_t launch_cnn_features(const FeatInst *fi_dev, int count, int H, int W, const double *F,
                               uint16_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3(blocks_for((int64_t)count * H * W)), dim3(256), 0, s, fi_dev, count, H, W,
                     F, out);
  return hipGetLastError();
}
hipError_t launch_cnn_extract(const FeatInst *fi_dev, int count, int H, int W, const float *u, double *x,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_extract, dim3(blocks_for((int64_t)count * (H - 2) * (W - 2))), dim3(256), 0, s, fi_dev,
                     count, H, W, u, x);
  return hipGetLastError();
}
}  // namespace adr

struct adr_cnn {
  int H = 0, W = 0, maxB = 0, tx = 0, ty = 0;
  int cus = 256;                    // compute units of the device (persistent grid size)
  hipStream_t stream = nullptr;
  float *param = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *wf[NLAYER] = {}, *wd[NLAYER] = {};
  float *bias[NLAYER] = {};
  float *z[NLAYER - 1] = {};        // pre-activations of the hidden layers
  uint16_t *act[NLAYER - 1] = {};   // their bf16 activations
  float *u = nullptr;               // output [maxB][H][W]
  uint16_t *g[2] = {};              // gradients entering a convolution (ping-pong)
  uint16_t *in = nullptr;           // input fields for the warm start
  float *part = nullptr;            // weight-gradient partials
  double *lpart = nullptr, *loss = nullptr;
  int64_t step = 0;
  bool have_grad = false;

  NetDev dev() const {
    NetDev nd;
    int64_t off = 0;
    for (int l = 0; l < NLAYER; ++l) {
      nd.L[l].off = off;
      nd.L[l].cin = CIN[l];
      nd.L[l].cout = COUT[l];
      nd.L[l].nout = cout_pad(l);
      nd.L[l].wf = wf[l];
      nd.L[l].wd = wd[l];
      nd.L[l].bias = bias[l];
      off += layer_size(l);
    }
    return nd;
  }
};

namespace {

#define CNN_TRY(expr)                                                                                      \
  do {                                                                                                     \
    hipError_t e_ = (expr);                                                                                \
    if (e_ != hipSuccess) {                                                                                \
      (void)hipGetLastError();                                                                             \
      return (adr_status)set_error(e_ == hipErrorOutOfMemory ? ADR_ERR_NOMEM : ADR_ERR_DEVICE, "%s: %s (%s:%d)", \
                                   #expr, hipGetErrorString(e_), __FILE__, __LINE__);                      \
    }                                                                                                      \
  } while (0)

template <class T>
hipError_t zalloc(T **p, size_t count) {
  *p = nullptr;
  hipError_t e = hipMalloc((void **)p, (count ? count : 1) * sizeof(T));
  if (e == hipSuccess) e = hipMemset(*p, 0, (count ? count : 1) * sizeof(T));
  return e;
}

int wgrad_blocks(int ntiles) { return ntiles < WGRAD_MAX_WG ? ntiles : WGRAD_MAX_WG; }

hipError_t conv(const adr_cnn *N, int mode, int nout, const uint16_t *in, const uint16_t *w, const float *bias,
                float *z, uint16_t *h, const float *zprev, float *u, int nb) {
  ConvArgs a;
  a.in = in;
  a.w = w;
  a.bias = bias;
  a.z = z;
  a.h = h;
  a.zprev = zprev;
  a.u = u;
  a.H = N->H;
  a.W = N->W;
  a.tx = N->tx;
  a.ty = N->ty;
  a.nb = nb;
  // persistent workgroups, as many as are resident at once (two per CU: the
  // kernels hold the layer's weights in registers)
  const int ntiles = nb * N->tx * N->ty;
  const dim3 grid((unsigned)std::min(ntiles, 2 * N->cus)), blk(256);
  if (mode == FWD_GELU && nout == 32 && z)
    hipLaunchKernelGGL((k_conv<32, FWD_GELU_Z>), grid, blk, 0, N->stream, a);
  else if (mode == FWD_GELU && nout == 32)
    hipLaunchKernelGGL((k_conv<32, FWD_GELU>), grid, blk, 0, N->stream, a);
  else if (mode == FWD_OUT && nout == 16)
    hipLaunchKernelGGL((k_conv<16, FWD_OUT>), grid, blk, 0, N->stream, a);
  else if (mode == BWD_GELU && nout == 32)
    hipLaunchKernelGGL((k_conv<32, BWD_GELU>), grid, blk, 0, N->stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t forward(adr_cnn *N, const uint16_t *in, int nb, float *u, bool keep_z) {
  const uint16_t *x = in;
  for (int l = 0; l < NLAYER - 1; ++l) {
    hipError_t e = conv(N, FWD_GELU, 32, x, N->wf[l], N->bias[l], keep_z ? N->z[l] : nullptr, N->act[l], nullptr,
                        nullptr, nb);
    if (e != hipSuccess) return e;
    x = N->act[l];
  }
  return conv(N, FWD_OUT, 16, x, N->wf[NLAYER - 1], N->bias[NLAYER - 1], nullptr, nullptr, nullptr, u, nb);
}

hipError_t wgrad(adr_cnn *N, int l, const uint16_t *h, const uint16_t *g, int nb, int64_t off) {
  WgArgs a;
  a.h = h;
  a.g = g;
  a.part = N->part;
  a.H = N->H;
  a.W = N->W;
  a.tx = N->tx;
  a.ty = N->ty;
  a.ntiles = nb * N->tx * N->ty;
  const int nwg = wgrad_blocks(a.ntiles);
  const int nout = cout_pad(l);
  if (nout == 32)
    hipLaunchKernelGGL(k_wgrad<32>, dim3(nwg), dim3(192), 0, N->stream, a);
  else
    hipLaunchKernelGGL(k_wgrad<16>, dim3(nwg), dim3(192), 0, N->stream, a);
  const int per = 9 * nout * CH + nout;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks_for(per)), dim3(256), 0, N->stream, (const float *)N->part, nwg,
                     nout, CIN[l], COUT[l], N->grad + off);
  return hipGetLastError();
}

adr_status check_batch(const adr_cnn *N, int nb) {
  if (!N) return (adr_status)set_error(ADR_ERR_ARG, "network is NULL");
  if (nb < 1 || nb > N->maxB)
    return (adr_status)set_error(ADR_ERR_ARG, "batch must be in [1, %d] (got %d)", N->maxB, nb);
  return ADR_OK;
}

}  // namespace

extern "C" {

int64_t adr_cnn_param_count(void) { return param_count(); }

void adr_cnn_destroy(adr_cnn *N) {
  if (!N) return;
  if (N->stream) (void)hipStreamSynchronize(N->stream);
  void *ptrs[] = {N->param, N->grad, N->m, N->v, N->u, N->g[0], N->g[1], N->in, N->part, N->lpart, N->loss};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  for (int l = 0; l < NLAYER; ++l) {
    if (N->wf[l]) (void)hipFree(N->wf[l]);
    if (N->wd[l]) (void)hipFree(N->wd[l]);
    if (N->bias[l]) (void)hipFree(N->bias[l]);
  }
  for (int l = 0; l < NLAYER - 1; ++l) {
    if (N->z[l]) (void)hipFree(N->z[l]);
    if (N->act[l]) (void)hipFree(N->act[l]);
  }
  delete N;
}

adr_status adr_cnn_create(int32_t height, int32_t width, int32_t max_batch, void *stream, adr_cnn **out) {
  clear_error();
  if (!out) return (adr_status)set_error(ADR_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (height < 3 || width < 3 || max_batch < 1)
    return (adr_status)set_error(ADR_ERR_ARG, "height, width must be >= 3 and max_batch >= 1 (got %d, %d, %d)",
                                 height, width, max_batch);
  const int64_t nodes = (int64_t)height * width * max_batch;
  if (nodes * CH > ((int64_t)1 << 40))
    return (adr_status)set_error(ADR_ERR_ARG, "network buffers too large");
  adr_cnn *N = new adr_cnn();
  N->H = height;
  N->W = width;
  N->maxB = max_batch;
  N->tx = (width + TS - 1) / TS;
  N->ty = (height + TS - 1) / TS;
  N->stream = (hipStream_t)stream;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      N->cus = cus;
  }
  auto bail = [&](hipError_t e) {
    adr_cnn_destroy(N);
    return (adr_status)set_error(e == hipErrorOutOfMemory ? ADR_ERR_NOMEM : ADR_ERR_DEVICE,
                                 "network allocation failed: %s", hipGetErrorString(e));
  };
  const int64_t np = param_count();
  hipError_t e = hipSuccess;
  float **pv[] = {&N->param, &N->grad, &N->m, &N->v};
  for (float **p : pv)
    if (e == hipSuccess) e = zalloc(p, (size_t)np);
  for (int l = 0; l < NLAYER && e == hipSuccess; ++l) {
    e = zalloc(&N->wf[l], (size_t)9 * cout_pad(l) * CH);
    if (e == hipSuccess && l > 0) e = zalloc(&N->wd[l], (size_t)9 * CH * CH);
    if (e == hipSuccess) e = zalloc(&N->bias[l], (size_t)cout_pad(l));
  }
  for (int l = 0; l < NLAYER - 1 && e == hipSuccess; ++l) {
    e = zalloc(&N->z[l], (size_t)nodes * CH);
    if (e == hipSuccess) e = zalloc(&N->act[l], (size_t)nodes * CH);
  }
  if (e == hipSuccess) e = zalloc(&N->u, (size_t)nodes);
  if (e == hipSuccess) e = zalloc(&N->g[0], (size_t)nodes * CH);
  if (e == hipSuccess) e = zalloc(&N->g[1], (size_t)nodes * CH);
  if (e == hipSuccess) e = zalloc(&N->in, (size_t)nodes * CH);
  if (e == hipSuccess) e = zalloc(&N->part, (size_t)WGRAD_MAX_WG * (9 * 32 * CH + 32));
  if (e == hipSuccess) e = zalloc(&N->lpart, (size_t)blocks_for(nodes));
  if (e == hipSuccess) e = zalloc(&N->loss, 1);
  if (e != hipSuccess) return bail(e);
  *out = N;
  return ADR_OK;
}

adr_status adr_cnn_set_params(adr_cnn *N, const float *params) {
  clear_error();
  if (!N || !params) return (adr_status)set_error(ADR_ERR_ARG, "NULL argument");
  const int64_t np = param_count();
  CNN_TRY(hipMemcpyAsync(N->param, params, (size_t)np * sizeof(float), hipMemcpyHostToDevice, N->stream));
  CNN_TRY(hipMemsetAsync(N->m, 0, (size_t)np * sizeof(float), N->stream));
  CNN_TRY(hipMemsetAsync(N->v, 0, (size_t)np * sizeof(float), N->stream));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(np)), dim3(256), 0, N->stream, N->dev(), N->param,
                     (const float *)N->grad, N->m, N->v, np, 0, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f);
  CNN_TRY(hipGetLastError());
  CNN_TRY(hipStreamSynchronize(N->stream));
  N->step = 0;
  N->have_grad = false;
  return ADR_OK;
}

adr_status adr_cnn_get_params(const adr_cnn *N, float *params) {
  clear_error();
  if (!N || !params) return (adr_status)set_error(ADR_ERR_ARG, "NULL argument");
  CNN_TRY(hipMemcpyAsync(params, N->param, (size_t)param_count() * sizeof(float), hipMemcpyDeviceToHost,
                         N->stream));
  CNN_TRY(hipStreamSynchronize(N->stream));
  return ADR_OK;
}

adr_status adr_cnn_forward(adr_cnn *N, const uint16_t *in, int32_t nb, float *u) {
  clear_error();
  adr_status st = check_batch(N, nb);
  if (st != ADR_OK) return st;
  if (!in || !u) return (adr_status)set_error(ADR_ERR_ARG, "NULL device pointer");
  CNN_TRY(forward(N, in, nb, u, false));
  CNN_TRY(hipStreamSynchronize(N->stream));
  return ADR_OK;
}

adr_status adr_cnn_gradient(adr_cnn *N, const uint16_t *in, const float *target, int32_t nb, float *u_out,
                            float *grad_host, double *loss_host) {
  clear_error();
  adr_status st = check_batch(N, nb);
  if (st != ADR_OK) return st;
  if (!in || !target) return (adr_status)set_error(ADR_ERR_ARG, "NULL device pointer");
  CNN_TRY(forward(N, in, nb, N->u, true));
  const int64_t nodes = (int64_t)nb * N->H * N->W;
  const double count = (double)nb * (N->H - 2) * (N->W - 2);
  const unsigned lb = blocks_for(nodes);
  hipLaunchKernelGGL(k_loss, dim3(lb), dim3(256), 0, N->stream, (const float *)N->u, target, N->g[0], nb, N->H,
                     N->W, (float)(1.0 / count), N->lpart);
  hipLaunchKernelGGL(k_loss_fin, dim3(1), dim3(256), 0, N->stream, (const double *)N->lpart, (int)lb, 1.0 / count,
                     N->loss);
  CNN_TRY(hipGetLastError());
  // backward: layer l's gradient sits in g[cur]; its input is act[l-1] (or the network input)
  const NetDev nd = N->dev();
  int cur = 0;
  for (int l = NLAYER - 1; l >= 0; --l) {
    const uint16_t *hin = l > 0 ? N->act[l - 1] : in;
    CNN_TRY(wgrad(N, l, hin, N->g[cur], nb, nd.L[l].off));
    if (l > 0) {
      CNN_TRY(conv(N, BWD_GELU, 32, N->g[cur], N->wd[l], nullptr, nullptr, N->g[cur ^ 1], N->z[l - 1], nullptr, nb));
      cur ^= 1;
    }
  }
  if (u_out)
    CNN_TRY(hipMemcpyAsync(u_out, N->u, (size_t)nodes * sizeof(float), hipMemcpyDeviceToDevice, N->stream));
  if (grad_host)
    CNN_TRY(hipMemcpyAsync(grad_host, N->grad, (size_t)param_count() * sizeof(float), hipMemcpyDeviceToHost,
                           N->stream));
  double loss = 0.0;
  CNN_TRY(hipMemcpyAsync(&loss, N->loss, sizeof(double), hipMemcpyDeviceToHost, N->stream));
  CNN_TRY(hipStreamSynchronize(N->stream));
  if (loss_host) *loss_host = loss;
  N->have_grad = true;
  return ADR_OK;
}

adr_status adr_cnn_adam(adr_cnn *N, float lr, float beta1, float beta2, float eps) {
  clear_error();
  if (!N) return (adr_status)set_error(ADR_ERR_ARG, "network is NULL");
  if (!N->have_grad) return (adr_status)set_error(ADR_ERR_STATE, "no gradient (call adr_cnn_gradient first)");
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return (adr_status)set_error(ADR_ERR_ARG, "bad Adam hyper-parameters");
  N->step += 1;
  const double c1 = 1.0 / (1.0 - std::pow((double)beta1, (double)N->step));
  const double c2 = 1.0 / (1.0 - std::pow((double)beta2, (double)N->step));
  const int64_t np = param_count();
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(np)), dim3(256), 0, N->stream, N->dev(), N->param,
                     (const float *)N->grad, N->m, N->v, np, 1, lr, beta1, beta2, eps, (float)c1, (float)c2);
  CNN_TRY(hipGetLastError());
  CNN_TRY(hipStreamSynchronize(N->stream));
  return ADR_OK;
}

adr_status adr_cnn_train_step(adr_cnn *N, const uint16_t *in, const float *target, int32_t nb, float lr,
                              double *loss_host) {
  adr_status st = adr_cnn_gradient(N, in, target, nb, nullptr, nullptr, loss_host);
  if (st != ADR_OK) return st;
  return adr_cnn_adam(N, lr, 0.9f, 0.999f, 1e-8f);
}

}  // extern "C"

namespace adr {
void cnn_shape(const adr_cnn *N, int *H, int *W, int *maxB, hipStream_t *s, uint16_t **in, float **u) {
  *H = N->H;
  *W = N->W;
  *maxB = N->maxB;
  *s = N->stream;
  *in = N->in;
  *u = N->u;
}
}  // namespace adr
