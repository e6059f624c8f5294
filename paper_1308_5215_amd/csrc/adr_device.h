// Device helpers shared by the streaming kernels (adr_kernels.hip) and the
// wavefront kernels (adr_sweeps.hip): double-double accumulation, block
// reductions of per-block partial sums, the five-point stencil at one point,
// and the batch and launch-geometry lookups.
#pragma once

#include <hip/hip_runtime.h>

#include "adr_internal.h"

#pragma clang fp contract(off)

namespace adr {

constexpr int BLK = 256;     // threads per block of the streaming kernels
constexpr int MAXSLOT = 4;   // partial-sum slots per block (3 dd sums + 1 max)

// ---------------------------------------------------------------------------
// Double-double arithmetic: TwoSum (Knuth), FastTwoSum (Dekker), TwoProd by
// fma, and the accurate double-word addition of Joldes, Muller & Popescu
// (ACM TOMS 2017).  An inner product accumulated this way and rounded once is
// the exact inner product rounded to nearest up to O(n u^2) sum|x_k y_k|, so
// it does not depend on how the sum is split over blocks and lanes.
// ---------------------------------------------------------------------------
struct dd {
  double hi, lo;
};

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void fast_two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  e = b - (s - a);
}
__device__ __forceinline__ dd dd_add(dd x, dd y) {
  double sh, sl, th, tl, vh, vl;
  two_sum(x.hi, y.hi, sh, sl);
  two_sum(x.lo, y.lo, th, tl);
  const double c = sl + th;
  fast_two_sum(sh, c, vh, vl);
  const double w = tl + vl;
  dd z;
  fast_two_sum(vh, w, z.hi, z.lo);
  return z;
}
__device__ __forceinline__ dd dd_prod(double a, double b) {
  const double p = a * b;
  return dd{p, fma(a, b, -p)};
}
__device__ __forceinline__ double nanmax(double a, double b) {
  return (a != a) ? a : ((b != b) ? b : (a > b ? a : b));
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) {
  return __shfl_xor(v, m, 64);
}
__device__ __forceinline__ dd wave_reduce_dd(dd v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    dd o{shfl_xor_d(v.hi, m), shfl_xor_d(v.lo, m)};
    v = dd_add(v, o);
  }
  return v;
}
__device__ __forceinline__ double wave_reduce_max(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = nanmax(v, shfl_xor_d(v, m));
  return v;
}

// Reduce NS dd values and one max over a block of NT threads; thread 0
// writes them to partials[(SLOT0 + q) * nblk + block] (q < NS) and the max
// to slot 3.
template <int NS, bool MAX, int NT = BLK, int SLOT0 = 0>
__device__ __forceinline__ void block_partials(const dd (&v)[NS > 0 ? NS : 1], double mx,
                                               double2 *partials, int nblk, int bid) {
  __shared__ dd sh[NS > 0 ? NS : 1][NT / 64];
  __shared__ double shm[NT / 64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    dd r = wave_reduce_dd(v[q]);
    if (l == 0) sh[q][w] = r;
  }
  if (MAX) {
    double m = wave_reduce_max(mx);
    if (l == 0) shm[w] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      dd r = sh[q][0];
#pragma unroll
      for (int u = 1; u < NT / 64; ++u) r = dd_add(r, sh[q][u]);
      partials[(size_t)(SLOT0 + q) * nblk + bid] = make_double2(r.hi, r.lo);
    }
    if (MAX) {
      double m = shm[0];
#pragma unroll
      for (int u = 1; u < NT / 64; ++u) m = nanmax(m, shm[u]);
      partials[(size_t)3 * nblk + bid] = make_double2(m, 0.0);
    }
  }
}

// Single-block fixed-order combine of the per-block partials of one slot.
// A thread takes partials b, b + BLK, ... in that order; CMB of them are
// loaded together before they are added, so the loads overlap.
constexpr int CMB = 8;
__device__ inline dd combine_dd(const double2 *part, int nblk) {
  __shared__ dd sh[BLK / 64];
  dd acc{0.0, 0.0};
  for (int b0 = threadIdx.x; b0 < nblk; b0 += CMB * BLK) {
    double2 q[CMB];
#pragma unroll
    for (int u = 0; u < CMB; ++u) q[u] = part[min(b0 + u * BLK, nblk - 1)];
#pragma unroll
    for (int u = 0; u < CMB; ++u)
      if (b0 + u * BLK < nblk) acc = dd_add(acc, dd{q[u].x, q[u].y});
  }
  dd r = wave_reduce_dd(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = r;
  __syncthreads();
  dd out = sh[0];
  for (int u = 1; u < BLK / 64; ++u) out = dd_add(out, sh[u]);
  __syncthreads();
  return out;  // same value in every thread
}
__device__ inline double combine_max(const double2 *part, int nblk) {
  __shared__ double sh[BLK / 64];
  double acc = 0.0;
  for (int b0 = threadIdx.x; b0 < nblk; b0 += CMB * BLK) {
    double q[CMB];
#pragma unroll
    for (int u = 0; u < CMB; ++u) q[u] = part[min(b0 + u * BLK, nblk - 1)].x;
#pragma unroll
    for (int u = 0; u < CMB; ++u)
      if (b0 + u * BLK < nblk) acc = nanmax(acc, q[u]);
  }
  double r = wave_reduce_max(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = r;
  __syncthreads();
  double out = sh[0];
  for (int u = 1; u < BLK / 64; ++u) out = nanmax(out, sh[u]);
  __syncthreads();
  return out;
}

// ---------------------------------------------------------------------------
// Launch geometry helpers.
// ---------------------------------------------------------------------------

// Blocks are dealt round-robin to the 8 XCDs (block b runs on XCD b % 8);
// give each XCD one contiguous range of tiles so that the rows above and
// below a tile (the +-nx neighbours of the stencil) sit in the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblk) {
  const int x = bid & 7, q = bid >> 3;
  const int per = nblk >> 3, rem = nblk & 7;
  return x * per + (x < rem ? x : rem) + q;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) {
  const uint32_t t = __umulhi(n, f.m);
  return (t + n) >> f.s;
}

// Neighbour values of point k (0 outside the grid).  Every load is issued
// unconditionally (an out-of-range neighbour reads x[k] and is then replaced
// by 0), so the five loads of a point, and of the points a thread handles
// together, are in flight at once instead of behind branches.
struct Nbr {
  double c, s, w, e, n;
};
__device__ __forceinline__ Nbr load_nbr(const double *__restrict__ x, int k, int i, int j, int nx, int ny) {
  const bool hs = j > 0, hw = i > 0, he = i < nx - 1, hn = j < ny - 1;
  const double vs = x[hs ? k - nx : k], vw = x[hw ? k - 1 : k], ve = x[he ? k + 1 : k];
  const double vn = x[hn ? k + nx : k], vc = x[k];
  return Nbr{vc, hs ? vs : 0.0, hw ? vw : 0.0, he ? ve : 0.0, hn ? vn : 0.0};
}

__device__ __forceinline__ double spmv_point(const Dia &A, const double *__restrict__ x, int k, int i,
                                             int j, int nx, int ny) {
  const Nbr v = load_nbr(x, k, i, j, nx, ny);
  const double xs = v.s, xw = v.w, xe = v.e, xn = v.n;
  double t = A.C[k] * v.c;
  t = fma(A.S[k], xs, t);
  t = fma(A.W[k], xw, t);
  t = fma(A.E[k], xe, t);
  t = fma(A.N[k], xn, t);
  return t;
}

// The same product with S, W, E, N read from the instance's stencil tables
// (tab = its Wc, Ec, Sr, Nr): the stored coefficients, so the same bits.
__device__ __forceinline__ double spmv_point_tab(const double *__restrict__ C, const double *__restrict__ tab,
                                                 const double *__restrict__ x, int k, int i, int j, int nx,
                                                 int ny) {
  const double *Wc = tab, *Ec = tab + nx, *Sr = tab + 2 * nx, *Nr = Sr + ny;
  const Nbr v = load_nbr(x, k, i, j, nx, ny);
  const double xs = v.s, xw = v.w, xe = v.e, xn = v.n;
  // S and N depend on the row only: when all active lanes of the wave are in
  // one row they are read once per wave, by scalar loads (the tables are
  // written by an earlier kernel and only read here).
  double sr, nr;
  const int j0 = __builtin_amdgcn_readfirstlane(j);
  if (__builtin_amdgcn_ballot_w64(j != j0) == 0) {
    typedef const __attribute__((address_space(4))) double *cdp;
    sr = ((cdp)Sr)[j0];
    nr = ((cdp)Nr)[j0];
  } else {
    sr = Sr[j];
    nr = Nr[j];
  }
  double t = C[k] * v.c;
  t = fma(sr, xs, t);
  t = fma(Wc[i], xw, t);
  t = fma(Ec[i], xe, t);
  t = fma(nr, xn, t);
  return t;
}

__device__ __forceinline__ bool finite(double v) { return isfinite(v); }

__device__ __forceinline__ int find_block_inst(const Inst *inst, int ninst, int b) {
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (inst[mid].blk0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace adr
