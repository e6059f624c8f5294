// Anti-diagonal wavefront kernels for gfx950: the ILU(0) factorisation of
// the five-point matrix and the forward (L) / backward (U) triangular sweeps
// that apply M^{-1} = U^{-1} L^{-1} (Section 5.1 of the paper).
//
// Every point of these recurrences depends on its predecessor in x and in y,
// so the points of one anti-diagonal (i + j = const) are independent.  The
// grid is cut into strips of R rows; one wave owns a strip and walks it
// column by column with a skew of one column per row (wave lane l handles
// strip row l-1 and, at step tau, sweep column tau - l), so at every step
// the wave holds R consecutive points of one anti-diagonal:
//   * the x-predecessor is the lane's own result of the previous step;
//   * the y-predecessor is the result of lane l-1 at the previous step,
//     moved one lane up with a DPP wave shift (no LDS, no barrier);
//   * lane 0 is a "ghost" row: it replays the last row of the strip below
//     (published by that strip's wave through a hand-off buffer in global
//     memory, one relaxed agent-scope atomic per value, with a sentinel
//     meaning "not yet written"), with coefficients chosen so that its
//     result is exactly the published value.
// Strip heights are multiples of the chunk width W = 16 (R = 16 or 32): the
// strip's last row then covers, in each chunk, exactly the 16 columns of one
// chunk of the next strip, which can start two chunks behind -- the same lag
// as R = 15 or 31 with one more row per strip.
// Coefficients and right-hand sides are brought in by coalesced loads of
// skewed R x W tiles into registers two chunks ahead, transposed through LDS,
// and the results leave the same way.  Strips start in ticket order, so a
// wave only ever waits for a wave that is already running.
// The per-point formulas are the fixed fma orders of include/adr.h; the
// wavefront order does not change a single rounding.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "adr_internal.h"

#pragma clang fp contract(off)

namespace adr {

namespace {

constexpr unsigned SPIN_LIMIT = 1u << 20;   // polls before a wait is declared failed
#ifndef ADR_SWEEP_THREADS
#define ADR_SWEEP_THREADS 512
#endif
#ifndef ADR_LOADER_DEPTH
#define ADR_LOADER_DEPTH 2
#endif
// chunks of loads in flight per loader wave: two where one workgroup holds
// the CU (32-row strips, deep ring: 256 registers per wave), one where two
// workgroups share it (128 registers per wave)
constexpr int LDEPTH_DEEP = ADR_LOADER_DEPTH;

__device__ __forceinline__ double dpp_up(double v) {
  // lane l receives lane l-1's value; lane 0 receives 0
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, 0x138, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), 0x138, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ float dpp_up(float v) {
  const int r = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true);
  return __int_as_float(r);
}

__device__ __forceinline__ void handoff_put(uint64_t *p, double v) {
  uint64_t b = (uint64_t)__double_as_longlong(v);
  if (b == HANDOFF_EMPTY) b = CANON_NAN;
  __hip_atomic_store(p, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t handoff_get(const uint64_t *p) {
  return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until this lane's hand-off value (if `need`) is written; returns it
// and marks the slot empty again for the next launch.  A wait that exceeds
// SPIN_LIMIT polls reports through *err and marks the wave `dead`, after
// which it no longer waits (the results are then invalid, but every wave
// still runs to its end).
__device__ __forceinline__ double handoff_take(const uint64_t *p, bool need, uint64_t prefetched, int *err,
                                               bool &dead) {
  uint64_t b = need ? prefetched : 0;
  unsigned spins = 0;
  while (!dead && __builtin_amdgcn_ballot_w64(need && b == HANDOFF_EMPTY) != 0ull) {
    if (need && b == HANDOFF_EMPTY) b = handoff_get(p);
    if (++spins > SPIN_LIMIT) {
      dead = true;
      if (threadIdx.x == 0) atomicOr(err, 1);
    } else {
      __builtin_amdgcn_s_sleep(1);
    }
  }
  if (need && b == HANDOFF_EMPTY) b = 0;
  if (need) __hip_atomic_store(const_cast<uint64_t *>(p), HANDOFF_EMPTY, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return need ? __longlong_as_double((long long)b) : 0.0;
}

// Pair loads for the loader waves: one 16-byte (FP64) or 8-byte (FP32) load
// of two adjacent row elements, aligned to the element only. The per-CU
// memory pipeline issues whole instructions at a fixed rate, so two elements
// per lane halve the instruction count.
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));
typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));
template <class T>
struct Pair {
  T x, y;   // the lane's first and second tile column
};
__device__ __forceinline__ int64_t rfl64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v), hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
// Buffer resource of the raw byte range [base, base + bytes), bytes < 2^32
// (gfx9 descriptor word 3: 32-bit data, no swizzle).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void *base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)(unsigned)bytes, 0x00020000);
}
// elements e + s and e + s + 1 of a buffer of T: lane offset e (a VGPR that
// stays put), uniform offset s (an SGPR per chunk); no address arithmetic
template <class T>
__device__ __forceinline__ Pair<T> ld_pair_buf(__amdgpu_buffer_rsrc_t r, unsigned e, int s) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  typedef float f2 __attribute__((ext_vector_type(2)));
  if constexpr (sizeof(T) == 8) {
    const d2 v = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)(e * 8u), s * 8, 0));
    return Pair<T>{v.x, v.y};
  } else {
    const f2 v = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)(e * 4u), s * 4, 0));
    return Pair<T>{v.x, v.y};
  }
}
// the same pair with its elements swapped (the U sweep walks columns from
// the right, so its first tile column is the higher grid column)
template <class T>
__device__ __forceinline__ Pair<T> swap_pair(Pair<T> r) {
  return Pair<T>{r.y, r.x};
}

// Instance owning strip ticket t: strips are numbered along the ticket order
// of the instances (ord, largest work first; null: table order), so strip0
// ascends along ord and a binary search over it finds the owner.
__device__ __forceinline__ int find_strip_inst(const Inst *inst, const int *ord, int ninst, int t) {
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (inst[ord ? ord[mid] : mid].strip0 <= t) lo = mid;
    else hi = mid - 1;
  }
  return ord ? ord[lo] : lo;
}

__device__ __forceinline__ void strip_finish(const SweepSync &sy, int nstrips) {
  if (threadIdx.x == 0) {
    const unsigned fin = atomicAdd(&sy.ticket[1], 1u);
    if (fin == (unsigned)nstrips - 1) {
      // every strip has taken its ticket and finished: reset for the next launch
      __hip_atomic_store(&sy.ticket[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&sy.ticket[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// L / U sweeps.
//   OP 0 (L): y = fma(-ls, y_s, fma(-lw, y_w, q))          inputs q, lw, ls
//   OP 1 (U): z = fma(-N, z_n, fma(-E, z_e, y)) * invd     inputs y, E, N, invd
// PREC 0: factors FP64; 1: factors FP32, arithmetic FP64; 2: arithmetic FP32.
// TAB: S, W, E, N come from the stencil tables: the U sweep reads E and N
// there, the FP64 L sweep forms lw = W invd_w and ls = S invd_s from invd in
// the factorisation's own operation order (one array instead of two).
// ---------------------------------------------------------------------------
struct SweepParams {
  BatchGeom g;
  const double *v;      // q (L) or y (U), batched
  const void *f1, *f2, *f3;   // lw, ls (L) or E, N, invd (U); double or float per PREC
                              // (TAB: L uses only f3 = invd, U only f3)
  const double *tab;    // stencil tables (TAB)
  double *out;
  SweepSync sync;
  const SolveState *st;  // per-instance state (null: always run)
};

// ---------------------------------------------------------------------------
// L / U sweeps, warp-specialised.  One workgroup per strip of R rows:
//   wave 0   compute: walks the strip chunk by chunk (W columns), reading its
//            inputs from an LDS ring, keeping the chunk's results in
//            registers, then writing them to an LDS output buffer and
//            publishing the strip's last row to the hand-off buffer;
//   wave 1   poller:  waits for the previous strip's published row and puts
//            it into the ring as tile row 0 (the ghost row);
//   wave 2   storer:  copies finished output tiles from LDS to global memory;
//   waves 3+ loaders: each owns every NLD-th chunk: coalesced global loads of
//            the skewed input tile into registers, then into its ring slot.
// The waves meet only through LDS flags (workgroup-scope acquire/release):
// per-slot "loaded" and "ghost" flags, and the compute / store counters.
// Many loader waves keep many chunks in flight, so the compute wave does not
// wait on memory latency; it waits only for the previous strip.
// ---------------------------------------------------------------------------
namespace {

__device__ __forceinline__ int lds_get(int *c) {
  return __hip_atomic_load(c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_put(int *c, int v) {
  __hip_atomic_store(c, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_wait_ge(int *c, int target) {
  while (lds_get(c) < target) __builtin_amdgcn_s_sleep(1);
}
__device__ __forceinline__ void lds_wait_eq(int *c, int target) {
  while (lds_get(c) != target) __builtin_amdgcn_s_sleep(1);
}
// relaxed read of a {loaded, ghost} flag pair (one LDS access)
__device__ __forceinline__ uint64_t lds_peek_pair(int *c) {
  return __hip_atomic_load((uint64_t *)c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int lds_peek(int *c) {
  return __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local"); }

template <int R, int NIN, int CTB, bool CMP, int NTH>
struct SweepShape {
  static constexpr int W = 16;                      // columns per chunk
  static constexpr int L = R + 1;                   // tile rows (row 0 = ghost)
  static constexpr int PITCH = W + 2;               // 16-byte aligned rows
  static constexpr int NT = NTH;                    // threads per workgroup
  static constexpr int NLD = NT / 64 - 3;           // loader waves
  // 76 KB (two workgroups per CU) for R = 16 and for compact 32-row strips
  // (tiles of at most three arrays, four or more slots), else 150 KB (one
  // workgroup per CU, a deeper ring)
  static constexpr int LDS_BUDGET = (R <= 16 || CMP) ? 76 * 1024 : 150 * 1024;
  static constexpr int OUT_BYTES = 2 * L * PITCH * 8;
  static constexpr int CHUNK_BYTES = NIN * L * PITCH * CTB;
  static constexpr int NC_FIT = (LDS_BUDGET - OUT_BYTES) / CHUNK_BYTES;
  static constexpr int NC = NC_FIT < 16 ? NC_FIT : 16;   // LDS ring depth (chunks)
  static_assert(NC >= 4, "LDS ring too small");
  static constexpr int RPP = 64 / W;                // tile rows per wave pass
  static constexpr int NP = (L - 1 + RPP - 1) / RPP;   // passes for rows 1..L-1
};

}  // namespace

// CMP: two workgroups share a CU, so each wave gets at most a quarter of a
// SIMD's registers (four waves per SIMD)
// NTH: threads per workgroup (three waves plus the loaders)
template <int R, int OP, int PREC, bool TAB, bool CMP, int NTH>
__global__ __launch_bounds__(NTH, CMP ? 4 : 1) void k_sweep_ws(SweepParams p) {
  static_assert(!TAB || OP == 1 || PREC == 0, "the L sweep forms its factors from tables only in FP64");
  using TF = typename std::conditional<PREC == 0, double, float>::type;
  using CT = typename std::conditional<PREC == 2, float, double>::type;
  constexpr int NIN = (OP == 0) ? 3 : 4;
  // The table-driven U sweep keeps N, which is the same along a strip row, in
  // a register of that row's lane: its ring tiles hold y, E and invd only.
  constexpr bool NREG = (OP == 1) && TAB;
  constexpr int NL = NREG ? 3 : NIN;   // arrays per ring tile (U: invd last)
  using Sh = SweepShape<R, NL, (int)sizeof(CT), CMP, NTH>;
  constexpr int W = Sh::W, L = Sh::L, PITCH = Sh::PITCH, NC = Sh::NC, NT = Sh::NT, NLD = Sh::NLD;
  constexpr int RPP = Sh::RPP, NP = Sh::NP;
  constexpr int LDEPTH = (R > 16 && !CMP) ? LDEPTH_DEEP : 1;
  static_assert(L <= 64, "strip too tall");
  __shared__ __align__(16) CT s_in[NC][NL][L][PITCH];
  __shared__ __align__(16) double s_out[2][L][PITCH];
  __shared__ __align__(8) int s_flag[NC][2];   // [slot]{loaded, ghost}: chunk index + 1
  __shared__ int s_computed, s_stored;
  __shared__ int s_strip, s_inst;

  // wave index and everything derived from the strip are wave-uniform; say
  // so (readfirstlane), so that branches on them stay scalar
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  if (p.g.xcd_group > 0) {
    // strips by workgroup index: XCD x = b mod 8 holds strips
    // [x G, x G + G); every strip is resident, so any wait ends
    const int b = blockIdx.x, t = (b & 7) * p.g.xcd_group + (b >> 3);
    if (t >= p.g.nstrips) return;   // padding workgroup: no strip
    if (tid == 0) {
      s_inst = 0;
      s_strip = t;
      s_computed = 0;
      s_stored = 0;
    }
  } else if (tid == 0) {
    const int t = (int)atomicAdd(&p.sync.ticket[0], 1u);
    const int ii = find_strip_inst(p.g.inst, p.g.sorder, p.g.ninst, t);
    s_inst = ii;
    s_strip = t - p.g.inst[ii].strip0;
    s_computed = 0;
    s_stored = 0;
  }
  if (tid < NC) {
    s_flag[tid][0] = 0;
    s_flag[tid][1] = 0;
  }
  // ghost row of every ring slot: zero values and coefficients (invd = 1)
  for (int e = tid; e < NC * NL * PITCH; e += NT) {
    const int sl = e / (NL * PITCH), m = (e / PITCH) % NL, w = e % PITCH;
    s_in[sl][m][0][w] = (OP == 1 && m == NL - 1) ? (CT)1 : (CT)0;
  }
  __syncthreads();
  const int strip = __builtin_amdgcn_readfirstlane(s_strip);
  const int sinst = __builtin_amdgcn_readfirstlane(s_inst);
  // the instance record, read with vector loads, made wave-uniform
  const Inst I = p.g.inst[sinst];
  const int64_t ioff = rfl64(I.off), itab = rfl64(I.tab_off), iho = rfl64(I.ho_off);
  // RUNNING: a pass; CHECK: the first pass of a possible restart (M^{-1} of
  // the true residual); any other phase: this instance has stopped
  if (p.st && p.st[sinst].phase != RUNNING && p.st[sinst].phase != CHECK) {
    strip_finish(p.sync, p.g.nstrips);
    return;
  }
  const int nx = __builtin_amdgcn_readfirstlane(I.nx), ny = __builtin_amdgcn_readfirstlane(I.ny);
  const int base = strip * R;
  const int rows = min(R, ny - base);
  const bool has_prev = strip > 0, has_next = base + R < ny;
  const int nchunks = (nx + rows + W - 1) / W;
  const int lr = lane / W, lc = lane % W;   // tile (row-in-pass, column) for loads and stores
  const double *vin = p.v + ioff;
  double *vout = p.out + ioff;
  const uint64_t *ho_base = p.sync.handoff + iho;
  auto grow = [&](int l) { return OP == 0 ? base + l - 1 : ny - base - l; };
  auto gcol = [&](int co) { return OP == 0 ? co : nx - 1 - co; };

  if (wave >= 3 && nx >= 2) {
    // ------------------------------------------------------- pair loaders
    // A lane holds two adjacent columns of one tile row per array (8 lanes
    // per row, 8 rows per pass).
    const TF *f1 = (const TF *)p.f1 + ioff, *f2 = (const TF *)p.f2 + ioff, *f3 = (const TF *)p.f3 + ioff;
    const double *tab = TAB ? p.tab + itab : nullptr;
    constexpr int RP2 = 8, NP2 = (L - 1 + RP2 - 1) / RP2;
    const int lr2 = lane >> 3, tc = 2 * (lane & 7);
    double rowv[TAB ? NP2 : 1];
    if (TAB) {
#pragma unroll
      for (int q = 0; q < NP2; ++q) {
        const int l = 1 + q * RP2 + lr2;
        const int gj = (l <= rows) ? grow(l) : 0;
        rowv[q] = tab[2 * nx + (OP == 0 ? 0 : ny) + gj];
      }
    }
    // Interior chunks take a fast path: chunks c in [cf0, cf1] of a full
    // strip have every column of every tile row inside the grid (and, for
    // the table-driven L sweep, its left neighbour too), so each pair window
    // moves by a fixed 16 elements per chunk and nothing is masked. Lane
    // offsets are taken at an anchor chunk (cf0 for L, cf1 for U) where all
    // of them are >= 0 and fit 32 bits; the chunk adds a uniform shift >= 0
    // (buffer loads: lane offset in a VGPR, shift in an SGPR).
    // Rows past the strip (l = L) reuse row L-1; they are never stored.
    // Edge chunks load each element at its clamped column and are masked in
    // commit, which recomputes the masks (no lane masks live across a tile).
    const int cf0 = (R + 16) / 16, cf1 = (nx - 15) / 16;
    const bool fastok = rows == L - 1 && (size_t)nx * ny < ((size_t)1 << 29);
    unsigned ek[NP2], eks[NP2], et[NP2];   // element offsets: row, row below, table
#pragma unroll
    for (int q = 0; q < NP2; ++q) {
      const int l = min(1 + q * RP2 + lr2, L - 1);
      const int gj = grow(l);
      const int o = OP == 0 ? tc - l + 16 * cf0 : nx - 2 - tc + l - 16 * cf1;
      et[q] = (unsigned)o;
      ek[q] = (unsigned)(gj * nx + o);
      eks[q] = (unsigned)((gj > 0 ? gj - 1 : gj) * nx + o);
    }
    const size_t abytes = (size_t)nx * ny * sizeof(double), fbytes = (size_t)nx * ny * sizeof(TF);
    const __amdgpu_buffer_rsrc_t rv = raw_rsrc(vin, abytes);
    const __amdgpu_buffer_rsrc_t r1 = raw_rsrc(f1, fbytes), r2 = raw_rsrc(f2, fbytes), r3 = raw_rsrc(f3, fbytes);
    const __amdgpu_buffer_rsrc_t rt = raw_rsrc(TAB ? tab : vin, TAB ? (size_t)(2 * nx + 2 * ny) * sizeof(double) : 0);
    struct Tile2 {
      bool fast;
      Pair<double> v[NP2];                 // q (L) or y (U)
      Pair<TF> f[NIN - 1][NP2];            // factor arrays (non-TAB), invd (U TAB)
      Pair<double> t[NP2];                 // the column table: W (L TAB) or E (U TAB)
      Pair<double> iw[TAB && OP == 0 ? NP2 : 1], is[TAB && OP == 0 ? NP2 : 1];
    };
    auto issue = [&](Tile2 &T, int c) {
      T.fast = fastok && c >= cf0 && c <= cf1;
      if (T.fast) {
        const int sh = OP == 0 ? 16 * (c - cf0) : 16 * (cf1 - c);
        auto ld = [&](auto tag, __amdgpu_buffer_rsrc_t r, unsigned e, int s) {
          using E = decltype(tag);
          return OP == 0 ? ld_pair_buf<E>(r, e, s) : swap_pair(ld_pair_buf<E>(r, e, s));
        };
#pragma unroll
        for (int q = 0; q < NP2; ++q) {
          T.v[q] = ld(double(), rv, ek[q], sh);
          if (TAB && OP == 0) {
            T.iw[q] = ld(double(), r3, ek[q] - 1, sh);    // invd
            T.is[q] = ld(double(), r3, eks[q], sh);
            T.t[q] = ld(double(), rt, et[q], sh);         // W(i)
          } else if (TAB) {
            T.t[q] = ld(double(), rt, et[q], nx + sh);    // E(i)
            T.f[NIN - 2][q] = ld(TF(), r3, ek[q], sh);
          } else {
            T.f[0][q] = ld(TF(), r1, ek[q], sh);
            T.f[1][q] = ld(TF(), r2, ek[q], sh);
            if (NIN == 4) T.f[NIN - 2][q] = ld(TF(), r3, ek[q], sh);
          }
        }
        return;
      }
#pragma unroll
      for (int q = 0; q < NP2; ++q) {
        const int l = 1 + q * RP2 + lr2;
        const int co0 = c * W + tc - l;
        const int gj = (l <= rows) ? grow(l) : 0;
        // grid columns of the lane's two tile columns, clamped into the row
        const int g0 = gcol(max(0, min(co0, nx - 1))), g1 = gcol(max(0, min(co0 + 1, nx - 1)));
        const size_t rb = (size_t)gj * nx;
        T.v[q].x = vin[rb + g0];
        T.v[q].y = vin[rb + g1];
        if (TAB && OP == 0) {
          // lw = W(i) invd(k-1) for i > 0, ls = S(j) invd(k-nx) for j > 0, else 0
          const double *invd = (const double *)f3;
          const size_t rs = gj > 0 ? rb - nx : rb;
          T.iw[q].x = invd[rb + max(g0 - 1, 0)];
          T.iw[q].y = invd[rb + max(g1 - 1, 0)];
          T.is[q].x = invd[rs + g0];
          T.is[q].y = invd[rs + g1];
          T.t[q].x = tab[g0];                        // W(i)
          T.t[q].y = tab[g1];
        } else if (TAB) {
          T.t[q].x = tab[nx + g0];                   // E(i)
          T.t[q].y = tab[nx + g1];
          T.f[NIN - 2][q].x = f3[rb + g0];
          T.f[NIN - 2][q].y = f3[rb + g1];
        } else {
#pragma unroll
          for (int m = 0; m < NIN - 1; ++m) {
            const TF *fm = m == 0 ? f1 : (m == 1 ? f2 : f3);
            T.f[m][q].x = fm[rb + g0];
            T.f[m][q].y = fm[rb + g1];
          }
        }
      }
    };
    auto commit = [&](Tile2 &T, int c) {
      // element values of the tile's arrays, masked on edge chunks
      CT v0[NP2][2];
      TF bf[NIN - 1][NP2][2];
      auto values = [&](auto fastc) {
        constexpr bool fast = decltype(fastc)::value;
#pragma unroll
      for (int q = 0; q < NP2; ++q) {
        const int l = 1 + q * RP2 + lr2;
        const int gj = (l <= rows) ? grow(l) : 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int co = c * W + tc - l + h;
          const bool ok = fast || (l <= rows && co >= 0 && co < nx);
          const double v = h == 0 ? T.v[q].x : T.v[q].y;
          v0[q][h] = ok ? (CT)v : (CT)0;
          if (TAB && OP == 0) {
            const bool fi = fast || gcol(co) > 0, fj = gj > 0;
            const double t = h == 0 ? T.t[q].x : T.t[q].y;
            const double iw = h == 0 ? T.iw[q].x : T.iw[q].y, is = h == 0 ? T.is[q].x : T.is[q].y;
            bf[0][q][h] = ok && fi ? (TF)(t * iw) : (TF)0;
            bf[1][q][h] = ok && fj ? (TF)(rowv[q] * is) : (TF)0;
          } else if (TAB) {
            bf[0][q][h] = ok ? (TF)(h == 0 ? T.t[q].x : T.t[q].y) : (TF)0;   // E(i)
            bf[1][q][h] = ok ? (TF)rowv[q] : (TF)0;                          // N(j)
            bf[NIN - 2][q][h] = ok ? (h == 0 ? T.f[NIN - 2][q].x : T.f[NIN - 2][q].y) : (TF)0;
          } else {
#pragma unroll
            for (int m = 0; m < NIN - 1; ++m)
              bf[m][q][h] = ok ? (h == 0 ? T.f[m][q].x : T.f[m][q].y) : (TF)0;
          }
        }
      }
      };
      if (T.fast) values(std::true_type{});
      else values(std::false_type{});
      lds_wait_ge(&s_computed, c - NC + 1);   // ring slot free
      const int sl = c % NC;
#pragma unroll
      for (int q = 0; q < NP2; ++q) {
        const int l = 1 + q * RP2 + lr2;
        if (l < L) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            s_in[sl][0][l][tc + h] = v0[q][h];
#pragma unroll
            for (int m = 1; m < NIN; ++m) {
              if (NREG && m == 2) continue;   // N: the compute wave's register
              s_in[sl][(NREG && m == 3) ? 2 : m][l][tc + h] = (CT)bf[m - 1][q][h];
            }
          }
        }
      }
      lds_put(&s_flag[sl][0], c + 1);
    };
    if (LDEPTH == 1) {
      for (int c = wave - 3; c < nchunks; c += NLD) {
        Tile2 T;
        issue(T, c);
        commit(T, c);
      }
    } else {
      // the scheduling barriers keep each tile's loads together and ahead of
      // the next tile's, so a commit waits for its own tile only
      Tile2 A, B;
      int c = wave - 3;
      if (c < nchunks) issue(A, c);
      __builtin_amdgcn_sched_barrier(0);
      while (c < nchunks) {
        issue(B, c + NLD);
        __builtin_amdgcn_sched_barrier(0);
        commit(A, c);
        __builtin_amdgcn_sched_barrier(0);
        c += NLD;
        if (c >= nchunks) break;
        issue(A, c + NLD);
        __builtin_amdgcn_sched_barrier(0);
        commit(B, c);
        __builtin_amdgcn_sched_barrier(0);
        c += NLD;
      }
    }
  } else if (wave >= 3) {
    // ---------------------------------------- element loaders (nx == 1)
    const TF *f1 = (const TF *)p.f1 + ioff, *f2 = (const TF *)p.f2 + ioff, *f3 = (const TF *)p.f3 + ioff;
    // stencil tables of the instance: Wc[nx], Ec[nx], Sr[ny], Nr[ny]
    const double *tab = TAB ? p.tab + itab : nullptr;
    // the row entry (S for L, N for U) of each strip row this lane loads is
    // the same in every chunk: read once
    double rowv[TAB ? NP : 1];
    if (TAB) {
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int l = 1 + q * RPP + lr;
        const int gj = (l <= rows) ? grow(l) : 0;
        rowv[q] = tab[2 * nx + (OP == 0 ? 0 : ny) + gj];
      }
    }
    // A loader keeps LDEPTH of its chunks in flight: the loads of the next
    // chunk it owns are issued before the previous one is written to the
    // ring, so each loader wave has up to LDEPTH tiles of loads outstanding.
    // Every load of a tile is issued before any is used (points outside the
    // strip load element 0 and are zeroed afterwards).
    struct Tile {
      double bv[NP];
      TF bf[NIN - 1][NP];
      bool okq[NP];
      double iw[TAB && OP == 0 ? NP : 1], is[TAB && OP == 0 ? NP : 1];   // invd of the x- and y-predecessor
      int fi[TAB && OP == 0 ? NP : 1], fj[TAB && OP == 0 ? NP : 1];
    };
    auto issue = [&](Tile &T, int c) {
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int l = 1 + q * RPP + lr;
        const int co = c * W + lc - l;
        const bool ok = (l <= rows) && (co >= 0) && (co < nx);
        const int gi = ok ? gcol(co) : 0, gj = ok ? grow(l) : 0;
        const size_t k = (size_t)gj * nx + gi;
        T.okq[q] = ok;
        T.bv[q] = vin[k];
        if (TAB && OP == 0) {
          // lw = W(i) invd(k-1) for i > 0, ls = S(j) invd(k-nx) for j > 0, else 0
          const double *invd = (const double *)f3;
          T.iw[q] = invd[gi > 0 ? k - 1 : k];
          T.is[q] = invd[gj > 0 ? k - nx : k];
          T.bf[0][q] = (TF)tab[gi];           // W(i)
          T.bf[1][q] = (TF)rowv[q];           // S(j)
          T.fi[q] = gi;
          T.fj[q] = gj;
        } else if (TAB) {
          T.bf[0][q] = (TF)tab[nx + gi];      // E(i)
          T.bf[1][q] = (TF)rowv[q];           // N(j)
          T.bf[NIN - 2][q] = f3[k];
        } else {
          T.bf[0][q] = f1[k];
          T.bf[1][q] = f2[k];
          if (NIN == 4) T.bf[NIN - 2][q] = f3[k];
        }
      }
    };
    auto commit = [&](Tile &T, int c) {
      if (TAB && OP == 0) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          T.bf[0][q] = T.fi[q] > 0 ? (TF)((double)T.bf[0][q] * T.iw[q]) : (TF)0;
          T.bf[1][q] = T.fj[q] > 0 ? (TF)((double)T.bf[1][q] * T.is[q]) : (TF)0;
        }
      }
      lds_wait_ge(&s_computed, c - NC + 1);   // ring slot free
      const int sl = c % NC;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int l = 1 + q * RPP + lr;
        if (l < L) {
          s_in[sl][0][l][lc] = T.okq[q] ? (CT)T.bv[q] : (CT)0;
#pragma unroll
          for (int m = 1; m < NIN; ++m) {
            if (NREG && m == 2) continue;   // N: the compute wave's register
            s_in[sl][(NREG && m == 3) ? 2 : m][l][lc] = T.okq[q] ? (CT)T.bf[m - 1][q] : (CT)0;
          }
        }
      }
      lds_put(&s_flag[sl][0], c + 1);
    };
    if (LDEPTH == 1) {
      for (int c = wave - 3; c < nchunks; c += NLD) {
        Tile T;
        issue(T, c);
        commit(T, c);
      }
    } else {
      // The next tile's loads are issued whether or not that chunk exists (a
      // chunk past the end has no point in the strip: its lanes load element
      // 0 and it is never committed), so the number of loads in flight is the
      // same on every path and each commit waits only for its own tile.
      Tile A, B;
      int c = wave - 3;
      if (c < nchunks) issue(A, c);
      while (c < nchunks) {
        issue(B, c + NLD);
        commit(A, c);
        c += NLD;
        if (c >= nchunks) break;
        issue(A, c + NLD);
        commit(B, c);
        c += NLD;
      }
    }
  } else if (wave == 1) {
    // ------------------------------------------------------------- poller
    // One relaxed load per lane covers a window of 64 / W chunks; NS such
    // samples are kept in flight, issued one after another, so a value that
    // lands is seen about one memory round trip later.  Every complete chunk
    // at the front of the window is delivered in order; the rest is polled
    // again.
    if (has_prev) {
      constexpr int CPW = 64 / W;   // chunks per window
      constexpr int NS = 1;         // samples in flight
      constexpr uint64_t GM = (W == 64) ? ~0ull : ((1ull << W) - 1);
      const uint64_t *ho_in = ho_base + (size_t)(strip - 1) * nx;
      unsigned idle = 0;
      bool dead = false;
      int next = 0;
      int ws[NS];
      uint64_t val[NS];
      auto sample = [&](int k) {
        ws[k] = next;
        const int co = next * W + lane;
        val[k] = (co < nx && next + lane / W < nchunks) ? handoff_get(ho_in + gcol(co)) : 0ull;
      };
#pragma unroll
      for (int k = 0; k < NS; ++k) sample(k);
      while (next < nchunks) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const int w0 = ws[k];
          const int co = w0 * W + lane;
          const bool need = co < nx && w0 + lane / W < nchunks;
          uint64_t b = val[k];
          if (dead && need && b == HANDOFF_EMPTY) b = 0;   // a failed wait delivers zeros
          const uint64_t okm = __builtin_amdgcn_ballot_w64(!need || b != HANDOFF_EMPTY);
          const int before = next;
#pragma unroll
          for (int q = 0; q < CPW; ++q) {
            const int c = w0 + q;
            if (c == next && c < nchunks && ((okm >> (q * W)) & GM) == GM) {
              lds_wait_ge(&s_computed, c - NC + 1);
              if (lane / W == q) s_in[c % NC][0][0][lane % W] = (CT)__longlong_as_double((long long)b);
              lds_put(&s_flag[c % NC][1], c + 1);
              ++next;
            }
          }
          // consumed slots are emptied again for the next launch
          const int cl = w0 + lane / W;
          if (need && cl >= before && cl < next)
            __hip_atomic_store(const_cast<uint64_t *>(ho_in + gcol(co)), HANDOFF_EMPTY, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
          if (next == before) {
            __builtin_amdgcn_s_sleep(2);
            if (++idle > SPIN_LIMIT && !dead) {
              dead = true;
              if (lane == 0) atomicOr(p.sync.err, 1);
            }
          } else {
            idle = 0;
          }
          if (next < nchunks) sample(k);
        }
      }
    }
  } else if (wave == 2) {
    // ------------------------------------------------------------- storer
    for (int c = 0; c < nchunks; ++c) {
      lds_wait_ge(&s_computed, c + 1);
      const int b = c & 1;
      // every LDS read of the tile first (one wait), then the stores
      double o[NP];
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int l = 1 + q * RPP + lr;
        o[q] = s_out[b][l < L ? l : L - 1][lc];
      }
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int l = 1 + q * RPP + lr;
        const int co = c * W + lc - l;
        const bool ok = (l <= rows) && (co >= 0) && (co < nx);
        if (ok) vout[(size_t)grow(l) * nx + gcol(co)] = o[q];
      }
      lds_put(&s_stored, c + 1);
    }
  } else {
    // ------------------------------------------------------------- compute
    uint64_t *ho_out = const_cast<uint64_t *>(ho_base) + (size_t)strip * nx;
    const int row = lane < L ? lane : L - 1;
    // NREG: N of this lane's strip row (0 for the ghost lane and rows past the
    // strip).  Unlike the tiles it is not zeroed at the (never stored) points
    // left or right of the grid; there y, E and invd are 0 and the value from
    // the row below is itself such a point's +-0, so they still come out +-0
    // (NaN only if the neighbour in x already is), as with a zero N.
    CT nrow = (CT)0;
    if (NREG && lane >= 1 && lane < L && lane <= rows)
      nrow = (CT)(TF)p.tab[itab + 2 * nx + ny + grow(lane)];
    CT west = (CT)0;
    uint64_t fl = lds_peek_pair(&s_flag[0][0]);
    for (int c = 0; c < nchunks; ++c) {
      const int sl = c % NC;
      const uint64_t want = has_prev ? ((uint64_t)(uint32_t)(c + 1) | ((uint64_t)(uint32_t)(c + 1) << 32))
                                     : (uint64_t)(uint32_t)(c + 1);
      const uint64_t mask = has_prev ? ~0ull : 0xffffffffull;
      if ((fl & mask) != want) {
        fl = lds_peek_pair(&s_flag[sl][0]);   // the read-ahead may predate the flags
        while ((fl & mask) != want) {
          __builtin_amdgcn_s_sleep(1);
          fl = lds_peek_pair(&s_flag[sl][0]);
        }
      }
      lds_acquire();
      int st = lds_peek(&s_stored);
      // the whole chunk's inputs into registers first, so that LDS latency is
      // paid once per chunk and not inside the dependent chain
      CT in[NL][W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
#pragma unroll
        for (int m = 0; m < NL; ++m) in[m][w] = s_in[sl][m][row][w];
      }
      __builtin_amdgcn_sched_barrier(0);
      CT res[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const CT south = dpp_up(west);
        CT v = fma(-(NREG ? nrow : in[2][w]), south, fma(-in[1][w], west, in[0][w]));
        if (OP == 1) v = v * in[NL - 1][w];
        res[w] = v;
        west = v;
      }
      fl = lds_peek_pair(&s_flag[(c + 1) % NC][0]);   // next chunk's flags, read ahead
      while (st < c - 1) {   // output buffer c & 1 is free
        __builtin_amdgcn_s_sleep(1);
        st = lds_peek(&s_stored);
      }
      lds_acquire();
      const int b = c & 1;
      if (lane < L) {
#pragma unroll
        for (int w = 0; w < W; ++w) s_out[b][lane][w] = (double)res[w];
      }
      if (has_next) {
        // publish this strip's last row: sweep columns c*W + w - rows
        const int co = c * W + lane - rows;
        if (lane < W && co >= 0 && co < nx) handoff_put(ho_out + gcol(co), s_out[b][rows][lane]);
      }
      lds_put(&s_computed, c + 1);
    }
  }
  __syncthreads();
  strip_finish(p.sync, p.g.nstrips);
}

// ---------------------------------------------------------------------------
// ILU(0) factorisation sweep (forward, like L).  Per point:
//   lw = W * invd_w,  ls = S * invd_s,  d = fma(-ls, N_s, fma(-lw, E_w, C)),
//   invd = 1 / d  (0 and a recorded bad index if d is 0 or not finite).
// Carried: invd and E of the x-predecessor (own lane); invd and N of the
// y-predecessor (lane below, DPP).  The ghost lane replays the last row of
// the strip below: its invd from the hand-off buffer, its N from A.
// ---------------------------------------------------------------------------
struct FactorParams {
  BatchGeom g;
  Dia A;
  Factors64 f;
  Factors32 h;   // optional FP32 copies (null pointers: not written)
  SweepSync sync;
  unsigned long long *bad;   // per instance: min over bad pivot indices (pre-set to ~0)
};

template <int R, int W>
__global__ __launch_bounds__(64) void k_ilu0(FactorParams p) {
  constexpr int L = R + 1, RPP = 64 / W, NP = (L + RPP - 1) / RPP, NIN = 5, NOUT = 3;
  __shared__ double s_in[NIN][L][W + 1];
  __shared__ double s_out[NOUT][L][W + 1];
  const int lane = threadIdx.x;
  unsigned tk = 0;
  if (lane == 0) tk = atomicAdd(&p.sync.ticket[0], 1u);
  const int t = __builtin_amdgcn_readfirstlane((int)tk);
  const int ii = find_strip_inst(p.g.inst, p.g.sorder, p.g.ninst, t);
  const Inst I = p.g.inst[ii];
  const int strip = t - I.strip0;
  const int nx = I.nx, ny = I.ny;
  const int base = strip * R;
  const int rows = min(R, ny - base);
  const bool has_prev = strip > 0, has_next = base + R < ny;
  const uint64_t *ho_in = p.sync.handoff + I.ho_off + (size_t)(has_prev ? strip - 1 : 0) * nx;
  uint64_t *ho_out = p.sync.handoff + I.ho_off + (size_t)strip * nx;
  const int nsteps = nx + rows;
  const int nchunks = (nsteps + W - 1) / W;
  const int lrow = lane / W, lcol = lane % W;
  bool dead = false;
  const int64_t o = I.off;
  const double *in[NIN] = {p.A.S + o, p.A.W + o, p.A.C + o, p.A.E + o, p.A.N + o};

  double stg[NIN][NP];
  auto issue = [&](int c) {
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const int l = q * RPP + lrow;
      const int co = c * W + lcol - l;
      const int row = base + l - 1;
      const bool inr = (co >= 0) && (co < nx);
      const bool ok = (l >= 1) && (l <= rows) && inr;
      const bool ghostN = (l == 0) && has_prev && inr;   // N of the row below the strip
      const size_t k = (ok || ghostN) ? (size_t)row * nx + co : 0;
#pragma unroll
      for (int m = 0; m < NIN; ++m) stg[m][q] = ok ? in[m][k] : 0.0;
      if (ghostN) stg[4][q] = in[4][k];
    }
  };
  auto to_lds = [&](int c) {
    const int co = c * W + lcol;
    const bool need = has_prev && lrow == 0 && co < nx;
    uint64_t pre = need ? handoff_get(ho_in + co) : 0ull;
    const double gv = handoff_take(ho_in + (need ? co : 0), need, pre, p.sync.err, dead);
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const int l = q * RPP + lrow;
      if (l < L) {
#pragma unroll
        for (int m = 0; m < NIN; ++m) s_in[m][l][lcol] = stg[m][q];
      }
    }
    if (lrow == 0) s_in[2][0][lcol] = gv;   // ghost: C slot carries the hand-off invd
  };

  double invd_w = 0.0, e_w = 0.0, n_prev = 0.0;
  const int lr = lane < L ? lane : L - 1;
  for (int c = 0; c < nchunks; ++c) {
    issue(c);
    to_lds(c);
    __syncthreads();
    for (int w = 0; w < W; ++w) {
      const double S = s_in[0][lr][w], Wc = s_in[1][lr][w], C = s_in[2][lr][w];
      const double E = s_in[3][lr][w], N = s_in[4][lr][w];
      const double invd_s = dpp_up(invd_w);
      const double n_s = dpp_up(n_prev);
      const double lw = Wc * invd_w;
      const double ls = S * invd_s;
      double d = fma(-lw, e_w, C);
      d = fma(-ls, n_s, d);
      const int co = c * W + w - lane;
      const bool valid = lane >= 1 && lane <= rows && co >= 0 && co < nx;
      const bool bad = valid && (d == 0.0 || !isfinite(d));
      double invd = (valid && !bad) ? 1.0 / d : 0.0;
      if (lane == 0) invd = C;
      if (bad) atomicMin(p.bad + ii, (unsigned long long)((size_t)(base + lane - 1) * nx + co));
      if (lane < L) {
        s_out[0][lane][w] = lw;
        s_out[1][lane][w] = ls;
        s_out[2][lane][w] = invd;
      }
      if (has_next && lane == rows && valid) handoff_put(ho_out + co, invd);
      invd_w = invd;
      e_w = E;
      n_prev = N;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const int l = q * RPP + lrow;
      const int co = c * W + lcol - l;
      const bool ok = (l >= 1) && (l <= rows) && (co >= 0) && (co < nx);
      if (ok) {
        const size_t k = (size_t)o + (size_t)(base + l - 1) * nx + co;
        p.f.lw[k] = s_out[0][l][lcol];
        p.f.ls[k] = s_out[1][l][lcol];
        p.f.invd[k] = s_out[2][l][lcol];
        if (p.h.lw) {
          p.h.lw[k] = (float)s_out[0][l][lcol];
          p.h.ls[k] = (float)s_out[1][l][lcol];
          p.h.invd[k] = (float)s_out[2][l][lcol];
          p.h.E[k] = (float)p.A.E[k];
          p.h.N[k] = (float)p.A.N[k];
        }
      }
    }
    __syncthreads();
  }
  strip_finish(p.sync, p.g.nstrips);
}

// ---------------------------------------------------------------------------
// Launchers.  One launch covers every strip of every instance of the batch.
// ---------------------------------------------------------------------------
hipError_t launch_ilu0(const Dia &A, const BatchGeom &g, Factors64 f64, Factors32 f32,
                       const SweepSync &sync, int64_t *bad, hipStream_t s) {
  FactorParams p;
  p.g = g;
  p.A = A;
  p.f = f64;
  p.h = f32;
  p.sync = sync;
  p.bad = (unsigned long long *)bad;
  switch (g.rows) {
    case 16: hipLaunchKernelGGL((k_ilu0<16, 32>), dim3(g.nstrips), dim3(64), 0, s, p); break;
    case 32: hipLaunchKernelGGL((k_ilu0<32, 32>), dim3(g.nstrips), dim3(64), 0, s, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Compact 32-row strips (two workgroups per CU, a four-slot ring) pay off when
// the strips outnumber the CUs well (batches); a grid whose strips about fill
// the CUs keeps the deeper ring.  Tiles of four arrays (the U sweep reading
// the diagonals) always take the deep ring.
template <int OP, int PREC, bool TAB>
static hipError_t launch_sweep_t(const SweepParams &p, hipStream_t s) {
  constexpr bool CAN_CMP = OP == 0 || TAB;   // three arrays per tile
  const int grid = p.g.xcd_group > 0 ? 8 * p.g.xcd_group : p.g.nstrips;
  switch (p.g.rows) {
    case 16:
      hipLaunchKernelGGL((k_sweep_ws<16, OP, PREC, TAB, false, ADR_SWEEP_THREADS>), dim3(p.g.nstrips),
                         dim3(ADR_SWEEP_THREADS), 0, s, p);
      break;
    case 32:
      if (CAN_CMP && p.g.compact == 2)   // compact ring, three loader waves
        hipLaunchKernelGGL((k_sweep_ws<32, OP, PREC, TAB, CAN_CMP, 384>), dim3(p.g.nstrips), dim3(384), 0, s, p);
      else if (CAN_CMP && p.g.compact)
        hipLaunchKernelGGL((k_sweep_ws<32, OP, PREC, TAB, CAN_CMP, ADR_SWEEP_THREADS>), dim3(p.g.nstrips),
                           dim3(ADR_SWEEP_THREADS), 0, s, p);
      else
        hipLaunchKernelGGL((k_sweep_ws<32, OP, PREC, TAB, false, ADR_SWEEP_THREADS>), dim3(grid),
                           dim3(ADR_SWEEP_THREADS), 0, s, p);
      break;

    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_lsweep(const BatchGeom &g, int precision, const Factors64 &f64, const Factors32 &f32,
                         const double *tab, const double *q, double *y, const SweepSync &sync,
                         const SolveState *st, hipStream_t s) {
  SweepParams p{};
  p.g = g;
  p.v = q;
  p.out = y;
  p.sync = sync;
  p.st = st;
  p.tab = tab;
  if (precision == 0) {
    p.f1 = f64.lw;
    p.f2 = f64.ls;
    p.f3 = f64.invd;
    return tab ? launch_sweep_t<0, 0, true>(p, s) : launch_sweep_t<0, 0, false>(p, s);
  }
  p.f1 = f32.lw;
  p.f2 = f32.ls;
  return precision == 1 ? launch_sweep_t<0, 1, false>(p, s) : launch_sweep_t<0, 2, false>(p, s);
}

hipError_t launch_usweep(const BatchGeom &g, int precision, const Dia &A, const Factors64 &f64,
                         const Factors32 &f32, const double *tab, const double *y, double *z,
                         const SweepSync &sync, const SolveState *st, hipStream_t s) {
  SweepParams p{};
  p.g = g;
  p.v = y;
  p.out = z;
  p.sync = sync;
  p.st = st;
  p.tab = tab;
  if (precision == 0) {
    p.f1 = A.E;
    p.f2 = A.N;
    p.f3 = f64.invd;
    return tab ? launch_sweep_t<1, 0, true>(p, s) : launch_sweep_t<1, 0, false>(p, s);
  }
  p.f1 = f32.E;
  p.f2 = f32.N;
  p.f3 = f32.invd;
  if (precision == 1) return tab ? launch_sweep_t<1, 1, true>(p, s) : launch_sweep_t<1, 1, false>(p, s);
  return tab ? launch_sweep_t<1, 2, true>(p, s) : launch_sweep_t<1, 2, false>(p, s);
}

}  // namespace adr
