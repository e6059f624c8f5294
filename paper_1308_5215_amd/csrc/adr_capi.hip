// Host runtime and C ABI (include/adr.h): argument checking, device memory,
// the 1-D tables of the discretisation, batch geometry, the sweep-height
// autotuner and the BiCGSTAB driver, which captures a chunk of passes into a
// HIP graph and replays it until the device-side states report that every
// instance has stopped.  A single problem is a batch of one instance.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/adr.h"
#include "../../include/adr_cnn.h"
#include "adr_internal.h"

#pragma clang fp contract(off)

using namespace adr;

namespace {

thread_local std::string g_last_error;

adr_status fail(adr_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
adr_status fail(adr_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                               \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) {                                                                         \
      (void)hipGetLastError();                                                                      \
      return fail(e_ == hipErrorOutOfMemory ? ADR_ERR_NOMEM : ADR_ERR_DEVICE, "%s: %s (%s:%d)", #expr, \
                  hipGetErrorString(e_), __FILE__, __LINE__);                                       \
    }                                                                                               \
  } while (0)

FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  uint32_t sh = 0;
  while ((1ull << sh) < d) ++sh;
  f.d = d;
  f.s = sh;
  f.m = (uint32_t)(((((uint64_t)1) << 32) * ((((uint64_t)1) << sh) - d)) / d + 1);
  return f;
}

// Streaming geometry of one instance: at most ~2048 blocks of 256 threads,
// each block a multiple of 1024 points (four per thread: the streaming pass
// kernels take four points per thread per loop trip).
void stream_geom(int64_t n, int &chunk, int &nblk) {
  int64_t c = (n + 2047) / 2048;
  c = ((c + 1023) / 1024) * 1024;
  if (c < 1024) c = 1024;
  chunk = (int)c;
  nblk = (int)((n + c - 1) / c);
  if (nblk < 1) nblk = 1;
}

Stream1D make_geom(int64_t n) {
  Stream1D g;
  g.n = (int)n;
  stream_geom(n, g.chunk, g.nblk);
  return g;
}

template <class T>
hipError_t dalloc(T **p, size_t count, size_t &bytes) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void **)p, count * sizeof(T));
  if (e == hipSuccess) bytes += count * sizeof(T);
  return e;
}
template <class T>
void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

// Buffers created after assembly (sync memory, factors, iteration vectors,
// solve states) come from the caller's workspace when one is bound, each
// rounded to 256 bytes; otherwise from hipMalloc.
constexpr size_t WS_ALIGN = 256;
size_t ws_round(size_t count, size_t elem) {
  const size_t b = (count ? count : 1) * elem;
  return (b + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN;
}

template <class T>
hipError_t palloc(adr_problem *P, T **p, size_t count);
template <class T>
void pfree(adr_problem *P, T *&p);

// Partial sums of adr_dot_noalloc: one 16-byte entry per streaming block of
// the inner product (at most 2048 blocks for n < 2^31, see stream_geom), in a
// fixed device array instead of per-call allocations.  Host code never uses
// the symbol itself as an address: dot_scratch() looks up this device's copy
// with hipGetSymbolAddress once and keeps the pointer per device.
constexpr int DOT_SCRATCH_BLOCKS = 2048;
static __device__ __align__(256) double2 scratch[DOT_SCRATCH_BLOCKS];

std::mutex g_scratch_mu;
constexpr int MAX_DEVICES = 64;
double2 *g_scratch[MAX_DEVICES] = {};

// Strip height used until the autotuner or the caller picks one: 32 rows
// (measured faster than 16 for every square grid from 128^2 to 4096^2: half
// as many strip hand-offs for one more chunk of lag each).
int default_rows(int /*max_ny*/) { return 32; }

}  // namespace

namespace adr {
int set_error(int st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}
void clear_error() { g_last_error.clear(); }
}  // namespace adr

struct adr_problem {
  int dev = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;   // private stream used only for graph capture
  int count = 0;
  std::vector<double> eps, X, Y;
  std::vector<int> nx, ny, scheme, bc;
  std::vector<Inst> inst;      // host copy of the instance table
  Inst *d_inst = nullptr;
  int *d_sorder = nullptr;   // instances in strip-ticket order
  int64_t ntot = 0;            // unknowns over the batch
  int nblk = 0, nstrips = 0, rows = 0, max_ny = 0;
  int compact = -1;            // 32-row sweep ring: -1 automatic, 0 deep, 1 compact
  int cus = 256;               // compute units of the device
  size_t bytes = 0;
  // matrix (batched)
  double *S = nullptr, *W = nullptr, *C = nullptr, *E = nullptr, *N = nullptr, *rhs = nullptr;
  double *F = nullptr;         // forcing f per unknown (input of the warm-start network)
  // stencil tables (separable S, W, E, N; verified against the diagonals)
  double *tab = nullptr;
  unsigned *tab_bad = nullptr;
  int64_t tab_len = 0;
  int has_tab = 0;    // tables match every point
  int tab_on = 1;     // the caller allows them (adr_use_stencil_tables)
  // factors
  double *lw = nullptr, *ls = nullptr, *invd = nullptr;
  float *lw32 = nullptr, *ls32 = nullptr, *invd32 = nullptr, *E32 = nullptr, *N32 = nullptr;
  int factored = 0, precision = 0;
  int max_restarts = 8;        // true-residual confirmation (adr_set_max_restarts)
  // iteration vectors
  double *r = nullptr, *rh = nullptr, *p = nullptr, *v = nullptr, *s = nullptr, *t = nullptr;
  double *ph = nullptr, *z = nullptr, *y = nullptr;
  // reductions, state, histories
  double2 *partials = nullptr;
  SolveState *st = nullptr;
  double *hist = nullptr;
  int hist_cap = 0;   // maxit + 1 the history buffer was sized for
  double *scal = nullptr;
  int64_t *bad = nullptr;
  FeatInst *d_feat = nullptr;  // per-instance table of the warm-start input fields
  // wavefront synchronisation
  unsigned *ticket = nullptr;
  uint64_t *handoff = nullptr;
  int64_t handoff_words = 0;
  int *err = nullptr;
  int sync_ready = 0;   // the three above allocated and initialised
  // caller workspace (adr_bind_workspace): the buffers created after assembly
  // are carved out of it instead of being allocated
  char *ws = nullptr;
  size_t ws_bytes = 0, ws_used = 0;
  // host pinned mirror of the states
  SolveState *h_st = nullptr;
  // events bracketing the kernels of a single-step call (and the autotuner)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t ev_chunk = nullptr;   // marks the state copy of a replayed chunk
  float last_ms = 0.f;
  // captured iteration chunk
  hipGraphExec_t gexec = nullptr;
  double *g_x = nullptr;
  double g_tol = -1;
  int g_maxit = -1, g_prec = -1, g_rows = -1, g_K = 0, g_tab = -1, g_cmp = -1, g_mr = -2;

  SweepSync sync() const { return SweepSync{ticket, handoff, err}; }
  Dia dia() const { return Dia{S, W, C, E, N}; }
  const double *stencil_tab() const { return (has_tab && tab_on) ? tab : nullptr; }
  // automatic: the compact ring when every strip has a CU of its own (its
  // smaller register and LDS footprint is 1 % faster per pass at 2048^2 and
  // 4096^2) or once the strips exceed 1.5 per CU (384 on 256 CUs); the deep
  // ring in between, where strips beyond one per CU would share a CU
  int ring_compact() const {
    return compact >= 0 ? compact : ((nstrips <= cus || 2 * nstrips > 3 * cus) ? 1 : 0);
  }
  // XCD-grouped strips: a single instance whose strips all fit on the
  // device at once (one workgroup per CU on the deep ring) places
  // consecutive strips on one XCD (workgroup b runs on XCD b mod 8)
  int xcd_group() const {
#ifdef ADR_NO_XCD_GROUPS
    return 0;
#else
    if (count != 1 || ring_compact() || rows != 32 || nstrips > cus) return 0;
    return (nstrips + 7) / 8;
#endif
  }
  BatchGeom geom() const {
    // the compact ring with three loader waves instead of five where every
    // strip has a CU of its own: the strips then wait on each other, not on
    // their loads, and fewer loads in flight shorten the hand-offs
    const int ring = ring_compact() == 1 && nstrips <= cus ? 2 : ring_compact();
    return BatchGeom{d_inst, count, nblk, nstrips, rows, ring, xcd_group(), d_sorder};
  }
};

namespace {

template <class T>
hipError_t palloc(adr_problem *P, T **p, size_t count) {
  if (!P->ws) return dalloc(p, count, P->bytes);
  const size_t b = ws_round(count, sizeof(T));
  *p = nullptr;
  if (P->ws_used + b > P->ws_bytes) return hipErrorOutOfMemory;
  *p = (T *)(P->ws + P->ws_used);
  P->ws_used += b;
  return hipSuccess;
}
template <class T>
void pfree(adr_problem *P, T *&p) {
  const char *c = (const char *)p;
  if (p && !(P->ws && c >= P->ws && c < P->ws + P->ws_bytes)) (void)hipFree((void *)p);
  p = nullptr;
}

// Hand-off words for the smallest strip height of every instance.
int64_t handoff_words(const adr_problem *P) {
  int64_t words = 0;
  for (int k = 0; k < P->count; ++k) words += (int64_t)((P->ny[k] + 15) / 16) * P->nx[k];
  return words;
}

// Workspace bytes: sync memory, factors of `precision`, iteration vectors and
// solve states, in the order and rounding palloc uses.
size_t workspace_bytes(const adr_problem *P, int precision) {
  const size_t n = (size_t)P->ntot;
  size_t b = ws_round(2, sizeof(unsigned)) + ws_round((size_t)handoff_words(P), sizeof(uint64_t)) +
             ws_round(1, sizeof(int));
  b += 3 * ws_round(n, sizeof(double));
  if (precision != ADR_FP64) b += 5 * ws_round(n, sizeof(float));
  b += 9 * ws_round(n, sizeof(double)) + ws_round((size_t)P->count, sizeof(SolveState));
  return b;
}

// (Re)build the instance table for strip height R and upload it.
adr_status build_table(adr_problem *P, int R) {
  int64_t off = 0, ho = 0, tabo = 0;
  int blk = 0, strip = 0;
  for (int k = 0; k < P->count; ++k) {
    Inst &I = P->inst[k];
    I.nx = P->nx[k];
    I.ny = P->ny[k];
    I.n = I.nx * I.ny;
    int nb;
    stream_geom(I.n, I.chunk, nb);
    I.off = off;
    I.blk0 = blk;
    I.nblk = (nb + 7) & ~7;   // whole XCD rounds: a block's XCD is its local index mod 8
    I.nstrips = (I.ny + R - 1) / R;
    I.ho_off = ho;
    I.fd = make_fastdiv((uint32_t)I.nx);
    I.pad = 0;
    I.tab_off = tabo;
    tabo += stencil_tab_len(I.nx, I.ny);
    off += I.n;
    blk += I.nblk;
    strip += I.nstrips;
    ho += (int64_t)I.nstrips * I.nx;
  }
  // Strip tickets go to the instances largest first (strips times chunks per
  // strip; ties in batch order), so that the long instances start early and
  // the short ones fill the tail (measured 8 % faster on a batch of 256
  // instances of 128^2..1024^2 than the batch order).  Strips of one
  // instance keep consecutive tickets.
  std::vector<int> ord(P->count);
  for (int k = 0; k < P->count; ++k) ord[k] = k;
  auto work = [&](int k) {
    const Inst &I = P->inst[k];
    return (int64_t)I.nstrips * ((I.nx + R + 15) / 16);
  };
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return work(a) > work(b); });
  int s0 = 0;
  for (int k : ord) {
    P->inst[k].strip0 = s0;
    s0 += P->inst[k].nstrips;
  }
  P->ntot = off;
  P->tab_len = tabo;
  P->nblk = blk;
  P->nstrips = strip;
  P->rows = R;
  if (!P->d_inst) HIP_TRY(dalloc(&P->d_inst, (size_t)P->count, P->bytes));
  if (!P->d_sorder) HIP_TRY(dalloc(&P->d_sorder, (size_t)P->count, P->bytes));
  HIP_TRY(hipMemcpyAsync(P->d_inst, P->inst.data(), sizeof(Inst) * (size_t)P->count, hipMemcpyHostToDevice,
                         P->stream));
  HIP_TRY(hipMemcpyAsync(P->d_sorder, ord.data(), sizeof(int) * (size_t)P->count, hipMemcpyHostToDevice,
                         P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return ADR_OK;
}

// Allocation helpers below allocate each missing buffer on its own, so a call
// that failed part-way (out of memory) leaves no null buffer behind a
// non-null one for the next call to trust.
adr_status ensure_sync(adr_problem *P) {
  if (P->sync_ready) return ADR_OK;
  const int64_t words = handoff_words(P);   // enough for the smallest strip height
  P->handoff_words = words;
  if (!P->ticket) HIP_TRY(palloc(P, &P->ticket, 2));
  if (!P->handoff) HIP_TRY(palloc(P, &P->handoff, (size_t)words));
  if (!P->err) HIP_TRY(palloc(P, &P->err, 1));
  HIP_TRY(launch_fill_u32(P->ticket, 2, 0u, P->stream));
  HIP_TRY(launch_fill_u64(P->handoff, words, HANDOFF_EMPTY, P->stream));
  HIP_TRY(hipMemsetAsync(P->err, 0, sizeof(int), P->stream));
  P->sync_ready = 1;
  return ADR_OK;
}

adr_status ensure_events(adr_problem *P) {
  if (!P->ev0) HIP_TRY(hipEventCreate(&P->ev0));
  if (!P->ev1) HIP_TRY(hipEventCreate(&P->ev1));
  if (!P->ev_chunk) HIP_TRY(hipEventCreateWithFlags(&P->ev_chunk, hipEventDisableTiming));
  return ADR_OK;
}

// Device time between the two events of the problem (after they completed).
adr_status read_call_ms(adr_problem *P) {
  HIP_TRY(hipEventSynchronize(P->ev1));
  HIP_TRY(hipEventElapsedTime(&P->last_ms, P->ev0, P->ev1));
  return ADR_OK;
}

adr_status check_device_fault(adr_problem *P) {
  int herr = 0;
  HIP_TRY(hipMemcpyAsync(&herr, P->err, sizeof(int), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  if (herr) {
    // a wavefront wait exceeded its spin limit: restore the sync memory
    HIP_TRY(launch_fill_u32(P->ticket, 2, 0u, P->stream));
    HIP_TRY(launch_fill_u64(P->handoff, P->handoff_words, HANDOFF_EMPTY, P->stream));
    HIP_TRY(hipMemsetAsync(P->err, 0, sizeof(int), P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    return fail(ADR_ERR_DEVICE, "wavefront hand-off wait exceeded its limit");
  }
  return ADR_OK;
}

adr_status ensure_iter_buffers(adr_problem *P, int maxit) {
  double **vecs[] = {&P->r, &P->rh, &P->p, &P->v, &P->s, &P->t, &P->ph, &P->z, &P->y};
  for (double **q : vecs)
    if (!*q) HIP_TRY(palloc(P, q, (size_t)P->ntot));
  if (!P->st) HIP_TRY(palloc(P, &P->st, (size_t)P->count));
  if (!P->h_st)
    HIP_TRY(hipHostMalloc((void **)&P->h_st, sizeof(SolveState) * (size_t)P->count, hipHostMallocDefault));
  if (P->hist_cap < maxit + 1) {
    dfree(P->hist);
    P->hist_cap = 0;
    HIP_TRY(dalloc(&P->hist, (size_t)P->count * 2 * (size_t)(maxit + 1), P->bytes));
    P->hist_cap = maxit + 1;
  }
  return ADR_OK;
}

IterBufs iter_bufs(adr_problem *P, double *x, double tol, int maxit) {
  IterBufs B;
  B.A = P->dia();
  B.tab = P->stencil_tab();
  B.b = P->rhs;
  B.x = x;
  B.r = P->r;
  B.rh = P->rh;
  B.p = P->p;
  B.v = P->v;
  B.s = P->s;
  B.t = P->t;
  B.ph = P->ph;
  B.z = P->z;
  B.partials = P->partials;
  B.st = P->st;
  B.hist = P->hist;
  B.tol = tol;
  B.maxit = maxit;
  B.max_restarts = P->max_restarts;
  return B;
}

Factors64 f64_of(const adr_problem *P) { return Factors64{P->lw, P->ls, P->invd}; }
Factors32 f32_of(const adr_problem *P) { return Factors32{P->lw32, P->ls32, P->invd32, P->E32, P->N32}; }

// One BiCGSTAB pass over the batch (13 kernels).
hipError_t enqueue_pass(adr_problem *P, const IterBufs &B, hipStream_t s) {
  const BatchGeom g = P->geom();
  const Factors64 f64 = f64_of(P);
  const Factors32 f32 = f32_of(P);
  const double *tab = P->stencil_tab();
  const int prec = P->precision;
  hipError_t e;
  if ((e = launch_pass_p(B, g, s)) != hipSuccess) return e;
  if ((e = launch_lsweep(g, prec, f64, f32, tab, P->p, P->y, P->sync(), P->st, s)) != hipSuccess) return e;
  if ((e = launch_usweep(g, prec, P->dia(), f64, f32, tab, P->y, P->ph, P->sync(), P->st, s)) != hipSuccess) return e;
  if ((e = launch_pass_v(B, g, s)) != hipSuccess) return e;
  if ((e = launch_pass_s(B, g, s)) != hipSuccess) return e;
  if ((e = launch_lsweep(g, prec, f64, f32, tab, P->s, P->y, P->sync(), P->st, s)) != hipSuccess) return e;
  if ((e = launch_usweep(g, prec, P->dia(), f64, f32, tab, P->y, P->z, P->sync(), P->st, s)) != hipSuccess) return e;
  if ((e = launch_pass_t(B, g, s)) != hipSuccess) return e;
  return launch_pass_xr(B, g, s);
}

adr_status build_graph(adr_problem *P, const IterBufs &B, int K) {
  if (P->gexec) {
    (void)hipGraphExecDestroy(P->gexec);
    P->gexec = nullptr;
  }
  if (!P->cap) HIP_TRY(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int k = 0; k < K && e == hipSuccess; ++k) e = enqueue_pass(P, B, P->cap);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(P->cap, &g);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    HIP_TRY(e);
  }
  HIP_TRY(e2);
  hipError_t e3 = hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIP_TRY(e3);
  P->g_K = K;
  return ADR_OK;
}

adr_status set_rows(adr_problem *P, int R) {
  if (R == P->rows) return ADR_OK;
  HIP_TRY(hipStreamSynchronize(P->stream));
  return build_table(P, R);
}

// Value v[i] of an item of problem data with `len` entries (1: broadcast).
inline double data_at(const double *v, int64_t len, int64_t i) { return v[len == 1 ? 0 : i]; }

// Assemble instance k into its slices of the batched arrays.  d: the
// caller's problem data (already validated), or NULL.
adr_status assemble_one(adr_problem *P, int k, const double *field_dev, double amp, const adr_problem_data *d) {
  const Inst &I = P->inst[k];
  const int nx = I.nx, ny = I.ny;
  const double eps = P->eps[k], X = P->X[k], Y = P->Y[k];
  const double dx = X / (double)(nx + 1), dy = Y / (double)(ny + 1);
  const double e1 = std::exp(-1.0);
  std::vector<double> tx(6 * (size_t)nx), ty(7 * (size_t)ny);
  double *xi = &tx[0], *ai = xi + nx, *exi = ai + nx, *uy0 = exi + nx, *uyY = uy0 + nx, *gyY = uyY + nx;
  double *yj = &ty[0], *bj = yj + ny, *eyj = bj + ny, *ebj = eyj + ny, *ux0 = ebj + ny, *uxX = ux0 + ny,
         *gxX = uxX + ny;
  // 1-D tables on the host (the same formulas and libm as the CPU reference)
  for (int i = 0; i < nx; ++i) {
    const double x = (double)(i + 1) * dx;
    xi[i] = x;
    ai[i] = 1.0 + x * x;
    exi[i] = std::exp(-x / X);
    uy0[i] = 0.0;
    uyY[i] = (exi[i] * (1.0 - e1)) * Y;
    gyY[i] = exi[i] * (e1 + (1.0 - e1));
  }
  for (int j = 0; j < ny; ++j) {
    const double y = (double)(j + 1) * dy;
    yj[j] = y;
    ebj[j] = std::exp(-y);
    bj[j] = X * std::exp(-y);
    eyj[j] = std::exp(-y / Y);
    ux0[j] = (1.0 - eyj[j]) * y;
    uxX[j] = (e1 * (1.0 - eyj[j])) * y;
    gxX[j] = (((-1.0 / X) * e1) * (1.0 - eyj[j])) * y;
  }
  // the caller's boundary data replaces the manufactured values (for the
  // Neumann sides it is the normal derivative)
  const bool neu = P->bc[k] == ADR_BC_NEUMANN_XY;
  if (d) {
    for (int j = 0; j < ny; ++j) {
      if (d->u_x0) ux0[j] = data_at(d->u_x0, d->u_x0_len, j);
      if (d->u_xX) (neu ? gxX : uxX)[j] = data_at(d->u_xX, d->u_xX_len, j);
    }
    for (int i = 0; i < nx; ++i) {
      if (d->u_y0) uy0[i] = data_at(d->u_y0, d->u_y0_len, i);
      if (d->u_yY) (neu ? gyY : uyY)[i] = data_at(d->u_yY, d->u_yY_len, i);
    }
  }
  double *dtab = nullptr;
  double *dfu = nullptr;      // host forcing array, uploaded
  size_t tb = 0;
  HIP_TRY(dalloc(&dtab, tx.size() + ty.size(), tb));
  hipError_t e = hipMemcpyAsync(dtab, tx.data(), tx.size() * sizeof(double), hipMemcpyHostToDevice, P->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dtab + tx.size(), ty.data(), ty.size() * sizeof(double), hipMemcpyHostToDevice, P->stream);
  AssembleArgs a;
  a.nx = nx; a.ny = ny; a.scheme = P->scheme[k]; a.bc = P->bc[k];
  a.eps = eps; a.X = X; a.Y = Y; a.dx = dx; a.dy = dy;
  const double *dx0 = dtab, *dy0 = dtab + tx.size();
  a.xi = dx0; a.ai = dx0 + nx; a.exi = dx0 + 2 * nx; a.uy0 = dx0 + 3 * nx; a.uyY = dx0 + 4 * nx; a.gyY = dx0 + 5 * nx;
  a.yj = dy0; a.bj = dy0 + ny; a.eyj = dy0 + 2 * ny; a.ebj = dy0 + 3 * ny; a.ux0 = dy0 + 4 * ny; a.uxX = dy0 + 5 * ny;
  a.gxX = dy0 + 6 * ny;
  a.field = field_dev ? field_dev + I.off : nullptr;
  a.amp = amp;
  a.fmode = 0;
  a.fuser = nullptr;
  a.fconst = 0.0;
  if (d && d->f) {
    if (d->f_len == 1 && !d->f_on_device) {
      a.fmode = 2;
      a.fconst = d->f[0];
    } else if (d->f_on_device) {
      a.fmode = 1;
      a.fuser = d->f;
    } else {
      a.fmode = 1;
      size_t fb = 0;
      if (e == hipSuccess) e = dalloc(&dfu, (size_t)I.n, fb);
      if (e == hipSuccess)
        e = hipMemcpyAsync(dfu, d->f, (size_t)I.n * sizeof(double), hipMemcpyHostToDevice, P->stream);
      a.fuser = dfu;
    }
  }
  a.S = P->S + I.off; a.W = P->W + I.off; a.C = P->C + I.off; a.E = P->E + I.off; a.N = P->N + I.off;
  a.rhs = P->rhs + I.off;
  a.F = P->F + I.off;
  a.partials = P->partials;
  a.fmax = P->scal;
  if (e == hipSuccess) e = launch_assemble(a, make_geom(I.n), P->stream);
  hipError_t es = hipStreamSynchronize(P->stream);
  (void)hipFree(dtab);
  if (dfu) (void)hipFree(dfu);
  HIP_TRY(e);
  HIP_TRY(es);
  return ADR_OK;
}

// Copy the stencil tables out of the diagonals and keep them only if every
// point's S, W, E, N equals its table entry (always so for assembled
// operators; a matrix given through adr_set_dia may not be separable).
adr_status refresh_stencil_tables(adr_problem *P) {
  P->has_tab = 0;
  if (!P->tab) HIP_TRY(dalloc(&P->tab, (size_t)P->tab_len, P->bytes));
  if (!P->tab_bad) HIP_TRY(dalloc(&P->tab_bad, 1, P->bytes));
  HIP_TRY(launch_fill_u32(P->tab_bad, 1, 0u, P->stream));
  HIP_TRY(launch_stencil_tables(P->dia(), P->geom(), P->tab, P->tab_bad, P->stream));
  unsigned bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, P->tab_bad, sizeof(unsigned), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  P->has_tab = bad == 0;
  return ADR_OK;
}

adr_status ensure_feat_table(adr_problem *P) {
  if (P->d_feat) return ADR_OK;
  std::vector<FeatInst> fi((size_t)P->count);
  for (int k = 0; k < P->count; ++k) {
    fi[k].eps = P->eps[k];
    fi[k].X = P->X[k];
    fi[k].Y = P->Y[k];
    fi[k].nx = P->nx[k];
    fi[k].ny = P->ny[k];
    fi[k].bc = P->bc[k];
    fi[k].scheme = P->scheme[k];
    fi[k].off = P->inst[k].off;
  }
  size_t b = 0;
  HIP_TRY(dalloc(&P->d_feat, fi.size(), b));
  HIP_TRY(hipMemcpy(P->d_feat, fi.data(), fi.size() * sizeof(FeatInst), hipMemcpyHostToDevice));
  P->bytes += b;
  return ADR_OK;
}

adr_status require_single(const adr_problem *P) {
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  if (P->count != 1) return fail(ADR_ERR_STATE, "this call needs a single-instance problem");
  return ADR_OK;
}

}  // namespace

extern "C" {

const char *adr_status_str(int32_t st) {
  switch (st) {
    case ADR_OK: return "ok";
    case ADR_ERR_ARG: return "invalid argument";
    case ADR_ERR_NOMEM: return "out of device memory";
    case ADR_ERR_DEVICE: return "device error";
    case ADR_ERR_STATE: return "call out of order";
    case ADR_MAXIT: return "maximum iterations reached";
    case ADR_BREAKDOWN_RHO: return "breakdown: rho = 0";
    case ADR_OMEGA_ZERO: return "omega = 0";
    case ADR_ZERO_PIVOT: return "zero or non-finite pivot";
    case ADR_NONFINITE: return "non-finite value";
    case ADR_INACCURATE: return "true residual above tolerance after the allowed restarts";
    default: return "unknown status";
  }
}

const char *adr_last_error(void) { return g_last_error.c_str(); }

void adr_destroy(adr_problem *P) {
  if (!P) return;
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
  if (P->cap) (void)hipStreamDestroy(P->cap);
  double *dv[] = {P->S, P->W, P->C, P->E, P->N, P->rhs, P->F, P->lw, P->ls, P->invd, P->r, P->rh,
                  P->p, P->v, P->s, P->t, P->ph, P->z, P->y, P->hist, P->scal, P->tab};
  for (double *q : dv) pfree(P, q);
  float *fv[] = {P->lw32, P->ls32, P->invd32, P->E32, P->N32};
  for (float *q : fv) pfree(P, q);
  dfree(P->partials);
  pfree(P, P->st);
  dfree(P->bad);
  pfree(P, P->ticket);
  pfree(P, P->handoff);
  pfree(P, P->err);
  dfree(P->d_inst);
  dfree(P->d_sorder);
  dfree(P->d_feat);
  dfree(P->tab_bad);
  if (P->h_st) (void)hipHostFree(P->h_st);
  if (P->ev0) (void)hipEventDestroy(P->ev0);
  if (P->ev1) (void)hipEventDestroy(P->ev1);
  if (P->ev_chunk) (void)hipEventDestroy(P->ev_chunk);
  delete P;
}

}  // extern "C"

namespace {

adr_status check_data(int k, int nx, int ny, const adr_problem_data &d) {
  struct Item {
    const char *name;
    const double *p;
    int64_t len, full;
  } items[] = {{"f", d.f, d.f_len, (int64_t)nx * ny}, {"u_x0", d.u_x0, d.u_x0_len, ny},
               {"u_xX", d.u_xX, d.u_xX_len, ny}, {"u_y0", d.u_y0, d.u_y0_len, nx},
               {"u_yY", d.u_yY, d.u_yY_len, nx}};
  for (const Item &it : items) {
    if (!it.p) {
      if (it.len != 0) return fail(ADR_ERR_ARG, "instance %d: %s is NULL but has length %lld", k, it.name, (long long)it.len);
      continue;
    }
    if (it.len != 1 && it.len != it.full)
      return fail(ADR_ERR_ARG, "instance %d: %s has %lld values; expected 1 or %lld", k, it.name, (long long)it.len,
                  (long long)it.full);
  }
  if (d.f_on_device && d.f && d.f_len != (int64_t)nx * ny)
    return fail(ADR_ERR_ARG, "instance %d: a device forcing array needs nx*ny = %lld values", k, (long long)nx * ny);
  if (d.f_on_device != 0 && d.f_on_device != 1) return fail(ADR_ERR_ARG, "instance %d: f_on_device must be 0 or 1", k);
  return ADR_OK;
}

adr_status batch_assemble(int32_t count, const double *eps, const double *X, const double *Y, const int32_t *nx,
                          const int32_t *ny, const int32_t *scheme, const int32_t *bc, const double *field_dev,
                          double amp, const adr_problem_data *data, void *stream, adr_problem **out) {
  if (!out) return fail(ADR_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (count < 1) return fail(ADR_ERR_ARG, "count must be >= 1 (got %d)", count);
  if (!eps || !X || !Y || !nx || !ny || !scheme || !bc) return fail(ADR_ERR_ARG, "NULL parameter array");
  for (int k = 0; k < count; ++k) {
    if (!(eps[k] > 0.0) || !std::isfinite(eps[k]))
      return fail(ADR_ERR_ARG, "instance %d: eps must be a finite number > 0 (got %g)", k, eps[k]);
    if (!(X[k] > 0.0) || !(Y[k] > 0.0) || !std::isfinite(X[k]) || !std::isfinite(Y[k]))
      return fail(ADR_ERR_ARG, "instance %d: X and Y must be finite and > 0 (got %g, %g)", k, X[k], Y[k]);
    if (nx[k] < 1 || ny[k] < 1)
      return fail(ADR_ERR_ARG, "instance %d: nx and ny must be >= 1 (got %d, %d)", k, nx[k], ny[k]);
    if (scheme[k] != ADR_UPWIND && scheme[k] != ADR_CENTERED)
      return fail(ADR_ERR_ARG, "instance %d: unknown scheme %d", k, scheme[k]);
    if (bc[k] != ADR_BC_DIRICHLET && bc[k] != ADR_BC_NEUMANN_XY)
      return fail(ADR_ERR_ARG, "instance %d: unknown bc %d", k, bc[k]);
    if ((int64_t)nx[k] * ny[k] > (int64_t)0x7fffffff)
      return fail(ADR_ERR_ARG, "instance %d: nx*ny must be < 2^31", k);
  }
  if (field_dev && !std::isfinite(amp)) return fail(ADR_ERR_ARG, "amp must be finite");
  if (data)
    for (int k = 0; k < count; ++k) {
      adr_status dst = check_data(k, nx[k], ny[k], data[k]);
      if (dst != ADR_OK) return dst;
    }

  adr_problem *P = new adr_problem();
  auto bail = [&](adr_status st) {
    adr_destroy(P);
    return st;
  };
  if (hipGetDevice(&P->dev) != hipSuccess) return bail(fail(ADR_ERR_DEVICE, "no HIP device"));
  if (hipDeviceGetAttribute(&P->cus, hipDeviceAttributeMultiprocessorCount, P->dev) != hipSuccess || P->cus < 1)
    return bail(fail(ADR_ERR_DEVICE, "cannot read the device's compute-unit count"));
  P->stream = (hipStream_t)stream;
  P->count = count;
  P->eps.assign(eps, eps + count);
  P->X.assign(X, X + count);
  P->Y.assign(Y, Y + count);
  P->nx.assign(nx, nx + count);
  P->ny.assign(ny, ny + count);
  P->scheme.assign(scheme, scheme + count);
  P->bc.assign(bc, bc + count);
  P->inst.resize(count);
  P->max_ny = *std::max_element(ny, ny + count);
  adr_status st = build_table(P, default_rows(P->max_ny));
  if (st != ADR_OK) return bail(st);
  double **arrs[] = {&P->S, &P->W, &P->C, &P->E, &P->N, &P->rhs, &P->F};
  for (double **q : arrs)
    if (dalloc(q, (size_t)P->ntot, P->bytes) != hipSuccess) return bail(fail(ADR_ERR_NOMEM, "device allocation failed"));
  // partials: 4 slots for every streaming block of the batch, and of one instance's assembly
  if (dalloc(&P->partials, (size_t)4 * P->nblk + 4 * 2048, P->bytes) != hipSuccess ||
      dalloc(&P->scal, 8, P->bytes) != hipSuccess || dalloc(&P->bad, (size_t)count, P->bytes) != hipSuccess)
    return bail(fail(ADR_ERR_NOMEM, "device allocation failed"));
  for (int k = 0; k < count; ++k) {
    st = assemble_one(P, k, data ? nullptr : field_dev, amp, data ? &data[k] : nullptr);
    if (st != ADR_OK) return bail(st);
  }
  st = refresh_stencil_tables(P);
  if (st != ADR_OK) return bail(st);
  *out = P;
  return ADR_OK;
}

}  // namespace

extern "C" {

adr_status adr_batch_assemble(int32_t count, const double *eps, const double *X, const double *Y,
                              const int32_t *nx, const int32_t *ny, const int32_t *scheme,
                              const int32_t *bc, const double *field_dev, double amp, void *stream,
                              adr_problem **out) {
  g_last_error.clear();
  return batch_assemble(count, eps, X, Y, nx, ny, scheme, bc, field_dev, amp, nullptr, stream, out);
}

adr_status adr_batch_assemble_data(int32_t count, const double *eps, const double *X, const double *Y,
                                   const int32_t *nx, const int32_t *ny, const int32_t *scheme,
                                   const int32_t *bc, const adr_problem_data *data, void *stream,
                                   adr_problem **out) {
  g_last_error.clear();
  return batch_assemble(count, eps, X, Y, nx, ny, scheme, bc, nullptr, 0.0, data, stream, out);
}

adr_status adr_assemble_data(double eps, double X, double Y, int32_t nx, int32_t ny, int32_t scheme, int32_t bc,
                             const adr_problem_data *data, void *stream, adr_problem **out) {
  g_last_error.clear();
  return batch_assemble(1, &eps, &X, &Y, &nx, &ny, &scheme, &bc, nullptr, 0.0, data, stream, out);
}

adr_status adr_assemble(double eps, double X, double Y, int32_t nx, int32_t ny, int32_t scheme,
                        int32_t bc, const double *field_dev, double amp, void *stream,
                        adr_problem **out) {
  return adr_batch_assemble(1, &eps, &X, &Y, &nx, &ny, &scheme, &bc, field_dev, amp, stream, out);
}

adr_status adr_batch_layout(const adr_problem *P, int32_t *count, int64_t *offsets) {
  g_last_error.clear();
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  if (count) *count = P->count;
  if (offsets) {
    for (int k = 0; k < P->count; ++k) offsets[k] = P->inst[k].off;
    offsets[P->count] = P->ntot;
  }
  return ADR_OK;
}

adr_status adr_get_dia(const adr_problem *P, double *S, double *W, double *C, double *E, double *N,
                       double *rhs) {
  g_last_error.clear();
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  const double *src[] = {P->S, P->W, P->C, P->E, P->N, P->rhs};
  double *dst[] = {S, W, C, E, N, rhs};
  for (int q = 0; q < 6; ++q)
    if (dst[q])
      HIP_TRY(hipMemcpyAsync(dst[q], src[q], (size_t)P->ntot * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return ADR_OK;
}

adr_status adr_set_dia(adr_problem *P, const double *S, const double *W, const double *C,
                       const double *E, const double *N, const double *rhs) {
  g_last_error.clear();
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  const double *src[] = {S, W, C, E, N, rhs};
  double *dst[] = {P->S, P->W, P->C, P->E, P->N, P->rhs};
  for (int q = 0; q < 6; ++q)
    if (!src[q]) return fail(ADR_ERR_ARG, "all six arrays are required");
  for (int q = 0; q < 6; ++q)
    HIP_TRY(hipMemcpyAsync(dst[q], src[q], (size_t)P->ntot * sizeof(double), hipMemcpyHostToDevice, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  P->factored = 0;
  return refresh_stencil_tables(P);
}

adr_status adr_get_factors(const adr_problem *P, double *lw, double *ls, double *invd) {
  g_last_error.clear();
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  if (!P->factored) return fail(ADR_ERR_STATE, "no factorisation (call adr_ilu0 first)");
  const double *src[] = {P->lw, P->ls, P->invd};
  double *dst[] = {lw, ls, invd};
  for (int q = 0; q < 3; ++q)
    if (dst[q])
      HIP_TRY(hipMemcpyAsync(dst[q], src[q], (size_t)P->ntot * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return ADR_OK;
}

adr_status adr_set_sweep_rows(adr_problem *P, int32_t rows) {
  g_last_error.clear();
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  if (rows != 0 && rows != 16 && rows != 32) return fail(ADR_ERR_ARG, "rows must be 0, 16 or 32 (got %d)", rows);
  P->compact = -1;
  return set_rows(P, rows ? rows : default_rows(P->max_ny));
}

adr_status adr_set_sweep_ring(adr_problem *P, int32_t mode) {
  g_last_error.clear();
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  if (mode < -1 || mode > 1) return fail(ADR_ERR_ARG, "ring mode must be -1, 0 or 1 (got %d)", mode);
  P->compact = mode;
  return ADR_OK;
}

int32_t adr_sweep_ring(const adr_problem *P) { return P ? P->ring_compact() : 0; }

size_t adr_device_bytes(const adr_problem *P) { return P ? P->bytes : 0; }

adr_status adr_use_stencil_tables(adr_problem *P, int32_t enable) {
  g_last_error.clear();
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  if (enable != 0 && enable != 1) return fail(ADR_ERR_ARG, "enable must be 0 or 1 (got %d)", enable);
  P->tab_on = enable;
  return ADR_OK;
}

int32_t adr_stencil_tables(const adr_problem *P) { return (P && P->stencil_tab()) ? 1 : 0; }

double adr_last_call_ms(const adr_problem *P) { return P ? (double)P->last_ms : 0.0; }

size_t adr_workspace_bytes(const adr_problem *P, int32_t precision) {
  if (!P || precision < ADR_FP64 || precision > ADR_FP32_SWEEPS) return 0;
  return workspace_bytes(P, precision);
}

adr_status adr_bind_workspace(adr_problem *P, void *dev_ptr, size_t bytes) {
  g_last_error.clear();
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  if (!dev_ptr) return fail(ADR_ERR_ARG, "workspace is NULL");
  if ((uintptr_t)dev_ptr % WS_ALIGN) return fail(ADR_ERR_ARG, "workspace must be %zu-byte aligned", WS_ALIGN);
  const size_t need = workspace_bytes(P, ADR_FP64);
  if (bytes < need) return fail(ADR_ERR_ARG, "workspace of %zu bytes is below the %zu the problem needs", bytes, need);
  if (P->ws || P->ticket || P->handoff || P->err || P->lw || P->ls || P->invd || P->lw32 || P->r || P->st)
    return fail(ADR_ERR_STATE, "bind the workspace once, before adr_ilu0 / adr_batch_ilu0 and any solve");
  P->ws = (char *)dev_ptr;
  P->ws_bytes = bytes;
  P->ws_used = 0;
  return ADR_OK;
}

adr_status adr_batch_ilu0(adr_problem *P, int32_t precision, int64_t *bad_index) {
  g_last_error.clear();
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  if (bad_index)
    for (int k = 0; k < P->count; ++k) bad_index[k] = -1;
  if (precision < ADR_FP64 || precision > ADR_FP32_SWEEPS) return fail(ADR_ERR_ARG, "unknown precision %d", precision);
  adr_status st = ensure_sync(P);
  if (st != ADR_OK) return st;
  double **dv[] = {&P->lw, &P->ls, &P->invd};
  for (double **q : dv)
    if (!*q) HIP_TRY(palloc(P, q, (size_t)P->ntot));
  if (precision != ADR_FP64) {
    float **fv[] = {&P->lw32, &P->ls32, &P->invd32, &P->E32, &P->N32};
    for (float **q : fv)
      if (!*q) HIP_TRY(palloc(P, q, (size_t)P->ntot));
  }
  P->factored = 0;
  HIP_TRY(launch_fill_u64((uint64_t *)P->bad, P->count, ~0ull, P->stream));
  Factors32 h{};
  if (precision != ADR_FP64) h = f32_of(P);
  HIP_TRY(launch_ilu0(P->dia(), P->geom(), f64_of(P), h, P->sync(), P->bad, P->stream));
  std::vector<uint64_t> hb((size_t)P->count);
  HIP_TRY(hipMemcpyAsync(hb.data(), P->bad, sizeof(uint64_t) * hb.size(), hipMemcpyDeviceToHost, P->stream));
  st = check_device_fault(P);
  if (st != ADR_OK) return st;
  int first_bad = -1;
  for (int k = 0; k < P->count; ++k)
    if (hb[k] != ~0ull) {
      if (bad_index) bad_index[k] = (int64_t)hb[k];
      if (first_bad < 0) first_bad = k;
    }
  if (first_bad >= 0)
    return fail(ADR_ZERO_PIVOT, "instance %d: zero or non-finite pivot at unknown %lld", first_bad,
                (long long)hb[first_bad]);
  P->factored = 1;
  P->precision = precision;
  return ADR_OK;
}

adr_status adr_ilu0(adr_problem *P, int32_t precision, int64_t *bad_index) {
  g_last_error.clear();
  adr_status st = require_single(P);
  if (st != ADR_OK) return st;
  return adr_batch_ilu0(P, precision, bad_index);
}

adr_status adr_spmv(adr_problem *P, const double *x, double *v) {
  g_last_error.clear();
  adr_status st = require_single(P);
  if (st != ADR_OK) return st;
  if (!x || !v) return fail(ADR_ERR_ARG, "NULL argument");
  const Inst &I = P->inst[0];
  st = ensure_events(P);
  if (st != ADR_OK) return st;
  HIP_TRY(hipEventRecord(P->ev0, P->stream));
  HIP_TRY(launch_spmv(P->dia(), I.fd, I.nx, I.ny, x, v, make_geom(I.n), P->stream));
  HIP_TRY(hipEventRecord(P->ev1, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return read_call_ms(P);
}

adr_status adr_lsolve(adr_problem *P, const double *q, double *y) {
  g_last_error.clear();
  if (!P || !q || !y) return fail(ADR_ERR_ARG, "NULL argument");
  if (!P->factored) return fail(ADR_ERR_STATE, "no factorisation (call adr_ilu0 first)");
  adr_status st = ensure_events(P);
  if (st != ADR_OK) return st;
  HIP_TRY(hipEventRecord(P->ev0, P->stream));
  HIP_TRY(launch_lsweep(P->geom(), P->precision, f64_of(P), f32_of(P), P->stencil_tab(), q, y, P->sync(), nullptr,
                        P->stream));
  HIP_TRY(hipEventRecord(P->ev1, P->stream));
  st = check_device_fault(P);
  return st != ADR_OK ? st : read_call_ms(P);
}

adr_status adr_usolve(adr_problem *P, const double *y, double *z) {
  g_last_error.clear();
  if (!P || !y || !z) return fail(ADR_ERR_ARG, "NULL argument");
  if (!P->factored) return fail(ADR_ERR_STATE, "no factorisation (call adr_ilu0 first)");
  adr_status st = ensure_events(P);
  if (st != ADR_OK) return st;
  HIP_TRY(hipEventRecord(P->ev0, P->stream));
  HIP_TRY(launch_usweep(P->geom(), P->precision, P->dia(), f64_of(P), f32_of(P), P->stencil_tab(), y, z, P->sync(),
                        nullptr, P->stream));
  HIP_TRY(hipEventRecord(P->ev1, P->stream));
  st = check_device_fault(P);
  return st != ADR_OK ? st : read_call_ms(P);
}

adr_status adr_precond(adr_problem *P, const double *q, double *z) {
  g_last_error.clear();
  if (!P || !q || !z) return fail(ADR_ERR_ARG, "NULL argument");
  if (!P->factored) return fail(ADR_ERR_STATE, "no factorisation (call adr_ilu0 first)");
  adr_status st = ensure_iter_buffers(P, 0);
  if (st == ADR_OK) st = ensure_events(P);
  if (st != ADR_OK) return st;
  HIP_TRY(hipEventRecord(P->ev0, P->stream));
  HIP_TRY(launch_lsweep(P->geom(), P->precision, f64_of(P), f32_of(P), P->stencil_tab(), q, P->y, P->sync(), nullptr,
                        P->stream));
  HIP_TRY(launch_usweep(P->geom(), P->precision, P->dia(), f64_of(P), f32_of(P), P->stencil_tab(), P->y, z, P->sync(),
                        nullptr, P->stream));
  HIP_TRY(hipEventRecord(P->ev1, P->stream));
  st = check_device_fault(P);
  return st != ADR_OK ? st : read_call_ms(P);
}

adr_status adr_autotune(adr_problem *P, int32_t *rows_chosen, double *ms_per_apply) {
  g_last_error.clear();
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  if (!P->factored) return fail(ADR_ERR_STATE, "no factorisation (call adr_ilu0 first)");
  adr_status st = ensure_iter_buffers(P, 0);
  if (st == ADR_OK) st = ensure_events(P);
  if (st != ADR_OK) return st;
  // time M^{-1} applied to the batch's right-hand sides for every strip
  // schedule: 16-row strips, 32-row strips with the deep ring, with the compact one
  const int cand[][2] = {{16, -1}, {32, 0}, {32, 1}};
  int best = P->rows, best_cmp = P->compact;
  float best_ms = -1.f;
  hipEvent_t e0 = P->ev0, e1 = P->ev1;
  for (const auto &c : cand) {
    const int R = c[0];
    P->compact = c[1];
    st = set_rows(P, R);
    if (st != ADR_OK) return st;
    float ms = 0.f;
    for (int rep = 0; rep < 3; ++rep) {
      HIP_TRY(hipEventRecord(e0, P->stream));
      HIP_TRY(launch_lsweep(P->geom(), P->precision, f64_of(P), f32_of(P), P->stencil_tab(), P->rhs, P->y, P->sync(), nullptr,
                            P->stream));
      HIP_TRY(launch_usweep(P->geom(), P->precision, P->dia(), f64_of(P), f32_of(P), P->stencil_tab(), P->y, P->z, P->sync(), nullptr,
                            P->stream));
      HIP_TRY(hipEventRecord(e1, P->stream));
      HIP_TRY(hipEventSynchronize(e1));
      float m = 0.f;
      HIP_TRY(hipEventElapsedTime(&m, e0, e1));
      if (rep > 0) ms += m / 2.f;   // the first application is a warm-up
    }
    st = check_device_fault(P);
    if (st != ADR_OK) return st;
    if (best_ms < 0.f || ms < best_ms) {
      best_ms = ms;
      best = R;
      best_cmp = c[1];
    }
  }
  P->compact = best_cmp;
  st = set_rows(P, best);
  if (st != ADR_OK) return st;
  if (rows_chosen) *rows_chosen = best;
  if (ms_per_apply) *ms_per_apply = best_ms;
  return ADR_OK;
}

adr_status adr_dot(const double *x, const double *y, int64_t n, void *stream, double *out) {
  g_last_error.clear();
  if (!x || !y || !out || n < 0 || n > 0x7fffffff) return fail(ADR_ERR_ARG, "bad argument");
  if (n == 0) {
    *out = 0.0;
    return ADR_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  Stream1D g = make_geom(n);
  double2 *part = nullptr;
  double *res = nullptr;
  size_t b = 0;
  HIP_TRY(dalloc(&part, (size_t)g.nblk, b));
  hipError_t e = dalloc(&res, 1, b);
  if (e == hipSuccess) e = launch_dot(x, y, g, part, res, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out, res, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(part);
  if (res) (void)hipFree(res);
  HIP_TRY(e);
  return ADR_OK;
}

adr_status adr_batch_solve(adr_problem *P, double tol, int32_t maxit, const double *x0, double *x,
                           double *hist_l2, double *hist_max, adr_solve_info *info) {
  g_last_error.clear();
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  if (info) memset(info, 0, sizeof(*info) * (size_t)P->count);
  if (!x) return fail(ADR_ERR_ARG, "x_dev is NULL");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(ADR_ERR_ARG, "tol must be finite and >= 0 (got %g)", tol);
  if (maxit < 0) return fail(ADR_ERR_ARG, "maxit must be >= 0 (got %d)", maxit);
  if (!P->factored) return fail(ADR_ERR_STATE, "no factorisation (call adr_ilu0 first)");
  adr_status st = ensure_iter_buffers(P, maxit);
  if (st != ADR_OK) return st;
  st = ensure_sync(P);
  if (st != ADR_OK) return st;
  const BatchGeom g = P->geom();
  const size_t vb = (size_t)P->ntot * sizeof(double);
  if (x0) {
    if (x0 != x) HIP_TRY(hipMemcpyAsync(x, x0, vb, hipMemcpyDeviceToDevice, P->stream));
  } else {
    HIP_TRY(launch_fill(x, P->ntot, 0.0, P->stream));
  }
  IterBufs B = iter_bufs(P, x, tol, maxit);
  // passes per graph replay: enough to amortise the host check
  int K = P->ntot >= (1 << 22) ? 4 : (P->ntot >= (1 << 18) ? 8 : 16);
  if (K > maxit && maxit > 0) K = maxit;
  if (!P->gexec || P->g_x != x || P->g_tol != tol || P->g_maxit != maxit || P->g_prec != P->precision ||
      P->g_rows != P->rows || P->g_K != K || P->g_tab != (P->stencil_tab() != nullptr) ||
      P->g_cmp != P->ring_compact() || P->g_mr != P->max_restarts) {
    st = build_graph(P, B, K);
    if (st != ADR_OK) return st;
    P->g_x = x;
    P->g_tol = tol;
    P->g_maxit = maxit;
    P->g_prec = P->precision;
    P->g_rows = P->rows;
    P->g_cmp = P->ring_compact();
    P->g_tab = P->stencil_tab() != nullptr;
    P->g_mr = P->max_restarts;
  }
  auto all_done = [&]() {
    for (int k = 0; k < P->count; ++k)
      if (P->h_st[k].phase != DONE) return false;
    return true;
  };
  const size_t stb = sizeof(SolveState) * (size_t)P->count;
  st = ensure_events(P);
  if (st != ADR_OK) return st;
  hipEvent_t e0 = P->ev0, e1 = P->ev1;
  HIP_TRY(hipEventRecord(e0, P->stream));
  HIP_TRY(launch_init(B, g, P->stream));
  // replay chunks; keep one chunk queued behind the one being checked
  const int max_chunks = maxit > 0 ? (maxit + K - 1) / K : 0;
  int launched = 0;
  bool done = false;
  if (max_chunks > 0) {
    HIP_TRY(hipGraphLaunch(P->gexec, P->stream));
    ++launched;
  }
  while (!done && launched > 0) {
    HIP_TRY(hipMemcpyAsync(P->h_st, P->st, stb, hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipEventRecord(P->ev_chunk, P->stream));
    if (launched < max_chunks) {
      HIP_TRY(hipGraphLaunch(P->gexec, P->stream));
      ++launched;
    }
    HIP_TRY(hipEventSynchronize(P->ev_chunk));
    if (all_done()) {
      done = true;
    } else if (launched >= max_chunks) {
      // the last chunk is queued; wait for it
      HIP_TRY(hipStreamSynchronize(P->stream));
      done = true;
    }
  }
  HIP_TRY(hipEventRecord(e1, P->stream));
  HIP_TRY(launch_true_residual(B, g, P->stream));
  HIP_TRY(hipMemcpyAsync(P->h_st, P->st, stb, hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  st = check_device_fault(P);
  if (st != ADR_OK) return st;
  adr_status result = ADR_OK;
  for (int k = 0; k < P->count; ++k) {
    const SolveState &S = P->h_st[k];
    if (S.phase != DONE) return fail(ADR_ERR_DEVICE, "instance %d did not reach a stopping state", k);
    const int hl = S.hist_len;
    const double *hsrc = P->hist + (size_t)k * 2 * (size_t)(maxit + 1);
    if (hist_l2 && hl > 0)
      HIP_TRY(hipMemcpy(hist_l2 + (size_t)k * (maxit + 1), hsrc, (size_t)hl * sizeof(double), hipMemcpyDeviceToHost));
    if (hist_max && hl > 0)
      HIP_TRY(hipMemcpy(hist_max + (size_t)k * (maxit + 1), hsrc + (maxit + 1), (size_t)hl * sizeof(double),
                        hipMemcpyDeviceToHost));
    if (info) {
      info[k].status = S.status;
      info[k].iters = S.iter;
      info[k].hist_len = hl;
      info[k].half_step = S.half_step;
      info[k].bnorm = S.bnorm;
      info[k].true_relres = S.bnorm > 0.0 ? std::sqrt(S.true_res2) / S.bnorm : 0.0;
      info[k].solve_ms = ms;
      info[k].restarts = S.restarts;
    }
    if (result == ADR_OK && S.status != ADR_OK) result = (adr_status)S.status;
  }
  return result;
}

adr_status adr_bicgstab_solve(adr_problem *P, double tol, int32_t maxit, const double *x0, double *x,
                              double *hist_l2, double *hist_max, adr_solve_info *info) {
  g_last_error.clear();
  adr_status st = require_single(P);
  if (st != ADR_OK) {
    if (info) memset(info, 0, sizeof(*info));
    return st;
  }
  return adr_batch_solve(P, tol, maxit, x0, x, hist_l2, hist_max, info);
}

adr_status adr_cnn_features(const adr_problem *P, int32_t first, int32_t count, uint16_t *out) {
  g_last_error.clear();
  if (!P || !out) return fail(ADR_ERR_ARG, "NULL argument");
  if (first < 0 || count < 1 || (int64_t)first + count > P->count)
    return fail(ADR_ERR_ARG, "instances [%d, %d) out of range [0, %d)", first, first + count, P->count);
  for (int k = first; k < first + count; ++k)
    if (P->nx[k] != P->nx[first] || P->ny[k] != P->ny[first])
      return fail(ADR_ERR_ARG, "instances %d and %d differ in size", first, k);
  adr_status st = ensure_feat_table(const_cast<adr_problem *>(P));
  if (st != ADR_OK) return st;
  const int H = P->ny[first] + 2, W = P->nx[first] + 2;
  HIP_TRY(launch_cnn_features(P->d_feat + first, count, H, W, P->F, out, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return ADR_OK;
}

adr_status adr_batch_warm_start(adr_problem *P, adr_cnn *net, double *x, int32_t *used) {
  g_last_error.clear();
  if (!P || !net || !x) return fail(ADR_ERR_ARG, "NULL argument");
  int H, W, maxB;
  hipStream_t ns;
  uint16_t *in;
  float *u;
  cnn_shape(net, &H, &W, &maxB, &ns, &in, &u);
  for (int k = 0; k < P->count; ++k)
    if (P->nx[k] != W - 2 || P->ny[k] != H - 2)
      return fail(ADR_ERR_ARG, "instance %d is %d x %d; the network takes %d x %d interior grids", k, P->nx[k],
                  P->ny[k], W - 2, H - 2);
  adr_status st = ensure_feat_table(P);
  if (st != ADR_OK) return st;
  st = ensure_iter_buffers(P, 0);
  if (st != ADR_OK) return st;
  HIP_TRY(hipStreamSynchronize(P->stream));
  for (int c0 = 0; c0 < P->count; c0 += maxB) {
    const int nb = std::min(maxB, P->count - c0);
    HIP_TRY(launch_cnn_features(P->d_feat + c0, nb, H, W, P->F, in, ns));
    st = adr_cnn_forward(net, in, nb, u);
    if (st != ADR_OK) return st;
    HIP_TRY(launch_cnn_extract(P->d_feat + c0, nb, H, W, u, x, ns));
  }
  HIP_TRY(hipStreamSynchronize(ns));
  // fallback test: keep the guess only where ||b - A x0||_2 is finite and below ||b||_2
  IterBufs B = iter_bufs(P, x, 0.0, 0);
  HIP_TRY(launch_init(B, P->geom(), P->stream));
  std::vector<double> h0((size_t)2 * P->count);
  HIP_TRY(hipMemcpyAsync(P->h_st, P->st, sizeof(SolveState) * (size_t)P->count, hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipMemcpyAsync(h0.data(), P->hist, h0.size() * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  for (int k = 0; k < P->count; ++k) {
    const double bn = P->h_st[k].bnorm, rn = h0[(size_t)2 * k];
    const bool keep = bn > 0.0 && std::isfinite(rn) && rn < bn;
    if (!keep) HIP_TRY(launch_fill(x + P->inst[k].off, P->inst[k].n, 0.0, P->stream));
    if (used) used[k] = keep ? 1 : 0;
  }
  HIP_TRY(hipStreamSynchronize(P->stream));
  return ADR_OK;
}

adr_status adr_set_max_restarts(adr_problem *P, int32_t n) {
  g_last_error.clear();
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  if (n < -1) return fail(ADR_ERR_ARG, "max_restarts must be >= -1 (got %d)", n);
  P->max_restarts = n;
  return ADR_OK;
}

adr_status adr_max_error(adr_problem *P, const double *x, double *err_host) {
  g_last_error.clear();
  if (!P || !x || !err_host) return fail(ADR_ERR_ARG, "NULL argument");
  double *res = P->scal + 1;   // device scalar (scal[0] is the assembly's max|f|)
  for (int k = 0; k < P->count; ++k) {
    const Inst &I = P->inst[k];
    MaxErrArgs a;
    a.nx = I.nx;
    a.ny = I.ny;
    a.bc = P->bc[k];
    a.X = P->X[k];
    a.Y = P->Y[k];
    a.dx = P->X[k] / (double)(I.nx + 1);
    a.dy = P->Y[k] / (double)(I.ny + 1);
    a.x = x + I.off;
    a.partials = P->partials;
    a.out = res;
    const int64_t nodes = (int64_t)(I.nx + 2) * (I.ny + 2);
    if (nodes > 0x7fffffff) return fail(ADR_ERR_ARG, "instance %d: grid too large for adr_max_error", k);
    HIP_TRY(launch_max_error(a, make_geom(nodes), P->stream));
    HIP_TRY(hipMemcpyAsync(err_host + k, res, sizeof(double), hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
  }
  return ADR_OK;
}

adr_status adr_classify(double eps, double X, double Y, int32_t nx, int32_t ny, int32_t scheme, int32_t bc,
                        double tol, adr_instance_class *out) {
  g_last_error.clear();
  if (!out) return fail(ADR_ERR_ARG, "out is NULL");
  memset(out, 0, sizeof(*out));
  if (!(eps > 0.0) || !(X > 0.0) || !(Y > 0.0) || !std::isfinite(eps) || !std::isfinite(X) || !std::isfinite(Y))
    return fail(ADR_ERR_ARG, "eps, X and Y must be finite and > 0");
  if (nx < 1 || ny < 1) return fail(ADR_ERR_ARG, "nx and ny must be >= 1 (got %d, %d)", nx, ny);
  if (scheme != ADR_UPWIND && scheme != ADR_CENTERED) return fail(ADR_ERR_ARG, "unknown scheme %d", scheme);
  if (bc != ADR_BC_DIRICHLET && bc != ADR_BC_NEUMANN_XY) return fail(ADR_ERR_ARG, "unknown bc %d", bc);
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(ADR_ERR_ARG, "tol must be finite and >= 0 (got %g)", tol);
  // the Section 4 coefficients, per column (through a) and per row (through
  // b), evaluated as the assembly kernel evaluates them
  const double dx = X / (double)(nx + 1), dy = Y / (double)(ny + 1);
  const double dx2 = dx * dx, dy2 = dy * dy;
  const double cx = eps * dy2, cy = eps * dx2, gx = dx * dy2, gy = dx2 * dy;
  std::vector<double> ax((size_t)nx), by((size_t)ny);
  double amax = 0.0, bmax = 0.0;
  for (int i = 0; i < nx; ++i) {
    const double x = (double)(i + 1) * dx;
    ax[i] = 1.0 + x * x;
    amax = std::max(amax, ax[i]);
  }
  for (int j = 0; j < ny; ++j) {
    by[j] = X * std::exp(-(double)(j + 1) * dy);
    bmax = std::max(bmax, by[j]);
  }
  out->pe_x = amax * dx / eps;
  out->pe_y = bmax * dy / eps;
  out->g_y = X * (1.0 - std::exp(-Y)) / eps;
  // negative couplings: W and E vary with the column only, S and N with the
  // row only; boundary couplings are absent (i = 0 has no W, ...)
  int64_t negw = 0, nege = 0, negs = 0, negn = 0;
  for (int i = 0; i < nx; ++i) {
    const double w = scheme == ADR_UPWIND ? cx - ax[i] * gx : cx - 0.5 * (ax[i] * gx);
    const double e = scheme == ADR_UPWIND ? cx : cx + 0.5 * (ax[i] * gx);
    negw += (i > 0 && w < 0.0);
    nege += (i < nx - 1 && e < 0.0);
  }
  for (int j = 0; j < ny; ++j) {
    const double sj = scheme == ADR_UPWIND ? cy - by[j] * gy : cy - 0.5 * (by[j] * gy);
    const double nj = scheme == ADR_UPWIND ? cy : cy + 0.5 * (by[j] * gy);
    negs += (j > 0 && sj < 0.0);
    negn += (j < ny - 1 && nj < 0.0);
  }
  out->neg_offdiag = (negw + nege) * ny + (negs + negn) * nx;
  // diagonal sign, point by point (the Neumann closure adds E, N on the
  // outer sides)
  int64_t nonneg = 0;
  for (int j = 0; j < ny; ++j) {
    const double nj = scheme == ADR_UPWIND ? cy : cy + 0.5 * (by[j] * gy);
    for (int i = 0; i < nx; ++i) {
      double c = scheme == ADR_UPWIND ? (ax[i] * gx + by[j] * gy) - 2.0 * (cx + cy) : -2.0 * (cx + cy);
      if (bc == ADR_BC_NEUMANN_XY) {
        if (i == nx - 1) c = c + (scheme == ADR_UPWIND ? cx : cx + 0.5 * (ax[i] * gx));
        if (j == ny - 1) c = c + nj;
      }
      nonneg += (c >= 0.0);
    }
  }
  out->nonneg_diag = nonneg;
  // expected failures: the Neumann residual floor u exp(g_y) above tol; a
  // diagonal that changes sign inside the grid (pivots through zero); the
  // downwind-differenced upwind scheme beyond cell Peclet 2
  const int64_t npts = (int64_t)nx * ny;
  const bool floor_above_tol = bc == ADR_BC_NEUMANN_XY && tol > 0.0 && out->g_y > std::log(tol / std::ldexp(1.0, -53));
  const bool sign_change = nonneg > 0 && nonneg < npts;
  const bool downwind = scheme == ADR_UPWIND && nonneg == 0 && std::max(out->pe_x, out->pe_y) > 2.0;
  out->expect_fail = (floor_above_tol || sign_change || downwind) ? 1 : 0;
  return ADR_OK;
}

adr_status adr_stream_copy(const double *src, double *dst, int64_t n, void *stream) {
  g_last_error.clear();
  if (!src || !dst || n < 0) return fail(ADR_ERR_ARG, "bad argument");
  if (n == 0) return ADR_OK;
  // one block per 64 KB segment (4096 pairs of doubles), at most 2^20 blocks
  const int64_t want = (n / 2 + 4095) / 4096;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)1 << 20));
  HIP_TRY(launch_stream_copy(src, dst, n, blocks, (hipStream_t)stream));
  return ADR_OK;
}

}  // extern "C"

namespace {

// This device's copy of the adr_dot_noalloc partial-sum array (looked up
// once per device, with that device current).
adr_status dot_scratch(double2 **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(ADR_ERR_DEVICE, "device %d beyond the %d supported", dev, MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(ADR_ERR_DEVICE, "no device address for the inner-product scratch array");
    g_scratch[dev] = (double2 *)p;
  }
  *out = g_scratch[dev];
  return ADR_OK;
}

}  // namespace

extern "C" {

adr_status adr_dot_noalloc(const double *x, const double *y, int64_t n, void *stream, double *out_dev) {
  g_last_error.clear();
  if (!x || !y || !out_dev) return fail(ADR_ERR_ARG, "NULL argument");
  if (n < 0 || n > 0x7fffffff) return fail(ADR_ERR_ARG, "n must be in [0, 2^31 - 1] (got %lld)", (long long)n);
  hipStream_t s = (hipStream_t)stream;
  if (n == 0) {
    HIP_TRY(launch_fill(out_dev, 1, 0.0, s));
    return ADR_OK;
  }
  const Stream1D g = make_geom(n);
  if (g.nblk > DOT_SCRATCH_BLOCKS)
    return fail(ADR_ERR_ARG, "n = %lld needs %d partial sums; the array holds %d", (long long)n, g.nblk,
                DOT_SCRATCH_BLOCKS);
  double2 *part = nullptr;
  adr_status st = dot_scratch(&part);
  if (st != ADR_OK) return st;
  HIP_TRY(launch_dot(x, y, g, part, out_dev, s));
  return ADR_OK;
}

}  // extern "C"
