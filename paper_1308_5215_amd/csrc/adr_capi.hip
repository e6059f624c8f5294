// Host runtime and C ABI (include/adr.h): argument checking, device memory,
// the 1-D tables of the discretisation, and the BiCGSTAB driver, which
// captures a chunk of passes into a HIP graph and replays it until the
// device-side state reports that the solve has stopped.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/adr.h"
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

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) {                                                               \
      (void)hipGetLastError();                                                            \
      return fail(e_ == hipErrorOutOfMemory ? ADR_ERR_NOMEM : ADR_ERR_DEVICE, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                      \
    }                                                                                     \
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

Stream1D make_geom(int64_t n) {
  Stream1D g;
  g.n = (int)n;
  const int64_t target = 2048;
  int64_t chunk = (n + target - 1) / target;
  chunk = ((chunk + 255) / 256) * 256;
  if (chunk < 256) chunk = 256;
  g.chunk = (int)chunk;
  g.nblk = (int)((n + chunk - 1) / chunk);
  if (g.nblk < 1) g.nblk = 1;
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

int auto_rows(int ny) {
  return ny >= 2048 ? 31 : 15;
}

}  // namespace

struct adr_problem {
  int dev = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;   // private stream used only for graph capture
  double eps = 0, X = 0, Y = 0;
  int nx = 0, ny = 0, scheme = 0, bc = 0;
  int64_t n = 0;
  size_t bytes = 0;
  Stream1D geom{};
  FastDiv fd{};
  // matrix
  double *S = nullptr, *W = nullptr, *C = nullptr, *E = nullptr, *N = nullptr, *rhs = nullptr;
  // factors
  double *lw = nullptr, *ls = nullptr, *invd = nullptr;
  float *lw32 = nullptr, *ls32 = nullptr, *invd32 = nullptr, *E32 = nullptr, *N32 = nullptr;
  int factored = 0, precision = 0;
  int rows = 0;   // sweep strip height (0 = automatic)
  // iteration vectors
  double *r = nullptr, *rh = nullptr, *p = nullptr, *v = nullptr, *s = nullptr, *t = nullptr;
  double *ph = nullptr, *z = nullptr, *y = nullptr;
  // reductions, state, histories
  double2 *partials = nullptr;
  SolveState *st = nullptr;
  double *hist = nullptr;
  int hist_cap = 0;
  double *scal = nullptr;      // scratch device scalars
  int64_t *bad = nullptr;
  // wavefront synchronisation
  unsigned *ticket = nullptr;
  uint64_t *handoff = nullptr;
  int *err = nullptr;
  // host pinned mirror of the state
  SolveState *h_st = nullptr;
  // captured iteration chunk
  hipGraphExec_t gexec = nullptr;
  double *g_x = nullptr;
  double g_tol = -1;
  int g_maxit = -1, g_prec = -1, g_rows = -1, g_K = 0;

  int sweep_rows() const { return rows ? rows : auto_rows(ny); }
  SweepSync sync() const { return SweepSync{ticket, handoff, err}; }
  Dia dia() const { return Dia{S, W, C, E, N}; }
};

namespace {

adr_status ensure_sync(adr_problem *P) {
  if (P->ticket) return ADR_OK;
  const int64_t slots = (int64_t)((P->ny + 14) / 15 + 1) * P->nx;
  HIP_TRY(dalloc(&P->ticket, 2, P->bytes));
  HIP_TRY(dalloc(&P->handoff, (size_t)slots, P->bytes));
  HIP_TRY(dalloc(&P->err, 1, P->bytes));
  HIP_TRY(launch_fill_u32(P->ticket, 2, 0u, P->stream));
  HIP_TRY(launch_fill_u64(P->handoff, slots, HANDOFF_EMPTY, P->stream));
  HIP_TRY(hipMemsetAsync(P->err, 0, sizeof(int), P->stream));
  return ADR_OK;
}

adr_status check_device_fault(adr_problem *P) {
  int herr = 0;
  HIP_TRY(hipMemcpyAsync(&herr, P->err, sizeof(int), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  if (herr) {
    // a wavefront wait exceeded its spin limit: restore the sync memory
    const int64_t slots = (int64_t)((P->ny + 14) / 15 + 1) * P->nx;
    HIP_TRY(launch_fill_u32(P->ticket, 2, 0u, P->stream));
    HIP_TRY(launch_fill_u64(P->handoff, slots, HANDOFF_EMPTY, P->stream));
    HIP_TRY(hipMemsetAsync(P->err, 0, sizeof(int), P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    return fail(ADR_ERR_DEVICE, "wavefront hand-off wait exceeded its limit");
  }
  return ADR_OK;
}

adr_status ensure_iter_buffers(adr_problem *P, int maxit) {
  if (!P->r) {
    double **vecs[] = {&P->r, &P->rh, &P->p, &P->v, &P->s, &P->t, &P->ph, &P->z, &P->y};
    for (double **q : vecs) HIP_TRY(dalloc(q, (size_t)P->n, P->bytes));
    HIP_TRY(dalloc(&P->st, 1, P->bytes));
    HIP_TRY(hipHostMalloc((void **)&P->h_st, sizeof(SolveState), hipHostMallocDefault));
  }
  if (P->hist_cap < maxit + 1) {
    dfree(P->hist);
    P->hist_cap = 0;
    HIP_TRY(dalloc(&P->hist, 2 * (size_t)(maxit + 1), P->bytes));
    P->hist_cap = maxit + 1;
  }
  return ADR_OK;
}

IterBufs iter_bufs(adr_problem *P, double *x, double tol, int maxit) {
  IterBufs B;
  B.A = P->dia();
  B.fd = P->fd;
  B.nx = P->nx;
  B.ny = P->ny;
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
  B.hist_l2 = P->hist;
  B.hist_max = P->hist + P->hist_cap;
  B.tol = tol;
  B.maxit = maxit;
  return B;
}

Factors64 f64_of(const adr_problem *P) { return Factors64{P->lw, P->ls, P->invd}; }
Factors32 f32_of(const adr_problem *P) { return Factors32{P->lw32, P->ls32, P->invd32, P->E32, P->N32}; }

// One BiCGSTAB pass (13 kernels).
hipError_t enqueue_pass(adr_problem *P, const IterBufs &B, hipStream_t s) {
  const int rows = P->sweep_rows();
  const int32_t *phase = &P->st->phase;
  hipError_t e;
  if ((e = launch_pass_p(B, P->geom, s)) != hipSuccess) return e;
  if ((e = launch_lsweep(P->nx, P->ny, rows, P->precision, f64_of(P), f32_of(P), P->p, P->y, P->sync(), phase, s)) != hipSuccess) return e;
  if ((e = launch_usweep(P->nx, P->ny, rows, P->precision, P->dia(), f64_of(P), f32_of(P), P->y, P->ph, P->sync(), phase, s)) != hipSuccess) return e;
  if ((e = launch_pass_v(B, P->geom, s)) != hipSuccess) return e;
  if ((e = launch_pass_s(B, P->geom, s)) != hipSuccess) return e;
  if ((e = launch_lsweep(P->nx, P->ny, rows, P->precision, f64_of(P), f32_of(P), P->s, P->y, P->sync(), phase, s)) != hipSuccess) return e;
  if ((e = launch_usweep(P->nx, P->ny, rows, P->precision, P->dia(), f64_of(P), f32_of(P), P->y, P->z, P->sync(), phase, s)) != hipSuccess) return e;
  if ((e = launch_pass_t(B, P->geom, s)) != hipSuccess) return e;
  return launch_pass_xr(B, P->geom, s);
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
    default: return "unknown status";
  }
}

const char *adr_last_error(void) { return g_last_error.c_str(); }

void adr_destroy(adr_problem *P) {
  if (!P) return;
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
  if (P->cap) (void)hipStreamDestroy(P->cap);
  double *dv[] = {P->S, P->W, P->C, P->E, P->N, P->rhs, P->lw, P->ls, P->invd, P->r, P->rh,
                  P->p, P->v, P->s, P->t, P->ph, P->z, P->y, P->hist, P->scal};
  for (double *q : dv) dfree(q);
  float *fv[] = {P->lw32, P->ls32, P->invd32, P->E32, P->N32};
  for (float *q : fv) dfree(q);
  dfree(P->partials);
  dfree(P->st);
  dfree(P->bad);
  dfree(P->ticket);
  dfree(P->handoff);
  dfree(P->err);
  if (P->h_st) (void)hipHostFree(P->h_st);
  delete P;
}

adr_status adr_assemble(double eps, double X, double Y, int32_t nx, int32_t ny, int32_t scheme,
                        int32_t bc, const double *field_dev, double amp, void *stream,
                        adr_problem **out) {
  g_last_error.clear();
  if (!out) return fail(ADR_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(ADR_ERR_ARG, "eps must be a finite number > 0 (got %g)", eps);
  if (!(X > 0.0) || !(Y > 0.0) || !std::isfinite(X) || !std::isfinite(Y))
    return fail(ADR_ERR_ARG, "X and Y must be finite and > 0 (got %g, %g)", X, Y);
  if (nx < 1 || ny < 1) return fail(ADR_ERR_ARG, "nx and ny must be >= 1 (got %d, %d)", nx, ny);
  if ((int64_t)nx * (int64_t)ny > (int64_t)0x7fffffff) return fail(ADR_ERR_ARG, "nx*ny must be < 2^31");
  if (scheme != ADR_UPWIND && scheme != ADR_CENTERED) return fail(ADR_ERR_ARG, "unknown scheme %d", scheme);
  if (bc != ADR_BC_DIRICHLET && bc != ADR_BC_NEUMANN_XY) return fail(ADR_ERR_ARG, "unknown bc %d", bc);
  if (field_dev && !std::isfinite(amp)) return fail(ADR_ERR_ARG, "amp must be finite");

  adr_problem *P = new adr_problem();
  HIP_TRY(hipGetDevice(&P->dev));
  P->stream = (hipStream_t)stream;
  P->eps = eps; P->X = X; P->Y = Y; P->nx = nx; P->ny = ny; P->scheme = scheme; P->bc = bc;
  P->n = (int64_t)nx * ny;
  P->geom = make_geom(P->n);
  P->fd = make_fastdiv((uint32_t)nx);

  auto cleanup_fail = [&](adr_status st) { adr_destroy(P); return st; };
#define TRY_P(expr)                                              \
  do {                                                           \
    hipError_t e_ = (expr);                                      \
    if (e_ != hipSuccess) {                                      \
      (void)hipGetLastError();                                   \
      adr_status st_ = fail(e_ == hipErrorOutOfMemory ? ADR_ERR_NOMEM : ADR_ERR_DEVICE, \
                            "%s: %s", #expr, hipGetErrorString(e_)); \
      return cleanup_fail(st_);                                  \
    }                                                            \
  } while (0)

  double **arrs[] = {&P->S, &P->W, &P->C, &P->E, &P->N, &P->rhs};
  for (double **q : arrs) TRY_P(dalloc(q, (size_t)P->n, P->bytes));
  TRY_P(dalloc(&P->partials, (size_t)4 * P->geom.nblk, P->bytes));
  TRY_P(dalloc(&P->scal, 8, P->bytes));
  TRY_P(dalloc(&P->bad, 1, P->bytes));

  // 1-D tables on the host (same formulas and libm as the CPU reference)
  const double dx = X / (double)(nx + 1), dy = Y / (double)(ny + 1);
  const double e1 = std::exp(-1.0);
  std::vector<double> tx(6 * (size_t)nx), ty(7 * (size_t)ny);
  double *xi = &tx[0], *ai = xi + nx, *exi = ai + nx, *uy0 = exi + nx, *uyY = uy0 + nx, *gyY = uyY + nx;
  double *yj = &ty[0], *bj = yj + ny, *eyj = bj + ny, *ebj = eyj + ny, *ux0 = ebj + ny, *uxX = ux0 + ny,
         *gxX = uxX + ny;
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
  double *dtab = nullptr;
  size_t tb = 0;
  TRY_P(dalloc(&dtab, tx.size() + ty.size(), tb));
  TRY_P(hipMemcpyAsync(dtab, tx.data(), tx.size() * sizeof(double), hipMemcpyHostToDevice, P->stream));
  TRY_P(hipMemcpyAsync(dtab + tx.size(), ty.data(), ty.size() * sizeof(double), hipMemcpyHostToDevice, P->stream));
  AssembleArgs a;
  a.nx = nx; a.ny = ny; a.scheme = scheme; a.bc = bc;
  a.eps = eps; a.X = X; a.Y = Y; a.dx = dx; a.dy = dy;
  const double *dx0 = dtab, *dy0 = dtab + tx.size();
  a.xi = dx0; a.ai = dx0 + nx; a.exi = dx0 + 2 * nx; a.uy0 = dx0 + 3 * nx; a.uyY = dx0 + 4 * nx; a.gyY = dx0 + 5 * nx;
  a.yj = dy0; a.bj = dy0 + ny; a.eyj = dy0 + 2 * ny; a.ebj = dy0 + 3 * ny; a.ux0 = dy0 + 4 * ny; a.uxX = dy0 + 5 * ny;
  a.gxX = dy0 + 6 * ny;
  a.field = field_dev;
  a.amp = amp;
  a.S = P->S; a.W = P->W; a.C = P->C; a.E = P->E; a.N = P->N; a.rhs = P->rhs;
  a.partials = P->partials;
  a.fmax = P->scal;
  hipError_t ea = launch_assemble(a, P->geom, P->stream);
  hipError_t es = hipStreamSynchronize(P->stream);
  (void)hipFree(dtab);
  TRY_P(ea);
  TRY_P(es);
#undef TRY_P
  *out = P;
  return ADR_OK;
}

adr_status adr_get_dia(const adr_problem *P, double *S, double *W, double *C, double *E, double *N,
                       double *rhs) {
  g_last_error.clear();
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  const double *src[] = {P->S, P->W, P->C, P->E, P->N, P->rhs};
  double *dst[] = {S, W, C, E, N, rhs};
  for (int q = 0; q < 6; ++q)
    if (dst[q]) HIP_TRY(hipMemcpyAsync(dst[q], src[q], (size_t)P->n * sizeof(double), hipMemcpyDeviceToHost, P->stream));
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
    HIP_TRY(hipMemcpyAsync(dst[q], src[q], (size_t)P->n * sizeof(double), hipMemcpyHostToDevice, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  P->factored = 0;
  return ADR_OK;
}

adr_status adr_get_factors(const adr_problem *P, double *lw, double *ls, double *invd) {
  g_last_error.clear();
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  if (!P->factored) return fail(ADR_ERR_STATE, "no factorisation (call adr_ilu0 first)");
  const double *src[] = {P->lw, P->ls, P->invd};
  double *dst[] = {lw, ls, invd};
  for (int q = 0; q < 3; ++q)
    if (dst[q]) HIP_TRY(hipMemcpyAsync(dst[q], src[q], (size_t)P->n * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return ADR_OK;
}

adr_status adr_set_sweep_rows(adr_problem *P, int32_t rows) {
  g_last_error.clear();
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  if (rows != 0 && rows != 15 && rows != 31)
    return fail(ADR_ERR_ARG, "rows must be 0, 15 or 31 (got %d)", rows);
  P->rows = rows;
  return ADR_OK;
}

size_t adr_device_bytes(const adr_problem *P) { return P ? P->bytes : 0; }

adr_status adr_ilu0(adr_problem *P, int32_t precision, int64_t *bad_index) {
  g_last_error.clear();
  if (bad_index) *bad_index = -1;
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  if (precision < ADR_FP64 || precision > ADR_FP32_SWEEPS) return fail(ADR_ERR_ARG, "unknown precision %d", precision);
  adr_status st = ensure_sync(P);
  if (st != ADR_OK) return st;
  if (!P->lw) {
    HIP_TRY(dalloc(&P->lw, (size_t)P->n, P->bytes));
    HIP_TRY(dalloc(&P->ls, (size_t)P->n, P->bytes));
    HIP_TRY(dalloc(&P->invd, (size_t)P->n, P->bytes));
  }
  if (precision != ADR_FP64 && !P->lw32) {
    float **fv[] = {&P->lw32, &P->ls32, &P->invd32, &P->E32, &P->N32};
    for (float **q : fv) HIP_TRY(dalloc(q, (size_t)P->n, P->bytes));
  }
  P->factored = 0;
  HIP_TRY(launch_fill_u64((uint64_t *)P->bad, 1, ~0ull, P->stream));
  Factors32 h{};
  if (precision != ADR_FP64) h = f32_of(P);
  HIP_TRY(launch_ilu0(P->dia(), P->nx, P->ny, P->sweep_rows(), f64_of(P), h, P->sync(), P->bad, P->stream));
  uint64_t hb = 0;
  HIP_TRY(hipMemcpyAsync(&hb, P->bad, sizeof(hb), hipMemcpyDeviceToHost, P->stream));
  st = check_device_fault(P);
  if (st != ADR_OK) return st;
  if (hb != ~0ull) {
    if (bad_index) *bad_index = (int64_t)hb;
    return fail(ADR_ZERO_PIVOT, "zero or non-finite pivot at unknown %lld", (long long)hb);
  }
  P->factored = 1;
  P->precision = precision;
  return ADR_OK;
}

adr_status adr_spmv(adr_problem *P, const double *x, double *v) {
  g_last_error.clear();
  if (!P || !x || !v) return fail(ADR_ERR_ARG, "NULL argument");
  HIP_TRY(launch_spmv(P->dia(), P->fd, P->nx, P->ny, x, v, P->geom, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return ADR_OK;
}

adr_status adr_precond(adr_problem *P, const double *q, double *z) {
  g_last_error.clear();
  if (!P || !q || !z) return fail(ADR_ERR_ARG, "NULL argument");
  if (!P->factored) return fail(ADR_ERR_STATE, "no factorisation (call adr_ilu0 first)");
  adr_status st = ensure_iter_buffers(P, 0);
  if (st != ADR_OK) return st;
  const int rows = P->sweep_rows();
  HIP_TRY(launch_lsweep(P->nx, P->ny, rows, P->precision, f64_of(P), f32_of(P), q, P->y, P->sync(), nullptr, P->stream));
  HIP_TRY(launch_usweep(P->nx, P->ny, rows, P->precision, P->dia(), f64_of(P), f32_of(P), P->y, z, P->sync(), nullptr, P->stream));
  return check_device_fault(P);
}

adr_status adr_lsolve(adr_problem *P, const double *q, double *y) {
  g_last_error.clear();
  if (!P || !q || !y) return fail(ADR_ERR_ARG, "NULL argument");
  if (!P->factored) return fail(ADR_ERR_STATE, "no factorisation (call adr_ilu0 first)");
  HIP_TRY(launch_lsweep(P->nx, P->ny, P->sweep_rows(), P->precision, f64_of(P), f32_of(P), q, y, P->sync(), nullptr, P->stream));
  return check_device_fault(P);
}

adr_status adr_usolve(adr_problem *P, const double *y, double *z) {
  g_last_error.clear();
  if (!P || !y || !z) return fail(ADR_ERR_ARG, "NULL argument");
  if (!P->factored) return fail(ADR_ERR_STATE, "no factorisation (call adr_ilu0 first)");
  HIP_TRY(launch_usweep(P->nx, P->ny, P->sweep_rows(), P->precision, P->dia(), f64_of(P), f32_of(P), y, z, P->sync(), nullptr, P->stream));
  return check_device_fault(P);
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

adr_status adr_bicgstab_solve(adr_problem *P, double tol, int32_t maxit, const double *x0,
                              double *x, double *hist_l2, double *hist_max, adr_solve_info *info) {
  g_last_error.clear();
  if (info) memset(info, 0, sizeof(*info));
  if (!P) return fail(ADR_ERR_ARG, "problem is NULL");
  if (!x) return fail(ADR_ERR_ARG, "x_dev is NULL");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(ADR_ERR_ARG, "tol must be finite and >= 0 (got %g)", tol);
  if (maxit < 0) return fail(ADR_ERR_ARG, "maxit must be >= 0 (got %d)", maxit);
  if (!P->factored) return fail(ADR_ERR_STATE, "no factorisation (call adr_ilu0 first)");
  adr_status st = ensure_iter_buffers(P, maxit);
  if (st != ADR_OK) return st;
  st = ensure_sync(P);
  if (st != ADR_OK) return st;
  const size_t vb = (size_t)P->n * sizeof(double);
  if (x0) {
    if (x0 != x) HIP_TRY(hipMemcpyAsync(x, x0, vb, hipMemcpyDeviceToDevice, P->stream));
  } else {
    HIP_TRY(launch_fill(x, P->n, 0.0, P->stream));
  }
  IterBufs B = iter_bufs(P, x, tol, maxit);
  // passes per graph replay: enough to amortise the host check
  int K = P->n >= (1 << 22) ? 4 : (P->n >= (1 << 18) ? 8 : 16);
  if (K > maxit && maxit > 0) K = maxit;
  if (!P->gexec || P->g_x != x || P->g_tol != tol || P->g_maxit != maxit || P->g_prec != P->precision ||
      P->g_rows != P->sweep_rows() || P->g_K != K) {
    st = build_graph(P, B, K);
    if (st != ADR_OK) return st;
    P->g_x = x; P->g_tol = tol; P->g_maxit = maxit; P->g_prec = P->precision; P->g_rows = P->sweep_rows();
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, P->stream));
  HIP_TRY(launch_init(B, P->geom, P->stream));
  // replay chunks; keep one chunk queued behind the one being checked
  const int max_chunks = maxit > 0 ? (maxit + K - 1) / K : 0;
  int launched = 0;
  bool done = false;
  if (max_chunks > 0) {
    HIP_TRY(hipGraphLaunch(P->gexec, P->stream));
    ++launched;
  }
  while (!done && launched > 0) {
    HIP_TRY(hipMemcpyAsync(P->h_st, P->st, sizeof(SolveState), hipMemcpyDeviceToHost, P->stream));
    hipEvent_t ev;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(ev, P->stream));
    if (launched < max_chunks) {
      HIP_TRY(hipGraphLaunch(P->gexec, P->stream));
      ++launched;
    }
    HIP_TRY(hipEventSynchronize(ev));
    (void)hipEventDestroy(ev);
    if (P->h_st->phase == DONE) done = true;
    else if (launched >= max_chunks) {
      // the last chunk is queued; wait for it
      HIP_TRY(hipMemcpyAsync(P->h_st, P->st, sizeof(SolveState), hipMemcpyDeviceToHost, P->stream));
      HIP_TRY(hipStreamSynchronize(P->stream));
      done = true;
    }
  }
  HIP_TRY(hipEventRecord(e1, P->stream));
  HIP_TRY(launch_true_residual(B, P->geom, P->scal + 1, P->stream));
  double tres = 0.0;
  HIP_TRY(hipMemcpyAsync(&tres, P->scal + 1, sizeof(double), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipMemcpyAsync(P->h_st, P->st, sizeof(SolveState), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  st = check_device_fault(P);
  if (st != ADR_OK) return st;
  const SolveState &S = *P->h_st;
  if (S.phase != DONE) return fail(ADR_ERR_DEVICE, "solve did not reach a stopping state");
  const int hl = S.hist_len;
  if (hist_l2 && hl > 0) HIP_TRY(hipMemcpy(hist_l2, P->hist, (size_t)hl * sizeof(double), hipMemcpyDeviceToHost));
  if (hist_max && hl > 0)
    HIP_TRY(hipMemcpy(hist_max, P->hist + P->hist_cap, (size_t)hl * sizeof(double), hipMemcpyDeviceToHost));
  if (info) {
    info->status = S.status;
    info->iters = S.iter;
    info->hist_len = hl;
    info->half_step = S.half_step;
    info->bnorm = S.bnorm;
    info->true_relres = S.bnorm > 0.0 ? std::sqrt(tres) / S.bnorm : 0.0;
    info->solve_ms = ms;
  }
  return (adr_status)S.status;
}

}  // extern "C"
