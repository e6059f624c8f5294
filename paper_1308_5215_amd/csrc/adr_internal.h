// Internal declarations shared by the library's kernel and host sources.
// Not part of the public ABI (see include/adr.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace adr {

// Device-resident scalar state of one BiCGSTAB solve.  Written only by the
// single-block finalize kernels (and the init kernel), read by every kernel
// of the iteration; kernels that find phase != RUNNING return at once, so
// iterations launched after the stop are no-ops and the pass count is exact.
enum Phase : int32_t { RUNNING = 0, HALF_STEP = 1, DONE = 2 };

struct SolveState {
  double rho, rho_prev, alpha, omega, beta;
  double bnorm, thr;
  int32_t iter;       // index of the pass in progress (passes started)
  int32_t status;     // adr_status once phase == DONE
  int32_t phase;      // Phase
  int32_t hist_len;   // valid history entries
  int32_t half_step;  // 1 if ended on the ||s|| test
  int32_t maxit;
  int32_t zero_x;     // b == 0: x must be cleared
  int32_t pad;
};

// Five diagonals (lexicographic order, x fastest).
struct Dia {
  const double *S, *W, *C, *E, *N;
};

// Magic-number unsigned division by a runtime constant d >= 1 for
// numerators below 2^31 (Granlund & Montgomery, PLDI 1994).
struct FastDiv {
  uint32_t d, m, s;
};

// Slots of the per-block double-double partial sums.
enum Slot : int { SLOT_A = 0, SLOT_B = 1, SLOT_C = 2, NSLOT = 3 };

// Launch geometry of the streaming kernels: nblk blocks of 256 threads,
// each owning `chunk` consecutive points (a multiple of 256).
struct Stream1D {
  int n, nblk, chunk;
};

// Wavefront sweep geometry and synchronisation memory.
struct SweepSync {
  unsigned *ticket;      // [2]: strip ticket, finished-strip counter
  uint64_t *handoff;     // [nstrips * nx]: last row of each strip, sentinel-filled
  int *err;              // device fault report (spin limit exceeded)
};

constexpr uint64_t HANDOFF_EMPTY = 0x7FF4DEADBEEF0001ull;  // a signalling-NaN pattern
constexpr uint64_t CANON_NAN = 0x7FF8000000000000ull;

// ---- launchers (adr_kernels.hip) ----
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s);
hipError_t launch_fill_u32(unsigned *p, int64_t n, unsigned v, hipStream_t s);

struct AssembleArgs {
  int nx, ny, scheme, bc;
  double eps, X, Y, dx, dy;
  // per-column tables (length nx) and per-row tables (length ny), device
  const double *xi, *ai, *exi, *uy0, *uyY, *gyY;
  const double *yj, *bj, *eyj, *ebj, *ux0, *uxX, *gxX;
  const double *field;  // optional
  double amp;
  double *S, *W, *C, *E, *N, *rhs;
  double2 *partials;   // workspace for the max|f| reduction
  double *fmax;        // device scalar
};
hipError_t launch_assemble(const AssembleArgs &a, const Stream1D &g, hipStream_t s);

hipError_t launch_spmv(const Dia &A, FastDiv fd, int nx, int ny, const double *x, double *v,
                       const Stream1D &g, hipStream_t s);
hipError_t launch_dot(const double *x, const double *y, const Stream1D &g, double2 *partials,
                      double *out, hipStream_t s);

// BiCGSTAB step kernels.
struct IterBufs {
  Dia A;
  FastDiv fd;
  int nx, ny;
  const double *b;
  double *x, *r, *rh, *p, *v, *s, *t, *ph, *z;
  double2 *partials;   // [NSLOT][maxblk] plus max slots
  SolveState *st;
  double *hist_l2, *hist_max;   // device, maxit+1
  double tol;
  int maxit;
};
hipError_t launch_init(const IterBufs &B, const Stream1D &g, hipStream_t s);
hipError_t launch_pass_p(const IterBufs &B, const Stream1D &g, hipStream_t s);
hipError_t launch_pass_v(const IterBufs &B, const Stream1D &g, hipStream_t s);
hipError_t launch_pass_s(const IterBufs &B, const Stream1D &g, hipStream_t s);
hipError_t launch_pass_t(const IterBufs &B, const Stream1D &g, hipStream_t s);
hipError_t launch_pass_xr(const IterBufs &B, const Stream1D &g, hipStream_t s);
hipError_t launch_true_residual(const IterBufs &B, const Stream1D &g, double *out, hipStream_t s);

// Wavefront kernels.  rows = strip height R (15, 31 or 63).
struct Factors64 {
  double *lw, *ls, *invd;
};
struct Factors32 {
  float *lw, *ls, *invd, *E, *N;
};
hipError_t launch_ilu0(const Dia &A, int nx, int ny, int rows, Factors64 f64, Factors32 f32,
                       const SweepSync &sync, int64_t *bad, hipStream_t s);
// precision: 0 = FP64 factors, 1 = FP32 factors/FP64 arithmetic, 2 = FP32 arithmetic
hipError_t launch_lsweep(int nx, int ny, int rows, int precision, const Factors64 &f64,
                         const Factors32 &f32, const double *q, double *y, const SweepSync &sync,
                         const int32_t *phase, hipStream_t s);
hipError_t launch_usweep(int nx, int ny, int rows, int precision, const Dia &A,
                         const Factors64 &f64, const Factors32 &f32, const double *y, double *z,
                         const SweepSync &sync, const int32_t *phase, hipStream_t s);

}  // namespace adr
