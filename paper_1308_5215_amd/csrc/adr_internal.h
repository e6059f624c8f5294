// Internal declarations shared by the library's kernel and host sources.
// Not part of the public ABI (see include/adr.h).
//
// Every iteration kernel works on a batch of independent instances (a single
// problem is a batch of one).  Instance k owns the slice [off, off + n) of
// each batched vector, the block range [blk0, blk0 + nblk) of the streaming
// kernels and the strip range [strip0, strip0 + nstrips) of the wavefront
// kernels; kernels find their instance by binary search over those starts.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

struct adr_cnn;

namespace adr {

// Device-resident scalar state of one BiCGSTAB solve.  Written only by the
// single-block finalize kernels (and the init kernel), read by every kernel
// of the iteration; kernels that find phase DONE return at once, so
// iterations launched after the stop are no-ops and the pass count is exact.
// CHECK: the recursively updated residual passed the stopping test; the next
// pass slot computes the true residual b - A x (written to r, r^ and p as the
// start of a restart) and its finalize step accepts the solve or restarts it.
enum Phase : int32_t { RUNNING = 0, HALF_STEP = 1, DONE = 2, CHECK = 3 };

struct SolveState {
  double rho, rho_prev, alpha, omega, beta;
  double bnorm, thr, true_res2;
  int32_t iter;       // index of the pass in progress (passes started)
  int32_t status;     // adr_status once phase == DONE
  int32_t phase;      // Phase
  int32_t hist_len;   // valid history entries
  int32_t half_step;  // 1 if ended on the ||s|| test
  int32_t maxit;
  int32_t zero_x;     // b == 0: x must be cleared
  int32_t restarts;   // restarts from the current iterate so far
  int32_t max_restarts;   // < 0: accept the recursive residual's test alone
  int32_t pad;
};

// Five diagonals (lexicographic order, x fastest), batched base pointers.
struct Dia {
  const double *S, *W, *C, *E, *N;
};

// Magic-number unsigned division by a runtime constant d >= 1 for
// numerators below 2^31 (Granlund & Montgomery, PLDI 1994).
struct FastDiv {
  uint32_t d, m, s;
};

// One instance of a batch.
struct Inst {
  int32_t nx, ny, n;
  int32_t chunk;            // points per streaming block (multiple of 1024)
  int64_t off;              // offset of the instance in every batched vector
  int32_t blk0, nblk;       // streaming blocks (blk0 and nblk multiples of 8)
  int32_t strip0, nstrips;  // wavefront strips (for the batch's strip height), numbered in ticket order
  int64_t ho_off;           // offset in the hand-off buffer (64-bit words)
  FastDiv fd;               // division by nx
  int32_t pad;
  int64_t tab_off;          // offset of the instance's stencil tables (below)
};

// Stencil tables.  The off-diagonals of the assembled operator are separable:
// W and E depend on the column i only, S and N on the row j only (Section 4:
// a = a(x), b = b(y), and the couplings to boundary nodes are zero in every
// row or column).  Instance k keeps, at tab + inst[k].tab_off,
//   Wc[nx], Ec[nx], Sr[ny], Nr[ny]   with W(i,j) = Wc[i], E(i,j) = Ec[i],
//                                         S(i,j) = Sr[j], N(i,j) = Nr[j],
// copied out of the diagonals themselves and verified against every point,
// so reading a table gives the stored coefficient bit for bit.  Kernels given
// tab == nullptr read the full diagonals.
inline int64_t stencil_tab_len(int nx, int ny) { return 2 * ((int64_t)nx + ny); }

// Launch geometry of a batch.
struct BatchGeom {
  const Inst *inst;   // device table
  int ninst;
  int nblk;           // total streaming blocks
  int nstrips;        // total strips
  int rows;           // strip height R
  int compact;        // 32-row sweeps: 0 deep ring; 1 compact ring (76 KB, two workgroups per CU);
                      // 2 compact ring with three loader waves (strips at most one per CU)
  int xcd_group;      // > 0: strips by workgroup index, xcd_group consecutive strips per XCD
  const int *sorder;  // device: instances in strip-ticket order (largest work first); strip0 ascends along it
};

// Single-instance streaming geometry (assembly, diagnostics).
struct Stream1D {
  int n, nblk, chunk;
};

// Wavefront synchronisation memory.
struct SweepSync {
  unsigned *ticket;      // [2]: strip ticket, finished-strip counter
  uint64_t *handoff;     // last row of each strip, sentinel-filled
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
  int fmode;            // 0: manufactured f (+ field); 1: f = fuser[k]; 2: f = fconst
  const double *fuser;  // device, fmode 1
  double fconst;        // fmode 2
  double *S, *W, *C, *E, *N, *rhs;
  double *F;           // optional: the forcing f at every unknown
  double2 *partials;   // workspace for the max|f| reduction
  double *fmax;        // device scalar
};
hipError_t launch_assemble(const AssembleArgs &a, const Stream1D &g, hipStream_t s);

hipError_t launch_spmv(const Dia &A, FastDiv fd, int nx, int ny, const double *x, double *v,
                       const Stream1D &g, hipStream_t s);
hipError_t launch_dot(const double *x, const double *y, const Stream1D &g, double2 *partials,
                      double *out, hipStream_t s);

// BiCGSTAB step kernels (batched).
struct IterBufs {
  Dia A;
  const double *tab;   // stencil tables, or nullptr: read S, W, E, N from A
  const double *b;
  double *x, *r, *rh, *p, *v, *s, *t, *ph, *z;
  double2 *partials;   // [4][total blocks]
  SolveState *st;      // [ninst]
  double *hist;        // [ninst][2][maxit + 1]
  double tol;
  int maxit;
  int max_restarts;    // see SolveState::max_restarts
};
hipError_t launch_init(const IterBufs &B, const BatchGeom &g, hipStream_t s);
hipError_t launch_pass_p(const IterBufs &B, const BatchGeom &g, hipStream_t s);
hipError_t launch_pass_v(const IterBufs &B, const BatchGeom &g, hipStream_t s);
hipError_t launch_pass_s(const IterBufs &B, const BatchGeom &g, hipStream_t s);
hipError_t launch_pass_t(const IterBufs &B, const BatchGeom &g, hipStream_t s);
hipError_t launch_pass_xr(const IterBufs &B, const BatchGeom &g, hipStream_t s);
hipError_t launch_true_residual(const IterBufs &B, const BatchGeom &g, hipStream_t s);

// max |U - u_exact| over the (nx+2) x (ny+2) nodes of one instance, U being
// the solution x with the boundary values (Dirichlet: exact u; Neumann edges
// reconstructed from the one-sided closure), into *out (device).
struct MaxErrArgs {
  int nx, ny, bc;
  double X, Y, dx, dy;
  const double *x;
  double2 *partials;
  double *out;
};
hipError_t launch_max_error(const MaxErrArgs &a, const Stream1D &g, hipStream_t s);
// dst[k] = src[k], k < n: a plain streaming copy (bandwidth reference).
hipError_t launch_stream_copy(const double *src, double *dst, int64_t n, int blocks, hipStream_t s);

// Wavefront kernels.  rows = strip height R (16 or 32).
struct Factors64 {
  double *lw, *ls, *invd;
};
struct Factors32 {
  float *lw, *ls, *invd, *E, *N;
};
hipError_t launch_ilu0(const Dia &A, const BatchGeom &g, Factors64 f64, Factors32 f32,
                       const SweepSync &sync, int64_t *bad, hipStream_t s);
// precision: 0 = FP64 factors, 1 = FP32 factors/FP64 arithmetic, 2 = FP32 arithmetic
// tab: stencil tables or nullptr.  With tables the FP64-factor L sweep forms
// lw = W invd_w and ls = S invd_s from invd (as the factorisation does) and
// the U sweep takes E and N from the tables.
hipError_t launch_lsweep(const BatchGeom &g, int precision, const Factors64 &f64,
                         const Factors32 &f32, const double *tab, const double *q, double *y,
                         const SweepSync &sync, const SolveState *st, hipStream_t s);
hipError_t launch_usweep(const BatchGeom &g, int precision, const Dia &A, const Factors64 &f64,
                         const Factors32 &f32, const double *tab, const double *y, double *z,
                         const SweepSync &sync, const SolveState *st, hipStream_t s);
// Copy the stencil tables of every instance out of the diagonals, then count
// the points whose S, W, E or N differ from their table entry (bitwise) into
// *mismatch (device, cleared by the caller).
hipError_t launch_stencil_tables(const Dia &A, const BatchGeom &g, double *tab, unsigned *mismatch,
                                 hipStream_t s);

// ---- error text shared by every C entry point (adr_capi.hip) ----
int set_error(int st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

// ---- warm-start network (adr_cnn.hip) ----
struct FeatInst {
  double eps, X, Y;
  int32_t nx, ny, bc, scheme;   // scheme: 0 upwind, 1 centered
  int64_t off;          // offset of the instance in the batched vectors
};
hipError_t launch_cnn_features(const FeatInst *fi_dev, int count, int H, int W, const double *F,
                               uint16_t *out, hipStream_t s);
hipError_t launch_cnn_extract(const FeatInst *fi_dev, int count, int H, int W, const float *u,
                              double *x, hipStream_t s);
// node grid, batch limit, stream and the input/output buffers of a network
void cnn_shape(const adr_cnn *net, int *H, int *W, int *maxB, hipStream_t *s, uint16_t **in, float **u);
}  // namespace adr
