// Internal interface between the HIP kernels (kernels.hip) and the host runtime (api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace socfv {

// Per-cell flag byte: bits 0..5 = face shared with a fibre voxel (x-, x+, y-, y+, z-, z+),
// bit 6 = pore cell.  Domain walls are not flagged (they are known from the position).
constexpr uint8_t FL_XM = 1, FL_XP = 2, FL_YM = 4, FL_YP = 8, FL_ZM = 16, FL_ZP = 32,
                  FL_FIBRE = 63, FL_PORE = 64;

// Reduction slots (double per block, NV values per block).
constexpr int NV = 4;

// One problem on the device.  Face velocities are stored per cell for the cell's lower
// x / y / z face (x = 0 face: inlet; y = 0 and z = 0 faces: walls, zero), plus the outlet
// plane wxo (ny * nz) for the x = nx faces; upper y / z wall faces are zero by contract.
template <typename T>
struct Faces {
  const T *wx, *wy, *wz, *wxo;
};

struct Grid {
  int nx, ny, nz;
  long long n;          // nx * ny * nz
};

// Arguments of one explicit sweep.
template <typename T>
struct SweepArgs {
  Grid g;
  const uint8_t *flags;
  Faces<T> w;
  const float *kappa;   // nullable: uniform activity 1
  const T *s;           // state (or correction) read
  T *s_new;             // state (or correction) written
  const float *r0;      // defect correction: frozen FP64 residual in FP32 (else null)
  T dt, s_in, s_eq, Da; // in the correction form s_in = s_eq = 0
  T gscale;             // transpose sweeps: g_P = gscale * w_out,P on outlet cells
  int pinned;
  double lo, hi;        // bound check on the written state (ignored for corrections)
  double *partial;      // nullable: per-block [sum R^2, violations, sum R, -]
  int zc;               // z cells per block
  const int *gate = nullptr;  // nullable: the launch returns at once unless *gate == 0
                              // (device-side stop of the solve loop)
};

// FP64 residual refresh for the defect correction:
//   t = s64 + delta;  s64_new = t;  r0 = R64(t) (stored FP32); partials of R64.
struct RefreshArgs {
  Grid g;
  const uint8_t *flags;
  Faces<double> w;
  const float *kappa;
  const double *s64;
  const float *delta;   // nullable: zero correction
  double *s64_new;
  float *r0;
  double s_in, s_eq, Da;
  int pinned;
  double lo, hi;
  double *partial;
  int zc;
};

// Adjoint sweep: psi_new = psi + dt (g - A^T psi) (reversed advection).
template <typename T>
struct AdjointArgs {
  Grid g;
  const uint8_t *flags;
  Faces<T> w;
  const float *kappa;
  const T *psi;
  T *psi_new;
  const float *r0;      // correction form: frozen FP64 adjoint residual (else null)
  T dt, Da, gscale;     // g_P = gscale * w_out,P on outlet cells (0 in correction form)
  int pinned;
  double *partial;
  int zc;
};

struct AdjRefreshArgs {
  Grid g;
  const uint8_t *flags;
  Faces<double> w;
  const float *kappa;
  const double *psi64;
  const float *delta;
  double *psi64_new;
  float *r0;
  double Da, gscale;
  int pinned;
  double *partial;
  int zc;
};

struct SolveCtl;

// One problem of a batched launch (device table entry).
struct BatchProb {
  int nx, ny, nz;
  int w, rx;            // two-sweep items: cells per lane, lanes per row segment
  const uint8_t *flags;
  const float *wx, *wy, *wz, *wxo;
  const float *kappa;
  float *s0, *s1;       // ping-pong buffers: parity 0 reads s0, writes s1
  const float *r0;      // correction form: frozen FP64 residual (else unused)
  float dt, Da, s_in, s_eq;
  double lo, hi;
  int pinned;
  int gx, gy, gz, zc;   // tile grid of this problem: 64 x ty lanes x zc planes, or for the
                        // two-sweep path tiles of shape (w, rx) (tile2_xy) x zc planes
  int tile0;            // index of its first tile in the work list
  int two;              // items of the two-sweep kernel (else of the single-sweep one)
  SolveCtl *ctl;        // device-side loop state of this problem
  const double *rpart;  // its refresh partials (rnblk blocks)
  int rnblk;
};

// work: tile numbers of the unfinished problems; *nwork (device) their count
void launch_batch_sweep(const BatchProb *probs, const int *tile_prob, const int *work,
                        const int *nwork, int nblocks, int ty, int parity, bool dc,
                        double *partial, hipStream_t st);
// two sweeps per launch over the work list's (problem, tile) items; correction form, no
// activity field.  grab: two device ints, zero before the first launch; each launch takes
// items from grab[0] and leaves both at zero when it ends
void launch_batch_sweep2(const BatchProb *probs, const int *tile_prob, const int *work,
                         const int *nwork, int *grab, int nblocks, int parity, double *partial,
                         hipStream_t st);
void launch_batch_reduce(const BatchProb *probs, int n, const double *partial, double *out,
                         hipStream_t st);

// Iterative upsampling (even nx, ny, nz): coarse mask (fibre iff all eight children are
// fibre), coarse staggered FP64 face velocities (half the sum of the four fine faces), and
// the prolongation of a coarse state to the fine pore cells.
void launch_coarse_mask(const Grid &g, const uint8_t *flags, uint8_t *solid_c, hipStream_t st);
void launch_restrict(const Grid &g, const Faces<double> &w, double *ux_c, double *uy_c,
                     double *uz_c, hipStream_t st);
void launch_prolong(const Grid &g, const uint8_t *flags, const double *s_c, double *s_f,
                    hipStream_t st);

// Launch shapes.
struct Tiles {
  int ty;   // threads (rows) along y per block; x is one 64-wide wave
  int zc;   // z cells marched per block
  int zc2;  // z cells per block of the two-sweep kernel
  int two;  // FP32 sweeps two per launch (shapes below 2^30 cells)
  int rx = 64;  // two-sweep tiles: lanes per row segment (64: one row per wave; 32: two)
};

// Two-sweep tiles: a block of 1024 lanes holds rows of rx lanes (rx = 64: 16 rows of one wave
// each; rx = 32: 32 rows, two per wave), w cells per lane, and writes its interior
// (rx - 2) w x (1024 / rx - 2) cells.  gx, gy: tiles along x and y.
inline void tile2_xy(int nx, int ny, int w, int rx, int &gx, int &gy) {
  const int ox = (rx - 2) * w, oy = 1024 / rx - 2;
  gx = (nx + ox - 1) / ox;
  gy = (ny + oy - 1) / oy;
}

// Relative cost per lane of 32-lane rows against 64-lane rows, measured on the 1024 x 512 x 256
// slab (10% longer per lane: a wave's loads span two rows).
constexpr double RX32_COST = 1.10;

// The row-segment width with the lower cost of the lanes it computes per plane (ties: 64).
inline int pick_rx(int nx, int ny, int w) {
  int ax, ay, bx, by;
  tile2_xy(nx, ny, w, 64, ax, ay);
  tile2_xy(nx, ny, w, 32, bx, by);
  return RX32_COST * bx * by < (double)ax * ay ? 32 : 64;
}

// Explicit Nernst model (FP64): transport step on every pore cell; electrode (reactive)
// cells take sigma(V - eta) with eta relaxed toward the overpotential balancing the
// transport step.  eta is updated in place (each cell touches only its own).
struct NernstArgs {
  Grid g;
  const uint8_t *flags;
  Faces<double> w;
  const float *kappa;   // nullable: uniform activity 1
  const double *s;
  double *s_new;
  double *eta;
  double s_in, dt, Da, omega, V, K;   // V = logit(s_eq), K = 1 / sqrt(s_eq (1 - s_eq))
  double *partial;      // nullable: per-block [sum ((s'-s)/dt)^2, non-finite, -, -]
  int zc;
};
void launch_nernst(const NernstArgs &a, const Tiles &t, hipStream_t st);

// ---- upstream flow step: steady Stokes flow by projection steps (flow.hip) ------------
// Face arrays in the staggered layout (x faces (nz, ny, nx+1), y faces (nz, ny+1, nx),
// z faces (nz+1, ny, nx)).  code[a][f]: bit 15 = open face; bits 2n..2n+1 = class of the
// neighbour face n (x-, x+, y-, y+, z-, z+) of the same orientation: 0 beyond the inlet /
// outlet plane (zero gradient), 1 open, 2 closed along the face normal, 3 wall across it.
constexpr uint16_t FC_OPEN = 0x8000;
// Scalar slots of the flow step (device doubles after the partials)
enum FlowSlot { FS_TARGET = 0, FS_DONE = 1, FS_CG_STEP = 2, FS_CG_TOTAL = 3, FS_N = 4 };
struct FlowArgs {
  Grid g;
  const uint8_t *flags;
  uint16_t *code[3];
  uint8_t *ccode;        // per cell: open-neighbour mask | inlet (64) | outlet (128); 0 = fibre
  double *u[3];          // velocity (updated in place by the projection)
  double *us[3];         // predictor output u*
  double *p, *r, *z, *q, *d[2];   // pressure and CG vectors (cells)
  double dt, p_in, theta2;        // theta2: (CG stop factor)^2
  int nbc, nbf;          // blocks of the cell kernels / per face array of the face kernels
  double *prz[2], *prr[2], *pdq;  // per-block CG partials (cell kernels), ping-pong by parity
  double *pdu;           // per-block [sum du^2, sum u^2] of the projection, (3 nbf) x 2
  double *pdiv;          // per-block [max |div u|, inlet flux] (cell kernels), nbc x 2
  double *pfl;           // per-block sum of b^2 + (diag p)^2 of the CG start (the floor)
  double *sc;            // FlowSlot scalars
};
int flow_cell_blocks(const Grid &g);
int flow_face_blocks(const Grid &g);
void launch_flow_codes(const FlowArgs &a, hipStream_t st);
void launch_flow_predict(const FlowArgs &a, hipStream_t st);
void launch_flow_cg_init(const FlowArgs &a, hipStream_t st);
void launch_flow_cg_iter(const FlowArgs &a, int j, hipStream_t st);   // both CG kernels
void launch_flow_project(const FlowArgs &a, hipStream_t st);
void launch_flow_check(const FlowArgs &a, hipStream_t st);   // fills pdiv


dim3 sweep_grid(const Grid &g, const Tiles &t);
// FP32 sweeps use four cells per lane when nx % 4 == 0 (grid: 256 x cells per block)
bool vec4_path(const Grid &g);
dim3 sweep_grid_v4(const Grid &g, const Tiles &t);
// two FP32 sweeps per launch (nx even): tiles of 124 x 14 output cells
bool two_path(const Grid &g);
int two_w(const Grid &g);   // cells per lane of the two-sweep kernel: 2 for even nx, 1 for odd
dim3 sweep2_grid(const Grid &g, const Tiles &t);
// adj: sweeps of the transpose system (correction form only)
void launch_sweep2(const SweepArgs<float> &a, const Tiles &t, hipStream_t st, bool adj = false);

// ---- kernels (launch wrappers; all enqueue on `st`) ---------------------------------

void launch_flags(const Grid &g, const uint8_t *solid, uint8_t *flags, double *partial,
                  int nblk, hipStream_t st);
int flags_blocks(const Grid &g);

// velocity ingest: writes FP32 and FP64 per-cell lower faces and the outlet plane.
// partial per block: [Q_in, max|div|, max|u|, bad-face count]
void launch_velocity(const Grid &g, const uint8_t *flags, const double *ux, const double *uy,
                     const double *uz, double q, float *w32[4], double *w64[4],
                     double *partial, int nblk, hipStream_t st);
int velocity_blocks(const Grid &g);

// max over updated cells of sum max(w,0) + sum G + lam (partial slot 0, max)
void launch_maxdiag(const Grid &g, const uint8_t *flags, Faces<double> w, const float *kappa,
                    double Da, int pinned, double *partial, int nblk, hipStream_t st);

template <typename T>
void launch_sweep(const SweepArgs<T> &a, const Tiles &t, hipStream_t st);
void launch_refresh(const RefreshArgs &a, const Tiles &t, hipStream_t st);
template <typename T>
void launch_adjoint(const AdjointArgs<T> &a, const Tiles &t, hipStream_t st);
void launch_adj_refresh(const AdjRefreshArgs &a, const Tiles &t, hipStream_t st);

// FP64 sweeps (any nx) by the FP64 plane march; partials as for launch_sweep
void launch_sweep64(const SweepArgs<double> &a, hipStream_t st);
int march64_blocks(const Grid &g);
// Batched FP64 sweeps (the polish of a batched solve): one entry per problem of a launch
struct BatchM64 {
  SweepArgs<double> a;   // geometry, faces, flags, activity, dt, s_in, s_eq, Da, bounds
  double *pair[2];       // the problem's two FP64 state buffers
  int c0;                // buffer read at parity 0
  int gx, gy, gz, zc;    // its march grid (march64_shape)
  int blk0;              // its first item
  int prob;              // its index in the batch (result slot)
};
void march64_shape(const Grid &g, int &gx, int &gy, int &gz, int &zc);
// one FP64 sweep of every problem in probs[0..nprob) over nitems items; with partial (NV
// doubles per item) also each problem's sums into out[NV prob]
void launch_batch_march64(const BatchM64 *probs, int nprob, const int *item_prob, int nitems,
                          int parity, double *partial, double *out, hipStream_t st);
   // blocks (partial slots) of any FP64 march launch

// outputs of a state: partial per block (NV2 = 8 slots):
// [sum_out w s, sum_out w, F_in, F_in_adv, reaction, sum_R, sum R^2, -]
constexpr int NV2 = 8;
void launch_outputs(const Grid &g, const uint8_t *flags, Faces<double> w, const float *kappa,
                    const double *s, double s_in, double s_eq, double Da, int pinned,
                    double *partial, int nblk, hipStream_t st);
int outputs_blocks(const Grid &g);

// gradients (one thread per cell, flags_blocks(g) blocks): dU_dkappa and partial
// [sum psi Radv, -, -, -]
void launch_gradients(const Grid &g, const uint8_t *flags, Faces<double> w, const double *s,
                      const double *psi, double s_in, double s_eq, double Da, int pinned,
                      double *dU_dkappa, double *partial, int nblk, hipStream_t st);

// deterministic second pass: out[k] = sum (or max if bit k of maxmask) over blocks
void launch_reduce(const double *partial, int nblk, int nv, unsigned maxmask, double *out,
                   hipStream_t st);

// Device-side control of the FP32 correction solve: the stop rule and the refresh decision of
// every chunk of sweeps are taken on the device, so the host enqueues many chunks between two
// reads of the state.  Sweeps run while state == CTL_RUN; the refresh while CTL_REFRESH; the
// corrections are zeroed before a chunk while `fill` is set.
enum { CTL_RUN = 0, CTL_REFRESH = 1, CTL_DONE = 2, CTL_STOP = 3, CTL_DIVERGED = 4 };
struct SolveCtl {
  int state;            // CTL_*
  int fill;             // zero the corrections before the next chunk
  int cur;              // s64 buffer holding the state
  int stall;            // chunks without a 0.1% residual decrease
  long long it;         // FP32 sweeps done
  long long max_iter;
  int cycles;           // refreshes after the first
  int pad;
  double tol, tau, npore, reduction;   // stop tolerance, time scale, pore cells, per-cycle drop
  double target, best, res, ri;        // cycle target, best correction residual, last FP64 /
                                       // correction residual
};
// after a chunk of k sweeps (its last launch wrote nblk x NV partials): the correction
// residual, the iteration count, the cycle's stop test (refresh when due)
void launch_ctl_chunk(SolveCtl *ctl, const double *partial, int nblk, int k, hipStream_t st);
// after the (gated) refresh: the FP64 residual, the stop rule of the solve, the next cycle
void launch_ctl_refresh(SolveCtl *ctl, const double *partial, int nblk, hipStream_t st);
// The batched loop on the device: BATCH_WORKLIST rebuilds the work lists from the problems'
// states; BATCH_FILL zeroes the corrections of the problems that start a cycle; BATCH_CHUNK
// takes every sweeping problem's decision from the reduced partials `out` of a chunk of k
// sweeps; BATCH_REFRESH applies the stop rule after the problems' gated refreshes.
enum { BATCH_WORKLIST = 0, BATCH_FILL = 1, BATCH_CHUNK = 2, BATCH_REFRESH = 3 };
void launch_batch_control(const BatchProb *probs, int n, int *work, int max_tiles, int *nwork,
                          int which, const double *out, int k, hipStream_t st);
// the refresh of the correction, gated on state == CTL_REFRESH, reading s64[ctl->cur] (+ delta)
// and writing s64[ctl->cur ^ 1]
void launch_refresh_gated(const RefreshArgs &a, double *s64_0, double *s64_1,
                          const SolveCtl *ctl, hipStream_t st);
// zero two FP32 buffers of n values when ctl->fill is set
void launch_fill_gated(float *a, float *b, long long n, const SolveCtl *ctl, hipStream_t st);

// Static scratch of the allocation-free entry point: SCRATCH_DOUBLES doubles of device memory
// per GPU.  scratch_address gives its device address on device dev (which must be current at
// the first call for that device; the address is looked up once and kept); returns 0 or a
// hipError_t.
constexpr long long SCRATCH_DOUBLES = 1ll << 19;      // 4 MiB
constexpr int SCRATCH_MAX_DEVICES = 64;
int scratch_address(int dev, double **out);

// helpers
void launch_fill_f32(float *p, long long n, float v, hipStream_t st);
void launch_fill_f64(double *p, long long n, double v, hipStream_t st);
void launch_init_state(const Grid &g, const uint8_t *flags, const double *s_init, double s_in,
                       double s_eq, int pinned, double *s64, hipStream_t st);
void launch_f64_to_f32(const double *a, float *b, long long n, hipStream_t st);
void launch_f32_to_f64(const float *a, double *b, long long n, hipStream_t st);
void launch_mask_held(const Grid &g, const uint8_t *flags, int pinned, double *p, hipStream_t st);

}  // namespace socfv
