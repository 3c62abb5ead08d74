// Host runtime of libsocfv: contexts, validation, the convergence loop, mixed precision,
// outputs, adjoint.  Implements the C ABI declared in include/socfv.h.
#include "../../include/socfv.h"
#include "internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <string>
#include <type_traits>
#include <vector>

using namespace socfv;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? SOCFV_OOM : SOCFV_HIP_ERROR, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                      \
  } while (0)

#define TRY(expr)            \
  do {                       \
    int r_ = (expr);         \
    if (r_ < 0) return r_;   \
  } while (0)

void hfree(void *ptr) {
  if (ptr) (void)hipFree(ptr);
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct socfv_ctx {
  Grid g{};
  hipStream_t st = nullptr;      // library stream (default priority)
  hipEvent_t ev = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;   // timing events around sweep chunks
  uint8_t *flags = nullptr;
  float *w32[4] = {nullptr, nullptr, nullptr, nullptr};
  double *w64[4] = {nullptr, nullptr, nullptr, nullptr};
  float *kappa = nullptr;
  float *s32[2] = {nullptr, nullptr};
  double *s64[2] = {nullptr, nullptr};
  float *r0 = nullptr;
  double *aux64 = nullptr;       // adjoint psi (FP64) ping-pong partner etc.
  double *aux64b = nullptr;
  double *partial = nullptr;
  long long partial_cap = 0;     // doubles
  double *dres = nullptr;        // device result slots
  double *hres = nullptr;        // pinned host mirror
  SolveCtl *dctl = nullptr;      // device-side control state of the FP32 solve
  SolveCtl *hctl = nullptr;      // pinned host mirror
  hipEvent_t evp[4 * 8] = {};    // timing events of a group of chunks
  long npore = 0, nreact = 0, ninlet = 0, noutlet = 0;
  bool have_velocity = false;
  double Q_in = 0, div_max = 0, u_max = 0;
  // the operator's version (velocity and activity; each set_* call bumps it) and the largest
  // diagonal last scanned for it at (Da, pinned), which fixes dt
  long long op_version = 0;
  long long md_version = -1;
  double md_Da = 0, md_value = 0;
  int md_pinned = -1;
  Tiles tiles{4, 8, 32, 1};
  bool tiles_fixed = false;
  int ncu = 1;                   // compute units of the device (for the tile choice)
  int dev = 0;                   // device holding the context's buffers
  // last forward solution
  bool have_state = false;
  int state_buf = 0;             // s64[state_buf] holds the last steady state
  socfv_params last_p{};
};

namespace {

Faces<float> faces32(const socfv_ctx *c) { return {c->w32[0], c->w32[1], c->w32[2], c->w32[3]}; }
Faces<double> faces64(const socfv_ctx *c) { return {c->w64[0], c->w64[1], c->w64[2], c->w64[3]}; }

// Two-sweep launches run one block per CU (its LDS and registers fill a CU), each block
// marching one tile of shape (W, rx) through a z chunk plus two extra planes.  The chunk
// count is chosen to minimise (rounds of blocks over the CUs) x (planes per block), with
// chunks of at least 8 planes unless nz is smaller.
int pick_zc2(const Grid &g, int ncu, int rx) {
  int gx, gy;
  tile2_xy(g.nx, g.ny, two_w(g), rx, gx, gy);
  const long long t2 = (long long)gx * gy;
  if (ncu < 1) ncu = 1;
  long long best = -1;
  int zbest = g.nz;
  for (int c = 1; c <= g.nz; ++c) {
    const int zc2 = (g.nz + c - 1) / c;
    if (c > 1 && zc2 < 8) break;
    const long long blocks = t2 * ((g.nz + zc2 - 1) / zc2);
    const long long cost = (blocks + ncu - 1) / ncu * (zc2 + 2);
    if (best < 0 || cost < best) {
      best = cost;
      zbest = zc2;
    }
  }
  return zbest;
}

Tiles auto_tiles(const Grid &g, int ty, int ncu) {
  long long txy = (long long)((g.nx + 63) / 64) * ((g.ny + ty - 1) / ty);
  long long zc = (long long)g.nz * txy / 8192;
  if (zc < 1) zc = 1;
  if (zc > 32) zc = 32;
  if (zc > g.nz) zc = g.nz;
  const int rx = pick_rx(g.nx, g.ny, two_w(g));
  Tiles t{ty, (int)zc, pick_zc2(g, ncu, rx), 1};
  t.rx = rx;
  return t;
}

long long sweep_blocks(const Grid &g, const Tiles &t) {
  dim3 d = sweep_grid(g, t);
  return (long long)d.x * d.y * d.z;
}

// doubles of per-block partials any sweep launch of this problem can write
long long partial_need(const Grid &g, const Tiles &t) {
  dim3 a = sweep_grid(g, t), b = sweep_grid_v4(g, t), c = sweep2_grid(g, t);
  long long m = (long long)a.x * a.y * a.z;
  m = std::max(m, (long long)b.x * b.y * b.z);
  m = std::max(m, (long long)c.x * c.y * c.z);
  return std::max(NV * m, (long long)NV2 * march64_blocks(g)) + 64;
}

int ensure_partial(socfv_ctx *c, long long doubles) {
  if (doubles <= c->partial_cap) return 0;
  if (c->partial) hfree(c->partial);
  c->partial = nullptr;
  c->partial_cap = 0;
  HIPCHK(hipMalloc(&c->partial, sizeof(double) * doubles));
  c->partial_cap = doubles;
  return 0;
}

// reduce nblk x nv partials (device, at `partial`) into the device slots `dres`, then into
// host values out[0..nv-1] through the context's pinned mirror
int reduce_via(socfv_ctx *c, const double *partial, double *dres, int nblk, int nv,
               unsigned maxmask, double *out) {
  launch_reduce(partial, nblk, nv, maxmask, dres, c->st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->hres, dres, sizeof(double) * nv, hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  for (int k = 0; k < nv; ++k) out[k] = c->hres[k];
  return 0;
}

// the same with the context's own partials and result slots
int reduce_to_host(socfv_ctx *c, int nblk, int nv, unsigned maxmask, double *out) {
  return reduce_via(c, c->partial, c->dres, nblk, nv, maxmask, out);
}

// join the caller's stream: library work starts after the caller's prior work
int enter(socfv_ctx *c, void *user_stream) {
  HIPCHK(hipEventRecord(c->ev, (hipStream_t)user_stream));
  HIPCHK(hipStreamWaitEvent(c->st, c->ev, 0));
  return 0;
}

// outputs complete before returning; the caller's stream waits on the library's
int leave(socfv_ctx *c, void *user_stream) {
  HIPCHK(hipEventRecord(c->ev, c->st));
  HIPCHK(hipStreamWaitEvent((hipStream_t)user_stream, c->ev, 0));
  HIPCHK(hipStreamSynchronize(c->st));
  return 0;
}

int ensure_state(socfv_ctx *c) {
  const size_t n = (size_t)c->g.n;
  for (int k = 0; k < 2; ++k) {
    if (!c->s64[k]) HIPCHK(hipMalloc(&c->s64[k], sizeof(double) * n));
    if (!c->s32[k]) HIPCHK(hipMalloc(&c->s32[k], sizeof(float) * n));
  }
  if (!c->r0) HIPCHK(hipMalloc(&c->r0, sizeof(float) * n));
  if (!c->dctl) HIPCHK(hipMalloc(&c->dctl, sizeof(SolveCtl)));
  if (!c->hctl) HIPCHK(hipHostMalloc(&c->hctl, sizeof(SolveCtl), hipHostMallocDefault));
  for (hipEvent_t &e : c->evp)
    if (!e) HIPCHK(hipEventCreate(&e));
  return ensure_partial(c, partial_need(c->g, c->tiles));
}

int ensure_adjoint(socfv_ctx *c) {
  const size_t n = (size_t)c->g.n;
  if (!c->aux64) HIPCHK(hipMalloc(&c->aux64, sizeof(double) * n));
  if (!c->aux64b) HIPCHK(hipMalloc(&c->aux64b, sizeof(double) * n));
  return 0;
}

int check_params(const socfv_params *p) {
  if (!p) return fail(SOCFV_INVALID_ARG, "params is NULL");
  if (!(p->cfl > 0.0 && p->cfl <= 1.0)) return fail(SOCFV_INVALID_ARG, "cfl must be in (0, 1]");
  if (!(p->tol >= 0.0)) return fail(SOCFV_INVALID_ARG, "tol must be >= 0");
  if (p->max_iter < 1) return fail(SOCFV_INVALID_ARG, "max_iter must be >= 1");
  if (p->check_every < 1) return fail(SOCFV_INVALID_ARG, "check_every must be >= 1");
  if (p->mode != SOCFV_FINITE_RATE && p->mode != SOCFV_PINNED)
    return fail(SOCFV_INVALID_ARG, "unknown mode %d", p->mode);
  if (p->precision < SOCFV_FP64 || p->precision > SOCFV_FP32_PLAIN)
    return fail(SOCFV_INVALID_ARG, "unknown precision %d", p->precision);
  if (!std::isfinite(p->s_in) || !std::isfinite(p->s_eq) || !std::isfinite(p->Da) || p->Da < 0)
    return fail(SOCFV_INVALID_ARG, "s_in, s_eq must be finite and Da >= 0");
  if (p->s_in == p->s_eq) return fail(SOCFV_INVALID_ARG, "s_in must differ from s_eq (U undefined)");
  return 0;
}

// Residual reduction per FP32 correction cycle before the next FP64 refresh.  The FP32
// update of a correction loses precision once its increments fall far below the correction
// itself (rounding relative to the correction, not to the increment), which slows the slowly
// decaying modes; short cycles keep each correction small against its increments, so the
// cycles take the FP64 iteration's sweep count (measured equal on every parity box and on
// the 1024 x 512 x 256 slab; a reduction of 1e-4 per cycle took up to 30% more sweeps).  A
// refresh costs about five FP32 sweeps.
constexpr double CYCLE_REDUCTION = 0.1;

struct Solver {
  socfv_ctx *c;
  const socfv_params *p;
  int pinned;
  double dt = 0, tau = 0;
  double lo = 0, hi = 0;
  long it = 0, it32 = 0, it64 = 0, sw64 = 0;
  int cycles = 0;
  double ms32 = 0, ms64 = 0, msref = 0;
  Tiles t;
  long long nblk = 0;

  int setup() {
    pinned = p->mode == SOCFV_PINNED;
    t = c->tiles;
    nblk = sweep_blocks(c->g, t);
    TRY(ensure_state(c));
    // time step: cfl over the largest diagonal of the updated cells (scanned once per
    // operator and (Da, pinned); repeated solves on one operator reuse it)
    double md = c->md_value;
    if (c->md_version != c->op_version || c->md_Da != p->Da || c->md_pinned != (int)pinned) {
      const int mb = flags_blocks(c->g);
      TRY(ensure_partial(c, (long long)mb * NV2 + 64));
      launch_maxdiag(c->g, c->flags, faces64(c), c->kappa, p->Da, pinned, c->partial, mb, c->st);
      HIPCHK(hipGetLastError());
      TRY(reduce_to_host(c, mb, 1, 1u, &md));
      c->md_version = c->op_version;
      c->md_Da = p->Da;
      c->md_pinned = (int)pinned;
      c->md_value = md;
    }
    if (!(md > 0)) return fail(SOCFV_BAD_VELOCITY, "no updated cell (max diagonal %g)", md);
    dt = p->cfl / md;
    tau = (double)c->g.n / c->Q_in;
    lo = std::fmin(p->s_in, p->s_eq) - 1e-6;
    hi = std::fmax(p->s_in, p->s_eq) + 1e-6;
    return 0;
  }

  double res_of(double ss) const { return tau * std::sqrt(ss / (double)c->npore); }

  template <typename T>
  SweepArgs<T> sweep_args(const T *s, T *s_new, bool dc, double *partial) {
    SweepArgs<T> a;
    a.g = c->g;
    a.flags = c->flags;
    a.kappa = c->kappa;
    a.s = s;
    a.s_new = s_new;
    a.r0 = dc ? c->r0 : nullptr;
    a.dt = (T)dt;
    a.s_in = dc ? T(0) : (T)p->s_in;
    a.s_eq = dc ? T(0) : (T)p->s_eq;
    a.Da = (T)p->Da;
    a.gscale = T(0);
    a.pinned = pinned;
    a.lo = lo;
    a.hi = hi;
    a.partial = partial;
    a.zc = t.zc;
    return a;
  }

  // Enqueue k sweeps ping-ponging buf[cur] -> buf[cur^1], partials from the last one (gate:
  // nullable device flag, see SweepArgs); returns the partials' block count.
  template <typename T>
  long long launch_sweeps(T *buf0, T *buf1, int &cur, int k, bool dc, Faces<T> w,
                          const int *gate) {
    T *buf[2] = {buf0, buf1};
    const bool two = sizeof(T) == 4 && two_path(c->g) && t.two;
    long long nb = nblk;
    int j = 0;
    if (two) {
      // two sweeps per launch; an odd remainder ends with one single sweep
      for (; j + 1 < k; j += 2) {
        const bool lastl = j + 2 >= k;
        SweepArgs<T> a = sweep_args<T>(buf[cur], buf[cur ^ 1], dc, lastl ? c->partial : nullptr);
        a.w = w;
        a.gate = gate;
        launch_sweep2(reinterpret_cast<const SweepArgs<float> &>(a), t, c->st);
        cur ^= 1;
      }
      dim3 g2 = sweep2_grid(c->g, t);
      nb = (long long)g2.x * g2.y * g2.z;
    }
    for (; j < k; ++j) {
      SweepArgs<T> a = sweep_args<T>(buf[cur], buf[cur ^ 1], dc, j == k - 1 ? c->partial : nullptr);
      a.w = w;
      a.gate = gate;
      if constexpr (sizeof(T) == 8) {
        launch_sweep64(a, c->st);
        nb = march64_blocks(c->g);
      } else {
        launch_sweep<T>(a, t, c->st);
        if (vec4_path(c->g)) {
          dim3 gv = sweep_grid_v4(c->g, t);
          nb = (long long)gv.x * gv.y * gv.z;
        } else {
          nb = nblk;
        }
      }
      cur ^= 1;
    }
    return nb;
  }

  // k sweeps (as launch_sweeps), timed, then their partials reduced on the host
  template <typename T>
  int chunk(T *buf0, T *buf1, int &cur, int k, bool dc, Faces<T> w, double out[NV]) {
    HIPCHK(hipEventRecord(c->t0, c->st));
    const long long nb = launch_sweeps<T>(buf0, buf1, cur, k, dc, w, nullptr);
    HIPCHK(hipEventRecord(c->t1, c->st));
    HIPCHK(hipGetLastError());
    TRY(reduce_to_host(c, (int)nb, NV, 0u, out));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, c->t0, c->t1));
    (sizeof(T) == 4 ? ms32 : ms64) += ms;
    return 0;
  }

  // FP64 refresh: s64[dst] = s64[src] + delta; r0 = R64; returns res and violations
  int refresh(int src, int dst, const float *delta, double out[NV]) {
    RefreshArgs a;
    a.g = c->g;
    a.flags = c->flags;
    a.w = faces64(c);
    a.kappa = c->kappa;
    a.s64 = c->s64[src];
    a.delta = delta;
    a.s64_new = c->s64[dst];
    a.r0 = c->r0;
    a.s_in = p->s_in;
    a.s_eq = p->s_eq;
    a.Da = p->Da;
    a.pinned = pinned;
    a.lo = lo;
    a.hi = hi;
    a.partial = c->partial;
    a.zc = t.zc;
    HIPCHK(hipEventRecord(c->t0, c->st));
    launch_refresh(a, t, c->st);
    HIPCHK(hipEventRecord(c->t1, c->st));
    HIPCHK(hipGetLastError());
    ++it64;
    TRY(reduce_to_host(c, march64_blocks(c->g), NV, 0u, out));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, c->t0, c->t1));
    msref += ms;
    return 0;
  }

  int check(const double out[NV], double res) {
    if (!std::isfinite(res) || out[1] > 0.0)
      return fail(SOCFV_DIVERGED, "iteration diverged at sweep %ld (residual %g, %g cells out of "
                  "bounds or non-finite)", it, res, out[1]);
    return 0;
  }

  int chunk_len() const {
    int k = p->check_every < 2 ? 2 : p->check_every;
    return k + (k & 1);
  }

  // FP64 sweeps from s64[cur] until res < tol or max_iter.  Returns status.
  int run_fp64(int &cur, double &res, long budget) {
    const int K = chunk_len();
    double out[NV];
    int status = SOCFV_NOT_CONVERGED;
    long done = 0;
    while (done < budget) {
      long k = std::min<long>(K, budget - done);
      TRY(chunk<double>(c->s64[0], c->s64[1], cur, (int)k, false, faces64(c), out));
      done += k;
      it += k;
      it64 += k;
      sw64 += k;
      res = res_of(out[0]);
      TRY(check(out, res));
      if (res < p->tol) { status = SOCFV_OK; break; }
    }
    return status;
  }

  // FP32 correction cycles with the loop's decisions on the device (SolveCtl): per chunk
  // of K sweeps, the corrections are zeroed if a cycle starts (k_fill2_gated), the sweeps run
  // while the state is CTL_RUN, k_ctl_chunk takes the correction residual and the cycle's end
  // test, the refresh runs if it asked for one, and k_ctl_refresh applies the stop rule and
  // starts the next cycle.  The host enqueues groups of chunks and reads the state once per
  // group; launches after the stop return at once.  From s64[cur] with FP64 residual res.
  int run_dc_device(int &cur, double &res) {
    constexpr int G = 8;                 // most chunks per group (4 events each)
    const int K = chunk_len();
    const long long n = c->g.n;
    SolveCtl &h = *c->hctl;
    h = SolveCtl{};
    h.state = CTL_RUN;
    h.fill = 1;
    h.cur = cur;
    h.max_iter = p->max_iter - it;
    h.tol = p->tol;
    h.tau = tau;
    h.npore = (double)c->npore;
    h.reduction = CYCLE_REDUCTION;
    h.target = std::fmax(p->tol, CYCLE_REDUCTION * res);
    h.best = INFINITY;
    h.res = res;
    h.ri = INFINITY;
    const long long budget = h.max_iter;
    HIPCHK(hipMemcpyAsync(c->dctl, c->hctl, sizeof(SolveCtl), hipMemcpyHostToDevice, c->st));
    const int nbr = march64_blocks(c->g);
    long long known = 0;                 // sweeps done at the last read of the state
    long long it_prev = -1;              // sweeps and correction residual at the read before
    double ri_prev = 0;
    int ng = 2;                          // chunks in the next group
    for (;;) {
      int ks[G];
      int nch = 0;
      long long enq = known;
      for (; nch < ng && enq < budget; ++nch) {
        const int k = (int)std::min<long long>(K, budget - enq);
        launch_fill_gated(c->s32[0], c->s32[1], n, c->dctl, c->st);
        HIPCHK(hipEventRecord(c->evp[4 * nch], c->st));
        int cd = 0;
        const long long nb = launch_sweeps<float>(c->s32[0], c->s32[1], cd, k, true, faces32(c),
                                                  &c->dctl->state);
        HIPCHK(hipEventRecord(c->evp[4 * nch + 1], c->st));
        launch_ctl_chunk(c->dctl, c->partial, (int)nb, k, c->st);
        RefreshArgs a;
        a.g = c->g; a.flags = c->flags; a.w = faces64(c); a.kappa = c->kappa;
        a.s64 = nullptr; a.delta = c->s32[cd]; a.s64_new = nullptr; a.r0 = c->r0;
        a.s_in = p->s_in; a.s_eq = p->s_eq; a.Da = p->Da; a.pinned = pinned;
        a.lo = lo; a.hi = hi; a.partial = c->partial; a.zc = t.zc;
        HIPCHK(hipEventRecord(c->evp[4 * nch + 2], c->st));
        launch_refresh_gated(a, c->s64[0], c->s64[1], c->dctl, c->st);
        HIPCHK(hipEventRecord(c->evp[4 * nch + 3], c->st));
        launch_ctl_refresh(c->dctl, c->partial, nbr, c->st);
        ks[nch] = k;
        enq += k;
      }
      HIPCHK(hipGetLastError());
      const int cyc0 = h.cycles;
      HIPCHK(hipMemcpyAsync(c->hctl, c->dctl, sizeof(SolveCtl), hipMemcpyDeviceToHost, c->st));
      HIPCHK(hipStreamSynchronize(c->st));
      // GPU time of the chunks whose sweeps ran (the first ones of the group), and of the
      // refreshes that ran (the longest refresh launches; the others returned at once)
      long long ran = h.it - known;
      float refresh_ms[G];
      for (int g = 0; g < nch; ++g) {
        float ms = 0;
        if (ran >= ks[g]) {
          HIPCHK(hipEventElapsedTime(&ms, c->evp[4 * g], c->evp[4 * g + 1]));
          ms32 += ms;
          ran -= ks[g];
        }
        HIPCHK(hipEventElapsedTime(&refresh_ms[g], c->evp[4 * g + 2], c->evp[4 * g + 3]));
      }
      std::sort(refresh_ms, refresh_ms + nch);
      for (int g = nch - 1; g >= 0 && g >= nch - (h.cycles - cyc0); --g) msref += refresh_ms[g];
      known = h.it;
      if (h.state == CTL_DIVERGED || h.state == CTL_DONE || h.state == CTL_STOP || nch == 0) break;
      // next group: about half the chunks the residual's decay rate since the last read
      // still needs to reach tol (the correction residual continues the explicit
      // iteration's residual across refreshes), between 1 and G, so that few launches are
      // enqueued past the stop
      ng = G;
      if (it_prev >= 0 && h.it > it_prev && ri_prev > 0 && h.ri > 0 && h.ri < ri_prev) {
        const double per = std::log(h.ri / ri_prev) / (double)(h.it - it_prev);
        const double left = std::log(p->tol / h.ri) / per;            // sweeps to tol
        ng = (int)std::max(1.0, std::min((double)G, std::floor(left / K / 2.0)));
      }
      it_prev = h.it;
      ri_prev = h.ri;
    }
    it += known;
    it32 += known;
    cycles += h.cycles;
    it64 += h.cycles;
    cur = h.cur;
    res = h.res;
    if (h.state == CTL_DIVERGED)
      return fail(SOCFV_DIVERGED, "correction sweeps or refresh diverged at sweep %ld "
                  "(residual %g)", it, std::isfinite(h.ri) ? h.res : h.ri);
    return 0;
  }

  int solve(const double *s_init, double *res_final, int *state_buf) {
    TRY(setup());
    const long long n = c->g.n;
    launch_init_state(c->g, c->flags, s_init, p->s_in, p->s_eq, pinned, c->s64[0], c->st);
    HIPCHK(hipGetLastError());
    double out[NV];
    double res = INFINITY;
    int status = SOCFV_NOT_CONVERGED;
    int cur = 0;
    if (p->precision == SOCFV_FP64) {
      launch_fill_f64(c->s64[1], n, 0.0, c->st);
      status = run_fp64(cur, res, p->max_iter);
    } else if (p->precision == SOCFV_FP32_PLAIN) {
      launch_f64_to_f32(c->s64[0], c->s32[0], n, c->st);
      launch_fill_f32(c->s32[1], n, 0.0f, c->st);
      const int K = chunk_len();
      double best = INFINITY;
      int stall = 0;
      int c32 = 0;
      while (it < p->max_iter) {
        long k = std::min<long>(K, p->max_iter - it);
        TRY(chunk<float>(c->s32[0], c->s32[1], c32, (int)k, false, faces32(c), out));
        it += k;
        it32 += k;
        res = res_of(out[0]);
        TRY(check(out, res));
        if (res < p->tol) { status = SOCFV_OK; break; }
        if (res < 0.999 * best) { best = res; stall = 0; }
        else if (++stall >= 8) break;            // FP32 stagnation
      }
      launch_f32_to_f64(c->s32[c32], c->s64[0], n, c->st);
      cur = 0;
    } else {
      // FP32 sweeps on a correction delta against the FP64 residual r0 of s64:
      //   delta <- delta + dt (r0 - A delta); s64 += delta; r0 = b - A s64 (FP64 refresh)
      TRY(refresh(0, 1, nullptr, out));
      cur = 1;
      res = res_of(out[0]);
      TRY(check(out, res));
      if (res >= p->tol && it < p->max_iter) TRY(run_dc_device(cur, res));
      if (res < p->tol) status = SOCFV_OK;
      // FP64 polish sweeps from the refreshed state, within what max_iter leaves
      long np = p->polish_iters > 0 ? p->polish_iters : chunk_len();
      np += np & 1;
      np = std::min<long>(np, p->max_iter - it);
      if (status == SOCFV_OK && np > 0) {
        int pc = cur;
        double pres = res;
        (void)run_fp64(pc, pres, np);
        cur = pc;
        res = pres;
        status = res < p->tol ? SOCFV_OK : SOCFV_NOT_CONVERGED;
      }
    }
    *res_final = res;
    *state_buf = cur;
    return status;
  }
};

// outputs of state s: per-block partials at `partial` (outputs_blocks x NV2 doubles), the
// reduced values at `dres` (NV2 doubles); both device memory the caller provides
int eval_outputs_into(socfv_ctx *c, const socfv_params *p, const double *s, double *partial,
                      double *dres, socfv_stats *st) {
  const int nb = outputs_blocks(c->g);
  launch_outputs(c->g, c->flags, faces64(c), c->kappa, s, p->s_in, p->s_eq, p->Da,
                 p->mode == SOCFV_PINNED, partial, nb, c->st);
  HIPCHK(hipGetLastError());
  double o[NV2];
  TRY(reduce_via(c, partial, dres, nb, NV2, 0u, o));
  st->s_out = o[0] / o[1];
  st->q_out = o[1];
  st->flux_out = o[0];
  st->flux_in = o[2];
  st->flux_in_adv = o[3];
  st->reaction = o[4];
  st->sum_R = o[5];
  st->U = (st->s_out - p->s_in) / (p->s_eq - p->s_in);
  const double tau = (double)c->g.n / c->Q_in;
  st->tau = tau;
  st->residual = tau * std::sqrt(o[6] / (double)c->npore);
  return 0;
}

int eval_outputs(socfv_ctx *c, const socfv_params *p, const double *s, socfv_stats *st) {
  TRY(ensure_partial(c, (long long)outputs_blocks(c->g) * NV2 + 64));
  return eval_outputs_into(c, p, s, c->partial, c->dres, st);
}

}  // namespace

// ======================================================================================
// C ABI
// ======================================================================================

extern "C" {

int socfv_version(void) { return 1; }

const char *socfv_last_error(void) { return g_err.c_str(); }

void socfv_default_params(socfv_params *p) {
  if (!p) return;
  p->s_in = 1.0;
  p->s_eq = 0.0;
  p->Da = 0.45;
  p->mode = SOCFV_FINITE_RATE;
  p->precision = SOCFV_FP32;
  p->cfl = 0.4;
  p->tol = 1e-8;
  p->max_iter = 100000000L;
  p->check_every = 200;
  p->polish_iters = 0;
}

void socfv_destroy(socfv_ctx *c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  hfree(c->flags);
  for (int k = 0; k < 4; ++k) { hfree(c->w32[k]); hfree(c->w64[k]); }
  hfree(c->kappa);
  for (int k = 0; k < 2; ++k) { hfree(c->s32[k]); hfree(c->s64[k]); }
  hfree(c->r0);
  hfree(c->aux64);
  hfree(c->aux64b);
  hfree(c->partial);
  hfree(c->dres);
  if (c->hres) (void)hipHostFree(c->hres);
  hfree(c->dctl);
  if (c->hctl) (void)hipHostFree(c->hctl);
  for (hipEvent_t e : c->evp)
    if (e) (void)hipEventDestroy(e);
  if (c->ev) (void)hipEventDestroy(c->ev);
  if (c->t0) (void)hipEventDestroy(c->t0);
  if (c->t1) (void)hipEventDestroy(c->t1);
  if (c->st) (void)hipStreamDestroy(c->st);
  delete c;
}

int socfv_setup_geometry(socfv_ctx **out, int nx, int ny, int nz, const uint8_t *solid,
                         void *hip_stream) {
  if (!out) return fail(SOCFV_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (nx < 1 || ny < 1 || nz < 1) return fail(SOCFV_INVALID_ARG, "bad dims %d %d %d", nx, ny, nz);
  if (!solid) return fail(SOCFV_INVALID_ARG, "solid is NULL");
  const long long n = (long long)nx * ny * nz;
  if (n > (1ll << 40)) return fail(SOCFV_INVALID_ARG, "grid too large");
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return fail(SOCFV_HIP_ERROR, "device query failed");
  socfv_ctx *c = new socfv_ctx();
  c->g = Grid{nx, ny, nz, n};
  c->ncu = ncu;
  c->dev = dev;
  {
    // the allocation-free entry point's scratch: its device address, once per device
    double *scr = nullptr;
    const int e = scratch_address(dev, &scr);
    if (e != 0) {
      delete c;
      return fail(SOCFV_HIP_ERROR, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString((hipError_t)e));
    }
  }
  c->tiles = auto_tiles(c->g, 16, ncu);
  auto bail = [&](int code) { socfv_destroy(c); return code; };
  if (hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreate(&c->t0) != hipSuccess || hipEventCreate(&c->t1) != hipSuccess)
    return bail(fail(SOCFV_HIP_ERROR, "stream/event creation failed"));
  if (hipMalloc(&c->flags, (size_t)n) != hipSuccess ||
      hipMalloc(&c->dres, sizeof(double) * 64) != hipSuccess ||
      hipHostMalloc(&c->hres, sizeof(double) * 64, hipHostMallocDefault) != hipSuccess)
    return bail(fail(SOCFV_OOM, "device allocation failed (%lld cells)", n));
  int r = enter(c, hip_stream);
  if (r < 0) return bail(r);
  const int nb = flags_blocks(c->g);
  if ((r = ensure_partial(c, 4ll * nb + 64)) < 0) return bail(r);
  launch_flags(c->g, solid, c->flags, c->partial, nb, c->st);
  if (hipGetLastError() != hipSuccess) return bail(fail(SOCFV_HIP_ERROR, "flags kernel launch"));
  double cnt[4];
  if ((r = reduce_to_host(c, nb, 4, 0u, cnt)) < 0) return bail(r);
  c->npore = (long)cnt[0];
  c->nreact = (long)cnt[1];
  c->ninlet = (long)cnt[2];
  c->noutlet = (long)cnt[3];
  if (c->ninlet == 0 || c->noutlet == 0)
    return bail(fail(SOCFV_BAD_GEOMETRY, "no pore cell in the %s plane",
                     c->ninlet == 0 ? "inlet" : "outlet"));
  // every pore cell must be face-connected to the inlet plane (host breadth-first search)
  std::vector<uint8_t> fl((size_t)n);
  if (hipMemcpyAsync(fl.data(), c->flags, (size_t)n, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
      hipStreamSynchronize(c->st) != hipSuccess)
    return bail(fail(SOCFV_HIP_ERROR, "flags copy"));
  std::vector<uint8_t> seen((size_t)n, 0);
  std::vector<long long> queue;
  queue.reserve((size_t)c->npore);
  const long long pl = (long long)nx * ny;
  for (long long z = 0; z < nz; ++z)
    for (long long y = 0; y < ny; ++y) {
      long long i = nx * (y + ny * z);
      if (fl[i] & FL_PORE) { seen[i] = 1; queue.push_back(i); }
    }
  for (size_t h = 0; h < queue.size(); ++h) {
    const long long i = queue[h];
    const long long x = i % nx, y = (i / nx) % ny, z = i / pl;
    const long long nb6[6] = {x > 0 ? i - 1 : -1, x < nx - 1 ? i + 1 : -1,
                              y > 0 ? i - nx : -1, y < ny - 1 ? i + nx : -1,
                              z > 0 ? i - pl : -1, z < nz - 1 ? i + pl : -1};
    for (long long j : nb6)
      if (j >= 0 && !seen[j] && (fl[j] & FL_PORE)) { seen[j] = 1; queue.push_back(j); }
  }
  const long long missing = c->npore - (long long)queue.size();
  if (missing != 0)
    return bail(fail(SOCFV_BAD_GEOMETRY, "%lld pore cells are not face-connected to the inlet",
                     missing));
  if ((r = leave(c, hip_stream)) < 0) return bail(r);
  *out = c;
  return SOCFV_OK;
}

int socfv_set_velocity(socfv_ctx *c, const double *ux, const double *uy, const double *uz,
                       double q, void *hip_stream) {
  if (!c || !ux || !uy || !uz) return fail(SOCFV_INVALID_ARG, "NULL argument");
  if (!std::isfinite(q) || q <= 0) return fail(SOCFV_INVALID_ARG, "q must be finite and > 0");
  const size_t n = (size_t)c->g.n, plane = (size_t)c->g.ny * c->g.nz;
  for (int k = 0; k < 3; ++k) {
    if (!c->w32[k]) HIPCHK(hipMalloc(&c->w32[k], sizeof(float) * n));
    if (!c->w64[k]) HIPCHK(hipMalloc(&c->w64[k], sizeof(double) * n));
  }
  if (!c->w32[3]) HIPCHK(hipMalloc(&c->w32[3], sizeof(float) * plane));
  if (!c->w64[3]) HIPCHK(hipMalloc(&c->w64[3], sizeof(double) * plane));
  TRY(enter(c, hip_stream));
  ++c->op_version;
  const int nb = velocity_blocks(c->g);
  TRY(ensure_partial(c, 4ll * nb + 64));
  launch_velocity(c->g, c->flags, ux, uy, uz, q, c->w32, c->w64, c->partial, nb, c->st);
  HIPCHK(hipGetLastError());
  double v[4];
  TRY(reduce_to_host(c, nb, 4, 0x6u, v));
  c->have_velocity = false;
  c->have_state = false;
  if (v[3] > 0)
    return fail(SOCFV_BAD_VELOCITY, "%.0f faces: non-finite or flux through a closed face", v[3]);
  if (!(v[0] > 0)) return fail(SOCFV_BAD_VELOCITY, "no net inflow (Q = %g)", v[0]);
  if (v[1] > 1e-6 * v[2])
    return fail(SOCFV_BAD_VELOCITY, "cell divergence %g exceeds 1e-6 x max velocity %g", v[1], v[2]);
  c->Q_in = v[0];
  c->div_max = v[1];
  c->u_max = v[2];
  c->have_velocity = true;
  TRY(leave(c, hip_stream));
  return SOCFV_OK;
}

int socfv_set_activity(socfv_ctx *c, const float *kappa, void *hip_stream) {
  if (!c) return fail(SOCFV_INVALID_ARG, "NULL context");
  c->have_state = false;
  ++c->op_version;
  if (!kappa) {
    if (c->kappa) hfree(c->kappa);
    c->kappa = nullptr;
    return SOCFV_OK;
  }
  if (!c->kappa) HIPCHK(hipMalloc(&c->kappa, sizeof(float) * (size_t)c->g.n));
  TRY(enter(c, hip_stream));
  HIPCHK(hipMemcpyAsync(c->kappa, kappa, sizeof(float) * (size_t)c->g.n, hipMemcpyDeviceToDevice,
                        c->st));
  TRY(leave(c, hip_stream));
  return SOCFV_OK;
}

int socfv_solve_soc_steady(socfv_ctx *c, const socfv_params *p, const double *s_init,
                           double *s_out, socfv_stats *st, void *hip_stream) {
  const double t0 = now_s();
  if (!c) return fail(SOCFV_INVALID_ARG, "NULL context");
  TRY(check_params(p));
  if (!c->have_velocity) return fail(SOCFV_INVALID_ARG, "velocity not set");
  TRY(enter(c, hip_stream));
  Solver S{c, p};
  double res = 0;
  int buf = 0;
  c->have_state = false;
  int status = S.solve(s_init, &res, &buf);
  if (status < 0) {
    (void)hipStreamSynchronize(c->st);
    return status;
  }
  c->have_state = true;
  c->state_buf = buf;
  c->last_p = *p;
  socfv_stats s{};
  TRY(eval_outputs(c, p, c->s64[buf], &s));
  if (s_out)
    HIPCHK(hipMemcpyAsync(s_out, c->s64[buf], sizeof(double) * (size_t)c->g.n,
                          hipMemcpyDeviceToDevice, c->st));
  TRY(leave(c, hip_stream));
  s.iterations = S.it;
  s.it_fp32 = S.it32;
  s.it_fp64 = S.it64;
  s.cycles = S.cycles;
  s.status = status;
  s.ms_fp32 = S.ms32;
  s.ms_fp64 = S.ms64;
  s.ms_refresh = S.msref;
  s.sweeps_fp64 = S.sw64;
  s.tile_y = S.t.ty;
  s.z_chunk = S.t.zc;
  s.dt = S.dt;
  s.tau = S.tau;
  s.residual = p->precision == SOCFV_FP64 ? res : s.residual;
  s.seconds = now_s() - t0;
  if (st) *st = s;
  if (status == SOCFV_NOT_CONVERGED)
    fail(SOCFV_NOT_CONVERGED, "not converged after %ld sweeps (residual %g)", S.it, res);
  return status;
}

int socfv_compute_umt(socfv_ctx *c, const socfv_params *p, double *U_mt, double *s_out,
                      socfv_stats *st, void *hip_stream) {
  socfv_params q;
  if (p) q = *p; else socfv_default_params(&q);
  q.mode = SOCFV_PINNED;
  q.s_in = 0.0;
  q.s_eq = 1.0;
  q.Da = 0.0;
  socfv_stats s{};
  int r = socfv_solve_soc_steady(c, &q, nullptr, s_out, &s, hip_stream);
  if (st) *st = s;
  if (U_mt && r >= 0) *U_mt = s.U;
  return r;
}

int socfv_evaluate(socfv_ctx *c, const socfv_params *p, const double *s, socfv_stats *st,
                   void *hip_stream) {
  if (!c || !st) return fail(SOCFV_INVALID_ARG, "NULL argument");
  TRY(check_params(p));
  if (!c->have_velocity) return fail(SOCFV_INVALID_ARG, "velocity not set");
  if (!s) {
    if (!c->have_state) return fail(SOCFV_INVALID_ARG, "no state in this context");
    s = c->s64[c->state_buf];
  }
  TRY(enter(c, hip_stream));
  socfv_stats o{};
  TRY(eval_outputs(c, p, s, &o));
  TRY(leave(c, hip_stream));
  st->U = o.U; st->s_out = o.s_out; st->flux_in = o.flux_in; st->flux_in_adv = o.flux_in_adv;
  st->flux_out = o.flux_out; st->reaction = o.reaction; st->sum_R = o.sum_R; st->q_out = o.q_out;
  st->residual = o.residual; st->tau = o.tau;
  return SOCFV_OK;
}

int socfv_evaluate_noalloc(socfv_ctx *c, const socfv_params *p, const double *s,
                           socfv_stats *st, void *hip_stream) {
  if (!c || !st) return fail(SOCFV_INVALID_ARG, "NULL argument");
  TRY(check_params(p));
  if (!c->have_velocity) return fail(SOCFV_INVALID_ARG, "velocity not set");
  if (!s) {
    if (!c->have_state) return fail(SOCFV_INVALID_ARG, "no state in this context");
    s = c->s64[c->state_buf];
  }
  int cur = -1;
  HIPCHK(hipGetDevice(&cur));
  if (cur != c->dev)
    return fail(SOCFV_INVALID_ARG, "context lives on device %d; device %d is current", c->dev,
                cur);
  double *scr = nullptr;
  const int e = scratch_address(c->dev, &scr);
  if (e != 0)
    return fail(SOCFV_HIP_ERROR, "static scratch of device %d: %s", c->dev,
                hipGetErrorString((hipError_t)e));
  const long long nb = outputs_blocks(c->g);
  if (nb * NV2 + NV2 > SCRATCH_DOUBLES)
    return fail(SOCFV_INVALID_ARG, "grid too large for the static scratch: %lld blocks x %d "
                "partials + %d results exceed %lld doubles (at most %lld blocks)", nb, NV2, NV2,
                SCRATCH_DOUBLES, (SCRATCH_DOUBLES - NV2) / NV2);
  TRY(enter(c, hip_stream));
  socfv_stats o{};
  TRY(eval_outputs_into(c, p, s, scr, scr + nb * NV2, &o));
  TRY(leave(c, hip_stream));
  st->U = o.U; st->s_out = o.s_out; st->flux_in = o.flux_in; st->flux_in_adv = o.flux_in_adv;
  st->flux_out = o.flux_out; st->reaction = o.reaction; st->sum_R = o.sum_R; st->q_out = o.q_out;
  st->residual = o.residual; st->tau = o.tau;
  return SOCFV_OK;
}

int socfv_solve_soc_adjoint(socfv_ctx *c, const socfv_params *p, double *dU_dkappa,
                            double *dU_dlnq, double *psi_out, socfv_stats *st,
                            void *hip_stream) {
  const double t0 = now_s();
  if (!c) return fail(SOCFV_INVALID_ARG, "NULL context");
  TRY(check_params(p));
  if (!c->have_state) return fail(SOCFV_INVALID_ARG, "no forward state: solve first");
  if (c->last_p.s_in != p->s_in || c->last_p.s_eq != p->s_eq || c->last_p.Da != p->Da ||
      c->last_p.mode != p->mode || c->last_p.cfl != p->cfl)
    return fail(SOCFV_INVALID_ARG, "parameters differ from the forward solve");
  TRY(ensure_adjoint(c));
  TRY(enter(c, hip_stream));
  Solver S{c, p};
  TRY(S.setup());
  const long long n = c->g.n;
  const int pinned = p->mode == SOCFV_PINNED;
  // g_P = w_out,P / (Q_out (s_eq - s_in)); Q_out from the outputs of the forward state
  socfv_stats o{};
  TRY(eval_outputs(c, p, c->s64[c->state_buf], &o));
  const double gscale = 1.0 / (o.q_out * (p->s_eq - p->s_in));
  double *psi[2] = {c->aux64, c->aux64b};
  launch_fill_f64(psi[0], n, 0.0, c->st);
  launch_fill_f64(psi[1], n, 0.0, c->st);
  const int K = S.chunk_len();
  double out[NV];
  // relative residual ||g - A^T psi|| / ||g||, ||g|| from psi = 0
  auto adj_refresh = [&](int src, int dst, const float *delta) -> int {
    AdjRefreshArgs a;
    a.g = c->g; a.flags = c->flags; a.w = faces64(c); a.kappa = c->kappa;
    a.psi64 = psi[src]; a.delta = delta; a.psi64_new = psi[dst]; a.r0 = c->r0;
    a.Da = p->Da; a.gscale = gscale; a.pinned = pinned; a.partial = c->partial; a.zc = S.t.zc;
    launch_adj_refresh(a, S.t, c->st);
    HIPCHK(hipGetLastError());
    ++S.it64;
    return reduce_to_host(c, (int)S.nblk, NV, 0u, out);
  };
  TRY(adj_refresh(0, 1, nullptr));
  int cur = 1;
  const double gnorm = std::sqrt(out[0]);
  if (!(gnorm > 0)) return fail(SOCFV_INVALID_ARG, "zero adjoint right-hand side");
  double rel = 1.0;
  int status = SOCFV_NOT_CONVERGED;
  auto adj_chunk = [&](auto *b0, auto *b1, int &cc, int k, bool dc, auto w, double gs) -> int {
    using T = std::remove_pointer_t<decltype(b0)>;
    T *b[2] = {b0, b1};
    long long nb = S.nblk;
    int j = 0;
    if constexpr (std::is_same_v<T, float>) {
      // FP32 corrections: two transpose sweeps per launch where the shape allows; an odd
      // remainder ends with one single sweep
      if (dc && two_path(c->g) && S.t.two) {
        for (; j + 1 < k; j += 2) {
          SweepArgs<float> a = S.sweep_args<float>(b[cc], b[cc ^ 1], true,
                                                   j + 2 >= k ? c->partial : nullptr);
          a.w = w;
          a.gscale = (float)gs;
          launch_sweep2(a, S.t, c->st, true);
          cc ^= 1;
        }
        const dim3 g2 = sweep2_grid(c->g, S.t);
        nb = (long long)g2.x * g2.y * g2.z;
      }
    }
    for (; j < k; ++j) {
      AdjointArgs<T> a;
      a.g = c->g; a.flags = c->flags; a.w = w; a.kappa = c->kappa;
      a.psi = b[cc]; a.psi_new = b[cc ^ 1]; a.r0 = dc ? c->r0 : nullptr;
      a.dt = (T)S.dt; a.Da = (T)p->Da; a.gscale = (T)gs; a.pinned = pinned;
      a.partial = j == k - 1 ? c->partial : nullptr; a.zc = S.t.zc;
      launch_adjoint<T>(a, S.t, c->st);
      cc ^= 1;
      nb = S.nblk;
    }
    HIPCHK(hipGetLastError());
    return reduce_to_host(c, (int)nb, NV, 0u, out);
  };
  if (p->precision == SOCFV_FP64) {
    while (S.it < p->max_iter) {
      long k = std::min<long>(K, p->max_iter - S.it);
      TRY(adj_chunk(psi[0], psi[1], cur, (int)k, false, faces64(c), gscale));
      S.it += k;
      S.it64 += k;
      rel = std::sqrt(out[0]) / gnorm;
      if (!std::isfinite(rel) || out[1] > 0) return fail(SOCFV_DIVERGED, "adjoint diverged");
      if (rel < p->tol) { status = SOCFV_OK; break; }
    }
  } else {
    rel = 1.0;
    while (rel >= p->tol && S.it < p->max_iter) {
      launch_fill_f32(c->s32[0], n, 0.0f, c->st);
      launch_fill_f32(c->s32[1], n, 0.0f, c->st);
      int cd = 0;
      const double target = std::fmax(p->tol, CYCLE_REDUCTION * rel);
      double best = INFINITY;
      int stall = 0;
      while (S.it < p->max_iter) {
        long k = std::min<long>(K, p->max_iter - S.it);
        TRY(adj_chunk(c->s32[0], c->s32[1], cd, (int)k, true, faces32(c), 0.0));
        S.it += k;
        S.it32 += k;
        const double ri = std::sqrt(out[0]) / gnorm;
        if (!std::isfinite(ri) || out[1] > 0) return fail(SOCFV_DIVERGED, "adjoint diverged");
        if (ri < target) break;
        if (ri < 0.999 * best) { best = ri; stall = 0; }
        else if (++stall >= 8) break;
      }
      TRY(adj_refresh(cur, cur ^ 1, c->s32[cd]));
      cur ^= 1;
      ++S.cycles;
      rel = std::sqrt(out[0]) / gnorm;
      if (!std::isfinite(rel)) return fail(SOCFV_DIVERGED, "adjoint diverged");
    }
    if (rel < p->tol) status = SOCFV_OK;
  }
  // gradients
  const int gb = flags_blocks(c->g);
  TRY(ensure_partial(c, (long long)gb * NV + 64));
  launch_gradients(c->g, c->flags, faces64(c), c->s64[c->state_buf], psi[cur], p->s_in, p->s_eq,
                   p->Da, pinned, dU_dkappa, c->partial, gb, c->st);
  HIPCHK(hipGetLastError());
  double gsum[NV];
  TRY(reduce_to_host(c, gb, NV, 0u, gsum));
  if (dU_dlnq) *dU_dlnq = gsum[0];
  if (psi_out)
    HIPCHK(hipMemcpyAsync(psi_out, psi[cur], sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice,
                          c->st));
  TRY(leave(c, hip_stream));
  if (st) {
    socfv_stats s{};
    s.iterations = S.it; s.it_fp32 = S.it32; s.it_fp64 = S.it64; s.cycles = S.cycles;
    s.status = status; s.residual = rel; s.dt = S.dt; s.tau = S.tau; s.U = o.U;
    s.seconds = now_s() - t0;
    *st = s;
  }
  if (status == SOCFV_NOT_CONVERGED) fail(status, "adjoint not converged (relative residual %g)", rel);
  return status;
}

int socfv_solve_nernst(socfv_ctx *c, const socfv_params *p, double omega, double *s_out,
                       double *eta_out, socfv_stats *st, void *hip_stream) {
  const double t0 = now_s();
  if (!c) return fail(SOCFV_INVALID_ARG, "NULL context");
  TRY(check_params(p));
  if (!c->have_velocity) return fail(SOCFV_INVALID_ARG, "velocity not set");
  if (p->mode != SOCFV_FINITE_RATE)
    return fail(SOCFV_INVALID_ARG, "the Nernst model is for finite-rate kinetics");
  if (!(p->s_eq > 0.0 && p->s_eq < 1.0) || !(p->Da > 0.0))
    return fail(SOCFV_INVALID_ARG, "the Nernst model needs 0 < s_eq < 1 and Da > 0");
  if (!(omega > 0.0 && omega <= 1.0)) return fail(SOCFV_INVALID_ARG, "omega must be in (0, 1]");
  const long long n = c->g.n;
  double *eta = nullptr;
  const int rc = [&]() -> int {
    TRY(enter(c, hip_stream));
    // time step from the transport-only diagonal (the reaction is on the electrode's value)
    socfv_params pt = *p;
    pt.Da = 0.0;
    Solver S{c, &pt};
    TRY(S.setup());
    HIPCHK(hipMalloc(&eta, sizeof(double) * (size_t)n));
    launch_fill_f64(eta, n, 0.0, c->st);
    // s_in on pore cells, s_eq = sigma(V - 0) on electrode cells
    launch_init_state(c->g, c->flags, nullptr, p->s_in, p->s_eq, 1, c->s64[0], c->st);
    HIPCHK(hipGetLastError());
    NernstArgs a;
    a.g = c->g; a.flags = c->flags; a.w = faces64(c); a.kappa = c->kappa; a.eta = eta;
    a.s_in = p->s_in; a.dt = S.dt; a.Da = p->Da; a.omega = omega;
    a.V = std::log(p->s_eq / (1.0 - p->s_eq));
    a.K = 1.0 / std::sqrt(p->s_eq * (1.0 - p->s_eq));
    a.zc = S.t.zc;
    const int K = S.chunk_len();
    int cur = 0, status = SOCFV_NOT_CONVERGED;
    double res = INFINITY, out[NV];
    while (S.it < p->max_iter) {
      const long k = std::min<long>(K, p->max_iter - S.it);
      for (long j = 0; j < k; ++j) {
        a.s = c->s64[cur];
        a.s_new = c->s64[cur ^ 1];
        a.partial = j == k - 1 ? c->partial : nullptr;
        launch_nernst(a, S.t, c->st);
        cur ^= 1;
      }
      HIPCHK(hipGetLastError());
      TRY(reduce_to_host(c, (int)S.nblk, NV, 0u, out));
      S.it += k;
      S.it64 += k;
      res = S.res_of(out[0]);
      if (!std::isfinite(res) || out[1] > 0)
        return fail(SOCFV_DIVERGED, "Nernst iteration diverged at %ld (residual %g; omega %g may "
                    "be too large for these kinetics)", S.it, res, omega);
      if (res < p->tol) { status = SOCFV_OK; break; }
    }
    // the Nernst steady state is the finite-rate model's: keep it as the context's state
    c->have_state = true;
    c->state_buf = cur;
    c->last_p = *p;
    socfv_stats s{};
    TRY(eval_outputs(c, p, c->s64[cur], &s));
    if (s_out)
      HIPCHK(hipMemcpyAsync(s_out, c->s64[cur], sizeof(double) * (size_t)n,
                            hipMemcpyDeviceToDevice, c->st));
    if (eta_out)
      HIPCHK(hipMemcpyAsync(eta_out, eta, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice,
                            c->st));
    TRY(leave(c, hip_stream));
    s.iterations = S.it; s.it_fp64 = S.it64; s.status = status; s.residual = res;
    s.dt = S.dt; s.tau = S.tau; s.sweeps_fp64 = S.it64;
    s.seconds = now_s() - t0;
    if (st) *st = s;
    if (status == SOCFV_NOT_CONVERGED) fail(status, "Nernst iteration not converged (%g)", res);
    return status;
  }();
  hfree(eta);
  return rc;
}

int socfv_coarsen(socfv_ctx *c, uint8_t *solid_c, double *ux_c, double *uy_c, double *uz_c,
                  void *hip_stream) {
  if (!c) return fail(SOCFV_INVALID_ARG, "NULL context");
  if (!solid_c || !ux_c || !uy_c || !uz_c) return fail(SOCFV_INVALID_ARG, "NULL output buffer");
  if (!c->have_velocity) return fail(SOCFV_INVALID_ARG, "velocity not set");
  const Grid &g = c->g;
  if ((g.nx | g.ny | g.nz) & 1)
    return fail(SOCFV_INVALID_ARG, "coarsening needs even dimensions (%d %d %d)", g.nx, g.ny, g.nz);
  TRY(enter(c, hip_stream));
  launch_coarse_mask(g, c->flags, solid_c, c->st);
  launch_restrict(g, faces64(c), ux_c, uy_c, uz_c, c->st);
  HIPCHK(hipGetLastError());
  return leave(c, hip_stream);
}

int socfv_solve_soc_upsampled(socfv_ctx *c, const socfv_params *p, double *s_out,
                              socfv_stats *st, socfv_stats *coarse_st, void *hip_stream) {
  const double t0 = now_s();
  if (!c) return fail(SOCFV_INVALID_ARG, "NULL context");
  TRY(check_params(p));
  const Grid g = c->g;
  const int nxc = g.nx / 2, nyc = g.ny / 2, nzc = g.nz / 2;
  const size_t nc = (size_t)nxc * nyc * nzc;
  uint8_t *solid = nullptr;
  double *ux = nullptr, *uy = nullptr, *uz = nullptr, *sc = nullptr, *sf = nullptr;
  socfv_ctx *cc = nullptr;
  const int rc = [&]() -> int {
    HIPCHK(hipMalloc(&solid, nc));
    HIPCHK(hipMalloc(&ux, sizeof(double) * (size_t)nzc * nyc * (nxc + 1)));
    HIPCHK(hipMalloc(&uy, sizeof(double) * (size_t)nzc * (nyc + 1) * nxc));
    HIPCHK(hipMalloc(&uz, sizeof(double) * (size_t)(nzc + 1) * nyc * nxc));
    HIPCHK(hipMalloc(&sc, sizeof(double) * nc));
    HIPCHK(hipMalloc(&sf, sizeof(double) * (size_t)g.n));
    TRY(socfv_coarsen(c, solid, ux, uy, uz, hip_stream));
    TRY(socfv_setup_geometry(&cc, nxc, nyc, nzc, solid, hip_stream));
    TRY(socfv_set_velocity(cc, ux, uy, uz, 1.0, hip_stream));
    socfv_params pc = *p;
    pc.Da = 2.0 * p->Da;
    socfv_stats cs{};
    // a coarse solve that stops at max_iter still gives a starting state
    TRY(socfv_solve_soc_steady(cc, &pc, nullptr, sc, &cs, hip_stream));
    if (coarse_st) *coarse_st = cs;
    TRY(enter(c, hip_stream));
    launch_prolong(g, c->flags, sc, sf, c->st);
    HIPCHK(hipGetLastError());
    TRY(leave(c, hip_stream));
    const int r = socfv_solve_soc_steady(c, p, sf, s_out, st, hip_stream);
    if (st) st->seconds = now_s() - t0;
    return r;
  }();
  if (cc) socfv_destroy(cc);
  hfree(solid); hfree(ux); hfree(uy); hfree(uz); hfree(sc); hfree(sf);
  return rc;
}

int socfv_set_tiles(socfv_ctx *c, int tile_y, int z_chunk, int z_chunk2, int two_sweeps) {
  if (!c) return fail(SOCFV_INVALID_ARG, "NULL context");
  if (tile_y != 0) {
    if (tile_y < 1 || tile_y > 16 || (tile_y & (tile_y - 1)))
      return fail(SOCFV_INVALID_ARG, "tile_y must be a power of two in [1, 16]");
    Tiles t = auto_tiles(c->g, tile_y, c->ncu);
    c->tiles.ty = tile_y;
    if (z_chunk == 0) c->tiles.zc = t.zc;
  }
  if (z_chunk != 0) {
    if (z_chunk < 1 || z_chunk > 4096) return fail(SOCFV_INVALID_ARG, "z_chunk must be in [1, 4096]");
    c->tiles.zc = z_chunk;
  }
  if (z_chunk2 != 0) {
    if (z_chunk2 < 1 || z_chunk2 > 4096)
      return fail(SOCFV_INVALID_ARG, "z_chunk2 must be in [1, 4096]");
    c->tiles.zc2 = z_chunk2;
  }
  if (two_sweeps > 3) return fail(SOCFV_INVALID_ARG, "two_sweeps must be -1, 0, 1, 2 or 3");
  if (two_sweeps >= 0) {
    c->tiles.two = two_sweeps ? 1 : 0;
    const int rx = two_sweeps == 2 ? 64 : two_sweeps == 3 ? 32
                                                           : pick_rx(c->g.nx, c->g.ny, two_w(c->g));
    if (two_sweeps > 0 && rx != c->tiles.rx) {
      c->tiles.rx = rx;
      if (z_chunk2 == 0) c->tiles.zc2 = pick_zc2(c->g, c->ncu, rx);
    }
  }
  c->tiles_fixed = true;
  return ensure_partial(c, partial_need(c->g, c->tiles));
}

int socfv_autotune(socfv_ctx *c, int sweeps, int best[3], void *hip_stream) {
  if (!c) return fail(SOCFV_INVALID_ARG, "NULL context");
  if (!c->have_velocity) return fail(SOCFV_INVALID_ARG, "velocity not set");
  if (sweeps < 2) sweeps = 2;
  TRY(ensure_state(c));
  TRY(enter(c, hip_stream));
  socfv_params p;
  socfv_default_params(&p);
  Solver S{c, &p};
  TRY(S.setup());
  const long long n = c->g.n;
  launch_init_state(c->g, c->flags, nullptr, p.s_in, p.s_eq, 0, c->s64[0], c->st);
  launch_f64_to_f32(c->s64[0], c->s32[0], n, c->st);
  launch_fill_f32(c->s32[1], n, 0.0f, c->st);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int tys[] = {1, 2, 4, 8, 16};
  const int zcs[] = {1, 2, 4, 8, 16, 32, 64};
  float best_ms = 1e30f;
  Tiles best_t = c->tiles;
  for (int ty : tys) {
    for (int zc : zcs) {
      if (zc > c->g.nz) continue;
      Tiles t{ty, zc, c->tiles.zc2, c->tiles.two};
      t.rx = c->tiles.rx;
      S.t = t;
      S.nblk = sweep_blocks(c->g, t);
      int cur = 0;
      // warm-up
      for (int j = 0; j < 2; ++j) {
        SweepArgs<float> a = S.sweep_args<float>(c->s32[cur], c->s32[cur ^ 1], false, nullptr);
        a.w = faces32(c);
        launch_sweep<float>(a, t, c->st);
        cur ^= 1;
      }
      HIPCHK(hipEventRecord(e0, c->st));
      for (int j = 0; j < sweeps; ++j) {
        SweepArgs<float> a = S.sweep_args<float>(c->s32[cur], c->s32[cur ^ 1], false, nullptr);
        a.w = faces32(c);
        launch_sweep<float>(a, t, c->st);
        cur ^= 1;
      }
      HIPCHK(hipEventRecord(e1, c->st));
      HIPCHK(hipEventSynchronize(e1));
      HIPCHK(hipGetLastError());
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) { best_ms = ms; best_t = t; }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // two-sweep kernel: z chunk
  float best2 = 1e30f;
  int best_zc2 = c->tiles.zc2;
  if (two_path(c->g)) {
    const int zc2s[] = {pick_zc2(c->g, c->ncu, c->tiles.rx), 8, 16, 32, 64, 128};
    for (int zc2 : zc2s) {
      if (zc2 > c->g.nz && zc2 != 8) continue;
      Tiles t = best_t;
      t.zc2 = zc2;
      int cur = 0;
      SweepArgs<float> a = S.sweep_args<float>(c->s32[cur], c->s32[cur ^ 1], false, nullptr);
      a.w = faces32(c);
      launch_sweep2(a, t, c->st);
      HIPCHK(hipEventRecord(e0, c->st));
      for (int j = 0; j < sweeps; j += 2) {
        SweepArgs<float> b = S.sweep_args<float>(c->s32[cur], c->s32[cur ^ 1], false, nullptr);
        b.w = faces32(c);
        launch_sweep2(b, t, c->st);
        cur ^= 1;
      }
      HIPCHK(hipEventRecord(e1, c->st));
      HIPCHK(hipEventSynchronize(e1));
      HIPCHK(hipGetLastError());
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best2) { best2 = ms; best_zc2 = zc2; }
    }
  }
  best_t.zc2 = best_zc2;
  best_t.two = c->tiles.two;
  c->tiles = best_t;
  c->tiles_fixed = true;
  TRY(ensure_partial(c, partial_need(c->g, c->tiles)));
  TRY(leave(c, hip_stream));
  if (best) { best[0] = best_t.ty; best[1] = best_t.zc; best[2] = best_t.zc2; }
  return SOCFV_OK;
}

int socfv_info(const socfv_ctx *c, int dims[3], long counts[3]) {
  if (!c) return fail(SOCFV_INVALID_ARG, "NULL context");
  if (dims) { dims[0] = c->g.nx; dims[1] = c->g.ny; dims[2] = c->g.nz; }
  if (counts) { counts[0] = c->npore; counts[1] = c->nreact; counts[2] = 0; }
  return SOCFV_OK;
}

int socfv_batch_solve(int n, socfv_ctx *const *ctxs, const socfv_params *p,
                      double *const *s_out, socfv_stats *st, void *hip_stream) {
  const double t0 = now_s();
  if (n < 0 || (n > 0 && (!ctxs || !p))) return fail(SOCFV_INVALID_ARG, "bad batch arguments");
  if (n == 0) return SOCFV_OK;
  bool batched = true;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return fail(SOCFV_INVALID_ARG, "context %d is NULL", i);
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(SOCFV_INVALID_ARG, "context %d repeated", i);
    TRY(check_params(&p[i]));
    if (!ctxs[i]->have_velocity) return fail(SOCFV_INVALID_ARG, "context %d: velocity not set", i);
    if (p[i].precision != SOCFV_FP32) batched = false;
  }
  if (!batched) {
    // FP64 / plain-FP32 problems: one solve after another
    int worst = SOCFV_OK;
    for (int i = 0; i < n; ++i) {
      socfv_stats s{};
      int r = socfv_solve_soc_steady(ctxs[i], &p[i], nullptr, s_out ? s_out[i] : nullptr, &s,
                                     hip_stream);
      if (st) st[i] = s;
      if (r < 0) return r;
      if (r > worst) worst = r;
    }
    return worst;
  }
  // One library stream for the whole batch (graph capture needs a non-default stream);
  // the contexts' own streams are swapped for it during the call.
  hipStream_t bs = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&bs, hipStreamNonBlocking));
  std::vector<hipStream_t> saved(n);
  for (int i = 0; i < n; ++i) { saved[i] = ctxs[i]->st; ctxs[i]->st = bs; }
  BatchProb *d_probs = nullptr;
  int *d_tiles = nullptr, *d_work = nullptr, *d_nwork = nullptr, *d_grab = nullptr,
      *h_work = nullptr;
  double *d_part = nullptr, *d_out = nullptr, *h_out = nullptr;
  BatchM64 *d_m = nullptr;               // batched FP64 polish: problem table, items, partials
  int *d_mitem = nullptr;
  double *d_mpart = nullptr;
  SolveCtl *d_ctl = nullptr, *h_ctl = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto cleanup = [&]() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamSynchronize(bs);
    hfree(d_probs); hfree(d_tiles); hfree(d_work); hfree(d_nwork); hfree(d_grab);
    hfree(d_part); hfree(d_out); hfree(d_ctl); hfree(d_m); hfree(d_mitem); hfree(d_mpart);
    if (h_work) (void)hipHostFree(h_work);
    if (h_out) (void)hipHostFree(h_out);
    if (h_ctl) (void)hipHostFree(h_ctl);
    for (int i = 0; i < n; ++i) ctxs[i]->st = saved[i];
    (void)hipStreamDestroy(bs);
  };
  int rc = [&]() -> int {
    TRY(enter(ctxs[0], hip_stream));
    std::vector<Solver> S;
    S.reserve(n);
    std::vector<double> res(n), target(n);
    std::vector<int> cur(n, 1), status(n, SOCFV_NOT_CONVERGED), done(n, 0);
    std::vector<double> out(NV);
    for (int i = 0; i < n; ++i) {
      S.push_back(Solver{ctxs[i], &p[i]});
      TRY(S[i].setup());
      socfv_ctx *c = ctxs[i];
      launch_init_state(c->g, c->flags, nullptr, p[i].s_in, p[i].s_eq, S[i].pinned, c->s64[0], bs);
      HIPCHK(hipGetLastError());
      TRY(S[i].refresh(0, 1, nullptr, out.data()));
      res[i] = S[i].res_of(out[0]);
      TRY(S[i].check(out.data(), res[i]));
      target[i] = std::fmax(p[i].tol, CYCLE_REDUCTION * res[i]);
      launch_fill_f32(c->s32[0], c->g.n, 0.0f, bs);
      launch_fill_f32(c->s32[1], c->g.n, 0.0f, bs);
      if (res[i] < p[i].tol) { done[i] = 1; status[i] = SOCFV_OK; }
    }
    // Problems whose shape allows it (nx even; no activity field in the batch) take two
    // sweeps per launch in the batched two-sweep kernel; the others take the batched
    // single-sweep kernel.  Its block shape is picked by timing a few sweeps per candidate;
    // the two-sweep z chunk comes from the same rounds x planes cost model as one problem's.
    bool any_kappa = false;
    for (int i = 0; i < n; ++i) any_kappa = any_kappa || ctxs[i]->kappa != nullptr;
    std::vector<int> two(n, 0), tw(n, 1), trx(n, 64);
    int n_two = 0;
    for (int i = 0; i < n; ++i) {
      two[i] = !any_kappa && two_path(ctxs[i]->g) && ctxs[i]->tiles.two;
      n_two += two[i];
      // item shape: two cells per lane for even nx (one for odd), and the row-segment width
      // with the lower cost of the lanes it computes per plane (one problem's rule)
      const Grid &g = ctxs[i]->g;
      tw[i] = two_w(g);
      trx[i] = pick_rx(g.nx, g.ny, tw[i]);
    }
    HIPCHK(hipMalloc(&d_ctl, sizeof(SolveCtl) * n));
    HIPCHK(hipHostMalloc(&h_ctl, sizeof(SolveCtl) * n, hipHostMallocDefault));
    int dev = 0, ncu = 256;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    // z chunk of the two-sweep items for the problems still running (act): the rounds x
    // planes cost model over their items; re-picked whenever a problem finishes, so that the
    // last problems of a batch still spread over the chip
    auto pick_zc2 = [&](const std::vector<int> &act) {
      long long best_cost = -1;
      int zbest = 8, zmax = 8;
      for (int i = 0; i < n; ++i)
        if (two[i] && act[i]) zmax = std::max(zmax, ctxs[i]->g.nz);
      for (int z = 8; z <= zmax; ++z) {
        long long items = 0;
        for (int i = 0; i < n; ++i) {
          if (!two[i] || !act[i]) continue;
          const Grid &g = ctxs[i]->g;
          const int zz = std::min(z, g.nz);
          int gx, gy;
          tile2_xy(g.nx, g.ny, tw[i], trx[i], gx, gy);
          items += (long long)gx * gy * ((g.nz + zz - 1) / zz);
        }
        const long long cost = (items + ncu - 1) / ncu * (z + 2);
        if (best_cost < 0 || cost < best_cost) { best_cost = cost; zbest = z; }
      }
      return zbest;
    };
    int zc2 = pick_zc2(std::vector<int>(n, 1));
    auto build = [&](int ty, int zc, std::vector<BatchProb> &hp, std::vector<int> &tp) {
      hp.assign(n, BatchProb{});
      tp.clear();
      for (int i = 0; i < n; ++i) {
        socfv_ctx *c = ctxs[i];
        BatchProb &b = hp[i];
        b.nx = c->g.nx; b.ny = c->g.ny; b.nz = c->g.nz;
        b.flags = c->flags;
        b.wx = c->w32[0]; b.wy = c->w32[1]; b.wz = c->w32[2]; b.wxo = c->w32[3];
        b.kappa = c->kappa;
        b.s0 = c->s32[0]; b.s1 = c->s32[1];
        b.r0 = c->r0;
        b.dt = (float)S[i].dt; b.Da = (float)p[i].Da; b.s_in = (float)p[i].s_in;
        b.s_eq = (float)p[i].s_eq; b.lo = S[i].lo; b.hi = S[i].hi; b.pinned = S[i].pinned;
        b.w = tw[i];
        b.rx = trx[i];
        b.two = two[i];
        b.ctl = d_ctl + i;
        b.rpart = c->partial;
        b.rnblk = march64_blocks(c->g);
        if (two[i]) {
          tile2_xy(c->g.nx, c->g.ny, tw[i], trx[i], b.gx, b.gy);
          b.zc = std::min(zc2, c->g.nz);
        } else {
          b.gx = (c->g.nx + 63) / 64; b.gy = (c->g.ny + ty - 1) / ty;
          b.zc = std::min(zc, c->g.nz);
        }
        b.gz = (c->g.nz + b.zc - 1) / b.zc;
        b.tile0 = (int)tp.size();
        for (int t = 0; t < b.gx * b.gy * b.gz; ++t) tp.push_back(i);
      }
    };
    std::vector<BatchProb> hp;
    std::vector<int> tp;
    size_t max_tiles = 0;
    const int tys[] = {2, 4, 8};
    const int zcs[] = {2, 4, 8, 16};
    {
      // buffers for every tiling used below: any candidate shape, two-sweep chunks down to 8
      const int zc2_run = zc2;
      for (int z2 : {8, zc2_run})
        for (int ty : tys)
          for (int zc : zcs) {
            zc2 = z2;
            build(ty, zc, hp, tp);
            max_tiles = std::max(max_tiles, tp.size());
          }
      zc2 = zc2_run;
    }
    HIPCHK(hipMalloc(&d_probs, sizeof(BatchProb) * n));
    HIPCHK(hipMalloc(&d_tiles, sizeof(int) * max_tiles));
    // work lists: two-sweep items at d_work, single-sweep items at d_work + max_tiles;
    // their counts at d_nwork[0] and d_nwork[1]
    HIPCHK(hipMalloc(&d_work, sizeof(int) * 2 * max_tiles));
    HIPCHK(hipMalloc(&d_nwork, sizeof(int) * 2));
    // item counter of the two-sweep launches (zeroed once by a copy; each launch leaves it
    // at zero)
    HIPCHK(hipMalloc(&d_grab, sizeof(int) * 2));
    {
      static const int zero2[2] = {0, 0};
      HIPCHK(hipMemcpy(d_grab, zero2, sizeof(int) * 2, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMalloc(&d_part, sizeof(double) * NV * max_tiles));
    HIPCHK(hipMalloc(&d_out, sizeof(double) * NV * n));
    HIPCHK(hipHostMalloc(&h_work, sizeof(int) * (2 * max_tiles + 2), hipHostMallocDefault));
    HIPCHK(hipHostMalloc(&h_out, sizeof(double) * NV * n, hipHostMallocDefault));
    // work lists = every tile of the unfinished problems, by path (counts at h_work[0..1])
    auto upload_work = [&](const std::vector<BatchProb> &hp_, const std::vector<int> &done_) -> int {
      int m[2] = {0, 0};
      int *lst[2] = {h_work + 2, h_work + 2 + max_tiles};
      for (int i = 0; i < n; ++i) {
        if (done_[i]) continue;
        const int k = two[i] ? 0 : 1;
        const int nt = hp_[i].gx * hp_[i].gy * hp_[i].gz;
        for (int t = 0; t < nt; ++t) lst[k][m[k]++] = hp_[i].tile0 + t;
      }
      h_work[0] = m[0];
      h_work[1] = m[1];
      HIPCHK(hipMemcpyAsync(d_nwork, h_work, sizeof(int) * 2, hipMemcpyHostToDevice, bs));
      for (int k = 0; k < 2; ++k)
        if (m[k])
          HIPCHK(hipMemcpyAsync(d_work + k * max_tiles, lst[k], sizeof(int) * m[k],
                                hipMemcpyHostToDevice, bs));
      HIPCHK(hipStreamSynchronize(bs));   // h_work is rewritten by the next upload
      return 0;
    };
    int n_one_tiles = 0, n_two_tiles = 0;
    auto count_tiles = [&](const std::vector<BatchProb> &hp_) {
      n_one_tiles = n_two_tiles = 0;
      for (int i = 0; i < n; ++i) (two[i] ? n_two_tiles : n_one_tiles) += hp_[i].gx * hp_[i].gy * hp_[i].gz;
    };
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best_ms = 1e30f;
    int bty = 4, bzc = 8;
    auto nblocks_for = [&](int ty, size_t ntiles) {
      // persistent grid: the blocks that fit the chip at once, never more than the tiles
      long long per_cu = std::max(1, 2048 / (64 * ty));
      long long nb = std::min<long long>((long long)ncu * per_cu, (long long)ntiles);
      return (int)std::max<long long>(nb, 1);
    };
    for (int ty : tys)
      for (int zc : zcs) {
        if (n_two == n) break;   // no single-sweep problems to time
        build(ty, zc, hp, tp);
        count_tiles(hp);
        HIPCHK(hipMemcpyAsync(d_probs, hp.data(), sizeof(BatchProb) * n, hipMemcpyHostToDevice, bs));
        HIPCHK(hipMemcpyAsync(d_tiles, tp.data(), sizeof(int) * tp.size(), hipMemcpyHostToDevice, bs));
        std::vector<int> none(n, 0);
        TRY(upload_work(hp, none));
        const int nb = nblocks_for(ty, n_one_tiles);
        // timing sweeps change the correction buffers: they are cleared again below
        launch_batch_sweep(d_probs, d_tiles, d_work + max_tiles, d_nwork + 1, nb, ty, 0, true,
                           nullptr, bs);
        HIPCHK(hipEventRecord(e0, bs));
        for (int j = 0; j < 4; ++j)
          launch_batch_sweep(d_probs, d_tiles, d_work + max_tiles, d_nwork + 1, nb, ty, j & 1,
                             true, nullptr, bs);
        HIPCHK(hipEventRecord(e1, bs));
        HIPCHK(hipEventSynchronize(e1));
        HIPCHK(hipGetLastError());
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) { best_ms = ms; bty = ty; bzc = zc; }
      }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    build(bty, bzc, hp, tp);
    count_tiles(hp);
    const int ntiles = (int)tp.size();
    const int nb = nblocks_for(bty, std::max(n_one_tiles, 1));
    const int nb2 = ncu;        // persistent two-sweep blocks (items may grow on re-tiling)
    HIPCHK(hipMemcpyAsync(d_probs, hp.data(), sizeof(BatchProb) * n, hipMemcpyHostToDevice, bs));
    HIPCHK(hipMemcpyAsync(d_tiles, tp.data(), sizeof(int) * ntiles, hipMemcpyHostToDevice, bs));
    TRY(upload_work(hp, done));
    for (int i = 0; i < n; ++i) {
      launch_fill_f32(ctxs[i]->s32[0], ctxs[i]->g.n, 0.0f, bs);
      launch_fill_f32(ctxs[i]->s32[1], ctxs[i]->g.n, 0.0f, bs);
    }
    // Each problem's loop runs on the device (SolveCtl, as one problem's solve): one chunk of
    // K sweeps, K a multiple of 4, is captured as a graph: the work lists of the problems
    // still sweeping, their corrections zeroed where a cycle starts, the sweeps (per pair of
    // sweeps one two-sweep launch, whose buffers flip once, and two single-sweep launches,
    // whose buffers flip twice, so after K sweeps every correction is back in s32[0]; partials
    // on the last launches), per-problem sums, each problem's decision, the refreshes asked
    // for (one gated launch per problem), and each refreshed problem's stop rule.  The host
    // replays the graph a few times between reads of the states, and re-tiles the remaining
    // problems when some have finished.
    int K = 4;
    for (int i = 0; i < n; ++i) K = std::max(K, S[i].chunk_len());
    K = (K + 3) / 4 * 4;
    for (int i = 0; i < n; ++i) {
      SolveCtl &h = h_ctl[i];
      h = SolveCtl{};
      h.state = done[i] ? CTL_DONE : CTL_RUN;
      h.fill = 0;                        // zeroed above
      h.cur = cur[i];
      h.max_iter = p[i].max_iter;
      h.tol = p[i].tol;
      h.tau = S[i].tau;
      h.npore = (double)ctxs[i]->npore;
      h.reduction = CYCLE_REDUCTION;
      h.target = target[i];
      h.best = INFINITY;
      h.res = res[i];
      h.ri = INFINITY;
    }
    HIPCHK(hipMemcpyAsync(d_ctl, h_ctl, sizeof(SolveCtl) * n, hipMemcpyHostToDevice, bs));
    HIPCHK(hipStreamSynchronize(bs));
    HIPCHK(hipStreamBeginCapture(bs, hipStreamCaptureModeThreadLocal));
    launch_batch_control(d_probs, n, d_work, (int)max_tiles, d_nwork, BATCH_WORKLIST, nullptr, 0,
                         bs);
    launch_batch_control(d_probs, n, d_work, (int)max_tiles, d_nwork, BATCH_FILL, nullptr, 0, bs);
    for (int j = 0; j < K / 2; ++j) {
      const bool lastp = j == K / 2 - 1;
      if (n_two_tiles)
        launch_batch_sweep2(d_probs, d_tiles, d_work, d_nwork, d_grab, nb2, j & 1,
                            lastp ? d_part : nullptr, bs);
      if (n_one_tiles) {
        launch_batch_sweep(d_probs, d_tiles, d_work + max_tiles, d_nwork + 1, nb, bty, 0, true,
                           nullptr, bs);
        launch_batch_sweep(d_probs, d_tiles, d_work + max_tiles, d_nwork + 1, nb, bty, 1, true,
                           lastp ? d_part : nullptr, bs);
      }
    }
    launch_batch_reduce(d_probs, n, d_part, d_out, bs);
    launch_batch_control(d_probs, n, d_work, (int)max_tiles, d_nwork, BATCH_CHUNK, d_out, K, bs);
    for (int i = 0; i < n; ++i) {
      socfv_ctx *c = ctxs[i];
      RefreshArgs a;
      a.g = c->g; a.flags = c->flags; a.w = faces64(c); a.kappa = c->kappa;
      a.s64 = nullptr; a.delta = c->s32[0]; a.s64_new = nullptr; a.r0 = c->r0;
      a.s_in = p[i].s_in; a.s_eq = p[i].s_eq; a.Da = p[i].Da; a.pinned = S[i].pinned;
      a.lo = S[i].lo; a.hi = S[i].hi; a.partial = c->partial; a.zc = S[i].t.zc;
      launch_refresh_gated(a, c->s64[0], c->s64[1], d_ctl + i, bs);
    }
    launch_batch_control(d_probs, n, d_work, (int)max_tiles, d_nwork, BATCH_REFRESH, nullptr, 0,
                         bs);
    HIPCHK(hipStreamEndCapture(bs, &graph));
    HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    int planned = 0;                     // problems sweeping at the last tiling
    for (int i = 0; i < n; ++i) planned += !done[i];
    int nact = planned;
    for (;;) {
      // chunks between reads of the states: four while many problems sweep, one near the
      // end (a launch after the last stop still dispatches its blocks, and the tail gains
      // from re-tiling soon after each finish)
      const int replays = nact > 4 ? 4 : 1;
      for (int g = 0; g < replays; ++g) HIPCHK(hipGraphLaunch(exec, bs));
      HIPCHK(hipMemcpyAsync(h_ctl, d_ctl, sizeof(SolveCtl) * n, hipMemcpyDeviceToHost, bs));
      HIPCHK(hipStreamSynchronize(bs));
      std::vector<int> act(n, 0);
      nact = 0;
      for (int i = 0; i < n; ++i) {
        if (h_ctl[i].state == CTL_DIVERGED)
          return fail(SOCFV_DIVERGED, "batch problem %d diverged at sweep %lld", i, h_ctl[i].it);
        act[i] = h_ctl[i].state == CTL_RUN;
        nact += act[i];
      }
      if (!nact) break;
      if (nact < planned) {
        // fewer problems left: shorter chunks for more items; single-sweep chunks halved
        // while their items are fewer than the persistent blocks (the next chunk's work
        // lists come from the new table)
        zc2 = pick_zc2(act);
        auto tiles1 = [&](int zc) {
          long long m = 0;
          for (int i = 0; i < n; ++i)
            if (act[i] && !two[i])
              m += (long long)((ctxs[i]->g.nx + 63) / 64) * ((ctxs[i]->g.ny + bty - 1) / bty) *
                   ((ctxs[i]->g.nz + std::min(zc, ctxs[i]->g.nz) - 1) / std::min(zc, ctxs[i]->g.nz));
          return m;
        };
        while (bzc > 2 && tiles1(bzc) < nb) bzc /= 2;
        build(bty, bzc, hp, tp);
        HIPCHK(hipMemcpyAsync(d_probs, hp.data(), sizeof(BatchProb) * n, hipMemcpyHostToDevice, bs));
        HIPCHK(hipMemcpyAsync(d_tiles, tp.data(), sizeof(int) * tp.size(), hipMemcpyHostToDevice, bs));
        planned = nact;
      }
    }
    for (int i = 0; i < n; ++i) {
      const SolveCtl &h = h_ctl[i];
      S[i].it += h.it;
      S[i].it32 += h.it;
      S[i].cycles += h.cycles;
      S[i].it64 += h.cycles;
      cur[i] = h.cur;
      res[i] = h.res;
      status[i] = h.state == CTL_DONE ? SOCFV_OK : SOCFV_NOT_CONVERGED;
    }
    // FP64 polish.  The first chunk of every converged problem's polish runs as batched FP64
    // sweeps: one launch per sweep over all of them (one problem at a time, their small
    // launches leave most of the chip idle and each costs a host launch).  Partials come from
    // the launches where some problem ends its chunk; each problem's sums are overwritten up
    // to its own last sweep.  A problem whose residual is still above tol after the chunk and
    // whose polish budget is longer continues alone, as the one-problem solve does.
    std::vector<long> npol(n, 0), nk(n, 0);
    long kmax = 0, items_max = 0;
    for (int i = 0; i < n; ++i) {
      long np = p[i].polish_iters > 0 ? p[i].polish_iters : S[i].chunk_len();
      np += np & 1;
      np = std::min<long>(np, p[i].max_iter - S[i].it);
      npol[i] = status[i] == SOCFV_OK && np > 0 ? np : 0;
      nk[i] = std::min<long>(npol[i], S[i].chunk_len());
      kmax = std::max(kmax, nk[i]);
      if (nk[i]) items_max += march64_blocks(ctxs[i]->g);
    }
    if (kmax > 0) {
      HIPCHK(hipMalloc(&d_m, sizeof(BatchM64) * n));
      HIPCHK(hipMalloc(&d_mitem, sizeof(int) * items_max));
      HIPCHK(hipMalloc(&d_mpart, sizeof(double) * NV * items_max));
      std::vector<BatchM64> hm;
      std::vector<int> hitem;
      // the problems still polishing at sweep j
      auto build_m = [&](long j) -> int {
        hm.clear();
        hitem.clear();
        for (int i = 0; i < n; ++i) {
          if (nk[i] <= j) continue;
          socfv_ctx *c = ctxs[i];
          BatchM64 b{};
          b.a = S[i].sweep_args<double>(nullptr, nullptr, false, nullptr);
          b.a.w = faces64(c);
          b.pair[0] = c->s64[0];
          b.pair[1] = c->s64[1];
          b.c0 = cur[i];
          march64_shape(c->g, b.gx, b.gy, b.gz, b.zc);
          b.blk0 = (int)hitem.size();
          b.prob = i;
          const int nb = b.gx * b.gy * b.gz;
          for (int t = 0; t < nb; ++t) hitem.push_back((int)hm.size());
          hm.push_back(b);
        }
        HIPCHK(hipStreamSynchronize(bs));   // the previous tables' launches are done
        HIPCHK(hipMemcpyAsync(d_m, hm.data(), sizeof(BatchM64) * hm.size(),
                              hipMemcpyHostToDevice, bs));
        HIPCHK(hipMemcpyAsync(d_mitem, hitem.data(), sizeof(int) * hitem.size(),
                              hipMemcpyHostToDevice, bs));
        HIPCHK(hipStreamSynchronize(bs));
        return 0;
      };
      TRY(build_m(0));
      std::vector<char> ends(kmax, 0);
      for (int i = 0; i < n; ++i)
        if (nk[i]) ends[nk[i] - 1] = 1;
      HIPCHK(hipEventRecord(ctxs[0]->t0, bs));
      for (long j = 0; j < kmax; ++j) {
        if (j > 0 && ends[j - 1]) TRY(build_m(j));
        launch_batch_march64(d_m, (int)hm.size(), d_mitem, (int)hitem.size(), (int)(j & 1),
                             ends[j] ? d_mpart : nullptr, d_out, bs);
      }
      HIPCHK(hipEventRecord(ctxs[0]->t1, bs));
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(h_out, d_out, sizeof(double) * NV * n, hipMemcpyDeviceToHost, bs));
      HIPCHK(hipStreamSynchronize(bs));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, ctxs[0]->t0, ctxs[0]->t1));
      for (int i = 0; i < n; ++i) {
        if (!nk[i]) continue;
        const double *out = h_out + (size_t)NV * i;
        S[i].it += nk[i];
        S[i].it64 += nk[i];
        S[i].sw64 += nk[i];
        S[i].ms64 += ms;             // the batched polish, shared by every problem in it
        cur[i] ^= (int)(nk[i] & 1);
        res[i] = S[i].res_of(out[0]);
        TRY(S[i].check(out, res[i]));
      }
    }
    // outputs and states per problem
    for (int i = 0; i < n; ++i) {
      socfv_ctx *c = ctxs[i];
      double pres = res[i];
      int pc = cur[i];
      if (nk[i] && pres >= p[i].tol && npol[i] > nk[i])
        (void)S[i].run_fp64(pc, pres, npol[i] - nk[i]);
      cur[i] = pc;
      res[i] = pres;
      status[i] = pres < p[i].tol ? SOCFV_OK : SOCFV_NOT_CONVERGED;
      c->have_state = true;
      c->state_buf = pc;
      c->last_p = p[i];
      socfv_stats s{};
      TRY(eval_outputs(c, &p[i], c->s64[pc], &s));
      if (s_out && s_out[i])
        HIPCHK(hipMemcpyAsync(s_out[i], c->s64[pc], sizeof(double) * (size_t)c->g.n,
                              hipMemcpyDeviceToDevice, bs));
      s.iterations = S[i].it; s.it_fp32 = S[i].it32; s.it_fp64 = S[i].it64;
      s.cycles = S[i].cycles; s.status = status[i]; s.dt = S[i].dt; s.tau = S[i].tau;
      s.ms_fp64 = S[i].ms64; s.ms_refresh = S[i].msref; s.sweeps_fp64 = S[i].sw64;
      s.tile_y = bty; s.z_chunk = bzc;
      if (st) st[i] = s;
    }
    TRY(leave(ctxs[0], hip_stream));
    const double el = now_s() - t0;
    int worst = SOCFV_OK;
    for (int i = 0; i < n; ++i) {
      if (st) st[i].seconds = el;
      worst = std::max(worst, status[i]);
    }
    if (worst == SOCFV_NOT_CONVERGED) fail(worst, "some batch problems did not converge");
    return worst;
  }();
  cleanup();
  return rc;
}

void socfv_default_flow_params(socfv_flow_params *p) {
  if (!p) return;
  p->p_in = 1.0;
  p->cfl = 0.5;
  p->tol = 1e-9;
  p->cg_theta = 0.1;
  p->max_steps = 10000000L;
  p->check_every = 50;
  p->cg_max = 256;
  p->resume = 0;
}

int socfv_solve_stokes(socfv_ctx *c, const socfv_flow_params *p, double *ux, double *uy,
                       double *uz, double *p_out, socfv_flow_stats *st, void *hip_stream) {
  const double t0 = now_s();
  if (!c) return fail(SOCFV_INVALID_ARG, "NULL context");
  if (!p) return fail(SOCFV_INVALID_ARG, "params is NULL");
  if (!ux || !uy || !uz) return fail(SOCFV_INVALID_ARG, "NULL velocity buffer");
  if (!(p->cfl > 0.0 && p->cfl < 4.0))
    return fail(SOCFV_INVALID_ARG, "cfl must be in (0, 4) (explicit diffusion stability)");
  if (!(p->tol >= 0.0) || !(p->cg_theta > 0.0) || !std::isfinite(p->p_in))
    return fail(SOCFV_INVALID_ARG, "tol >= 0, cg_theta > 0 and a finite p_in are required");
  if (p->max_steps < 1 || p->check_every < 1 || p->cg_max < 1)
    return fail(SOCFV_INVALID_ARG, "max_steps, check_every and cg_max must be >= 1");
  const Grid &g = c->g;
  const long long n = g.n;
  // the flow kernels decompose face and cell indices in 32 bits
  if ((long long)(g.nx + 1) * (g.ny + 1) * (g.nz + 1) >= (1ll << 32))
    return fail(SOCFV_INVALID_ARG, "grid too large for the flow step (2^32 faces)");
  const long long nf[3] = {(long long)(g.nx + 1) * g.ny * g.nz,
                           (long long)g.nx * (g.ny + 1) * g.nz,
                           (long long)g.nx * g.ny * (g.nz + 1)};
  FlowArgs a{};
  a.g = g;
  a.flags = c->flags;
  a.u[0] = ux; a.u[1] = uy; a.u[2] = uz;
  a.nbc = flow_cell_blocks(g);
  a.nbf = flow_face_blocks(g);
  // Eq. (time-step-flow) with C_V = 2 mu / rho * 3 / h^2 = 6 and no advective or force term
  a.dt = 0.5 * p->cfl / (2.0 * 6.0);
  a.p_in = p->p_in;
  a.theta2 = p->cg_theta * p->cg_theta;
  std::vector<void *> mem;
  auto alloc = [&](void **ptr, size_t bytes) -> int {
    HIPCHK(hipMalloc(ptr, bytes));
    mem.push_back(*ptr);
    return 0;
  };
  const int rc = [&]() -> int {
    for (int k = 0; k < 3; ++k) {
      TRY(alloc((void **)&a.code[k], sizeof(uint16_t) * (size_t)nf[k]));
      TRY(alloc((void **)&a.us[k], sizeof(double) * (size_t)nf[k]));
    }
    double **cellv[6] = {&a.p, &a.r, &a.z, &a.q, &a.d[0], &a.d[1]};
    for (double **v : cellv) TRY(alloc((void **)v, sizeof(double) * (size_t)n));
    TRY(alloc((void **)&a.ccode, (size_t)n));
    const long long npart = 6ll * a.nbc + 6ll * a.nbf + 4ll * a.nbc + FS_N;
    double *part = nullptr;
    TRY(alloc((void **)&part, sizeof(double) * (size_t)npart));
    a.prz[0] = part;
    a.prz[1] = part + a.nbc;
    a.prr[0] = part + 2ll * a.nbc;
    a.prr[1] = part + 3ll * a.nbc;
    a.pdq = part + 4ll * a.nbc;
    a.pdu = part + 5ll * a.nbc;
    a.pdiv = a.pdu + 6ll * a.nbf;
    a.pfl = a.pdiv + 4ll * a.nbc;
    a.sc = a.pfl + a.nbc;
    TRY(enter(c, hip_stream));
    // start from rest with zero pressure, or resume from the caller's velocity and pressure;
    // zero partials make the first step's CG run to its cap
    if (!p->resume)
      for (int k = 0; k < 3; ++k) launch_fill_f64(a.u[k], nf[k], 0.0, c->st);
    for (double **v : cellv) launch_fill_f64(*v, n, 0.0, c->st);
    if (p->resume && p_out)
      HIPCHK(hipMemcpyAsync(a.p, p_out, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice,
                            c->st));
    launch_fill_f64(part, npart, 0.0, c->st);
    launch_flow_codes(a, c->st);
    HIPCHK(hipGetLastError());
    long steps = 0;
    double total_prev = 0.0, du = INFINITY, un = 0.0;
    int m = p->cg_max;
    int status = SOCFV_NOT_CONVERGED;
    while (steps < p->max_steps) {
      const long k = std::min<long>(p->check_every, p->max_steps - steps);
      for (long s = 0; s < k; ++s) {
        launch_flow_predict(a, c->st);
        launch_flow_cg_init(a, c->st);
        for (int j = 0; j < m; ++j) launch_flow_cg_iter(a, j, c->st);
        launch_flow_project(a, c->st);
      }
      HIPCHK(hipGetLastError());
      launch_reduce(a.pdu, 3 * a.nbf, 2, 0u, c->dres, c->st);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(c->hres, c->dres, sizeof(double) * 2, hipMemcpyDeviceToHost, c->st));
      HIPCHK(hipMemcpyAsync(c->hres + 2, a.sc + FS_CG_TOTAL, sizeof(double),
                            hipMemcpyDeviceToHost, c->st));
      HIPCHK(hipStreamSynchronize(c->st));
      steps += k;
      du = std::sqrt(c->hres[0]);
      un = std::sqrt(c->hres[1]);
      const double total = c->hres[2];
      if (!std::isfinite(du) || !std::isfinite(un))
        return fail(SOCFV_DIVERGED, "flow steps diverged at step %ld", steps);
      // launch enough CG iterations for this phase: twice the recent average plus 4, at
      // least 8 (kernels past the stop return at once, at about 2 us each)
      const double avg = (total - total_prev) / (double)k;
      total_prev = total;
      m = std::min(p->cg_max, std::max(8, (int)std::ceil(2.0 * avg) + 4));
      if (un > 0.0 && du < p->tol * un) {
        status = SOCFV_OK;
        break;
      }
    }
    launch_flow_check(a, c->st);
    HIPCHK(hipGetLastError());
    launch_reduce(a.pdiv, a.nbc, 4, 0x5u, c->dres, c->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->hres, c->dres, sizeof(double) * 4, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(c->hres + 4, a.sc + FS_CG_TOTAL, sizeof(double),
                          hipMemcpyDeviceToHost, c->st));
    if (p_out)
      HIPCHK(hipMemcpyAsync(p_out, a.p, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice,
                            c->st));
    TRY(leave(c, hip_stream));
    socfv_flow_stats s{};
    s.steps = steps;
    s.cg_iterations = (long)c->hres[4];
    s.change = un > 0.0 ? du / un : INFINITY;
    s.divergence = c->hres[0];
    s.Q = c->hres[1];
    s.u_max = c->hres[2];
    s.Q_out = c->hres[3];
    s.dt = a.dt;
    s.status = status;
    s.seconds = now_s() - t0;
    if (st) *st = s;
    if (status == SOCFV_NOT_CONVERGED)
      fail(status, "flow not converged after %ld steps (relative change %g)", steps, s.change);
    return status;
  }();
  if (rc < 0 && c->st) (void)hipStreamSynchronize(c->st);
  for (void *ptr : mem) hfree(ptr);
  return rc;
}

}  // extern "C"
