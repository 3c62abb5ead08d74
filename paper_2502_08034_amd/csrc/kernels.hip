// HIP kernels (gfx950) of the steady state-of-charge solve.
//
// Finite-volume residual of the SOC transport equation (Eq. (nernst-planck-soc)) with the
// affine Butler-Volmer source (Eq. (rate-from-soc-gen)), explicit pseudo-time sweeps as in
// the Algorithm "SOC at Mass Transport Limit", the residual norm of
// Eq. (convergence-bv-change), the utilisation of Eq. (utilization-def) / Eq. (umt-def)
// and the electron-flow balance of Eqs. (electron-flow)-(convergence-bv-flow).
//
// The sweep is bandwidth bound (about 35 flops per 21 bytes in FP32), so the kernels are
// organised around memory traffic, not arithmetic: each thread owns one (x, y) column
// and marches a chunk of z, carrying s and the z-face velocity of the planes below and
// above in registers, so every z plane of s and of the z velocities is fetched once per
// chunk; x and y neighbours come from the same or adjacent rows that the block's other
// lanes fetch at the same time (coalesced 64-wide rows, served from L1/L2).  All
// reductions are two-pass and deterministic: 64-lane shuffles, then a fixed-order sum
// of per-wave values in LDS, then one block over the per-block partials.
#include "internal.h"

#include <cmath>
#include <mutex>
#include <type_traits>

namespace socfv {

// ------------------------------------------------------------------------------------
// Reductions
// ------------------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Reduce K values over the block and store them at out[0..K-1] (thread 0).  Bit k of
// maxmask selects max instead of sum for value k.  Must be reached by every thread.
template <int K>
__device__ __forceinline__ void block_store(double (&v)[K], unsigned maxmask, double *out) {
  __shared__ double sh[16][K];
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nthreads = blockDim.x * blockDim.y * blockDim.z;
  const int lane = tid & 63, wid = tid >> 6, nw = (nthreads + 63) >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = ((maxmask >> k) & 1u) ? wave_max(v[k]) : wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) sh[wid][k] = v[k];
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double acc = sh[0][k];
      for (int w = 1; w < nw; ++w) acc = ((maxmask >> k) & 1u) ? fmax(acc, sh[w][k]) : acc + sh[w][k];
      out[k] = acc;
    }
  }
}

__global__ void __launch_bounds__(256) k_reduce(const double *__restrict__ partial, int nblk,
                                                int nv, unsigned maxmask,
                                                double *__restrict__ out) {
  __shared__ double sh[256];
  for (int k = 0; k < nv; ++k) {
    const bool mx = (maxmask >> k) & 1u;
    double acc = mx ? -INFINITY : 0.0;
    for (int j = threadIdx.x; j < nblk; j += 256) {
      double v = partial[(long long)j * nv + k];
      acc = mx ? fmax(acc, v) : acc + v;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        double b = sh[threadIdx.x + s];
        sh[threadIdx.x] = mx ? fmax(sh[threadIdx.x], b) : sh[threadIdx.x] + b;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sh[0];
    __syncthreads();
  }
}

void launch_reduce(const double *partial, int nblk, int nv, unsigned maxmask, double *out,
                   hipStream_t st) {
  k_reduce<<<1, 256, 0, st>>>(partial, nblk, nv, maxmask, out);
}

// ------------------------------------------------------------------------------------
// Geometry flags
// ------------------------------------------------------------------------------------

int flags_blocks(const Grid &g) { return (int)((g.n + 255) / 256); }

// partial per block: [pore cells, reactive cells, inlet pore cells, outlet pore cells]
__global__ void __launch_bounds__(256) k_flags(Grid g, const uint8_t *__restrict__ solid,
                                               uint8_t *__restrict__ flags,
                                               double *__restrict__ partial) {
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  double v[4] = {0, 0, 0, 0};
  if (i < g.n) {
    const int x = (int)(i % g.nx);
    const int y = (int)((i / g.nx) % g.ny);
    const int z = (int)(i / ((long long)g.nx * g.ny));
    const long long pl = (long long)g.nx * g.ny;
    uint8_t f = 0;
    if (!solid[i]) {
      f = FL_PORE;
      if (x > 0 && solid[i - 1]) f |= FL_XM;
      if (x < g.nx - 1 && solid[i + 1]) f |= FL_XP;
      if (y > 0 && solid[i - g.nx]) f |= FL_YM;
      if (y < g.ny - 1 && solid[i + g.nx]) f |= FL_YP;
      if (z > 0 && solid[i - pl]) f |= FL_ZM;
      if (z < g.nz - 1 && solid[i + pl]) f |= FL_ZP;
      v[0] = 1.0;
      v[1] = (f & FL_FIBRE) ? 1.0 : 0.0;
      v[2] = x == 0 ? 1.0 : 0.0;
      v[3] = x == g.nx - 1 ? 1.0 : 0.0;
    }
    flags[i] = f;
  }
  block_store<4>(v, 0u, partial + 4ll * blockIdx.x);
}

void launch_flags(const Grid &g, const uint8_t *solid, uint8_t *flags, double *partial,
                  int nblk, hipStream_t st) {
  k_flags<<<nblk, 256, 0, st>>>(g, solid, flags, partial);
}

// ------------------------------------------------------------------------------------
// Velocity ingest and validation
// ------------------------------------------------------------------------------------

int velocity_blocks(const Grid &g) { return (int)((g.n + 255) / 256); }

// One thread per cell: the cell's lower x / y / z faces, its outlet face (x = nx-1) and
// its upper wall faces (y = ny-1, z = nz-1).  A face with a pore cell on one side and a
// fibre voxel or a wall on the other must carry zero velocity.  Inlet and outlet faces may
// carry flow either way (upwinded like every face).  Faces without a pore cell on either
// side are stored as zero.
// partial per block: [Q_in, max|div|, max|u|, bad faces]
__global__ void __launch_bounds__(256) k_velocity(Grid g, const uint8_t *__restrict__ flags,
                                                  const double *__restrict__ ux,
                                                  const double *__restrict__ uy,
                                                  const double *__restrict__ uz, double q,
                                                  float *wx32, float *wy32, float *wz32,
                                                  float *wxo32, double *wx64, double *wy64,
                                                  double *wz64, double *wxo64,
                                                  double *__restrict__ partial) {
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  double v[4] = {0, 0, 0, 0};
  if (i < g.n) {
    const long long nx = g.nx, ny = g.ny, nz = g.nz;
    const int x = (int)(i % nx);
    const int y = (int)((i / nx) % ny);
    const int z = (int)(i / (nx * ny));
    const bool pore = flags[i] & FL_PORE;
    const long long pl = nx * ny;
    const bool pxm = x > 0 && (flags[i - 1] & FL_PORE);
    const bool pym = y > 0 && (flags[i - nx] & FL_PORE);
    const bool pzm = z > 0 && (flags[i - pl] & FL_PORE);
    double bad = 0.0;
    // lower x face (x = 0: inlet)
    double a = ux[x + (nx + 1) * (y + ny * z)] * q;
    double b = uy[x + nx * (y + (ny + 1) * z)] * q;
    double c = uz[x + nx * (y + ny * z)] * q;
    if (!isfinite(a) || !isfinite(b) || !isfinite(c)) bad += 1.0;
    // x face: open iff both sides pore (x > 0), or the inlet face of a pore cell
    const bool ox = (x == 0) ? pore : (pore && pxm);
    const bool oy = pore && pym;
    const bool oz = pore && pzm;
    if (!ox && (pore || pxm) && a != 0.0) bad += 1.0;
    if (!oy && (pore || pym) && b != 0.0) bad += 1.0;
    if (!oz && (pore || pzm) && c != 0.0) bad += 1.0;
    if (!ox) a = 0.0;
    if (!oy) b = 0.0;
    if (!oz) c = 0.0;
    wx64[i] = a; wy64[i] = b; wz64[i] = c;
    wx32[i] = (float)a; wy32[i] = (float)b; wz32[i] = (float)c;
    double umax = fmax(fabs(a), fmax(fabs(b), fabs(c)));
    // upper faces of this cell, for the divergence and the wall / outlet checks
    double ax = 0.0, by = 0.0, cz = 0.0;
    if (x == nx - 1) {
      double o = ux[nx + (nx + 1) * (y + ny * z)] * q;
      if (!isfinite(o)) bad += 1.0;
      if (!pore && o != 0.0) o = 0.0;   // outlet face of a fibre voxel: unused
      wxo64[y + ny * z] = o;
      wxo32[y + ny * z] = (float)o;
      ax = o;
    } else {
      double t = ux[(x + 1) + (nx + 1) * (y + ny * z)] * q;
      ax = (pore && (flags[i + 1] & FL_PORE)) ? t : 0.0;
    }
    if (y == ny - 1) {
      double t = uy[x + nx * (ny + (ny + 1) * z)] * q;
      if (!isfinite(t) || (pore && t != 0.0)) bad += 1.0;
    } else {
      double t = uy[x + nx * ((y + 1) + (ny + 1) * z)] * q;
      by = (pore && (flags[i + nx] & FL_PORE)) ? t : 0.0;
    }
    if (z == nz - 1) {
      double t = uz[x + nx * (y + ny * nz)] * q;
      if (!isfinite(t) || (pore && t != 0.0)) bad += 1.0;
    } else {
      double t = uz[x + nx * (y + ny * (z + 1))] * q;
      cz = (pore && (flags[i + pl] & FL_PORE)) ? t : 0.0;
    }
    if (pore) {
      v[1] = fabs((ax - a) + (by - b) + (cz - c));
      umax = fmax(umax, fmax(fabs(ax), fmax(fabs(by), fabs(cz))));
    }
    v[0] = (x == 0 && pore) ? a : 0.0;
    v[2] = umax;
    v[3] = bad;
  }
  block_store<4>(v, 0x6u, partial + 4ll * blockIdx.x);
}

void launch_velocity(const Grid &g, const uint8_t *flags, const double *ux, const double *uy,
                     const double *uz, double q, float *w32[4], double *w64[4],
                     double *partial, int nblk, hipStream_t st) {
  k_velocity<<<nblk, 256, 0, st>>>(g, flags, ux, uy, uz, q, w32[0], w32[1], w32[2], w32[3],
                                   w64[0], w64[1], w64[2], w64[3], partial);
}

// ------------------------------------------------------------------------------------
// The finite-volume residual of one cell
// ------------------------------------------------------------------------------------

// Neighbourhood of cell P: values on the six faces' far sides and the outward velocities.
template <typename T>
struct Cell {
  T c, xm, xp, ym, yp, zm, zp;          // s (or psi) of P and its neighbours
  T wxm, wxp, wym, wyp, wzm, wzp;       // face velocities along +axis (lower / upper faces)
  T gxm, gxp, gym, gyp, gzm, gzp;       // diffusive coefficients G_f
};

// R_P = sum_f [inflow brings the upwind value, outflow removes s_P, G_f (s_nb - s_P)]
//       + lam (s_eq - s_P).
// Lower faces have outward normal -axis, so their inflow velocity is +w; upper faces +axis.
// At the inlet the caller passes s_in as xm and G = 2; at the outlet s_P as xp and G = 0.
template <typename T>
__device__ __forceinline__ T residual(const Cell<T> &q, T lam, T s_eq) {
  const T z = T(0);
  T r = lam * (s_eq - q.c);
  r += fmax(q.wxm, z) * q.xm - fmax(-q.wxm, z) * q.c + q.gxm * (q.xm - q.c);
  r += fmax(-q.wxp, z) * q.xp - fmax(q.wxp, z) * q.c + q.gxp * (q.xp - q.c);
  r += fmax(q.wym, z) * q.ym - fmax(-q.wym, z) * q.c + q.gym * (q.ym - q.c);
  r += fmax(-q.wyp, z) * q.yp - fmax(q.wyp, z) * q.c + q.gyp * (q.yp - q.c);
  r += fmax(q.wzm, z) * q.zm - fmax(-q.wzm, z) * q.c + q.gzm * (q.zm - q.c);
  r += fmax(-q.wzp, z) * q.zp - fmax(q.wzp, z) * q.c + q.gzp * (q.zp - q.c);
  return r;
}

// The same residual, rearranged for the FP32 sweeps with fewer operations:
// max(w,0) s_nb - max(-w,0) s_P = max(w,0)(s_nb - s_P) + w s_P for a face with inflow
// velocity w, so
//   R_P = sum_f (max(win_f, 0) + G_f)(s_nb(f) - s_P) - s_P div_P + lam (s_eq - s_P),
//   div_P = sum of outward face velocities.
// Closed faces have w = 0 and G = 0; the outlet face takes s_nb = s_P.  G_f comes from
// one byte of closed-face bits (fibre faces, plus the walls and the outlet of this cell).
__device__ __forceinline__ float gbit(unsigned closed, int k) {
  return (float)(((~closed) >> k) & 1u);
}

__device__ __forceinline__ float residual_fast(float c, float xm, float xp, float ym, float yp,
                                               float zm, float zp, float wxm, float wxp,
                                               float wym, float wyp, float wzm, float wzp,
                                               unsigned closed, float gxm_inlet, float lam,
                                               float s_eq) {
  const float div = (wxp - wxm) + (wyp - wym) + (wzp - wzm);
  float r = lam * (s_eq - c) - c * div;
  r += (fmaxf(wxm, 0.f) + (gbit(closed, 0) + gxm_inlet)) * (xm - c);
  r += (fmaxf(-wxp, 0.f) + gbit(closed, 1)) * (xp - c);
  r += (fmaxf(wym, 0.f) + gbit(closed, 2)) * (ym - c);
  r += (fmaxf(-wyp, 0.f) + gbit(closed, 3)) * (yp - c);
  r += (fmaxf(wzm, 0.f) + gbit(closed, 4)) * (zm - c);
  r += (fmaxf(-wzp, 0.f) + gbit(closed, 5)) * (zp - c);
  return r;
}

// Reversed-advection (transpose) action at P: (A^T psi)_P for updated cells, with the
// neighbours' psi (zero on held and fibre cells, which cannot couple):
//   sum_f (max(w_f,0) + G_f)(psi_P - psi_nb) + outlet w psi_P + lam psi_P,
// w_f the outward velocity; the inlet has psi_nb = 0 and G = 2, the outlet uses w (any
// sign) on psi_P with no neighbour.
template <typename T>
__device__ __forceinline__ T transpose_action(const Cell<T> &q, T lam, bool outlet) {
  const T z = T(0);
  T a = lam * q.c;
  a += (fmax(-q.wxm, z) + q.gxm) * (q.c - q.xm);
  a += outlet ? q.wxp * q.c : (fmax(q.wxp, z) + q.gxp) * (q.c - q.xp);
  a += (fmax(-q.wym, z) + q.gym) * (q.c - q.ym);
  a += (fmax(q.wyp, z) + q.gyp) * (q.c - q.yp);
  a += (fmax(-q.wzm, z) + q.gzm) * (q.c - q.zm);
  a += (fmax(q.wzp, z) + q.gzp) * (q.c - q.zp);
  return a;
}

// Fill the in-plane part of a Cell (x and y neighbours, x / y velocities, G) for cell i at
// (x, y, z); xm_bc is the value behind the inlet face (s_in, 0 for corrections / psi),
// outlet_self selects s_P (forward) or 0 (adjoint) behind the outlet face.
template <typename T>
__device__ __forceinline__ void load_plane(Cell<T> &q, const T *__restrict__ s,
                                           const Faces<T> &w, uint8_t f, const Grid &g,
                                           int x, int y, int z, long long i, T xm_bc,
                                           bool outlet_self) {
  const int nx = g.nx, ny = g.ny;
  const bool xl = x > 0, xr = x < nx - 1, yl = y > 0, yr = y < ny - 1;
  q.xm = xl ? s[i - 1] : xm_bc;
  q.xp = xr ? s[i + 1] : (outlet_self ? q.c : T(0));
  q.ym = yl ? s[i - nx] : T(0);
  q.yp = yr ? s[i + nx] : T(0);
  q.wxm = w.wx[i];
  q.wxp = xr ? w.wx[i + 1] : w.wxo[y + (long long)ny * z];
  q.wym = w.wy[i];
  q.wyp = yr ? w.wy[i + nx] : T(0);
  q.gxm = xl ? ((f & FL_XM) ? T(0) : T(1)) : T(2);
  q.gxp = xr ? ((f & FL_XP) ? T(0) : T(1)) : T(0);
  q.gym = (yl && !(f & FL_YM)) ? T(1) : T(0);
  q.gyp = (yr && !(f & FL_YP)) ? T(1) : T(0);
}

// ------------------------------------------------------------------------------------
// Explicit sweep: s_new = s + dt R(s)  (or the correction form with r0)
// ------------------------------------------------------------------------------------

dim3 sweep_grid(const Grid &g, const Tiles &t) {
  return dim3((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + t.ty - 1) / t.ty),
              (unsigned)((g.nz + t.zc - 1) / t.zc));
}

template <typename T, bool DC, bool RES>
__global__ void __launch_bounds__(1024) k_sweep(SweepArgs<T> a) {
  if (a.gate && *a.gate != CTL_RUN) return;
  const Grid g = a.g;
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z0 = blockIdx.z * a.zc;
  const int z1 = min(z0 + a.zc, g.nz);
  const long long pl = (long long)g.nx * g.ny;
  double acc[NV] = {0, 0, 0, 0};
  if (x < g.nx && y < g.ny && z0 < z1) {
    long long i = x + (long long)g.nx * (y + (long long)g.ny * z0);
    Cell<T> q;
    T s_c = a.s[i];
    T s_dn = z0 > 0 ? a.s[i - pl] : T(0);
    T wz_c = a.w.wz[i];
    for (int z = z0; z < z1; ++z, i += pl) {
      const bool up = z + 1 < g.nz;
      const T s_up = up ? a.s[i + pl] : T(0);
      const T wz_u = up ? a.w.wz[i + pl] : T(0);
      const uint8_t f = a.flags[i];
      T out = T(0);
      if (f & FL_PORE) {
        q.c = s_c;
        q.zm = s_dn;
        q.zp = s_up;
        q.wzm = wz_c;
        q.wzp = wz_u;
        q.gzm = (z > 0 && !(f & FL_ZM)) ? T(1) : T(0);
        q.gzp = (up && !(f & FL_ZP)) ? T(1) : T(0);
        load_plane<T>(q, a.s, a.w, f, g, x, y, z, i, a.s_in, true);
        const int nf = __popc((unsigned)(f & FL_FIBRE));
        const bool held = a.pinned && nf > 0;
        const T kap = a.kappa ? (T)a.kappa[i] : T(1);
        const T lam = a.Da * kap * (T)nf;
        T r = residual<T>(q, lam, a.s_eq);
        if (DC) r += (T)a.r0[i];
        if (held) r = T(0);
        out = held ? (DC ? T(0) : a.s_eq) : s_c + a.dt * r;
        if (RES) {
          const double rd = (double)r;
          acc[0] += rd * rd;
          acc[2] += rd;
          if (!DC) {
            const double o = (double)out;
            if (!(o >= a.lo && o <= a.hi)) acc[1] += 1.0;
          } else if (!isfinite(rd)) {
            acc[1] += 1.0;
          }
        }
      }
      a.s_new[i] = out;
      s_dn = s_c;
      s_c = s_up;
      wz_c = wz_u;
    }
  }
  if (RES) block_store<NV>(acc, 0u, a.partial + (long long)NV * (blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)));
}

// Block order across the eight XCDs: hardware hands consecutive workgroups to the XCDs
// in turn, so logical tile L is given to workgroup b with L contiguous per XCD.  Tiles that
// are neighbours in y and z then run on the same XCD and share its L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, k = b >> 3;
  return x * q + min(x, r) + k;
}

// FP32 sweep with four consecutive x cells per lane (16-byte loads and stores); rows of
// 256 cells per wave.  Used when nx is a multiple of 4.  The x neighbours of a lane's
// group come from the adjacent lanes by shuffles; the wave's edge lanes load them.
template <bool DC, bool RES, bool ACT>
__global__ void __launch_bounds__(1024) k_sweep_v4(SweepArgs<float> a, int gx, int gy, int gz);

// Two sweeps per launch (time skewing along the z march).  A block of 1024 lanes holds a
// tile of rows of RX lanes (RX = 64: 16 rows, one per wave; RX = 32: 32 rows, two per wave,
// which fits narrow boxes with less waste), W consecutive x cells per lane (W = 2 for even nx,
// 1 for odd), and writes the second sweep on its interior (RX - 2) W x (1024 / RX - 2) cells;
// tiles overlap by one lane in x and one row in y on each side, where the first sweep is
// recomputed.  Marching plane j,
// the block computes the first sweep s1(j) from s(j-1..j+1) over the whole tile, stages
// s1(j) in LDS (two plane slots, one barrier per plane), and the second sweep at plane j-1
// from s1(j-2..j).  State, velocities, flags and the frozen residual come from HBM once for
// two sweeps.  Each sweep is the arithmetic of one k_sweep_v4 sweep, cell by cell.
constexpr int T2_ROWS = 16;   // thread rows of a two-sweep block (64 x 16 = 1024 lanes)

template <int W>
struct VecW {
  float v[W];
};

// Device-memory accesses through global-address-space pointers.  Array pointers read from a
// table in memory (the batched kernels) would otherwise be generic, and the compiler would
// emit flat accesses, which also count against the LDS wait counter and so make every LDS
// wait of a step wait for the loads in flight as well.
#define GMEM __attribute__((address_space(1)))
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <int W>
__device__ __forceinline__ VecW<W> ldw(const float *p) {
  VecW<W> r;
  if constexpr (W == 4) {
    const f4v t = *(GMEM const f4v *)p;
    r.v[0] = t.x; r.v[1] = t.y; r.v[2] = t.z; r.v[3] = t.w;
  } else if constexpr (W == 2) {
    const f2v t = *(GMEM const f2v *)p;
    r.v[0] = t.x; r.v[1] = t.y;
  } else {
    r.v[0] = *(GMEM const float *)p;
  }
  return r;
}

template <int W>
__device__ __forceinline__ void stw(float *p, const VecW<W> &r) {
  if constexpr (W == 4) {
    f4v t;
    t.x = r.v[0]; t.y = r.v[1]; t.z = r.v[2]; t.w = r.v[3];
    *(GMEM f4v *)p = t;
  } else if constexpr (W == 2) {
    f2v t;
    t.x = r.v[0]; t.y = r.v[1];
    *(GMEM f2v *)p = t;
  } else {
    *(GMEM float *)p = r.v[0];
  }
}

template <int W>
__device__ __forceinline__ unsigned ldflags(const uint8_t *p) {
  if constexpr (W == 4) return *(GMEM const unsigned *)p;
  else if constexpr (W == 2) return *(GMEM const unsigned short *)p;
  else return *(GMEM const uint8_t *)p;
}

template <int W>
__device__ __forceinline__ VecW<W> zerow() {
  VecW<W> r;
#pragma unroll
  for (int k = 0; k < W; ++k) r.v[k] = 0.f;
  return r;
}

template <int W>
struct CoefW {        // per-lane coefficients of one plane (W cells)
  VecW<W> wx, wym, wyp, wzl, wzu, r0;
  VecW<W> kap;        // per-cell activity (kernels instantiated for an activity field)
  float wxr;          // x face velocity after the lane's last cell
  unsigned fl;
};

// Resolved coefficients of W cells for the FP32 residual in the form
//   R_P = src_P - s_P e_P + sum_f a_f (s_nb(f) - s_P),
// a_f = max(inflow velocity through f, 0) + G_f (zero on closed faces and on the outlet
// face, whose advective flux s_P w is part of e), e_P = div_P + lam_P, and src_P = lam_P s_eq,
// or the frozen FP64 residual r0 for a correction (whose s_in and s_eq are 0).  Cells that
// are not updated (fibre, held) get zero coefficients, so R = 0 there and a sweep keeps their
// value, which the initial state sets (0 on fibre cells, s_eq or 0 on held cells).
template <int W>
struct ResW {
  VecW<W> axm, axp, aym, ayp, azm, azp, e, src;
};

// max(w, 0) + G with one rounding (h = 1/2): w + |w| is 2w or 0 exactly.  With h = 0 and
// G = 0 the coefficient is 0, which is how cells that are not updated get theirs without
// a branch.
__device__ __forceinline__ float inflow_coef(float h, float w, float G) {
  return fmaf(h, w + fabsf(w), G);
}

// ACT: the activity field is set and its values came with the plane's loads (a load here
// would make the step wait for every load in flight).  ADJ: coefficients of the transpose
// system A^T psi = g in the same form, r = src - psi e + sum_f b_f (psi_nb - psi): b_f takes
// the outflow velocity through f (max(w_out, 0) + G_f), the outlet face's flux w psi_P goes
// to the diagonal, e = lam + w_out at the outlet, and src = g_P = gscale w_out on outlet
// cells (plus r0 for a correction).  Behind the inlet psi_nb = 0, as s_in is 0.
template <bool DC, bool ACT, bool ADJ, int W>
__device__ __forceinline__ void resolvew(const SweepArgs<float> &a, const CoefW<W> &c, int x,
                                         int y, int z, bool up, ResW<W> &q) {
  const int nx = a.g.nx, ny = a.g.ny;
  // walls of this row / plane as closed-face bits (y, z)
  const unsigned wall = (y > 0 ? 0u : (unsigned)FL_YM) | (y < ny - 1 ? 0u : (unsigned)FL_YP) |
                        (z > 0 ? 0u : (unsigned)FL_ZM) | (up ? 0u : (unsigned)FL_ZP);
  const float sg = ADJ ? -1.f : 1.f;     // inflow (forward) or outflow (transpose) velocity
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const unsigned f = (c.fl >> (8 * k)) & 0xffu;
    const int xk = x + k;
    const bool outlet = xk == nx - 1;
    const int nf = __popc(f & FL_FIBRE);
    const bool upd = (f & FL_PORE) && !(a.pinned && nf > 0);
    // not updated: every face closed and no advective part
    const unsigned closed = upd ? (f | wall) : (unsigned)FL_FIBRE;
    const float h = upd ? 0.5f : 0.f;
    const float lam = a.Da * (ACT ? c.kap.v[k] : 1.f) * (float)nf;
    const float wxm = c.wx.v[k], wxp = k == W - 1 ? c.wxr : c.wx.v[k + 1];
    // inlet face: Dirichlet value on the face, G = 2 (closed bit 0 is never set there); the
    // outlet face's flux is all on the diagonal
    q.axm.v[k] = inflow_coef(h, sg * wxm, gbit(closed, 0) + (upd && xk == 0 ? 1.f : 0.f));
    q.axp.v[k] = inflow_coef(h, outlet ? 0.f : -sg * wxp, outlet ? 0.f : gbit(closed, 1));
    q.aym.v[k] = inflow_coef(h, sg * c.wym.v[k], gbit(closed, 2));
    q.ayp.v[k] = inflow_coef(h, -sg * c.wyp.v[k], gbit(closed, 3));
    q.azm.v[k] = inflow_coef(h, sg * c.wzl.v[k], gbit(closed, 4));
    q.azp.v[k] = inflow_coef(h, -sg * c.wzu.v[k], gbit(closed, 5));
    float e, src;
    if (ADJ) {
      e = lam + (outlet ? wxp : 0.f);
      src = (outlet ? a.gscale * wxp : 0.f) + (DC ? c.r0.v[k] : 0.f);
    } else {
      const float div = (wxp - wxm) + (c.wyp.v[k] - c.wym.v[k]) + (c.wzu.v[k] - c.wzl.v[k]);
      e = div + lam;
      src = DC ? c.r0.v[k] : lam * a.s_eq;
    }
    q.e.v[k] = upd ? e : 0.f;
    q.src.v[k] = upd ? src : 0.f;
  }
}

// One explicit FP32 update of W cells from resolved coefficients: out = s + dt R(s),
// rout = R.  left / right are the x neighbours beyond the lane's first / last cell.
template <int W>
__device__ __forceinline__ void applyw(const ResW<W> &q, float dt, const VecW<W> &sc,
                                       float left, float right, const VecW<W> &sdn,
                                       const VecW<W> &sup, const VecW<W> &sym,
                                       const VecW<W> &syp, VecW<W> &out, VecW<W> &rout) {
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const float c0 = sc.v[k];
    const float xm = k == 0 ? left : sc.v[k - 1];
    const float xp = k == W - 1 ? right : sc.v[k + 1];
    float r = fmaf(-c0, q.e.v[k], q.src.v[k]);
    r = fmaf(q.axm.v[k], xm - c0, r);
    r = fmaf(q.axp.v[k], xp - c0, r);
    r = fmaf(q.aym.v[k], sym.v[k] - c0, r);
    r = fmaf(q.ayp.v[k], syp.v[k] - c0, r);
    r = fmaf(q.azm.v[k], sdn.v[k] - c0, r);
    r = fmaf(q.azp.v[k], sup.v[k] - c0, r);
    out.v[k] = fmaf(dt, r, c0);
    rout.v[k] = r;
  }
}

// One explicit FP32 sweep of W cells: out = s + dt (R(s) [+ r0]), rout = the residual used.
template <bool DC, bool ACT, int W>
__device__ __forceinline__ void sweepw(const SweepArgs<float> &a, const CoefW<W> &c,
                                       const VecW<W> &sc, float left, float right,
                                       const VecW<W> &sdn, const VecW<W> &sup,
                                       const VecW<W> &sym, const VecW<W> &syp, int x, int y,
                                       int z, bool up, VecW<W> &out, VecW<W> &rout) {
  ResW<W> q;
  resolvew<DC, ACT, false, W>(a, c, x, y, z, up, q);
  applyw<W>(q, a.dt, sc, left, right, sdn, sup, sym, syp, out, rout);
}

// Everything a lane (W cells) reads from plane j: the state one plane up, the state of
// rows y-1 / y+1, the coefficients, and the x-edge values its wave's edge lanes need.
template <int W>
struct PlaneW {
  VecW<W> s_up, sym, syp;
  CoefW<W> c;
  float left, right;
};

// One-lane shifts across the wave by DPP wave shifts (one VALU move, no LDS round trip):
// lane i receives lane i-1's value (from below) or lane i+1's (from above); the wave's
// first / last lane receives 0.  Every lane whose value is read must be active.
__device__ __forceinline__ float lane_from_below(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x138, 0xf, 0xf, false));
}

__device__ __forceinline__ float lane_from_above(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x130, 0xf, 0xf, false));
}

// A lane's resolved coefficients (W cells, 8 W floats) parked in LDS between its two sweeps
// of a plane: 2 W float4 per lane, lane-private (no barrier needed), two plane slots.
template <int W>
__device__ __forceinline__ void park_coef(float4 (*slot)[64 * T2_ROWS], int t, const ResW<W> &q) {
  if constexpr (W == 2) {
    slot[0][t] = make_float4(q.axm.v[0], q.axm.v[1], q.axp.v[0], q.axp.v[1]);
    slot[1][t] = make_float4(q.aym.v[0], q.aym.v[1], q.ayp.v[0], q.ayp.v[1]);
    slot[2][t] = make_float4(q.azm.v[0], q.azm.v[1], q.azp.v[0], q.azp.v[1]);
    slot[3][t] = make_float4(q.e.v[0], q.e.v[1], q.src.v[0], q.src.v[1]);
  } else {
    slot[0][t] = make_float4(q.axm.v[0], q.axp.v[0], q.aym.v[0], q.ayp.v[0]);
    slot[1][t] = make_float4(q.azm.v[0], q.azp.v[0], q.e.v[0], q.src.v[0]);
  }
}

template <int W>
__device__ __forceinline__ ResW<W> fetch_coef(float4 (*slot)[64 * T2_ROWS], int t) {
  ResW<W> q;
  if constexpr (W == 2) {
    float4 v = slot[0][t];
    q.axm.v[0] = v.x; q.axm.v[1] = v.y; q.axp.v[0] = v.z; q.axp.v[1] = v.w;
    v = slot[1][t];
    q.aym.v[0] = v.x; q.aym.v[1] = v.y; q.ayp.v[0] = v.z; q.ayp.v[1] = v.w;
    v = slot[2][t];
    q.azm.v[0] = v.x; q.azm.v[1] = v.y; q.azp.v[0] = v.z; q.azp.v[1] = v.w;
    v = slot[3][t];
    q.e.v[0] = v.x; q.e.v[1] = v.y; q.src.v[0] = v.z; q.src.v[1] = v.w;
  } else {
    float4 v = slot[0][t];
    q.axm.v[0] = v.x; q.axp.v[0] = v.y; q.aym.v[0] = v.z; q.ayp.v[0] = v.w;
    v = slot[1][t];
    q.azm.v[0] = v.x; q.azp.v[0] = v.y; q.e.v[0] = v.z; q.src.v[0] = v.w;
  }
  return q;
}

// Loads and stores at a 32-bit byte offset from a kernel-argument base: the compiler then
// addresses with the scalar base plus one 32-bit VGPR offset per lane, with no 64-bit
// address arithmetic per access.  Every FP32 array of the two-sweep path is below 4 GiB.
template <int W>
__device__ __forceinline__ VecW<W> ldo(const float *base, unsigned off) {
  return ldw<W>(reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + off));
}

__device__ __forceinline__ float ldo1(const float *base, unsigned off) {
  return ldw<1>(reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + off)).v[0];
}

template <int W>
__device__ __forceinline__ void sto(float *base, unsigned off, const VecW<W> &v) {
  stw<W>(reinterpret_cast<float *>(reinterpret_cast<char *>(base) + off), v);
}

// Loads at clamped 32-bit offsets (every address valid; out-of-range planes, rows and
// lanes read a copy of a valid cell and their results meet only zero-coefficient faces),
// then selects for the wall velocities that must be zero.  With UPZ the plane's upper
// z-face velocity is loaded too; without, the caller takes it from the next plane's lower
// face.
template <bool DC, bool UPZ, bool ACT, int W, int RX>
__device__ __forceinline__ void load_plane2(const SweepArgs<float> &a, PlaneW<W> &d,
                                            unsigned ib, unsigned pl, int j, int xc, int yc,
                                            int lx, bool last, bool yl, bool yr) {
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int jj = min(j, nz - 1);
  const bool up = jj + 1 < nz;
  const unsigned o = ib + pl * (unsigned)jj;
  const unsigned o4 = 4u * o;
  const unsigned oup = o4 + (up ? 4u * pl : 0u);
  const unsigned oyp = o4 + (yr ? 4u * (unsigned)nx : 0u);
  const unsigned oym = o4 - (yl ? 4u * (unsigned)nx : 0u);
  // the lower z face first: the step before this plane's reads it as its upper face, and
  // load counters complete in issue order
  d.c.wzl = ldo<W>(a.w.wz, o4);
  d.s_up = ldo<W>(a.s, oup);
  d.sym = ldo<W>(a.s, oym);
  d.syp = ldo<W>(a.s, oyp);
  d.c.wx = ldo<W>(a.w.wx, o4);
  d.c.wym = ldo<W>(a.w.wy, o4);
  const VecW<W> wyp = ldo<W>(a.w.wy, oyp);
  if (UPZ) {
    const VecW<W> wzu = ldo<W>(a.w.wz, oup);
#pragma unroll
    for (int k = 0; k < W; ++k) d.c.wzu.v[k] = up ? wzu.v[k] : 0.f;
  }
#pragma unroll
  for (int k = 0; k < W; ++k) d.c.wyp.v[k] = yr ? wyp.v[k] : 0.f;
  d.c.fl = ldflags<W>(a.flags + o);
  if (DC) d.c.r0 = ldo<W>(a.r0, o4);
  else d.c.r0 = zerow<W>();
  if (ACT) d.c.kap = ldo<W>(a.kappa, o4);
  d.left = a.s_in;
  d.right = 0.f;
  d.c.wxr = 0.f;
  if (lx == 0 && xc > 0) d.left = ldo1(a.s, o4 - 4u);
  if (last) d.c.wxr = ldo1(a.w.wxo, 4u * (yc + (unsigned)ny * (unsigned)jj));
  else if (lx == RX - 1) {
    d.right = ldo1(a.s, o4 + 4u * W);
    d.c.wxr = ldo1(a.w.wx, o4 + 4u * W);
  }
}

template <bool DC, bool RES, bool ACT, bool ADJ, int W, int RX>
__device__ __forceinline__ void sweep2_tile(const SweepArgs<float> &a, int gx, int gy, int L,
                                            float (*lds)[1024 / RX][RX * W],
                                            float4 (*qlds)[2 * W][64 * T2_ROWS], double *part) {
  constexpr int RY = 1024 / RX;
  const Grid g = a.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int bx = L % gx, by = (L / gx) % gy, bz = L / (gx * gy);
  const int lane = threadIdx.x, tid = lane + 64 * threadIdx.y;
  // position in the tile: lane lx of row ry (RX = 64: the wave's lane and the wave's row)
  const int lx = tid % RX, row = tid / RX;
  const int x = bx * ((RX - 2) * W) - W + W * lx;
  const int y = by * (RY - 2) - 1 + row;
  const int z0 = bz * a.zc;
  const int z1 = min(z0 + a.zc, nz);
  const bool act = x >= 0 && x < nx && y >= 0 && y < ny;
  const bool outc = act && lx >= 1 && lx <= RX - 2 && row >= 1 && row <= RY - 2;
  const int xc = min(max(x, 0), nx - W);
  const int yc = min(max(y, 0), ny - 1);
  const bool yl = yc > 0, yr = yc < ny - 1;
  const bool last = xc + W >= nx;
  const unsigned pl = (unsigned)nx * (unsigned)ny;
  const unsigned ib = (unsigned)xc + (unsigned)nx * (unsigned)yc;
  const VecW<W> zw = zerow<W>();
  double acc[NV] = {0, 0, 0, 0};
  // March j over [jb, je]: first sweep at plane j, second sweep at plane j-1 from the LDS
  // copy of s1(j-1) staged in the previous step, stage s1(j).  Plane data sit in a ring of
  // four: j is swept, j-1 keeps s(j) (its s_up), and the loads of the next PD planes are in
  // flight (two ahead; one in the variant that also accumulates the residual, whose extra
  // registers would not fit two).  The loop is unrolled by four so every ring index is a
  // compile-time constant.
  constexpr int PD = RES || ACT ? 1 : 2;
  const int jb = max(z0 - 1, 0);
  const int je = min(z1, nz);            // inclusive; j == nz only finishes plane nz-1
  PlaneW<W> P[4];
  VecW<W> sdn;                           // s(j-1)
  // first-sweep planes below the box are closed walls: their LDS copy must be finite
#pragma unroll
  for (int k = 0; k < W; ++k) lds[0][row][W * lx + k] = lds[1][row][W * lx + k] = 0.f;
  {
    const unsigned o = ib + pl * (unsigned)jb;
    sdn = jb > 0 ? ldo<W>(a.s, 4u * (o - pl)) : zw;
    P[3].s_up = ldo<W>(a.s, 4u * o);     // s(jb)
    P[3].c.fl = 0u;
    load_plane2<DC, PD == 1, ACT, W, RX>(a, P[0], ib, pl, jb, xc, yc, lx, last, yl, yr);
    if (PD == 2)
      load_plane2<DC, false, ACT, W, RX>(a, P[1], ib, pl, jb + 1, xc, yc, lx, last, yl, yr);
  }
  auto step = [&](PlaneW<W> &cur, const PlaneW<W> &prev, const PlaneW<W> &nxt, PlaneW<W> &ld,
                  int j) {
    load_plane2<DC, PD == 1, ACT, W, RX>(a, ld, ib, pl, j + PD, xc, yc, lx, last, yl, yr);
    if (PD == 2) {
      // upper z face of plane j = lower z face of plane j+1 (closed above the top plane)
#pragma unroll
      for (int k = 0; k < W; ++k) cur.c.wzu.v[k] = j + 1 < nz ? nxt.c.wzl.v[k] : 0.f;
    }
    const VecW<W> &s_c = prev.s_up;      // s(j)
    float left = lane_from_below(s_c.v[W - 1]);
    float right = lane_from_above(s_c.v[0]);
    float wxr = lane_from_above(cur.c.wx.v[0]);
    // the segment's edge lanes take what they loaded (the shifts cross segments there)
    if (lx == 0) left = cur.left;
    if (lx == RX - 1 || last) {
      right = cur.right;
      wxr = cur.c.wxr;
    }
    if (x == 0) left = a.s_in;
    cur.c.wxr = wxr;
    VecW<W> r1, s1_j;
    if (j < nz) {
      ResW<W> q;
      resolvew<DC, ACT, ADJ, W>(a, cur.c, xc, yc, j, j + 1 < nz, q);
      applyw<W>(q, a.dt, s_c, left, right, sdn, cur.s_up, cur.sym, cur.syp, s1_j, r1);
      park_coef<W>(qlds[j & 1], tid, q);
    } else {
      s1_j = zw;
    }
    sdn = s_c;
    // second sweep at plane p = j - 1 on the interior.  The lane's own s1(p) is read and
    // its x neighbours shifted in from the adjacent lanes with every lane active (the halo
    // lanes take no part in the update below but supply these values).
    const int p = j - 1;
    const int bp = p & 1;
    VecW<W> c1;
#pragma unroll
    for (int k = 0; k < W; ++k) c1.v[k] = lds[bp][row][W * lx + k];
    const float c1_left = lane_from_below(c1.v[W - 1]);
    const float c1_right = lane_from_above(c1.v[0]);
    if (p >= z0 && p < z1 && outc) {
      // y neighbours of s1(p), and the lane's own s1(p-1) below: the other slot still
      // holds it, as s1(j) is staged only at the end of this step
      VecW<W> ym1, yp1, dn1;
#pragma unroll
      for (int k = 0; k < W; ++k) {
        ym1.v[k] = lds[bp][row - 1][W * lx + k];
        yp1.v[k] = lds[bp][row + 1][W * lx + k];
        dn1.v[k] = lds[bp ^ 1][row][W * lx + k];
      }
      const float lft = x == 0 ? a.s_in : c1_left;
      const float rgt = c1_right;
      const unsigned ip = ib + pl * (unsigned)p;
      VecW<W> s2, r2;
      applyw<W>(fetch_coef<W>(qlds[bp], tid), a.dt, c1, lft, rgt, dn1, s1_j, ym1, yp1, s2, r2);
      sto<W>(a.s_new, 4u * ip, s2);
      if (RES) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const unsigned f = (prev.c.fl >> (8 * k)) & 0xffu;
          if (!(f & FL_PORE)) continue;
          const double rd = (double)r2.v[k];
          acc[0] += rd * rd;
          acc[2] += rd;
          if (!DC) {
            const double od = (double)s2.v[k];
            if (!(od >= a.lo && od <= a.hi)) acc[1] += 1.0;
          } else if (!isfinite(rd)) {
            acc[1] += 1.0;
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < W; ++k) lds[j & 1][row][W * lx + k] = s1_j.v[k];
    __syncthreads();
  };
  for (int j = jb; j <= je; j += 4) {
    step(P[0], P[3], P[1], P[(PD + 0) & 3], j);
    if (j + 1 > je) break;
    step(P[1], P[0], P[2], P[(PD + 1) & 3], j + 1);
    if (j + 2 > je) break;
    step(P[2], P[1], P[3], P[(PD + 2) & 3], j + 2);
    if (j + 3 > je) break;
    step(P[3], P[2], P[0], P[(PD + 3) & 3], j + 3);
  }
  if (RES) block_store<NV>(acc, 0u, part);
}

// One tile march per block; tiles go to workgroups XCD by XCD.
template <bool DC, bool RES, bool ACT, bool ADJ, int W, int RX>
__global__ void __launch_bounds__(1024) k_sweep2(SweepArgs<float> a, int gx, int gy, int gz) {
  __shared__ float lds[2][1024 / RX][RX * W];
  __shared__ float4 qlds[2][2 * W][64 * T2_ROWS];
  if (a.gate && *a.gate != CTL_RUN) return;
  const int L = xcd_tile(blockIdx.x, gx * gy * gz);
  sweep2_tile<DC, RES, ACT, ADJ, W, RX>(a, gx, gy, L, lds, qlds,
                                        RES ? a.partial + (long long)NV * blockIdx.x : nullptr);
}

template <bool DC, bool RES, bool ACT>
__global__ void __launch_bounds__(1024) k_sweep_v4(SweepArgs<float> a, int gx, int gy, int gz) {
  if (a.gate && *a.gate != CTL_RUN) return;
  constexpr int W = 4;
  const Grid g = a.g;
  const int nx = g.nx, ny = g.ny;
  const int nb = gx * gy * gz;
  const int L = xcd_tile(blockIdx.x, nb);
  const int bx = L % gx, by = (L / gx) % gy, bz = L / (gx * gy);
  const int lane = threadIdx.x;
  const int x = bx * 256 + W * lane;
  const int y = by * blockDim.y + threadIdx.y;
  const int z0 = bz * a.zc;
  const int z1 = min(z0 + a.zc, g.nz);
  const long long pl = (long long)nx * ny;
  const bool act = x < nx && y < ny;
  const bool yl = y > 0, yr = y < ny - 1;
  const bool last = x + W >= nx;          // this group holds the outlet cell
  double acc[NV] = {0, 0, 0, 0};
  const VecW<W> zw = zerow<W>();
  long long i = act ? x + (long long)nx * (y + (long long)ny * z0) : 0;
  VecW<W> sc = zw, sdn = zw, wzc = zw;
  if (act) {
    sc = ldw<W>(a.s + i);
    if (z0 > 0) sdn = ldw<W>(a.s + i - pl);
    wzc = ldw<W>(a.w.wz + i);
  }
  for (int z = z0; z < z1; ++z, i += pl) {
    const bool up = z + 1 < g.nz;
    CoefW<W> cc;
    cc.wx = cc.wym = cc.wyp = cc.wzu = cc.r0 = zw;
    cc.wzl = wzc;
    cc.fl = 0u;
    VecW<W> sup = zw, sym = zw, syp = zw;
    if (act) {
      if (up) {
        sup = ldw<W>(a.s + i + pl);
        cc.wzu = ldw<W>(a.w.wz + i + pl);
      }
      cc.wx = ldw<W>(a.w.wx + i);
      cc.wym = ldw<W>(a.w.wy + i);
      if (yr) {
        cc.wyp = ldw<W>(a.w.wy + i + nx);
        syp = ldw<W>(a.s + i + nx);
      }
      if (yl) sym = ldw<W>(a.s + i - nx);
      cc.fl = ldflags<W>(a.flags + i);
      if (DC) cc.r0 = ldw<W>(a.r0 + i);
      if (ACT) cc.kap = ldw<W>(a.kappa + i);
    }
    // x neighbours: lane-1 holds x-1, lane+1 holds x+4 and the face velocity at x+4
    float left = __shfl_up(sc.v[W - 1], 1, 64);
    float right = __shfl_down(sc.v[0], 1, 64);
    float wxr = __shfl_down(cc.wx.v[0], 1, 64);
    if (act) {
      if (x == 0) left = a.s_in;
      else if (lane == 0) left = a.s[i - 1];
      if (last) {
        wxr = a.w.wxo[y + (long long)ny * z];
        right = 0.f;
      } else if (lane == 63) {
        right = a.s[i + W];
        wxr = a.w.wx[i + W];
      }
    }
    cc.wxr = wxr;
    if (act) {
      VecW<W> out, r;
      sweepw<DC, ACT, W>(a, cc, sc, left, right, sdn, sup, sym, syp, x, y, z, up, out, r);
      stw<W>(a.s_new + i, out);
      if (RES) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const unsigned f = (cc.fl >> (8 * k)) & 0xffu;
          if (!(f & FL_PORE)) continue;
          const double rd = (double)r.v[k];
          acc[0] += rd * rd;
          acc[2] += rd;
          if (!DC) {
            const double od = (double)out.v[k];
            if (!(od >= a.lo && od <= a.hi)) acc[1] += 1.0;
          } else if (!isfinite(rd)) {
            acc[1] += 1.0;
          }
        }
      }
    }
    sdn = sc;
    sc = sup;
    wzc = cc.wzu;
  }
  if (RES) block_store<NV>(acc, 0u, a.partial + (long long)NV * blockIdx.x);
}

bool vec4_path(const Grid &g) { return (g.nx & 3) == 0; }

// 32-bit byte offsets for every FP32 array
bool two_path(const Grid &g) { return g.n < (1ll << 30); }

int two_w(const Grid &g) { return (g.nx & 1) ? 1 : 2; }

dim3 sweep2_grid(const Grid &g, const Tiles &t) {
  int gx, gy;
  tile2_xy(g.nx, g.ny, two_w(g), t.rx, gx, gy);
  return dim3((unsigned)gx, (unsigned)gy, (unsigned)((g.nz + t.zc2 - 1) / t.zc2));
}

// Calls f with three std::bool_constant arguments, so one launch line covers the eight
// instantiations of a kernel template over (correction, residual, activity).
template <typename F>
void with_flags(bool a, bool b, bool c, F &&f) {
  using T = std::true_type;
  using N = std::false_type;
  if (a) {
    if (b) { if (c) f(T{}, T{}, T{}); else f(T{}, T{}, N{}); }
    else { if (c) f(T{}, N{}, T{}); else f(T{}, N{}, N{}); }
  } else {
    if (b) { if (c) f(N{}, T{}, T{}); else f(N{}, T{}, N{}); }
    else { if (c) f(N{}, N{}, T{}); else f(N{}, N{}, N{}); }
  }
}

void launch_sweep2(const SweepArgs<float> &a, const Tiles &t, hipStream_t st, bool adj) {
  dim3 gv = sweep2_grid(a.g, t);
  const unsigned nb = gv.x * gv.y * gv.z;
  SweepArgs<float> b = a;
  b.zc = t.zc2;
  dim3 block(64, T2_ROWS, 1);
  auto go = [&](auto w, auto rx) {
    constexpr int W = decltype(w)::value, RX = decltype(rx)::value;
    if (adj) {
      // transpose sweeps run only in the correction form
      with_flags(true, a.partial != nullptr, a.kappa != nullptr, [&](auto, auto res, auto act) {
        k_sweep2<true, res.value, act.value, true, W, RX><<<nb, block, 0, st>>>(b, gv.x, gv.y,
                                                                               gv.z);
      });
      return;
    }
    with_flags(a.r0 != nullptr, a.partial != nullptr, a.kappa != nullptr,
               [&](auto dc, auto res, auto act) {
                 k_sweep2<dc.value, res.value, act.value, false, W, RX><<<nb, block, 0, st>>>(
                     b, gv.x, gv.y, gv.z);
               });
  };
  using I2 = std::integral_constant<int, 2>;
  using I1 = std::integral_constant<int, 1>;
  using R64 = std::integral_constant<int, 64>;
  using R32 = std::integral_constant<int, 32>;
  if (two_w(a.g) == 2) {
    if (t.rx == 32) go(I2{}, R32{});
    else go(I2{}, R64{});
  } else {
    if (t.rx == 32) go(I1{}, R32{});
    else go(I1{}, R64{});
  }
}

dim3 sweep_grid_v4(const Grid &g, const Tiles &t) {
  return dim3((unsigned)((g.nx + 255) / 256), (unsigned)((g.ny + t.ty - 1) / t.ty),
              (unsigned)((g.nz + t.zc - 1) / t.zc));
}

template <typename T>
void launch_sweep(const SweepArgs<T> &a, const Tiles &t, hipStream_t st) {
  if (sizeof(T) == 4 && vec4_path(a.g)) {
    const SweepArgs<float> &af = reinterpret_cast<const SweepArgs<float> &>(a);
    dim3 gv = sweep_grid_v4(a.g, t);
    const unsigned nb = gv.x * gv.y * gv.z;
    dim3 block(64, t.ty, 1);
    with_flags(a.r0 != nullptr, a.partial != nullptr, a.kappa != nullptr,
               [&](auto dc, auto res, auto act) {
                 k_sweep_v4<dc.value, res.value, act.value><<<nb, block, 0, st>>>(af, gv.x, gv.y,
                                                                                 gv.z);
               });
    return;
  }
  dim3 grid = sweep_grid(a.g, t), block(64, t.ty, 1);
  const bool dc = a.r0 != nullptr, res = a.partial != nullptr;
  if (dc) {
    if (res) k_sweep<T, true, true><<<grid, block, 0, st>>>(a);
    else k_sweep<T, true, false><<<grid, block, 0, st>>>(a);
  } else {
    if (res) k_sweep<T, false, true><<<grid, block, 0, st>>>(a);
    else k_sweep<T, false, false><<<grid, block, 0, st>>>(a);
  }
}
template void launch_sweep<float>(const SweepArgs<float> &, const Tiles &, hipStream_t);
template void launch_sweep<double>(const SweepArgs<double> &, const Tiles &, hipStream_t);

// ------------------------------------------------------------------------------------
// Batched sweeps: many problems of uneven size in one launch
// ------------------------------------------------------------------------------------

// One launch sweeps every unfinished problem once.  The tiles of all problems are numbered
// (each tile: 64 x ty lanes, one cell per lane, zc cells along z); the work list holds
// the tiles of the unfinished problems, and a fixed set of persistent blocks splits it
// into contiguous runs, placed XCD by XCD so that neighbouring tiles share an L2.
// Finished problems are not swept, so their buffers keep their parity.  With RES the
// residual partials are written per tile; k_batch_reduce sums each problem's tiles in a
// fixed order.
template <bool DC, bool RES>
__global__ void __launch_bounds__(1024) k_batch_sweep(const BatchProb *__restrict__ probs,
                                                     const int *__restrict__ tile_prob,
                                                     const int *__restrict__ work,
                                                     const int *__restrict__ nwork, int parity,
                                                     double *__restrict__ partial) {
  // the work list holds the tiles of the unfinished problems; its length lives in device
  // memory so that a captured graph keeps working as problems finish
  const int nw = *nwork;
  const int per = (nw + (int)gridDim.x - 1) / (int)gridDim.x;
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int w0 = b * per;
  const int w1 = min(w0 + per, nw);
  const int lane = threadIdx.x, row = threadIdx.y;
  for (int w = w0; w < w1; ++w) {
    const int t = work[w];
    const int pi = tile_prob[t];
    const BatchProb &q = probs[pi];
    double acc[NV] = {0, 0, 0, 0};
    {
      const int nx = q.nx, ny = q.ny, nz = q.nz;
      const long long pl = (long long)nx * ny;
      const int lt = t - q.tile0;
      const int bx = lt % q.gx, by = (lt / q.gx) % q.gy, bz = lt / (q.gx * q.gy);
      const int x = bx * 64 + lane;
      const int y = by * blockDim.y + row;
      const int z0 = bz * q.zc;
      const int z1 = min(z0 + q.zc, nz);
      const float *s = parity ? q.s1 : q.s0;
      float *s_new = parity ? q.s0 : q.s1;
      if (x < nx && y < ny) {
        const bool xl = x > 0, xr = x < nx - 1, yl = y > 0, yr = y < ny - 1;
        const float xm_bc = DC ? 0.f : q.s_in;
        long long i = x + (long long)nx * (y + (long long)ny * z0);
        float s_c = s[i];
        float s_dn = z0 > 0 ? s[i - pl] : 0.f;
        float wz_c = q.wz[i];
        const unsigned ywall = (yl ? 0u : (unsigned)FL_YM) | (yr ? 0u : (unsigned)FL_YP) |
                               (xr ? 0u : (unsigned)FL_XP);
        for (int z = z0; z < z1; ++z, i += pl) {
          const bool up = z + 1 < nz;
          const float s_up = up ? s[i + pl] : 0.f;
          const float wz_u = up ? q.wz[i + pl] : 0.f;
          const unsigned f = q.flags[i];
          float out = 0.f;
          if (f & FL_PORE) {
            const unsigned closed = f | ywall | (z > 0 ? 0u : (unsigned)FL_ZM) |
                                    (up ? 0u : (unsigned)FL_ZP);
            const float xm = xl ? s[i - 1] : xm_bc;
            const float xp = xr ? s[i + 1] : s_c;
            const float ym = yl ? s[i - nx] : 0.f;
            const float yp = yr ? s[i + nx] : 0.f;
            const float wxm = q.wx[i];
            const float wxp = xr ? q.wx[i + 1] : q.wxo[y + (long long)ny * z];
            const float wym = q.wy[i];
            const float wyp = yr ? q.wy[i + nx] : 0.f;
            const int nf = __popc(f & FL_FIBRE);
            const bool held = q.pinned && nf > 0;
            const float kap = q.kappa ? q.kappa[i] : 1.f;
            float r = residual_fast(s_c, xm, xp, ym, yp, s_dn, s_up, wxm, wxp, wym, wyp, wz_c, wz_u,
                                    closed, xl ? 0.f : 1.f, q.Da * kap * (float)nf,
                                    DC ? 0.f : q.s_eq);
            if (DC) r += q.r0[i];
            if (held) r = 0.f;
            out = held ? (DC ? 0.f : q.s_eq) : s_c + q.dt * r;
            if (RES) {
              const double rd = (double)r;
              acc[0] += rd * rd;
              acc[2] += rd;
              if (!DC) {
                const double od = (double)out;
                if (!(od >= q.lo && od <= q.hi)) acc[1] += 1.0;
              } else if (!isfinite(rd)) {
                acc[1] += 1.0;
              }
            }
          }
          s_new[i] = out;
          s_dn = s_c;
          s_c = s_up;
          wz_c = wz_u;
        }
      }
    }
    if (RES) block_store<NV>(acc, 0u, partial + (long long)NV * t);
  }
}

// Batched two-sweep launches, correction form, no activity field: persistent blocks (one per
// CU) take the items of the work list of (problem, tile) items one at a time from a counter
// in device memory; each item is one tile march of the two-sweep kernel on its problem,
// whose residual partials go to the item's tile number.  Items differ in cost (tile shapes
// and z chunks differ between problems), so taking them as blocks free up keeps every CU
// busy until the list runs out, where contiguous runs per block left the last runs alone
// (3.62 s against 4.58 s for the 48-problem benchmark batch).  grab[0] is the next item,
// grab[1] the blocks done; the last block to finish resets both to zero for the next
// launch (every block's last take precedes its count in grab[1]).
template <bool RES>
__global__ void __launch_bounds__(1024) k_batch_sweep2(const BatchProb *__restrict__ probs,
                                                      const int *__restrict__ tile_prob,
                                                      const int *__restrict__ work,
                                                      const int *__restrict__ nwork,
                                                      int *__restrict__ grab, int parity,
                                                      double *__restrict__ partial) {
  // LDS for the largest item shape (two cells per lane); every (w, rx) shape uses a view of
  // the same arrays
  __shared__ float lds[2 * 1024 * 2];
  __shared__ float4 qlds[2 * 4 * 64 * T2_ROWS];
  const int nw = *nwork;
  __shared__ int next;
  const int tid = threadIdx.x + 64 * threadIdx.y;
  for (;;) {
    if (tid == 0) next = atomicAdd(grab, 1);
    __syncthreads();
    const int w = next;
    __syncthreads();
    if (w >= nw) break;
    const int t = work[w];
    const BatchProb &q = probs[tile_prob[t]];
    SweepArgs<float> a;
    a.g = Grid{q.nx, q.ny, q.nz, (long long)q.nx * q.ny * q.nz};
    a.flags = q.flags;
    a.w = Faces<float>{q.wx, q.wy, q.wz, q.wxo};
    a.kappa = nullptr;
    a.s = parity ? q.s1 : q.s0;
    a.s_new = parity ? q.s0 : q.s1;
    a.r0 = q.r0;
    a.dt = q.dt;
    a.s_in = 0.f;
    a.s_eq = 0.f;
    a.Da = q.Da;
    a.gscale = 0.f;
    a.pinned = q.pinned;
    a.lo = q.lo;
    a.hi = q.hi;
    a.partial = nullptr;
    a.zc = q.zc;
    double *pp = RES ? partial + (long long)NV * t : nullptr;
    const int lt = t - q.tile0;
    auto item = [&](auto wc, auto rxc) {
      constexpr int W = decltype(wc)::value, RX = decltype(rxc)::value;
      sweep2_tile<true, RES, false, false, W, RX>(
          a, q.gx, q.gy, lt, reinterpret_cast<float (*)[1024 / RX][RX * W]>(lds),
          reinterpret_cast<float4 (*)[2 * W][64 * T2_ROWS]>(qlds), pp);
    };
    using I2 = std::integral_constant<int, 2>;
    using I1 = std::integral_constant<int, 1>;
    using R64 = std::integral_constant<int, 64>;
    using R32 = std::integral_constant<int, 32>;
    if (q.w == 2) {
      if (q.rx == 32) item(I2{}, R32{});
      else item(I2{}, R64{});
    } else {
      if (q.rx == 32) item(I1{}, R32{});
      else item(I1{}, R64{});
    }
  }
  if (tid == 0) {
    __threadfence();
    if (atomicAdd(grab + 1, 1) == (int)gridDim.x - 1) {
      grab[0] = 0;
      grab[1] = 0;
      __threadfence();
    }
  }
}

void launch_batch_sweep2(const BatchProb *probs, const int *tile_prob, const int *work,
                         const int *nwork, int *grab, int nblocks, int parity, double *partial,
                         hipStream_t st) {
  dim3 block(64, T2_ROWS, 1);
  if (partial)
    k_batch_sweep2<true><<<nblocks, block, 0, st>>>(probs, tile_prob, work, nwork, grab, parity,
                                                   partial);
  else
    k_batch_sweep2<false><<<nblocks, block, 0, st>>>(probs, tile_prob, work, nwork, grab, parity,
                                                    partial);
}

// out[p * NV + k] = sum over problem p's tiles of partial[tile * NV + k], fixed order
__global__ void __launch_bounds__(256) k_batch_reduce(const BatchProb *__restrict__ probs,
                                                     const double *__restrict__ partial,
                                                     double *__restrict__ out) {
  __shared__ double sh[256];
  const BatchProb &q = probs[blockIdx.x];
  const int ntile = q.gx * q.gy * q.gz;
  for (int k = 0; k < NV; ++k) {
    double acc = 0.0;
    for (int j = threadIdx.x; j < ntile; j += 256) acc += partial[(long long)NV * (q.tile0 + j) + k];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[(long long)NV * blockIdx.x + k] = sh[0];
    __syncthreads();
  }
}

void launch_batch_sweep(const BatchProb *probs, const int *tile_prob, const int *work,
                        const int *nwork, int nblocks, int ty, int parity, bool dc,
                        double *partial, hipStream_t st) {
  dim3 block(64, ty, 1);
  if (dc) {
    if (partial) k_batch_sweep<true, true><<<nblocks, block, 0, st>>>(probs, tile_prob, work, nwork, parity, partial);
    else k_batch_sweep<true, false><<<nblocks, block, 0, st>>>(probs, tile_prob, work, nwork, parity, partial);
  } else {
    if (partial) k_batch_sweep<false, true><<<nblocks, block, 0, st>>>(probs, tile_prob, work, nwork, parity, partial);
    else k_batch_sweep<false, false><<<nblocks, block, 0, st>>>(probs, tile_prob, work, nwork, parity, partial);
  }
}

void launch_batch_reduce(const BatchProb *probs, int n, const double *partial, double *out,
                         hipStream_t st) {
  k_batch_reduce<<<n, 256, 0, st>>>(probs, partial, out);
}

// ------------------------------------------------------------------------------------
// FP64 plane march: FP64 sweeps, the FP64 refresh of the defect correction, the outputs
// ------------------------------------------------------------------------------------

// Blocks of 64 x M64_ROWS lanes, W consecutive x cells per lane (W = 2 for even nx, which
// makes every row start 16-byte aligned; 1 for odd nx), each block marching a chunk of z.
// A lane keeps the state of planes j-1 and j in registers and loads plane j+1; rows y-1 and
// y+1 are loads that the block's neighbouring rows fetch too (cache hits); x neighbours come
// from the adjacent lanes by DPP shifts, and the wave's edge lanes load theirs.  Small blocks
// give many waves per CU to hide the load latency.  The per-cell
// arithmetic is residual<double>, the same as every other FP64 kernel's.
constexpr int M64_ROWS = 4;

template <int W>
struct DW {
  double v[W];
};

typedef double d2v __attribute__((ext_vector_type(2)));

template <int W>
__device__ __forceinline__ DW<W> ldd(const double *p) {
  DW<W> r;
  if constexpr (W == 2) {
    const d2v t = *(GMEM const d2v *)p;
    r.v[0] = t.x; r.v[1] = t.y;
  } else {
    r.v[0] = *(GMEM const double *)p;
  }
  return r;
}

template <int W>
__device__ __forceinline__ void std2(double *p, const DW<W> &r) {
  if constexpr (W == 2) {
    d2v t;
    t.x = r.v[0]; t.y = r.v[1];
    *(GMEM d2v *)p = t;
  } else {
    *(GMEM double *)p = r.v[0];
  }
}

// s64 + delta at W cells (delta nullable), the state the refresh evaluates
template <int W, bool DELTA>
__device__ __forceinline__ DW<W> ldstate(const double *s, const float *d, long long i) {
  DW<W> r = ldd<W>(s + i);
  if (DELTA) {
    const VecW<W> e = ldw<W>(d + i);
#pragma unroll
    for (int k = 0; k < W; ++k) r.v[k] += (double)e.v[k];
  }
  return r;
}

// 64-bit lane shifts: lane i receives lane i-1's value (from below) or lane i+1's (from
// above), as two 32-bit DPP moves; the wave's first / last lane receives 0.
__device__ __forceinline__ double dlane_from_below(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x138, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double dlane_from_above(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x130, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

enum { M64_SWEEP = 0, M64_REFRESH = 1, M64_OUTPUTS = 2 };

// Arguments of every FP64 march kernel (the fields an operation does not use are unset).
struct March64Args {
  Grid g;
  const uint8_t *flags;
  Faces<double> w;
  const float *kappa;
  const double *s;      // state (refresh: base state s64)
  const float *delta;   // refresh: FP32 correction added to s (nullable)
  double *s_new;        // sweep: s + dt R; refresh: s + delta (held cells s_eq)
  float *r0;            // refresh: R(s + delta) in FP32
  double dt, s_in, s_eq, Da;
  int pinned;
  double lo, hi;        // bound check on the written state
  double *partial;      // per block: sweep / refresh NV values, outputs NV2 values
  int zc;
  const int *gate;      // nullable: run only if *gate == gate_val
  int gate_val;
  const int *sel;       // nullable: s = pair[*sel], s_new = pair[*sel ^ 1]
  double *pair[2];
};

template <int OP>
struct M64Acc {
  static constexpr int K = OP == M64_OUTPUTS ? NV2 : NV;
};

// OP = M64_SWEEP: s_new = s + dt R(s) (held cells s_eq); with RES the partials
// [sum R^2, cells out of bounds, sum R, -] over updated cells.
// OP = M64_REFRESH: t = s + delta; s_new = t (held cells s_eq); r0 = R(t) in FP32 (held 0);
// partials as for the sweep (RES always).
// OP = M64_OUTPUTS: partials [sum_out w s, sum_out w, F_in, F_in_adv, reaction, sum R,
// sum R^2, -] of the state s (as the outputs entry points document).
// One block of the march: block (bx, by, bz) of the grid, its partials (RES, OUTPUTS) to part.
template <int W, int OP, bool RES, bool DELTA>
__device__ __forceinline__ void march64_block(const March64Args &a, int bx, int by, int bz,
                                              double *part) {
  constexpr int K = M64Acc<OP>::K;
  const Grid g = a.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int lane = threadIdx.x;
  const int x = bx * (64 * W) + W * lane;
  const int y = by * M64_ROWS + threadIdx.y;
  const int z0 = bz * a.zc;
  const int z1 = min(z0 + a.zc, nz);
  const bool act = x < nx && y < ny;
  const bool yl = y > 0, yr = y < ny - 1;
  const bool last = x + W >= nx;         // this lane holds the outlet cell
  const long long pl = (long long)nx * ny;
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  DW<W> sc, sdn, wzc;
#pragma unroll
  for (int k = 0; k < W; ++k) sc.v[k] = sdn.v[k] = wzc.v[k] = 0.0;
  long long i = act ? x + (long long)nx * (y + (long long)ny * z0) : 0;
  if (act) {
    sc = ldstate<W, DELTA>(a.s, a.delta, i);
    if (z0 > 0) sdn = ldstate<W, DELTA>(a.s, a.delta, i - pl);
    wzc = ldd<W>(a.w.wz + i);
  }
  for (int z = z0; z < z1; ++z, i += pl) {
    const bool up = z + 1 < nz;
    DW<W> sup, sym, syp, wx, wym, wyp, wzu;
    VecW<W> kap;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      sup.v[k] = sym.v[k] = syp.v[k] = wx.v[k] = wym.v[k] = wyp.v[k] = wzu.v[k] = 0.0;
      kap.v[k] = 1.f;
    }
    unsigned fl = 0u;
    if (act) {
      if (up) {
        sup = ldstate<W, DELTA>(a.s, a.delta, i + pl);
        wzu = ldd<W>(a.w.wz + i + pl);
      }
      if (yl) sym = ldstate<W, DELTA>(a.s, a.delta, i - nx);
      if (yr) {
        syp = ldstate<W, DELTA>(a.s, a.delta, i + nx);
        wyp = ldd<W>(a.w.wy + i + nx);
      }
      wx = ldd<W>(a.w.wx + i);
      wym = ldd<W>(a.w.wy + i);
      fl = ldflags<W>(a.flags + i);
      if (a.kappa) kap = ldw<W>(a.kappa + i);
    }
    // x neighbours: the lane below holds x-1, the lane above x+W and the face velocity there
    double left = dlane_from_below(sc.v[W - 1]);
    double right = dlane_from_above(sc.v[0]);
    double wxr = dlane_from_above(wx.v[0]);
    if (act) {
      if (x == 0) left = a.s_in;
      else if (lane == 0) left = ldstate<1, DELTA>(a.s, a.delta, i - 1).v[0];
      if (last) {
        wxr = a.w.wxo[y + (long long)ny * z];
      } else if (lane == 63) {
        right = ldstate<1, DELTA>(a.s, a.delta, i + W).v[0];
        wxr = a.w.wx[i + W];
      }
    }
    DW<W> out;
    VecW<W> rout;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      out.v[k] = 0.0;
      rout.v[k] = 0.f;
      const unsigned f = (fl >> (8 * k)) & 0xffu;
      const int xk = x + k;
      if (!act || !(f & FL_PORE)) continue;
      Cell<double> q;
      q.c = sc.v[k];
      q.zm = sdn.v[k];
      q.zp = up ? sup.v[k] : 0.0;
      q.wzm = wzc.v[k];
      q.wzp = up ? wzu.v[k] : 0.0;
      q.gzm = (z > 0 && !(f & FL_ZM)) ? 1.0 : 0.0;
      q.gzp = (up && !(f & FL_ZP)) ? 1.0 : 0.0;
      const bool xl = xk > 0, xr = xk < nx - 1;
      q.xm = k == 0 ? left : sc.v[k - 1];
      q.xp = xr ? (k == W - 1 ? right : sc.v[k + 1]) : q.c;
      q.ym = yl ? sym.v[k] : 0.0;
      q.yp = yr ? syp.v[k] : 0.0;
      q.wxm = wx.v[k];
      q.wxp = k == W - 1 ? wxr : wx.v[k + 1];
      q.wym = wym.v[k];
      q.wyp = yr ? wyp.v[k] : 0.0;
      q.gxm = xl ? ((f & FL_XM) ? 0.0 : 1.0) : 2.0;
      q.gxp = xr ? ((f & FL_XP) ? 0.0 : 1.0) : 0.0;
      q.gym = (yl && !(f & FL_YM)) ? 1.0 : 0.0;
      q.gyp = (yr && !(f & FL_YP)) ? 1.0 : 0.0;
      const int nf = __popc(f & FL_FIBRE);
      const bool held = a.pinned && nf > 0;
      const double lam = a.Da * (double)kap.v[k] * (double)nf;
      if (OP == M64_OUTPUTS) {
        if (xk == nx - 1) {
          acc[0] += q.wxp * q.c;
          acc[1] += q.wxp;
        }
        if (xk == 0) {
          // upwind: inflow brings s_in, outflow through the inlet carries s_P
          const double adv = fmax(q.wxm, 0.0) * a.s_in + fmin(q.wxm, 0.0) * q.c;
          acc[2] += adv + 2.0 * (a.s_in - q.c);
          acc[3] += adv;
        }
        if (held) {
          acc[4] += residual<double>(q, 0.0, a.s_eq);     // absorbed by the electrode cell
        } else {
          const double r = residual<double>(q, lam, a.s_eq);
          acc[4] += lam * (q.c - a.s_eq);
          acc[5] += r;
          acc[6] += r * r;
        }
      } else {
        const double r = held ? 0.0 : residual<double>(q, lam, a.s_eq);
        out.v[k] = held ? a.s_eq : (OP == M64_SWEEP ? q.c + a.dt * r : q.c);
        rout.v[k] = (float)r;
        if (RES && !held) {
          acc[0] += r * r;
          acc[2] += r;
        }
        if (RES && !(out.v[k] >= a.lo && out.v[k] <= a.hi)) acc[1] += 1.0;
      }
    }
    if (OP != M64_OUTPUTS && act) {
      std2<W>(a.s_new + i, out);
      if (OP == M64_REFRESH) stw<W>(a.r0 + i, rout);
    }
    sdn = sc;
    sc = sup;
    wzc = wzu;
  }
  if (RES || OP == M64_OUTPUTS) block_store<K>(acc, 0u, part);
}

template <int W, int OP, bool RES, bool DELTA>
__global__ void __launch_bounds__(64 * M64_ROWS) k_march64(March64Args a, int gx, int gy,
                                                             int gz) {
  if (a.gate && *a.gate != a.gate_val) return;
  if (a.sel) {
    const int c = *a.sel;
    a.s = a.pair[c];
    a.s_new = a.pair[c ^ 1];
  }
  const int L = xcd_tile(blockIdx.x, gx * gy * gz);
  march64_block<W, OP, RES, DELTA>(
      a, L % gx, (L / gx) % gy, L / (gx * gy),
      RES || OP == M64_OUTPUTS ? a.partial + (long long)M64Acc<OP>::K * blockIdx.x : nullptr);
}

// Blocks of the march resident at once on the chip: 256 CUs x 3 blocks of four waves (the
// occupancy of the FP64 epilogues, three waves per SIMD).
constexpr int M64_RESIDENT = 768;

// z chunk of the march: the power of two from 128 planes down with the lowest
// (rounds of resident blocks) x (planes a block marches + 8), the 8 standing for a block's
// start (the plane below re-read, the first plane's loads with nothing to overlap them).
// Measured per FP64 sweep, against halving the chunk while the grid had under 2048 blocks:
// 1024x512x256 1.19 ms either way (128 planes), 256x128x128 39 us against 54, 175x89x89
// 30 us against 48, 96x78x78 15 us against 19.5, 64x32x32 7.4 us either way (2 planes).
static int march64_zc(const Grid &g) {
  const int W = (g.nx & 1) ? 1 : 2;
  const long long gxy = (long long)((g.nx + 64 * W - 1) / (64 * W)) * ((g.ny + M64_ROWS - 1) / M64_ROWS);
  int best = 128;
  long long best_cost = -1;
  for (int zc = 128; zc >= 2; zc /= 2) {
    const long long blocks = gxy * ((g.nz + zc - 1) / zc);
    const long long cost =
        (blocks + M64_RESIDENT - 1) / M64_RESIDENT * (std::min(zc, g.nz) + 8);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = zc;
    }
  }
  return best;
}

static dim3 march64_grid(const Grid &g, int zc) {
  const int W = (g.nx & 1) ? 1 : 2;
  return dim3((unsigned)((g.nx + 64 * W - 1) / (64 * W)),
              (unsigned)((g.ny + M64_ROWS - 1) / M64_ROWS), (unsigned)((g.nz + zc - 1) / zc));
}

int march64_blocks(const Grid &g) {
  const dim3 d = march64_grid(g, march64_zc(g));
  return (int)(d.x * d.y * d.z);
}

template <int OP, bool RES, bool DELTA>
static void launch_march64(March64Args a, hipStream_t st) {
  a.zc = march64_zc(a.g);
  const dim3 d = march64_grid(a.g, a.zc);
  const unsigned nb = d.x * d.y * d.z;
  const dim3 block(64, M64_ROWS, 1);
  if (a.g.nx & 1) k_march64<1, OP, RES, DELTA><<<nb, block, 0, st>>>(a, d.x, d.y, d.z);
  else k_march64<2, OP, RES, DELTA><<<nb, block, 0, st>>>(a, d.x, d.y, d.z);
}

void launch_sweep64(const SweepArgs<double> &s, hipStream_t st) {
  March64Args a{};
  a.g = s.g; a.flags = s.flags; a.w = s.w; a.kappa = s.kappa;
  a.s = s.s; a.s_new = s.s_new; a.dt = s.dt; a.s_in = s.s_in; a.s_eq = s.s_eq; a.Da = s.Da;
  a.pinned = s.pinned; a.lo = s.lo; a.hi = s.hi; a.partial = s.partial;
  if (s.partial) launch_march64<M64_SWEEP, true, false>(a, st);
  else launch_march64<M64_SWEEP, false, false>(a, st);
}

// Batched FP64 sweeps: one block per (problem, march block) item over every problem of the
// table; item w belongs to problem item_prob[w] and is its block w - blk0.  Each problem's
// buffers alternate with the launch parity (s = pair[c0 ^ parity]).  With RES the partials
// [sum R^2, cells out of bounds, sum R, -] of item w go to partial[NV w].
template <bool RES>
__global__ void __launch_bounds__(64 * M64_ROWS) k_batch_march64(const BatchM64 *__restrict__ probs,
                                                                 const int *__restrict__ item_prob,
                                                                 int parity,
                                                                 double *__restrict__ partial) {
  const int w = blockIdx.x;
  const BatchM64 &q = probs[item_prob[w]];
  March64Args a{};
  a.g = q.a.g;
  a.flags = q.a.flags;
  a.w = q.a.w;
  a.kappa = q.a.kappa;
  a.s = q.pair[q.c0 ^ parity];
  a.s_new = q.pair[q.c0 ^ parity ^ 1];
  a.dt = q.a.dt;
  a.s_in = q.a.s_in;
  a.s_eq = q.a.s_eq;
  a.Da = q.a.Da;
  a.pinned = q.a.pinned;
  a.lo = q.a.lo;
  a.hi = q.a.hi;
  a.zc = q.zc;
  const int L = w - q.blk0;
  const int bx = L % q.gx, by = (L / q.gx) % q.gy, bz = L / (q.gx * q.gy);
  double *part = RES ? partial + (long long)NV * w : nullptr;
  if (q.a.g.nx & 1) march64_block<1, M64_SWEEP, RES, false>(a, bx, by, bz, part);
  else march64_block<2, M64_SWEEP, RES, false>(a, bx, by, bz, part);
}

// out[NV p] = sums of problem p's item partials (items blk0 .. blk0 + nblk - 1), fixed order
__global__ void __launch_bounds__(256) k_batch_march64_reduce(const BatchM64 *__restrict__ probs,
                                                              const double *__restrict__ partial,
                                                              double *__restrict__ out) {
  __shared__ double sh[256];
  const BatchM64 &q = probs[blockIdx.x];
  const int nb = q.gx * q.gy * q.gz;
  for (int k = 0; k < NV; ++k) {
    double acc = 0.0;
    for (int j = threadIdx.x; j < nb; j += 256) acc += partial[(long long)NV * (q.blk0 + j) + k];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
      if (threadIdx.x < s2) sh[threadIdx.x] += sh[threadIdx.x + s2];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[(long long)NV * q.prob + k] = sh[0];
    __syncthreads();
  }
}

void march64_shape(const Grid &g, int &gx, int &gy, int &gz, int &zc) {
  zc = march64_zc(g);
  const dim3 d = march64_grid(g, zc);
  gx = (int)d.x;
  gy = (int)d.y;
  gz = (int)d.z;
}

void launch_batch_march64(const BatchM64 *probs, int nprob, const int *item_prob, int nitems,
                          int parity, double *partial, double *out, hipStream_t st) {
  const dim3 block(64, M64_ROWS, 1);
  if (partial) {
    k_batch_march64<true><<<nitems, block, 0, st>>>(probs, item_prob, parity, partial);
    k_batch_march64_reduce<<<nprob, 256, 0, st>>>(probs, partial, out);
  } else {
    k_batch_march64<false><<<nitems, block, 0, st>>>(probs, item_prob, parity, nullptr);
  }
}

void launch_refresh(const RefreshArgs &r, const Tiles &, hipStream_t st) {
  March64Args a{};
  a.g = r.g; a.flags = r.flags; a.w = r.w; a.kappa = r.kappa;
  a.s = r.s64; a.delta = r.delta; a.s_new = r.s64_new; a.r0 = r.r0;
  a.s_in = r.s_in; a.s_eq = r.s_eq; a.Da = r.Da; a.pinned = r.pinned; a.lo = r.lo; a.hi = r.hi;
  a.partial = r.partial;
  if (r.delta) launch_march64<M64_REFRESH, true, true>(a, st);
  else launch_march64<M64_REFRESH, true, false>(a, st);
}

void launch_refresh_gated(const RefreshArgs &r, double *s64_0, double *s64_1,
                          const SolveCtl *ctl, hipStream_t st) {
  March64Args a{};
  a.g = r.g; a.flags = r.flags; a.w = r.w; a.kappa = r.kappa;
  a.delta = r.delta; a.r0 = r.r0;
  a.s_in = r.s_in; a.s_eq = r.s_eq; a.Da = r.Da; a.pinned = r.pinned; a.lo = r.lo; a.hi = r.hi;
  a.partial = r.partial;
  a.gate = &ctl->state;
  a.gate_val = CTL_REFRESH;
  a.sel = &ctl->cur;
  a.pair[0] = s64_0;
  a.pair[1] = s64_1;
  if (r.delta) launch_march64<M64_REFRESH, true, true>(a, st);
  else launch_march64<M64_REFRESH, true, false>(a, st);
}

// ---- device-side control of the FP32 correction solve ---------------------------------

// sums of partial values 0 (sum R^2) and 1 (violations) over nblk blocks, fixed order;
// every thread returns them
__device__ __forceinline__ void ctl_sums(const double *__restrict__ partial, int nblk,
                                         double &ss, double &viol) {
  __shared__ double sh[2][256];
  double a = 0.0, b = 0.0;
  for (int j = threadIdx.x; j < nblk; j += 256) {
    a += partial[(long long)NV * j];
    b += partial[(long long)NV * j + 1];
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  ss = sh[0][0];
  viol = sh[1][0];
}

// After a chunk of k correction sweeps whose last launch summed ss = sum R^2 and viol
// (non-finite cells): the correction residual tau rms(r0 - A delta), then the cycle's end
// test (target reached, max_iter, or no 0.1% decrease in 8 chunks).
__device__ void ctl_after_chunk(SolveCtl *ctl, double ss, double viol, int k) {
  ctl->fill = 0;
  ctl->it += k;
  const double ri = ctl->tau * sqrt(ss / ctl->npore);
  ctl->ri = ri;
  if (!isfinite(ri) || viol > 0.0) {
    ctl->state = CTL_DIVERGED;
    return;
  }
  bool refresh = ri < ctl->target || ctl->it >= ctl->max_iter;
  if (!refresh) {
    if (ri < 0.999 * ctl->best) {
      ctl->best = ri;
      ctl->stall = 0;
    } else if (++ctl->stall >= 8) {
      refresh = true;
    }
  }
  if (refresh) ctl->state = CTL_REFRESH;
}

// After the refresh (ss, viol of the FP64 residual of s64 + delta): the solve's stop rule
// (Eq. (convergence-bv-change)) and the next cycle's target.
__device__ void ctl_after_refresh(SolveCtl *ctl, double ss, double viol) {
  const double res = ctl->tau * sqrt(ss / ctl->npore);
  ctl->res = res;
  ctl->cycles += 1;
  ctl->cur ^= 1;
  if (!isfinite(res) || viol > 0.0) {
    ctl->state = CTL_DIVERGED;
  } else if (res < ctl->tol) {
    ctl->state = CTL_DONE;
  } else if (ctl->it >= ctl->max_iter) {
    ctl->state = CTL_STOP;
  } else {
    ctl->target = fmax(ctl->tol, ctl->reduction * res);
    ctl->best = INFINITY;
    ctl->stall = 0;
    ctl->fill = 1;
    ctl->state = CTL_RUN;
  }
}

__global__ void __launch_bounds__(256) k_ctl_chunk(SolveCtl *ctl, const double *partial,
                                                   int nblk, int k) {
  if (ctl->state != CTL_RUN) return;
  double ss, viol;
  ctl_sums(partial, nblk, ss, viol);
  if (threadIdx.x == 0) ctl_after_chunk(ctl, ss, viol, k);
}

__global__ void __launch_bounds__(256) k_ctl_refresh(SolveCtl *ctl, const double *partial,
                                                     int nblk) {
  if (ctl->state != CTL_REFRESH) return;
  double ss, viol;
  ctl_sums(partial, nblk, ss, viol);
  if (threadIdx.x == 0) ctl_after_refresh(ctl, ss, viol);
}

// ---- the batched solve's loop on the device -------------------------------------------

// Work lists of the problems still sweeping (state CTL_RUN): the tile numbers of every such
// problem, two-sweep items at work[0..] and single-sweep items at work[max_tiles..], their
// counts at nwork[0] and nwork[1].  One block; problems in order, tiles in order.
__global__ void __launch_bounds__(256) k_batch_worklist(const BatchProb *__restrict__ probs,
                                                        int n, int *__restrict__ work,
                                                        int max_tiles, int *__restrict__ nwork) {
  int m[2] = {0, 0};
  for (int i = 0; i < n; ++i) {
    const BatchProb &q = probs[i];
    if (q.ctl->state != CTL_RUN) continue;
    const int path = q.two ? 0 : 1;
    const int nt = q.gx * q.gy * q.gz;
    int *dst = work + (long long)path * max_tiles + m[path];
    for (int t = threadIdx.x; t < nt; t += 256) dst[t] = q.tile0 + t;
    m[path] += nt;
  }
  if (threadIdx.x == 0) {
    nwork[0] = m[0];
    nwork[1] = m[1];
  }
}

// Zero the corrections of the problems that start a cycle (ctl->fill); 16 blocks per problem.
__global__ void __launch_bounds__(256) k_batch_fill_gated(const BatchProb *__restrict__ probs) {
  const BatchProb &q = probs[blockIdx.x / 16];
  if (!q.ctl->fill) return;
  const long long nc = (long long)q.nx * q.ny * q.nz;
  for (long long i = (blockIdx.x % 16) * 256ll + threadIdx.x; i < nc; i += 16 * 256ll) {
    q.s0[i] = 0.f;
    q.s1[i] = 0.f;
  }
}

// After a chunk of k sweeps: each sweeping problem's decision from its reduced partials
// out[NV i ..] (k_batch_reduce); one thread per problem.
__global__ void __launch_bounds__(64) k_batch_ctl_chunk(const BatchProb *__restrict__ probs,
                                                        const double *__restrict__ out, int n,
                                                        int k) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= n || probs[i].ctl->state != CTL_RUN) return;
  ctl_after_chunk(probs[i].ctl, out[(long long)NV * i], out[(long long)NV * i + 1], k);
}

// After the (gated, per-problem) refreshes: block i applies problem i's stop rule from its
// refresh partials.
__global__ void __launch_bounds__(256) k_batch_ctl_refresh(const BatchProb *__restrict__ probs) {
  const BatchProb &q = probs[blockIdx.x];
  if (q.ctl->state != CTL_REFRESH) return;
  double ss, viol;
  ctl_sums(q.rpart, q.rnblk, ss, viol);
  if (threadIdx.x == 0) ctl_after_refresh(q.ctl, ss, viol);
}

void launch_batch_control(const BatchProb *probs, int n, int *work, int max_tiles, int *nwork,
                          int which, const double *out, int k, hipStream_t st) {
  switch (which) {
    case BATCH_WORKLIST:
      k_batch_worklist<<<1, 256, 0, st>>>(probs, n, work, max_tiles, nwork);
      break;
    case BATCH_FILL:
      k_batch_fill_gated<<<16 * n, 256, 0, st>>>(probs);
      break;
    case BATCH_CHUNK:
      k_batch_ctl_chunk<<<(n + 63) / 64, 64, 0, st>>>(probs, out, n, k);
      break;
    default:
      k_batch_ctl_refresh<<<n, 256, 0, st>>>(probs);
      break;
  }
}

void launch_ctl_chunk(SolveCtl *ctl, const double *partial, int nblk, int k, hipStream_t st) {
  k_ctl_chunk<<<1, 256, 0, st>>>(ctl, partial, nblk, k);
}

void launch_ctl_refresh(SolveCtl *ctl, const double *partial, int nblk, hipStream_t st) {
  k_ctl_refresh<<<1, 256, 0, st>>>(ctl, partial, nblk);
}

int outputs_blocks(const Grid &g) { return march64_blocks(g); }

void launch_outputs(const Grid &g, const uint8_t *flags, Faces<double> w, const float *kappa,
                    const double *s, double s_in, double s_eq, double Da, int pinned,
                    double *partial, int nblk, hipStream_t st) {
  (void)nblk;
  March64Args a{};
  a.g = g; a.flags = flags; a.w = w; a.kappa = kappa; a.s = s;
  a.s_in = s_in; a.s_eq = s_eq; a.Da = Da; a.pinned = pinned; a.partial = partial;
  launch_march64<M64_OUTPUTS, false, false>(a, st);
}

// ------------------------------------------------------------------------------------
// Time-step bound
// ------------------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_maxdiag(Grid g, const uint8_t *__restrict__ flags,
                                                 Faces<double> w, const float *kappa,
                                                 double Da, int pinned, double *partial) {
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  double v[1] = {0.0};
  if (i < g.n) {
    const uint8_t f = flags[i];
    if (f & FL_PORE) {
      const int nx = g.nx, ny = g.ny;
      const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((long long)nx * ny));
      const int nf = __popc((unsigned)(f & FL_FIBRE));
      if (!(pinned && nf > 0)) {
        const long long pl = (long long)nx * ny;
        const bool xr = x < nx - 1, yr = y < ny - 1, zr = z < g.nz - 1;
        double d = Da * (kappa ? (double)kappa[i] : 1.0) * nf;
        d += fmax(-w.wx[i], 0.0) + fmax(xr ? w.wx[i + 1] : w.wxo[y + (long long)ny * z], 0.0);
        d += fmax(-w.wy[i], 0.0) + fmax(yr ? w.wy[i + nx] : 0.0, 0.0);
        d += fmax(-w.wz[i], 0.0) + fmax(zr ? w.wz[i + pl] : 0.0, 0.0);
        d += (x > 0) ? ((f & FL_XM) ? 0.0 : 1.0) : 2.0;
        d += (xr && !(f & FL_XP)) ? 1.0 : 0.0;
        d += (y > 0 && !(f & FL_YM)) ? 1.0 : 0.0;
        d += (yr && !(f & FL_YP)) ? 1.0 : 0.0;
        d += (z > 0 && !(f & FL_ZM)) ? 1.0 : 0.0;
        d += (zr && !(f & FL_ZP)) ? 1.0 : 0.0;
        v[0] = d;
      }
    }
  }
  block_store<1>(v, 1u, partial + blockIdx.x);
}

void launch_maxdiag(const Grid &g, const uint8_t *flags, Faces<double> w, const float *kappa,
                    double Da, int pinned, double *partial, int nblk, hipStream_t st) {
  k_maxdiag<<<nblk, 256, 0, st>>>(g, flags, w, kappa, Da, pinned, partial);
}

// ------------------------------------------------------------------------------------
// Adjoint sweeps: psi_new = psi + dt (g - A^T psi)
// ------------------------------------------------------------------------------------

template <typename T, bool DC, bool RES>
__global__ void __launch_bounds__(1024) k_adjoint(AdjointArgs<T> a) {
  const Grid g = a.g;
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z0 = blockIdx.z * a.zc;
  const int z1 = min(z0 + a.zc, g.nz);
  const long long pl = (long long)g.nx * g.ny;
  double acc[NV] = {0, 0, 0, 0};
  if (x < g.nx && y < g.ny && z0 < z1) {
    long long i = x + (long long)g.nx * (y + (long long)g.ny * z0);
    Cell<T> q;
    T p_c = a.psi[i];
    T p_dn = z0 > 0 ? a.psi[i - pl] : T(0);
    T wz_c = a.w.wz[i];
    for (int z = z0; z < z1; ++z, i += pl) {
      const bool up = z + 1 < g.nz;
      const T p_up = up ? a.psi[i + pl] : T(0);
      const T wz_u = up ? a.w.wz[i + pl] : T(0);
      const uint8_t f = a.flags[i];
      T out = T(0);
      if (f & FL_PORE) {
        const int nf = __popc((unsigned)(f & FL_FIBRE));
        const bool held = a.pinned && nf > 0;
        if (!held) {
          q.c = p_c; q.zm = p_dn; q.zp = p_up; q.wzm = wz_c; q.wzp = wz_u;
          q.gzm = (z > 0 && !(f & FL_ZM)) ? T(1) : T(0);
          q.gzp = (up && !(f & FL_ZP)) ? T(1) : T(0);
          load_plane<T>(q, a.psi, a.w, f, g, x, y, z, i, T(0), false);
          const bool outlet = x == g.nx - 1;
          const T lam = a.Da * (a.kappa ? (T)a.kappa[i] : T(1)) * (T)nf;
          T r = -transpose_action<T>(q, lam, outlet);
          if (outlet) r += a.gscale * q.wxp;
          if (DC) r += (T)a.r0[i];
          out = p_c + a.dt * r;
          if (RES) {
            const double rd = (double)r;
            acc[0] += rd * rd;
            if (!isfinite(rd)) acc[1] += 1.0;
          }
        }
      }
      a.psi_new[i] = out;
      p_dn = p_c;
      p_c = p_up;
      wz_c = wz_u;
    }
  }
  if (RES) block_store<NV>(acc, 0u, a.partial + (long long)NV * (blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)));
}

template <typename T>
void launch_adjoint(const AdjointArgs<T> &a, const Tiles &t, hipStream_t st) {
  dim3 grid = sweep_grid(a.g, t), block(64, t.ty, 1);
  const bool dc = a.r0 != nullptr, res = a.partial != nullptr;
  if (dc) {
    if (res) k_adjoint<T, true, true><<<grid, block, 0, st>>>(a);
    else k_adjoint<T, true, false><<<grid, block, 0, st>>>(a);
  } else {
    if (res) k_adjoint<T, false, true><<<grid, block, 0, st>>>(a);
    else k_adjoint<T, false, false><<<grid, block, 0, st>>>(a);
  }
}
template void launch_adjoint<float>(const AdjointArgs<float> &, const Tiles &, hipStream_t);
template void launch_adjoint<double>(const AdjointArgs<double> &, const Tiles &, hipStream_t);

__global__ void __launch_bounds__(1024) k_adj_refresh(AdjRefreshArgs a) {
  const Grid g = a.g;
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z0 = blockIdx.z * a.zc;
  const int z1 = min(z0 + a.zc, g.nz);
  const long long pl = (long long)g.nx * g.ny;
  double acc[NV] = {0, 0, 0, 0};
  if (x < g.nx && y < g.ny && z0 < z1) {
    const int nx = g.nx, ny = g.ny;
    const bool xl = x > 0, xr = x < nx - 1, yl = y > 0, yr = y < ny - 1;
    const float *d = a.delta;
    auto val = [&](long long j) -> double { return a.psi64[j] + (d ? (double)d[j] : 0.0); };
    long long i = x + (long long)nx * (y + (long long)ny * z0);
    double p_c = val(i);
    double p_dn = z0 > 0 ? val(i - pl) : 0.0;
    double wz_c = a.w.wz[i];
    for (int z = z0; z < z1; ++z, i += pl) {
      const bool up = z + 1 < g.nz;
      const double p_up = up ? val(i + pl) : 0.0;
      const double wz_u = up ? a.w.wz[i + pl] : 0.0;
      const uint8_t f = a.flags[i];
      double nv = 0.0;
      float r0 = 0.0f;
      if (f & FL_PORE) {
        const int nf = __popc((unsigned)(f & FL_FIBRE));
        const bool held = a.pinned && nf > 0;
        if (!held) {
          Cell<double> q;
          q.c = p_c; q.zm = p_dn; q.zp = p_up; q.wzm = wz_c; q.wzp = wz_u;
          q.gzm = (z > 0 && !(f & FL_ZM)) ? 1.0 : 0.0;
          q.gzp = (up && !(f & FL_ZP)) ? 1.0 : 0.0;
          q.xm = xl ? val(i - 1) : 0.0;
          q.xp = xr ? val(i + 1) : 0.0;
          q.ym = yl ? val(i - nx) : 0.0;
          q.yp = yr ? val(i + nx) : 0.0;
          q.wxm = a.w.wx[i];
          q.wxp = xr ? a.w.wx[i + 1] : a.w.wxo[y + (long long)ny * z];
          q.wym = a.w.wy[i];
          q.wyp = yr ? a.w.wy[i + nx] : 0.0;
          q.gxm = xl ? ((f & FL_XM) ? 0.0 : 1.0) : 2.0;
          q.gxp = xr ? ((f & FL_XP) ? 0.0 : 1.0) : 0.0;
          q.gym = (yl && !(f & FL_YM)) ? 1.0 : 0.0;
          q.gyp = (yr && !(f & FL_YP)) ? 1.0 : 0.0;
          const double lam = a.Da * (a.kappa ? (double)a.kappa[i] : 1.0) * (double)nf;
          const bool outlet = x == nx - 1;
          double r = -transpose_action<double>(q, lam, outlet);
          if (outlet) r += a.gscale * q.wxp;
          nv = p_c;
          r0 = (float)r;
          acc[0] += r * r;
          if (!isfinite(r)) acc[1] += 1.0;
        }
      }
      a.psi64_new[i] = nv;
      a.r0[i] = r0;
      p_dn = p_c;
      p_c = p_up;
      wz_c = wz_u;
    }
  }
  block_store<NV>(acc, 0u, a.partial + (long long)NV * (blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)));
}

void launch_adj_refresh(const AdjRefreshArgs &a, const Tiles &t, hipStream_t st) {
  k_adj_refresh<<<sweep_grid(a.g, t), dim3(64, t.ty, 1), 0, st>>>(a);
}

// ------------------------------------------------------------------------------------
// Gradients from the adjoint state
// ------------------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_gradients(Grid g, const uint8_t *__restrict__ flags,
                                                   Faces<double> w, const double *__restrict__ s,
                                                   const double *__restrict__ psi, double s_in,
                                                   double s_eq, double Da, int pinned,
                                                   double *dU_dkappa, double *partial) {
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  double v[NV] = {0, 0, 0, 0};
  if (i < g.n) {
    const uint8_t f = flags[i];
    double gk = 0.0;
    if (f & FL_PORE) {
      const int nf = __popc((unsigned)(f & FL_FIBRE));
      const bool held = pinned && nf > 0;
      if (!held) {
        const int nx = g.nx, ny = g.ny;
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((long long)nx * ny));
        const long long pl = (long long)nx * ny;
        const bool up = z + 1 < g.nz;
        Cell<double> q;
        q.c = s[i];
        q.zm = z > 0 ? s[i - pl] : 0.0;
        q.zp = up ? s[i + pl] : 0.0;
        q.wzm = w.wz[i];
        q.wzp = up ? w.wz[i + pl] : 0.0;
        load_plane<double>(q, s, w, f, g, x, y, z, i, s_in, true);
        // advective residual: every G and the reaction set to zero
        q.gxm = q.gxp = q.gym = q.gyp = q.gzm = q.gzp = 0.0;
        q.gzm = 0.0;
        const double radv = residual<double>(q, 0.0, s_eq);
        v[0] = psi[i] * radv;
        if (!pinned && nf > 0) gk = Da * (double)nf * psi[i] * (s_eq - q.c);
      }
    }
    if (dU_dkappa) dU_dkappa[i] = gk;
  }
  block_store<NV>(v, 0u, partial + (long long)NV * blockIdx.x);
}

void launch_gradients(const Grid &g, const uint8_t *flags, Faces<double> w, const double *s,
                      const double *psi, double s_in, double s_eq, double Da, int pinned,
                      double *dU_dkappa, double *partial, int nblk, hipStream_t st) {
  k_gradients<<<nblk, 256, 0, st>>>(g, flags, w, s, psi, s_in, s_eq, Da, pinned, dU_dkappa,
                                    partial);
}

// ------------------------------------------------------------------------------------
// Small helpers
// ------------------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(256) k_fill(T *p, long long n, T v) {
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) p[i] = v;
}

// ------------------------------------------------------------------------------------
// Static scratch of the allocation-free entry point
// ------------------------------------------------------------------------------------

// Per-block partials and reduced values of socfv_evaluate_noalloc, in device memory that the
// code object holds (each GPU its own copy, for the life of the process), so that the call
// needs no allocation.  In host code `scratch` names a host-side stand-in, never the device
// memory: its device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

int scratch_address(int dev, double **out) {
  static std::mutex mu;
  static double *addr[SCRATCH_MAX_DEVICES] = {};
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return (int)e;
    if (cur != dev) return (int)hipErrorInvalidDevice;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    addr[dev] = static_cast<double *>(p);
  }
  *out = addr[dev];
  return 0;
}

__global__ void __launch_bounds__(256) k_fill2_gated(float *a, float *b, long long n,
                                                     const SolveCtl *ctl) {
  if (!ctl->fill) return;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
    a[i] = 0.f;
    b[i] = 0.f;
  }
}

static unsigned fill_blocks(long long n) {
  long long b = (n + 255) / 256;
  return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

void launch_fill_gated(float *a, float *b, long long n, const SolveCtl *ctl, hipStream_t st) {
  k_fill2_gated<<<fill_blocks(n), 256, 0, st>>>(a, b, n, ctl);
}

void launch_fill_f32(float *p, long long n, float v, hipStream_t st) {
  k_fill<float><<<fill_blocks(n), 256, 0, st>>>(p, n, v);
}
void launch_fill_f64(double *p, long long n, double v, hipStream_t st) {
  k_fill<double><<<fill_blocks(n), 256, 0, st>>>(p, n, v);
}

// ------------------------------------------------------------------------------------
// Explicit Nernst model (Sec. "Steady State Reaction Model (Nernst)", Algorithm "Explicit
// Nernst Model"; electrode value of Eq. (nernst-model-s-update)), FP64
// ------------------------------------------------------------------------------------

// One iteration: s' = s + dt R_t(s) on pore cells (R_t: advection and diffusion, the
// reaction term left out); on electrode cells eta_I = 2 asinh(-R_t / (2 c sqrt(s (1 - s))))
// (Eq. (nernst-eta-inst-def) with D lap s replaced by the transport rate), c = a k0 =
// Da kappa n_f / K, eta <- (1 - omega) eta + omega eta_I (Eq. (nernst-model-eta-update)) and
// s' = sigma(V - eta).  With RES the partials hold sum ((s' - s) / dt)^2 over pore cells.
template <bool RES>
__global__ void __launch_bounds__(1024) k_nernst(NernstArgs a) {
  const Grid g = a.g;
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z0 = blockIdx.z * a.zc;
  const int z1 = min(z0 + a.zc, g.nz);
  const long long pl = (long long)g.nx * g.ny;
  double acc[NV] = {0, 0, 0, 0};
  if (x < g.nx && y < g.ny && z0 < z1) {
    long long i = x + (long long)g.nx * (y + (long long)g.ny * z0);
    Cell<double> q;
    double s_c = a.s[i];
    double s_dn = z0 > 0 ? a.s[i - pl] : 0.0;
    double wz_c = a.w.wz[i];
    for (int z = z0; z < z1; ++z, i += pl) {
      const bool up = z + 1 < g.nz;
      const double s_up = up ? a.s[i + pl] : 0.0;
      const double wz_u = up ? a.w.wz[i + pl] : 0.0;
      const uint8_t f = a.flags[i];
      double out = 0.0;
      if (f & FL_PORE) {
        q.c = s_c;
        q.zm = s_dn;
        q.zp = s_up;
        q.wzm = wz_c;
        q.wzp = wz_u;
        q.gzm = (z > 0 && !(f & FL_ZM)) ? 1.0 : 0.0;
        q.gzp = (up && !(f & FL_ZP)) ? 1.0 : 0.0;
        load_plane<double>(q, a.s, a.w, f, g, x, y, z, i, a.s_in, true);
        const double r = residual<double>(q, 0.0, 0.0);
        out = s_c + a.dt * r;
        const int nf = __popc((unsigned)(f & FL_FIBRE));
        if (nf > 0) {
          const double c = a.Da * (a.kappa ? (double)a.kappa[i] : 1.0) * (double)nf / a.K;
          const double eta_i = 2.0 * asinh(-r / (2.0 * c * sqrt(s_c * (1.0 - s_c))));
          const double eta = (1.0 - a.omega) * a.eta[i] + a.omega * eta_i;
          a.eta[i] = eta;
          out = 1.0 / (1.0 + exp(eta - a.V));
        }
        if (RES) {
          const double d = (out - s_c) / a.dt;
          acc[0] += d * d;
          if (!isfinite(d)) acc[1] += 1.0;
        }
      }
      a.s_new[i] = out;
      s_dn = s_c;
      s_c = s_up;
      wz_c = wz_u;
    }
  }
  if (RES) block_store<NV>(acc, 0u, a.partial + (long long)NV * (blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)));
}

void launch_nernst(const NernstArgs &a, const Tiles &t, hipStream_t st) {
  dim3 grid = sweep_grid(a.g, t), block(64, t.ty, 1);
  if (a.partial) k_nernst<true><<<grid, block, 0, st>>>(a);
  else k_nernst<false><<<grid, block, 0, st>>>(a);
}

// ------------------------------------------------------------------------------------
// Iterative upsampling: the problem coarsened by two in every direction, and the
// prolongation of its steady state (converge on the unrefined grid, then start the refined
// problem from the interpolated state; Sec. "Incompressible Fluid Flow")
// ------------------------------------------------------------------------------------

// coarse cell fibre iff all eight children are fibre
__global__ void __launch_bounds__(256) k_coarse_mask(Grid g, const uint8_t *__restrict__ flags,
                                                     uint8_t *__restrict__ solid_c) {
  const int nxc = g.nx / 2, nyc = g.ny / 2;
  const long long nc = (long long)nxc * nyc * (g.nz / 2);
  for (long long c = blockIdx.x * 256ll + threadIdx.x; c < nc; c += 256ll * gridDim.x) {
    const int ic = (int)(c % nxc), jc = (int)((c / nxc) % nyc), kc = (int)(c / ((long long)nxc * nyc));
    bool all = true;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int d = 0; d < 2; ++d) {
          const long long i = (2 * ic + d) + (long long)g.nx * ((2 * jc + b) + (long long)g.ny * (2 * kc + a));
          all = all && !(flags[i] & FL_PORE);
        }
    solid_c[c] = all ? 1 : 0;
  }
}

// Coarse staggered face velocities in coarse grid units (h doubled, same physical flux):
// ((v00 + v01) + (v10 + v11)) / 2 over the four fine faces of a coarse face, v_ab with a the
// offset along the slower transverse axis (z for x and y faces, y for z faces) and b along
// the faster one.  Fine faces come from the per-cell lower faces and the outlet faces; the
// top y and z walls carry 0.  One thread per coarse face over ux, then uy, then uz.
__global__ void __launch_bounds__(256) k_restrict(Grid g, Faces<double> w, double *__restrict__ ux_c,
                                                  double *__restrict__ uy_c,
                                                  double *__restrict__ uz_c) {
  const int nx = g.nx, ny = g.ny;
  const int nxc = g.nx / 2, nyc = g.ny / 2, nzc = g.nz / 2;
  const long long nux = (long long)nzc * nyc * (nxc + 1);
  const long long nuy = (long long)nzc * (nyc + 1) * nxc;
  const long long nuz = (long long)(nzc + 1) * nyc * nxc;
  auto at = [&](int x, int y, int z) { return x + (long long)nx * (y + (long long)ny * z); };
  for (long long t = blockIdx.x * 256ll + threadIdx.x; t < nux + nuy + nuz; t += 256ll * gridDim.x) {
    double v[2][2];
    if (t < nux) {
      const int ic = (int)(t % (nxc + 1)), jc = (int)((t / (nxc + 1)) % nyc);
      const int kc = (int)(t / ((long long)(nxc + 1) * nyc));
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          const int y = 2 * jc + b, z = 2 * kc + a;
          v[a][b] = ic < nxc ? w.wx[at(2 * ic, y, z)] : w.wxo[y + (long long)ny * z];
        }
      ux_c[t] = ((v[0][0] + v[0][1]) + (v[1][0] + v[1][1])) * 0.5;
    } else if (t < nux + nuy) {
      const long long u = t - nux;
      const int ic = (int)(u % nxc), jc = (int)((u / nxc) % (nyc + 1));
      const int kc = (int)(u / ((long long)nxc * (nyc + 1)));
      if (jc == nyc) {
        uy_c[u] = 0.0;
        continue;
      }
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) v[a][b] = w.wy[at(2 * ic + b, 2 * jc, 2 * kc + a)];
      uy_c[u] = ((v[0][0] + v[0][1]) + (v[1][0] + v[1][1])) * 0.5;
    } else {
      const long long u = t - nux - nuy;
      const int ic = (int)(u % nxc), jc = (int)((u / nxc) % nyc);
      const int kc = (int)(u / ((long long)nxc * nyc));
      if (kc == nzc) {
        uz_c[u] = 0.0;
        continue;
      }
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) v[a][b] = w.wz[at(2 * ic + b, 2 * jc + a, 2 * kc)];
      uz_c[u] = ((v[0][0] + v[0][1]) + (v[1][0] + v[1][1])) * 0.5;
    }
  }
}

// fine starting state: each pore cell takes its parent's coarse value, fibre cells 0
__global__ void __launch_bounds__(256) k_prolong(Grid g, const uint8_t *__restrict__ flags,
                                                 const double *__restrict__ s_c,
                                                 double *__restrict__ s_f) {
  const int nxc = g.nx / 2, nyc = g.ny / 2;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < g.n; i += 256ll * gridDim.x) {
    const int x = (int)(i % g.nx), y = (int)((i / g.nx) % g.ny);
    const int z = (int)(i / ((long long)g.nx * g.ny));
    const long long c = (x / 2) + (long long)nxc * ((y / 2) + (long long)nyc * (z / 2));
    s_f[i] = (flags[i] & FL_PORE) ? s_c[c] : 0.0;
  }
}

void launch_coarse_mask(const Grid &g, const uint8_t *flags, uint8_t *solid_c, hipStream_t st) {
  k_coarse_mask<<<fill_blocks(g.n / 8 + 1), 256, 0, st>>>(g, flags, solid_c);
}

void launch_restrict(const Grid &g, const Faces<double> &w, double *ux_c, double *uy_c,
                     double *uz_c, hipStream_t st) {
  k_restrict<<<fill_blocks(g.n / 8 * 3 + 1), 256, 0, st>>>(g, w, ux_c, uy_c, uz_c);
}

void launch_prolong(const Grid &g, const uint8_t *flags, const double *s_c, double *s_f,
                    hipStream_t st) {
  k_prolong<<<fill_blocks(g.n), 256, 0, st>>>(g, flags, s_c, s_f);
}

__global__ void __launch_bounds__(256) k_init_state(Grid g, const uint8_t *__restrict__ flags,
                                                    const double *__restrict__ s_init,
                                                    double s_in, double s_eq, int pinned,
                                                    double *__restrict__ s64) {
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < g.n; i += 256ll * gridDim.x) {
    const uint8_t f = flags[i];
    double v = 0.0;
    if (f & FL_PORE) {
      const bool held = pinned && (f & FL_FIBRE);
      v = held ? s_eq : (s_init ? s_init[i] : s_in);
    }
    s64[i] = v;
  }
}

void launch_init_state(const Grid &g, const uint8_t *flags, const double *s_init, double s_in,
                       double s_eq, int pinned, double *s64, hipStream_t st) {
  k_init_state<<<fill_blocks(g.n), 256, 0, st>>>(g, flags, s_init, s_in, s_eq, pinned, s64);
}

__global__ void __launch_bounds__(256) k_f64_to_f32(const double *a, float *b, long long n) {
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) b[i] = (float)a[i];
}
__global__ void __launch_bounds__(256) k_f32_to_f64(const float *a, double *b, long long n) {
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) b[i] = (double)a[i];
}
void launch_f64_to_f32(const double *a, float *b, long long n, hipStream_t st) {
  k_f64_to_f32<<<fill_blocks(n), 256, 0, st>>>(a, b, n);
}
void launch_f32_to_f64(const float *a, double *b, long long n, hipStream_t st) {
  k_f32_to_f64<<<fill_blocks(n), 256, 0, st>>>(a, b, n);
}

__global__ void __launch_bounds__(256) k_mask_held(Grid g, const uint8_t *__restrict__ flags,
                                                   int pinned, double *p) {
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < g.n; i += 256ll * gridDim.x) {
    const uint8_t f = flags[i];
    if (!(f & FL_PORE) || (pinned && (f & FL_FIBRE))) p[i] = 0.0;
  }
}
void launch_mask_held(const Grid &g, const uint8_t *flags, int pinned, double *p, hipStream_t st) {
  k_mask_held<<<fill_blocks(g.n), 256, 0, st>>>(g, flags, pinned, p);
}

}  // namespace socfv
