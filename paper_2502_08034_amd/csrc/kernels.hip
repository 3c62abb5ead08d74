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
// fibre voxel or a wall on the other must carry zero velocity; an inlet face must not
// carry backflow.  Faces without a pore cell on either side are stored as zero.
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
    if (x == 0 && pore && a < 0.0) bad += 1.0;       // inlet backflow
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

template <typename T>
void launch_sweep(const SweepArgs<T> &a, const Tiles &t, hipStream_t st) {
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
// FP64 refresh of the defect correction: t = s64 + delta, r0 = R64(t)
// ------------------------------------------------------------------------------------

__global__ void __launch_bounds__(1024) k_refresh(RefreshArgs a) {
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
    auto val = [&](long long j) -> double { return a.s64[j] + (d ? (double)d[j] : 0.0); };
    long long i = x + (long long)nx * (y + (long long)ny * z0);
    double s_c = val(i);
    double s_dn = z0 > 0 ? val(i - pl) : 0.0;
    double wz_c = a.w.wz[i];
    for (int z = z0; z < z1; ++z, i += pl) {
      const bool up = z + 1 < g.nz;
      const double s_up = up ? val(i + pl) : 0.0;
      const double wz_u = up ? a.w.wz[i + pl] : 0.0;
      const uint8_t f = a.flags[i];
      double nv = 0.0;
      float r0 = 0.0f;
      if (f & FL_PORE) {
        Cell<double> q;
        q.c = s_c; q.zm = s_dn; q.zp = s_up; q.wzm = wz_c; q.wzp = wz_u;
        q.gzm = (z > 0 && !(f & FL_ZM)) ? 1.0 : 0.0;
        q.gzp = (up && !(f & FL_ZP)) ? 1.0 : 0.0;
        q.xm = xl ? val(i - 1) : a.s_in;
        q.xp = xr ? val(i + 1) : s_c;
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
        const int nf = __popc((unsigned)(f & FL_FIBRE));
        const bool held = a.pinned && nf > 0;
        const double lam = a.Da * (a.kappa ? (double)a.kappa[i] : 1.0) * (double)nf;
        double r = held ? 0.0 : residual<double>(q, lam, a.s_eq);
        nv = held ? a.s_eq : s_c;
        r0 = (float)r;
        acc[0] += r * r;
        acc[2] += r;
        if (!(nv >= a.lo && nv <= a.hi)) acc[1] += 1.0;
      }
      a.s64_new[i] = nv;
      a.r0[i] = r0;
      s_dn = s_c;
      s_c = s_up;
      wz_c = wz_u;
    }
  }
  block_store<NV>(acc, 0u, a.partial + (long long)NV * (blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)));
}

void launch_refresh(const RefreshArgs &a, const Tiles &t, hipStream_t st) {
  k_refresh<<<sweep_grid(a.g, t), dim3(64, t.ty, 1), 0, st>>>(a);
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
// Outputs of a state: utilisation and the balance of fluxes
// ------------------------------------------------------------------------------------

int outputs_blocks(const Grid &g) { return (int)((g.n + 255) / 256); }

__global__ void __launch_bounds__(256) k_outputs(Grid g, const uint8_t *__restrict__ flags,
                                                 Faces<double> w, const float *kappa,
                                                 const double *__restrict__ s, double s_in,
                                                 double s_eq, double Da, int pinned,
                                                 double *partial) {
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  double v[NV2] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (i < g.n) {
    const uint8_t f = flags[i];
    if (f & FL_PORE) {
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
      q.gzm = (z > 0 && !(f & FL_ZM)) ? 1.0 : 0.0;
      q.gzp = (up && !(f & FL_ZP)) ? 1.0 : 0.0;
      load_plane<double>(q, s, w, f, g, x, y, z, i, s_in, true);
      const int nf = __popc((unsigned)(f & FL_FIBRE));
      const bool held = pinned && nf > 0;
      if (x == nx - 1) {
        const double wo = w.wxo[y + (long long)ny * z];
        v[0] = wo * q.c;
        v[1] = wo;
      }
      if (x == 0) {
        const double u = w.wx[i];
        v[2] = u * s_in + 2.0 * (s_in - q.c);
        v[3] = u * s_in;
      }
      if (held) {
        v[4] = residual<double>(q, 0.0, s_eq);        // absorbed by the electrode cell
      } else {
        const double lam = Da * (kappa ? (double)kappa[i] : 1.0) * nf;
        const double r = residual<double>(q, lam, s_eq);
        v[4] = lam * (q.c - s_eq);
        v[5] = r;
        v[6] = r * r;
      }
    }
  }
  block_store<NV2>(v, 0u, partial + (long long)NV2 * blockIdx.x);
}

void launch_outputs(const Grid &g, const uint8_t *flags, Faces<double> w, const float *kappa,
                    const double *s, double s_in, double s_eq, double Da, int pinned,
                    double *partial, int nblk, hipStream_t st) {
  k_outputs<<<nblk, 256, 0, st>>>(g, flags, w, kappa, s, s_in, s_eq, Da, pinned, partial);
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

static unsigned fill_blocks(long long n) {
  long long b = (n + 255) / 256;
  return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

void launch_fill_f32(float *p, long long n, float v, hipStream_t st) {
  k_fill<float><<<fill_blocks(n), 256, 0, st>>>(p, n, v);
}
void launch_fill_f64(double *p, long long n, double v, hipStream_t st) {
  k_fill<double><<<fill_blocks(n), 256, 0, st>>>(p, n, v);
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
