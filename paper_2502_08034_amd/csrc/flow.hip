// HIP kernels (gfx950) of the upstream flow step: steady Stokes flow through the voxel pore
// space by the projection method (Eqs. (cp1)-(cp4), Algorithm "Flow Simulation" with explicit
// momentum diffusion), in the Stokes regime of Eq. (stokes-flow) (no momentum advection).
//
// Discretisation (nondimensional: h = rho = mu = 1): normal velocity on open faces (both
// cells pore, or the inlet / outlet face of a pore cell), pressure in pore cells, applied
// pressure p_in at the inlet face and 0 at the outlet face (half a cell from the first / last
// cell centre), no-slip on fibre voxel faces and the y / z walls, zero normal gradient of the
// velocity across the inlet and outlet planes.  One step:
//   predictor   u* = u + dt L u                       (Eq. (cp1) without advection)
//   pressure    (-D G) p = D gbc - D u* / dt           (Eq. (cp4)), Jacobi-preconditioned CG
//   projection  u' = u* - dt (G p + gbc)               (Eq. (cp2))
// The CG starts from the previous step's pressure and stops once dt ||r|| (the divergence
// the projection leaves) is below theta times the previous step's velocity change, or at the
// per-step cap.  A fixed point of the step satisfies the pressure equation exactly (a CG
// started at its solution does not move), so it is the discrete Stokes solution L u = G p,
// D u = 0 whatever the inner tolerance; the tolerance only sets how fast the steps get there.
//
// Everything is FP64 (the velocity is an FP64 input of the state-of-charge solve).  The step
// is bandwidth bound (a few flops per 8-byte value); kernels are grid-stride loops over
// faces or cells with coalesced rows.  The CG's scalars are never sent to the host: every
// block of the next kernel sums the previous kernel's per-block partials itself, in a fixed
// order, so all blocks take the same (deterministic) values and the same stop decision.
#include "internal.h"

namespace socfv {

namespace {

constexpr int FB = 256;        // threads per block of every flow kernel
constexpr int FLOW_MAX_BLOCKS = 2048;

__device__ __forceinline__ double fwave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double fwave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Block-wide sum (or max) of v, returned to every thread; fixed order.  Every thread of the
// block must reach it.
__device__ __forceinline__ double block_total(double v, bool mx, double *sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = mx ? fwave_max(v) : fwave_sum(v);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = sh[0];
#pragma unroll
  for (int k = 1; k < FB / 64; ++k) t = mx ? fmax(t, sh[k]) : t + sh[k];
  return t;
}

// Sum of a[k * stride] for k < n by the whole block (same value in every thread and block).
// Eight loads per thread are in flight at once (indices past n read a[0], selected away).
__device__ __forceinline__ double sum_partials(const double *a, int n, int stride, double *sh) {
  double v = 0.0;
  for (int k0 = 0; k0 < n; k0 += 8 * FB) {
    double t[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + j * FB + (int)threadIdx.x;
      t[j] = a[(long long)(k < n ? k : 0) * stride];
      t[j] = k < n ? t[j] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) v += t[j];
  }
  return block_total(v, false, sh);
}

// Workgroups go to the eight XCDs in turn (block b to XCD b % 8), each XCD with its own L2.
// Renumbering them so that every XCD works one contiguous run of logical blocks keeps a
// cell's row neighbours (the next block) in the same L2.  A bijection on [0, nb).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned x = b % 8u, k = b / 8u, q = nb / 8u, r = nb % 8u;
  return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ bool pore_at(const uint8_t *fl, const Grid &g, int x, int y, int z) {
  return (fl[x + (long long)g.nx * (y + (long long)g.ny * z)] & FL_PORE) != 0;
}

struct FaceDims {
  int fx, fy, fz;
  long long n;
};
__device__ __forceinline__ FaceDims face_dims(const Grid &g, int a) {
  FaceDims d{g.nx + (a == 0), g.ny + (a == 1), g.nz + (a == 2), 0};
  d.n = (long long)d.fx * d.fy * d.fz;
  return d;
}

// Is the face of orientation a at (x, y, z) of its face array open?
__device__ __forceinline__ bool face_open(const uint8_t *fl, const Grid &g, int a, int x, int y,
                                          int z) {
  if (a == 0) {
    if (x == 0) return pore_at(fl, g, 0, y, z);
    if (x == g.nx) return pore_at(fl, g, g.nx - 1, y, z);
    return pore_at(fl, g, x - 1, y, z) && pore_at(fl, g, x, y, z);
  }
  if (a == 1) {
    if (y == 0 || y == g.ny) return false;
    return pore_at(fl, g, x, y - 1, z) && pore_at(fl, g, x, y, z);
  }
  if (z == 0 || z == g.nz) return false;
  return pore_at(fl, g, x, y, z - 1) && pore_at(fl, g, x, y, z);
}

// Pressure-operator row of a pore cell: diagonal and the open-neighbour mask (bit n for
// neighbour n = x-, x+, y-, y+, z-, z+).  Inlet / outlet faces add 2 to the diagonal.
struct PRow {
  double diag;
  unsigned nb;
};
__device__ __forceinline__ PRow prow(uint8_t fl, const Grid &g, int x, int y, int z) {
  PRow r{0.0, 0u};
  if (x > 0) { if (!(fl & FL_XM)) { r.nb |= 1u; r.diag += 1.0; } } else r.diag += 2.0;
  if (x < g.nx - 1) { if (!(fl & FL_XP)) { r.nb |= 2u; r.diag += 1.0; } } else r.diag += 2.0;
  if (y > 0 && !(fl & FL_YM)) { r.nb |= 4u; r.diag += 1.0; }
  if (y < g.ny - 1 && !(fl & FL_YP)) { r.nb |= 8u; r.diag += 1.0; }
  if (z > 0 && !(fl & FL_ZM)) { r.nb |= 16u; r.diag += 1.0; }
  if (z < g.nz - 1 && !(fl & FL_ZP)) { r.nb |= 32u; r.diag += 1.0; }
  return r;
}

// Cell code byte (built once per call): bits 0..5 the open-neighbour mask, bit 6 the inlet
// face, bit 7 the outlet face; 0 for fibre cells (a pore cell always has an open face or the
// inlet: it is face-connected to the inlet).  The CG kernels need nothing else of the cell.
constexpr unsigned CC_INLET = 64u, CC_OUTLET = 128u;
__device__ __forceinline__ PRow prow_code(unsigned cc) {
  return PRow{(double)(__popc(cc & 63u) + 2 * ((cc >> 6) & 1u) + 2 * ((cc >> 7) & 1u)),
              cc & 63u};
}

// Sum of v over the open neighbours of a cell.  Branch-free: a closed neighbour's index is
// replaced by the cell's own (always in bounds) and its value selected away, so all six loads
// are in flight together (a load under a branch makes the join wait for every load).
__device__ __forceinline__ double nb_sum(const double *__restrict__ v, long long c, unsigned nb,
                                         long long sy, long long sz) {
  const double a0 = v[(nb & 1u) ? c - 1 : c];
  const double a1 = v[(nb & 2u) ? c + 1 : c];
  const double a2 = v[(nb & 4u) ? c - sy : c];
  const double a3 = v[(nb & 8u) ? c + sy : c];
  const double a4 = v[(nb & 16u) ? c - sz : c];
  const double a5 = v[(nb & 32u) ? c + sz : c];
  return (((nb & 1u) ? a0 : 0.0) + ((nb & 2u) ? a1 : 0.0)) +
         (((nb & 4u) ? a2 : 0.0) + ((nb & 8u) ? a3 : 0.0)) +
         (((nb & 16u) ? a4 : 0.0) + ((nb & 32u) ? a5 : 0.0));
}

// ---- face classification ---------------------------------------------------------------
__global__ void __launch_bounds__(FB) k_flow_codes(FlowArgs a) {
  const Grid g = a.g;
  const int o = blockIdx.y;
  const FaceDims d = face_dims(g, o);
  uint16_t *code = a.code[o];
  for (long long f = (long long)xcd_block(blockIdx.x, gridDim.x) * FB + threadIdx.x; f < d.n;
       f += (long long)gridDim.x * FB) {
    const unsigned fu = (unsigned)f, t = fu / (unsigned)d.fx;
    const int x = (int)(fu - t * (unsigned)d.fx);
    const int y = (int)(t % (unsigned)d.fy), z = (int)(t / (unsigned)d.fy);
    uint16_t c = 0;
    if (face_open(a.flags, g, o, x, y, z)) {
      c = FC_OPEN;
      for (int n = 0; n < 6; ++n) {
        const int b = n >> 1, s = (n & 1) ? 1 : -1;
        const int xx = x + (b == 0 ? s : 0), yy = y + (b == 1 ? s : 0), zz = z + (b == 2 ? s : 0);
        const bool inside = xx >= 0 && xx < d.fx && yy >= 0 && yy < d.fy && zz >= 0 && zz < d.fz;
        unsigned cls;
        if (!inside) cls = (b == 0) ? 0u : 3u;      // open plane: zero gradient; y / z wall
        else if (face_open(a.flags, g, o, xx, yy, zz)) cls = 1u;
        else cls = (b == o) ? 2u : 3u;
        c |= (uint16_t)(cls << (2 * n));
      }
    }
    code[f] = c;
  }
}

__global__ void __launch_bounds__(FB) k_flow_cell_codes(FlowArgs a) {
  const Grid g = a.g;
  for (long long c = (long long)xcd_block(blockIdx.x, gridDim.x) * FB + threadIdx.x; c < g.n;
       c += (long long)gridDim.x * FB) {
    const uint8_t fl = a.flags[c];
    unsigned cc = 0;
    if (fl & FL_PORE) {
      const unsigned cu = (unsigned)c, row = cu / (unsigned)g.nx;
      const int x = (int)(cu - row * (unsigned)g.nx);
      const int y = (int)(row % (unsigned)g.ny), z = (int)(row / (unsigned)g.ny);
      cc = prow(fl, g, x, y, z).nb | (x == 0 ? CC_INLET : 0u) | (x == g.nx - 1 ? CC_OUTLET : 0u);
    }
    a.ccode[c] = (uint8_t)cc;
  }
}

// ---- predictor: u* = u + dt L u ----------------------------------------------------------
__global__ void __launch_bounds__(FB) k_flow_predict(FlowArgs a) {
  const Grid g = a.g;
  const int o = blockIdx.y;
  const FaceDims d = face_dims(g, o);
  const uint16_t *__restrict__ code = a.code[o];
  const double *__restrict__ u = a.u[o];
  double *__restrict__ us = a.us[o];
  const long long off[6] = {-1, 1, -(long long)d.fx, (long long)d.fx,
                            -(long long)d.fx * d.fy, (long long)d.fx * d.fy};
  for (long long f = (long long)xcd_block(blockIdx.x, gridDim.x) * FB + threadIdx.x; f < d.n;
       f += (long long)gridDim.x * FB) {
    const unsigned c = code[f];
    double out = 0.0;
    if (c & FC_OPEN) {
      const double u0 = u[f];
      double nbv[6];
#pragma unroll
      for (int n = 0; n < 6; ++n)      // branch-free gather: closed neighbours read the face
        nbv[n] = u[((c >> (2 * n)) & 3u) == 1u ? f + off[n] : f];
      double acc = 0.0, diag = 0.0;
#pragma unroll
      for (int n = 0; n < 6; ++n) {
        const unsigned cls = (c >> (2 * n)) & 3u;
        acc += cls == 1u ? nbv[n] : 0.0;
        diag += cls == 3u ? 2.0 : (cls != 0u ? 1.0 : 0.0);
      }
      out = u0 + a.dt * (acc - diag * u0);
    }
    us[f] = out;
  }
}

// ---- pressure CG -------------------------------------------------------------------------
// init: r = b - A p with b = D gbc - D u* / dt, z = r / diag; partials of r.z, r.r into
// parity 0.  Block 0 also sets the step's stop target from the last projection's partials.
__global__ void __launch_bounds__(FB) k_flow_cg_init(FlowArgs a) {
  __shared__ double sh[FB / 64];
  const Grid g = a.g;
  if (blockIdx.x == 0) {
    const double du2 = sum_partials(a.pdu, 3 * a.nbf, 2, sh);
    if (threadIdx.x == 0) {
      a.sc[FS_TARGET] = a.theta2 * du2 / (a.dt * a.dt);
      a.sc[FS_DONE] = 0.0;
      a.sc[FS_CG_STEP] = 0.0;
    }
  }
  const long long sy = g.nx, sz = (long long)g.nx * g.ny;
  double rz = 0.0, rr = 0.0, fl = 0.0;
  for (long long c = (long long)xcd_block(blockIdx.x, gridDim.x) * FB + threadIdx.x; c < g.n;
       c += (long long)gridDim.x * FB) {
    const unsigned cc = a.ccode[c];
    double rv = 0.0, zv = 0.0;
    if (cc) {
      // x faces: index c + (y + ny z); y faces: c + nx z
      const unsigned row = (unsigned)c / (unsigned)g.nx, z = row / (unsigned)g.ny;
      const long long ix = c + row;
      const long long iy = c + (long long)g.nx * z;
      const double div = (a.us[0][ix + 1] - a.us[0][ix]) + (a.us[1][iy + g.nx] - a.us[1][iy]) +
                         (a.us[2][c + sz] - a.us[2][c]);
      const double b = ((cc & CC_INLET) ? 2.0 * a.p_in : 0.0) - div / a.dt;
      const PRow pr = prow_code(cc);
      const double ap = pr.diag * a.p[c] - nb_sum(a.p, c, pr.nb, sy, sz);
      rv = b - ap;
      zv = rv / pr.diag;
      rz += rv * zv;
      rr += rv * rv;
      const double dp = pr.diag * a.p[c];
      fl += b * b + dp * dp;
    }
    a.r[c] = rv;
    a.z[c] = zv;
  }
  rz = block_total(rz, false, sh);
  rr = block_total(rr, false, sh);
  fl = block_total(fl, false, sh);
  if (threadIdx.x == 0) {
    a.prz[0][blockIdx.x] = rz;
    a.prr[0][blockIdx.x] = rr;
    a.pfl[blockIdx.x] = fl;
  }
}

// Floor of the CG stop target: about what the recursively updated residual reaches in FP64,
// (CG_FLOOR eps)^2 (||b||^2 + ||diag p||^2) at the step's start.  Near the steady state the
// target (theta times the last velocity change) falls with the change; the floor keeps a
// target below rounding level from running the CG to the per-step cap.  It binds only there
// (the step's fixed point does not depend on it).
constexpr double CG_FLOOR = 16.0;

// iteration j, first half: stop test; d = z + beta d_old; q = A d; partials of d.q
__global__ void __launch_bounds__(FB) k_flow_cg_a(FlowArgs a, int j) {
  __shared__ double sh[FB / 64];
  if (a.sc[FS_DONE] != 0.0) return;
  const Grid g = a.g;
  const int par = j & 1;
  const double rz = sum_partials(a.prz[par], a.nbc, 1, sh);
  const double rr = sum_partials(a.prr[par], a.nbc, 1, sh);
  const double floor2 = (CG_FLOOR * 2.220446049250313e-16) * (CG_FLOOR * 2.220446049250313e-16) *
                        sum_partials(a.pfl, a.nbc, 1, sh);
  if (rr <= fmax(a.sc[FS_TARGET], floor2)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) a.sc[FS_DONE] = 1.0;
    return;
  }
  const double beta = j == 0 ? 0.0 : rz / sum_partials(a.prz[par ^ 1], a.nbc, 1, sh);
  const double *__restrict__ zz = a.z;
  const double *__restrict__ dold = a.d[par ^ 1];
  double *__restrict__ dn = a.d[par];
  const long long sy = g.nx, sz = (long long)g.nx * g.ny;
  double dq = 0.0;
  for (long long c = (long long)xcd_block(blockIdx.x, gridDim.x) * FB + threadIdx.x; c < g.n;
       c += (long long)gridDim.x * FB) {
    const unsigned cc = a.ccode[c];
    double dv = 0.0, qv = 0.0;
    if (cc) {
      const PRow pr = prow_code(cc);
      double nbs;
      if (j == 0) {
        dv = zz[c];
        nbs = nb_sum(zz, c, pr.nb, sy, sz);
      } else {
        dv = zz[c] + beta * dold[c];
        nbs = nb_sum(zz, c, pr.nb, sy, sz) + beta * nb_sum(dold, c, pr.nb, sy, sz);
      }
      qv = pr.diag * dv - nbs;
      dq += dv * qv;
    }
    dn[c] = dv;
    a.q[c] = qv;
  }
  dq = block_total(dq, false, sh);
  if (threadIdx.x == 0) a.pdq[blockIdx.x] = dq;
}

// iteration j, second half: alpha = r.z / d.q; p += alpha d; r -= alpha q; z = r / diag;
// partials of the new r.z, r.r into the other parity
__global__ void __launch_bounds__(FB) k_flow_cg_b(FlowArgs a, int j) {
  __shared__ double sh[FB / 64];
  if (a.sc[FS_DONE] != 0.0) return;
  const Grid g = a.g;
  const int par = j & 1;
  const double rz = sum_partials(a.prz[par], a.nbc, 1, sh);
  const double dq = sum_partials(a.pdq, a.nbc, 1, sh);
  const double alpha = rz / dq;
  const double *__restrict__ dn = a.d[par];
  double rzn = 0.0, rrn = 0.0;
  for (long long c = (long long)xcd_block(blockIdx.x, gridDim.x) * FB + threadIdx.x; c < g.n;
       c += (long long)gridDim.x * FB) {
    const unsigned cc = a.ccode[c];
    if (!cc) continue;
    const PRow pr = prow_code(cc);
    a.p[c] += alpha * dn[c];
    const double rv = a.r[c] - alpha * a.q[c];
    const double zv = rv / pr.diag;
    a.r[c] = rv;
    a.z[c] = zv;
    rzn += rv * zv;
    rrn += rv * rv;
  }
  rzn = block_total(rzn, false, sh);
  rrn = block_total(rrn, false, sh);
  if (threadIdx.x == 0) {
    a.prz[par ^ 1][blockIdx.x] = rzn;
    a.prr[par ^ 1][blockIdx.x] = rrn;
    if (blockIdx.x == 0) a.sc[FS_CG_STEP] = (double)(j + 1);
  }
}

// ---- projection: u' = u* - dt (G p + gbc); partials [sum (u' - u)^2, sum u'^2] -----------
__global__ void __launch_bounds__(FB) k_flow_project(FlowArgs a) {
  __shared__ double sh[FB / 64];
  const Grid g = a.g;
  const int o = blockIdx.y;
  const FaceDims d = face_dims(g, o);
  const uint16_t *__restrict__ code = a.code[o];
  const double *__restrict__ us = a.us[o];
  double *__restrict__ u = a.u[o];
  const double *__restrict__ p = a.p;
  double du2 = 0.0, u2 = 0.0;
  for (long long f = (long long)xcd_block(blockIdx.x, gridDim.x) * FB + threadIdx.x; f < d.n;
       f += (long long)gridDim.x * FB) {
    double un = 0.0;
    if (code[f] & FC_OPEN) {
      const unsigned fu = (unsigned)f, t = fu / (unsigned)d.fx;
      const int x = (int)(fu - t * (unsigned)d.fx);
      const int y = (int)(t % (unsigned)d.fy), z = (int)(t / (unsigned)d.fy);
      double gp;
      if (o == 0) {
        const long long c = (long long)x + (long long)g.nx * (y + (long long)g.ny * z);
        if (x == 0) gp = 2.0 * (p[c] - a.p_in);
        else if (x == g.nx) gp = -2.0 * p[c - 1];
        else gp = p[c] - p[c - 1];
      } else if (o == 1) {
        const long long c = (long long)x + (long long)g.nx * (y + (long long)g.ny * z);
        gp = p[c] - p[c - g.nx];
      } else {
        const long long c = (long long)x + (long long)g.nx * (y + (long long)g.ny * z);
        gp = p[c] - p[c - (long long)g.nx * g.ny];
      }
      un = us[f] - a.dt * gp;
    }
    const double dv = un - u[f];
    du2 += dv * dv;
    u2 += un * un;
    u[f] = un;
  }
  du2 = block_total(du2, false, sh);
  u2 = block_total(u2, false, sh);
  if (threadIdx.x == 0) {
    const long long b = (long long)o * a.nbf + blockIdx.x;
    a.pdu[2 * b] = du2;
    a.pdu[2 * b + 1] = u2;
    if (o == 0 && blockIdx.x == 0) a.sc[FS_CG_TOTAL] += a.sc[FS_CG_STEP];
  }
}

// ---- outputs: per block [max |D u|, inlet flux, max |u| over cell faces, outlet flux] ----
__global__ void __launch_bounds__(FB) k_flow_check(FlowArgs a) {
  __shared__ double sh[FB / 64];
  const Grid g = a.g;
  const long long sz = (long long)g.nx * g.ny;
  double dmax = 0.0, qin = 0.0, umax = 0.0, qout = 0.0;
  for (long long c = (long long)xcd_block(blockIdx.x, gridDim.x) * FB + threadIdx.x; c < g.n;
       c += (long long)gridDim.x * FB) {
    const unsigned cc = a.ccode[c];
    if (!cc) continue;
    const unsigned row = (unsigned)c / (unsigned)g.nx, z = row / (unsigned)g.ny;
    const long long ix = c + row;
    const long long iy = c + (long long)g.nx * z;
    const double v[6] = {a.u[0][ix], a.u[0][ix + 1], a.u[1][iy], a.u[1][iy + g.nx], a.u[2][c],
                         a.u[2][c + sz]};
    dmax = fmax(dmax, fabs((v[1] - v[0]) + (v[3] - v[2]) + (v[5] - v[4])));
    for (int k = 0; k < 6; ++k) umax = fmax(umax, fabs(v[k]));
    if (cc & CC_INLET) qin += v[0];
    if (cc & CC_OUTLET) qout += v[1];
  }
  dmax = block_total(dmax, true, sh);
  qin = block_total(qin, false, sh);
  umax = block_total(umax, true, sh);
  qout = block_total(qout, false, sh);
  if (threadIdx.x == 0) {
    double *o = a.pdiv + 4ll * blockIdx.x;
    o[0] = dmax;
    o[1] = qin;
    o[2] = umax;
    o[3] = qout;
  }
}

}  // namespace

int flow_cell_blocks(const Grid &g) {
  const long long b = (g.n + FB - 1) / FB;
  return (int)(b < FLOW_MAX_BLOCKS ? b : FLOW_MAX_BLOCKS);
}

int flow_face_blocks(const Grid &g) {
  const long long nmax = (long long)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
  const long long b = (nmax + FB - 1) / FB;
  return (int)(b < FLOW_MAX_BLOCKS ? b : FLOW_MAX_BLOCKS);
}

void launch_flow_codes(const FlowArgs &a, hipStream_t st) {
  k_flow_codes<<<dim3(a.nbf, 3), FB, 0, st>>>(a);
  k_flow_cell_codes<<<a.nbc, FB, 0, st>>>(a);
}
void launch_flow_predict(const FlowArgs &a, hipStream_t st) {
  k_flow_predict<<<dim3(a.nbf, 3), FB, 0, st>>>(a);
}
void launch_flow_cg_init(const FlowArgs &a, hipStream_t st) {
  k_flow_cg_init<<<a.nbc, FB, 0, st>>>(a);
}
void launch_flow_cg_iter(const FlowArgs &a, int j, hipStream_t st) {
  k_flow_cg_a<<<a.nbc, FB, 0, st>>>(a, j);
  k_flow_cg_b<<<a.nbc, FB, 0, st>>>(a, j);
}
void launch_flow_project(const FlowArgs &a, hipStream_t st) {
  k_flow_project<<<dim3(a.nbf, 3), FB, 0, st>>>(a);
}
void launch_flow_check(const FlowArgs &a, hipStream_t st) {
  k_flow_check<<<a.nbc, FB, 0, st>>>(a);
}

}  // namespace socfv
