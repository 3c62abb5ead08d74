/*
 * FP64 CPU oracle for the steady state-of-charge (SOC) solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls this
 * file; only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
 * It shares no source with the GPU library.
 *
 * What it computes (paper: Sec. "Reaction Steady State from Nernst Equilibrium Boundary
 * Condition", the SOC transport equation Eq. (nernst-planck-soc) with the affine rate of
 * Eq. (rate-from-soc-gen); the explicit iteration of Algorithm "SOC at Mass Transport
 * Limit"; utilisation Eq. (utilization-def) / Eq. (umt-def); electron flows
 * Eqs. (electron-flow)-(convergence-bv-flow); convergence rule Eq. (convergence-bv-change)).
 *
 * Discretisation (nondimensional: h = 1, D = 1, time in h^2/D), finite volumes on a voxel
 * grid, x fastest, cell index P = x + nx*(y + ny*z).  Every pore cell P has six faces f
 * with outward normal velocity w_f (staggered face velocities, positive along +axis):
 *
 *   face class                    upwind value        diffusive coefficient G_f
 *   interior (pore both sides)    s of the neighbour  1
 *   inlet  (x- face of x = 0)     s_in (s_P where     2   (Dirichlet value on the face)
 *                                 the flow leaves)
 *   outlet (x+ face of x = nx-1)  s_P                 0   (no concentration gradient)
 *   fibre face, y/z domain wall   no flux             0   (w_f must be 0)
 *
 *   R_P(s) = sum_f [ -max(w_f,0) s_P - min(w_f,0) s_up(f) + G_f (s_nb(f) - s_P) ]
 *            + lam_P (s_eq - s_P)
 *
 * which is written here as R = b - A s with one routine (row_of) producing row P of A and
 * b; the residual gathers it and the adjoint scatters it (A^T), so both use one definition.
 * lam_P = Da * kappa_P * n_f(P), n_f = number of faces P shares with fibre voxels (domain
 * walls do not react).  In the mass-transport limit (pinned mode) every pore cell with
 * n_f > 0 is held at s_eq (Dirichlet on the electrode surface, Eqs. (np-fast-interior),
 * (np-fast-boundary)) and has R = 0.
 *
 * Iteration: s <- s + dt R(s), dt = cfl / max_P diag_P, diag_P = sum_f max(w_f,0) +
 * sum_f G_f + lam_P over updated cells.  Residual res = tau * sqrt(sum_P R_P^2 / N_pore)
 * = (tau/dt) ||s^{n+1} - s^n||_rms, tau = nx*ny*nz / Q, Q = sum of inlet face velocities.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { F_INTERIOR = 0, F_INLET = 1, F_OUTLET = 2, F_CLOSED = 3 };

typedef struct {
    int nx, ny, nz;
    const uint8_t *solid;        /* 1 = fibre voxel */
    const double *ux, *uy, *uz;  /* (nz,ny,nx+1), (nz,ny+1,nx), (nz+1,ny,nx) */
    const double *lam;           /* per-cell reaction coefficient (NULL: none) */
    double s_in, s_eq;
    int pinned;                  /* 1: reactive cells held at s_eq */
    const int8_t *nf;            /* fibre-face count per cell, -1 for fibre cells */
} prob_t;

typedef struct {
    double diag;      /* A_PP */
    double dtdiag;    /* sum max(w,0) + sum G + lam (time-step bound) */
    double rhs;       /* b_P */
    long nb[6];       /* neighbour index or -1 */
    double coef[6];   /* A_P,nb */
    int held;         /* pinned cell: identity row, not updated */
} row_t;

void orc_export_rows(int nx, int ny, int nz, const uint8_t *solid, const double *ux,
                     const double *uy, const double *uz, const double *lam, const int8_t *nf,
                     double s_in, double s_eq, int pinned, double *diag, double *rhs,
                     uint8_t *held, long *nb, double *coef);

static inline long cidx(const prob_t *p, long x, long y, long z) {
    return x + (long)p->nx * (y + (long)p->ny * z);
}

/* outward normal velocity and class of face f (0:x-,1:x+,2:y-,3:y+,4:z-,5:z+) of cell */
static void face_of(const prob_t *p, long x, long y, long z, int f,
                    double *w, int *cls, long *nb) {
    long nx = p->nx, ny = p->ny, nz = p->nz;
    long xn = x, yn = y, zn = z;
    int at_edge = 0;
    switch (f) {
    case 0: *w = -p->ux[x + (nx + 1) * (y + ny * z)]; xn = x - 1; at_edge = (x == 0); break;
    case 1: *w = p->ux[(x + 1) + (nx + 1) * (y + ny * z)]; xn = x + 1; at_edge = (x == nx - 1); break;
    case 2: *w = -p->uy[x + nx * (y + (ny + 1) * z)]; yn = y - 1; at_edge = (y == 0); break;
    case 3: *w = p->uy[x + nx * ((y + 1) + (ny + 1) * z)]; yn = y + 1; at_edge = (y == ny - 1); break;
    case 4: *w = -p->uz[x + nx * (y + ny * z)]; zn = z - 1; at_edge = (z == 0); break;
    default: *w = p->uz[x + nx * (y + ny * (z + 1))]; zn = z + 1; at_edge = (z == nz - 1); break;
    }
    *nb = -1;
    if (at_edge) {
        if (f == 0) *cls = F_INLET;
        else if (f == 1) *cls = F_OUTLET;
        else *cls = F_CLOSED;
        return;
    }
    long q = cidx(p, xn, yn, zn);
    if (p->solid[q]) { *cls = F_CLOSED; return; }
    *cls = F_INTERIOR;
    *nb = q;
}

static inline double dmax(double a, double b) { return a > b ? a : b; }
static inline double dmin(double a, double b) { return a < b ? a : b; }

/* Row P of A s = b (pore cells only). */
static void row_of(const prob_t *p, long x, long y, long z, row_t *r) {
    long P = cidx(p, x, y, z);
    double lam = p->lam ? p->lam[P] : 0.0;
    r->diag = 0.0; r->dtdiag = 0.0; r->rhs = 0.0; r->held = 0;
    for (int f = 0; f < 6; ++f) { r->nb[f] = -1; r->coef[f] = 0.0; }
    if (p->pinned && p->nf[P] > 0) {
        r->held = 1; r->diag = 1.0; r->rhs = p->s_eq;
        return;
    }
    for (int f = 0; f < 6; ++f) {
        double w; int cls; long q;
        face_of(p, x, y, z, f, &w, &cls, &q);
        switch (cls) {
        case F_INTERIOR:
            r->diag += dmax(w, 0.0) + 1.0;
            r->dtdiag += dmax(w, 0.0) + 1.0;
            r->nb[f] = q;
            r->coef[f] = dmin(w, 0.0) - 1.0;
            break;
        case F_INLET:
            r->diag += dmax(w, 0.0) + 2.0;
            r->dtdiag += dmax(w, 0.0) + 2.0;
            r->rhs += -dmin(w, 0.0) * p->s_in + 2.0 * p->s_in;
            break;
        case F_OUTLET:
            r->diag += dmax(w, 0.0) + dmin(w, 0.0);
            r->dtdiag += dmax(w, 0.0);
            break;
        default:
            break;
        }
    }
    r->diag += lam;
    r->dtdiag += lam;
    r->rhs += lam * p->s_eq;
}

static prob_t mkprob(int nx, int ny, int nz, const uint8_t *solid, const double *ux,
                     const double *uy, const double *uz, const double *lam,
                     const int8_t *nf, double s_in, double s_eq, int pinned) {
    prob_t p;
    p.nx = nx; p.ny = ny; p.nz = nz; p.solid = solid;
    p.ux = ux; p.uy = uy; p.uz = uz; p.lam = lam; p.nf = nf;
    p.s_in = s_in; p.s_eq = s_eq; p.pinned = pinned;
    return p;
}

/* ------------------------------------------------------------------------------------ */
/* Geometry: fibre-face counts and connectivity                                           */
/* ------------------------------------------------------------------------------------ */

/* nf[P] = faces of pore cell P shared with a fibre voxel (walls excluded); -1 on fibre.
 * Returns the number of reactive (nf > 0) pore cells. */
long orc_fibre_faces(int nx, int ny, int nz, const uint8_t *solid, int8_t *nf) {
    long n = (long)nx * ny * nz, cnt = 0;
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                long P = x + nx * (y + ny * z);
                if (solid[P]) { nf[P] = -1; continue; }
                int c = 0;
                if (x > 0 && solid[P - 1]) ++c;
                if (x < nx - 1 && solid[P + 1]) ++c;
                if (y > 0 && solid[P - nx]) ++c;
                if (y < ny - 1 && solid[P + nx]) ++c;
                if (z > 0 && solid[P - (long)nx * ny]) ++c;
                if (z < nz - 1 && solid[P + (long)nx * ny]) ++c;
                nf[P] = (int8_t)c;
                if (c) ++cnt;
            }
    (void)n;
    return cnt;
}

/* Pore cells not face-connected to a pore cell of the inlet plane (breadth-first). */
long orc_disconnected(int nx, int ny, int nz, const uint8_t *solid) {
    long n = (long)nx * ny * nz;
    uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
    long *queue = (long *)malloc(sizeof(long) * (size_t)n);
    long head = 0, tail = 0, npore = 0;
    for (long P = 0; P < n; ++P) npore += !solid[P];
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y) {
            long P = nx * (y + ny * z);
            if (!solid[P]) { seen[P] = 1; queue[tail++] = P; }
        }
    while (head < tail) {
        long P = queue[head++];
        long x = P % nx, y = (P / nx) % ny, z = P / ((long)nx * ny);
        long nbs[6]; int k = 0;
        if (x > 0) nbs[k++] = P - 1;
        if (x < nx - 1) nbs[k++] = P + 1;
        if (y > 0) nbs[k++] = P - nx;
        if (y < ny - 1) nbs[k++] = P + nx;
        if (z > 0) nbs[k++] = P - (long)nx * ny;
        if (z < nz - 1) nbs[k++] = P + (long)nx * ny;
        for (int i = 0; i < k; ++i) {
            long q = nbs[i];
            if (!solid[q] && !seen[q]) { seen[q] = 1; queue[tail++] = q; }
        }
    }
    free(seen); free(queue);
    return npore - tail;
}

/* lam[P] = Da * kappa[P] * nf[P] on pore cells (kappa NULL: 1). */
void orc_reaction_coeff(int nx, int ny, int nz, const int8_t *nf, const double *kappa,
                        double Da, double *lam) {
    long n = (long)nx * ny * nz;
    for (long P = 0; P < n; ++P)
        lam[P] = nf[P] > 0 ? Da * (kappa ? kappa[P] : 1.0) * (double)nf[P] : 0.0;
}

/* ------------------------------------------------------------------------------------ */
/* Residual, time step, residual norm                                                     */
/* ------------------------------------------------------------------------------------ */

/* R = b - A s on every pore cell (0 on fibre and pinned cells).  Returns sum R^2. */
double orc_residual(int nx, int ny, int nz, const uint8_t *solid, const double *ux,
                    const double *uy, const double *uz, const double *lam, const int8_t *nf,
                    double s_in, double s_eq, int pinned, const double *s, double *R) {
    prob_t p = mkprob(nx, ny, nz, solid, ux, uy, uz, lam, nf, s_in, s_eq, pinned);
    double acc = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : acc)
    for (long z = 0; z < nz; ++z) {
        row_t r;
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                long P = cidx(&p, x, y, z);
                if (solid[P]) { R[P] = 0.0; continue; }
                row_of(&p, x, y, z, &r);
                if (r.held) { R[P] = 0.0; continue; }
                double v = r.rhs - r.diag * s[P];
                for (int f = 0; f < 6; ++f)
                    if (r.nb[f] >= 0) v -= r.coef[f] * s[r.nb[f]];
                R[P] = v;
                acc += v * v;
            }
    }
    return acc;
}

/* Time-step bound: max over updated pore cells of sum max(w,0) + sum G + lam. */
double orc_max_diag(int nx, int ny, int nz, const uint8_t *solid, const double *ux,
                    const double *uy, const double *uz, const double *lam, const int8_t *nf,
                    int pinned) {
    prob_t p = mkprob(nx, ny, nz, solid, ux, uy, uz, lam, nf, 0.0, 0.0, pinned);
    double m = 0.0;
    row_t r;
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                long P = cidx(&p, x, y, z);
                if (solid[P]) continue;
                row_of(&p, x, y, z, &r);
                if (!r.held && r.dtdiag > m) m = r.dtdiag;
            }
    return m;
}

/* Inlet volumetric flow Q = sum of +x face velocities over inlet pore cells. */
double orc_inflow(int nx, int ny, int nz, const uint8_t *solid, const double *ux) {
    double Q = 0.0;
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y) {
            long P = (long)nx * (y + (long)ny * z);
            if (!solid[P]) Q += ux[(nx + 1) * (y + (long)ny * z)];
        }
    return Q;
}

static long count_pore(long n, const uint8_t *solid) {
    long c = 0;
    for (long P = 0; P < n; ++P) c += !solid[P];
    return c;
}

/* ------------------------------------------------------------------------------------ */
/* Explicit pseudo-time iteration to steady state                                         */
/* ------------------------------------------------------------------------------------ */

/*
 * s (in/out): start state on entry (held cells are reset to s_eq), final state on exit.
 * Each iteration: R = R(s^n); s^{n+1} = s^n + dt R.  After every check_every iterations
 * the residual of the last update, tau*rms(R) = (tau/dt)||s^{n+1}-s^n||_rms, is compared
 * with tol.  out[0] = iterations, out[1] = final residual, out[2] = dt, out[3] = tau.
 * Returns 0 converged, 1 not converged within max_iter.
 */
int orc_solve(int nx, int ny, int nz, const uint8_t *solid, const double *ux,
              const double *uy, const double *uz, const double *lam, const int8_t *nf,
              double s_in, double s_eq, int pinned, double cfl, double tol, long max_iter,
              int check_every, double *s, double *out) {
    long n = (long)nx * ny * nz;
    prob_t p = mkprob(nx, ny, nz, solid, ux, uy, uz, lam, nf, s_in, s_eq, pinned);
    double dt = cfl / orc_max_diag(nx, ny, nz, solid, ux, uy, uz, lam, nf, pinned);
    double tau = (double)n / orc_inflow(nx, ny, nz, solid, ux);
    double npore = (double)count_pore(n, solid);
    double *R = (double *)malloc(sizeof(double) * (size_t)n);
    for (long P = 0; P < n; ++P) {
        if (solid[P]) s[P] = 0.0;
        else if (pinned && nf[P] > 0) s[P] = s_eq;
    }
    long it = 0;
    double res = INFINITY;
    int status = 1;
    if (check_every < 1) check_every = 1;
    while (it < max_iter) {
        double ss = orc_residual(nx, ny, nz, solid, ux, uy, uz, lam, nf, s_in, s_eq, pinned, s, R);
#pragma omp parallel for schedule(static)
        for (long P = 0; P < n; ++P) s[P] += dt * R[P];
        ++it;
        if (it % check_every == 0) {
            res = tau * sqrt(ss / npore);
            if (res < tol) { status = 0; break; }
        }
    }
    (void)p;
    free(R);
    out[0] = (double)it; out[1] = res; out[2] = dt; out[3] = tau;
    return status;
}

/*
 * Explicit Nernst model (Sec. "Steady State Reaction Model (Nernst)", Algorithm "Explicit
 * Nernst Model", with the electrode value of Eq. (nernst-model-s-update)).  Electrode cells
 * are the reactive pore cells (n_f > 0).  One iteration:
 *   1. transport step on every pore cell, s' = s + dt R_t(s), R_t the residual without the
 *      reaction term (advection and diffusion: the same faces and boundary values);
 *   2. on electrode cells, the instantaneous overpotential of Eq. (nernst-eta-inst-def) with
 *      D lap s replaced by the transport rate (s' - s) / dt = R_t:
 *        eta_I = 2 asinh(-R_t / (2 c sqrt(s (1 - s)))),  c = a k0 per cell = lam / K,
 *      K = e^{V/2} + e^{-V/2} = 1 / sqrt(s_eq (1 - s_eq)) the affine rate's slope at
 *      alpha = 1/2 (lam = Da kappa n_f carries a k0 K);
 *   3. eta <- (1 - omega) eta + omega eta_I (Eq. (nernst-model-eta-update));
 *   4. s' = sigma(V - eta) on electrode cells (Eq. (nernst-model-s-update)), V = logit(s_eq).
 * Stop when tau rms((s' - s) / dt) < tol, checked every check_every iterations; dt from the
 * transport-only diagonal.  The caller passes the start (s on pore cells, eta on electrode
 * cells); electrode cells start at sigma(V - eta).  0 < s_eq < 1, lam > 0 on electrode cells.
 * out: [iterations, residual, dt, tau].  Returns 0 on convergence, 1 otherwise.
 */
int orc_nernst(int nx, int ny, int nz, const uint8_t *solid, const double *ux,
               const double *uy, const double *uz, const double *lam, const int8_t *nf,
               double s_in, double s_eq, double omega, double cfl, double tol, long max_iter,
               int check_every, double *s, double *eta, double *out) {
    long n = (long)nx * ny * nz;
    double *lam0 = (double *)calloc((size_t)n, sizeof(double));
    double *R = (double *)malloc(sizeof(double) * (size_t)n);
    double dt = cfl / orc_max_diag(nx, ny, nz, solid, ux, uy, uz, lam0, nf, 0);
    double tau = (double)n / orc_inflow(nx, ny, nz, solid, ux);
    double npore = (double)count_pore(n, solid);
    double V = log(s_eq / (1.0 - s_eq));
    double K = 1.0 / sqrt(s_eq * (1.0 - s_eq));
    for (long P = 0; P < n; ++P) {
        if (solid[P]) { s[P] = 0.0; eta[P] = 0.0; }
        else if (nf[P] > 0) s[P] = 1.0 / (1.0 + exp(eta[P] - V));
        else eta[P] = 0.0;
    }
    long it = 0;
    double res = INFINITY;
    int status = 1;
    if (check_every < 1) check_every = 1;
    while (it < max_iter) {
        orc_residual(nx, ny, nz, solid, ux, uy, uz, lam0, nf, s_in, s_eq, 0, s, R);
        double ss = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : ss)
        for (long P = 0; P < n; ++P) {
            if (solid[P]) continue;
            double sn = s[P] + dt * R[P];
            if (nf[P] > 0) {
                double c = lam[P] / K;
                double sp = s[P];
                double eta_i = 2.0 * asinh(-R[P] / (2.0 * c * sqrt(sp * (1.0 - sp))));
                eta[P] = (1.0 - omega) * eta[P] + omega * eta_i;
                sn = 1.0 / (1.0 + exp(eta[P] - V));
            }
            double d = (sn - s[P]) / dt;
            ss += d * d;
            s[P] = sn;
        }
        ++it;
        if (it % check_every == 0) {
            res = tau * sqrt(ss / npore);
            if (!(res == res)) break;
            if (res < tol) { status = 0; break; }
        }
    }
    free(lam0);
    free(R);
    out[0] = (double)it; out[1] = res; out[2] = dt; out[3] = tau;
    return status;
}

/*
 * Fixed number of iterations (no residual checks): the timing leg uses this.
 */
void orc_iterate(int nx, int ny, int nz, const uint8_t *solid, const double *ux,
                 const double *uy, const double *uz, const double *lam, const int8_t *nf,
                 double s_in, double s_eq, int pinned, double dt, long iters, double *s,
                 double *R) {
    long n = (long)nx * ny * nz;
    for (long k = 0; k < iters; ++k) {
        orc_residual(nx, ny, nz, solid, ux, uy, uz, lam, nf, s_in, s_eq, pinned, s, R);
#pragma omp parallel for schedule(static)
        for (long P = 0; P < n; ++P) s[P] += dt * R[P];
    }
}

/* ------------------------------------------------------------------------------------ */
/* Outputs: utilisation and the flow / reaction balance                                   */
/* ------------------------------------------------------------------------------------ */

/*
 * out[0] U         = (sbar_out - s_in) / (s_eq - s_in)
 * out[1] sbar_out  = sum_outlet w s_P / sum_outlet w
 * out[2] F_in      = total (advective + diffusive) flux of s entering through the inlet
 * out[3] F_in_adv  = advective part only, sum_inlet u_x s_up (electron-flow definition;
 *                    s_up = s_in where u_x > 0, s_P where the flow leaves through the inlet)
 * out[4] F_out     = sum_outlet w s_P
 * out[5] reaction  = sum_P lam_P (s_P - s_eq)          (finite rate), or
 *                    sum over held cells of T_P (pinned), T_P = R_P without the
 *                    reaction term = what the electrode removes from cell P
 * out[6] sum_R     = sum over updated cells of R_P (F_in - F_out - reaction = sum_R)
 * out[7] Q_out     = sum_outlet w
 */
void orc_outputs(int nx, int ny, int nz, const uint8_t *solid, const double *ux,
                 const double *uy, const double *uz, const double *lam, const int8_t *nf,
                 double s_in, double s_eq, int pinned, const double *s, double *out) {
    prob_t p = mkprob(nx, ny, nz, solid, ux, uy, uz, lam, nf, s_in, s_eq, pinned);
    double fin = 0, fin_adv = 0, fout = 0, qout = 0, react = 0, sumR = 0;
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y) {
            long P0 = cidx(&p, 0, y, z), P1 = cidx(&p, nx - 1, y, z);
            if (!solid[P0]) {
                /* upwind: inflow brings s_in, outflow through the inlet carries s_P */
                double u = ux[(nx + 1) * (y + (long)ny * z)];
                double adv = dmax(u, 0.0) * s_in + dmin(u, 0.0) * s[P0];
                fin += adv + 2.0 * (s_in - s[P0]);
                fin_adv += adv;
            }
            if (!solid[P1]) {
                double w = ux[nx + (nx + 1) * (y + (long)ny * z)];
                fout += w * s[P1];
                qout += w;
            }
        }
    /* transport-only residual T_P (R without the reaction term) for the pinned balance */
    prob_t pt = p; pt.lam = NULL; pt.pinned = 0;
    row_t r;
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                long P = cidx(&p, x, y, z);
                if (solid[P]) continue;
                int held = pinned && nf[P] > 0;
                if (!held) {
                    if (lam) react += lam[P] * (s[P] - s_eq);
                    row_of(&p, x, y, z, &r);
                } else {
                    row_of(&pt, x, y, z, &r);
                }
                double v = r.rhs - r.diag * s[P];
                for (int f = 0; f < 6; ++f)
                    if (r.nb[f] >= 0) v -= r.coef[f] * s[r.nb[f]];
                if (held) react += v;           /* absorbed by the held electrode cell */
                else sumR += v;
            }
    out[0] = (fout / qout - s_in) / (s_eq - s_in);
    out[1] = fout / qout;
    out[2] = fin; out[3] = fin_adv; out[4] = fout; out[5] = react; out[6] = sumR;
    out[7] = qout;
}

/* ------------------------------------------------------------------------------------ */
/* Adjoint: A^T psi = g, g = dU/ds                                                        */
/* ------------------------------------------------------------------------------------ */

/* out = A^T psi restricted to updated (non-held) pore cells, by scattering each row. */
static void apply_AT(const prob_t *p, const double *psi, double *out) {
    long n = (long)p->nx * p->ny * p->nz;
    memset(out, 0, sizeof(double) * (size_t)n);
    row_t r;
    for (long z = 0; z < p->nz; ++z)
        for (long y = 0; y < p->ny; ++y)
            for (long x = 0; x < p->nx; ++x) {
                long Q = cidx(p, x, y, z);
                if (p->solid[Q]) { out[Q] += psi[Q]; continue; }
                row_of(p, x, y, z, &r);
                out[Q] += r.diag * psi[Q];
                for (int f = 0; f < 6; ++f)
                    if (r.nb[f] >= 0) out[r.nb[f]] += r.coef[f] * psi[Q];
            }
}

/* g_P = w_out,P / (sum_outlet w * (s_eq - s_in)) on outlet pore cells. */
void orc_adjoint_rhs(int nx, int ny, int nz, const uint8_t *solid, const double *ux,
                     double s_in, double s_eq, double *g) {
    long n = (long)nx * ny * nz;
    double qout = 0.0;
    memset(g, 0, sizeof(double) * (size_t)n);
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            if (!solid[(nx - 1) + (long)nx * (y + (long)ny * z)])
                qout += ux[nx + (nx + 1) * (y + (long)ny * z)];
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y) {
            long P = (nx - 1) + (long)nx * (y + (long)ny * z);
            if (!solid[P]) g[P] = ux[nx + (nx + 1) * (y + (long)ny * z)] / (qout * (s_eq - s_in));
        }
}

/*
 * psi <- psi + dt (g - A^T psi) on updated cells, from psi = 0, until
 * ||g - A^T psi||_2 / ||g||_2 < tol (checked every check_every iterations).  In pinned
 * mode the held cells' psi follows afterwards from their own column:
 * psi_P = g_P - sum_{Q != P} A_QP psi_Q.
 * The rows are stored once; A^T psi is formed per cell by gathering A_QP from each
 * neighbour Q's row at the face pointing back to P (a stencil couples faces in pairs:
 * face f of P is face f^1 of its neighbour), which the tests check against the
 * row-scatter product apply_AT and against SciPy's transpose.
 * out[0] = iterations, out[1] = final relative residual.  Returns 0 / 1 as orc_solve.
 */
static void gather_AT(int nx, int ny, int nz, const uint8_t *solid, const double *diag,
                      const long *nb, const double *coef, const double *psi, double *out) {
    long n = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (long P = 0; P < n; ++P) {
        double v = diag[P] * psi[P];
        if (!solid[P]) {
            long x = P % nx, y = (P / nx) % ny, z = P / ((long)nx * ny);
            long Qs[6] = {x > 0 ? P - 1 : -1, x < nx - 1 ? P + 1 : -1,
                          y > 0 ? P - nx : -1, y < ny - 1 ? P + nx : -1,
                          z > 0 ? P - (long)nx * ny : -1,
                          z < nz - 1 ? P + (long)nx * ny : -1};
            for (int f = 0; f < 6; ++f) {
                long Q = Qs[f];
                if (Q < 0 || solid[Q]) continue;
                /* Q sees P through the paired face f^1 (its row may not couple: held) */
                if (nb[6 * Q + (f ^ 1)] == P) v += coef[6 * Q + (f ^ 1)] * psi[Q];
            }
        }
        out[P] = v;
    }
}

/* t = A^T psi by gathering (exported for tests). */
void orc_apply_AT(int nx, int ny, int nz, const uint8_t *solid, const double *ux,
                  const double *uy, const double *uz, const double *lam, const int8_t *nf,
                  int pinned, const double *psi, double *t, int scatter) {
    long n = (long)nx * ny * nz;
    prob_t p = mkprob(nx, ny, nz, solid, ux, uy, uz, lam, nf, 0.0, 0.0, pinned);
    if (scatter) { apply_AT(&p, psi, t); return; }
    double *diag = (double *)malloc(sizeof(double) * (size_t)n);
    double *rhs = (double *)malloc(sizeof(double) * (size_t)n);
    uint8_t *held = (uint8_t *)malloc((size_t)n);
    long *nb = (long *)malloc(sizeof(long) * 6 * (size_t)n);
    double *coef = (double *)malloc(sizeof(double) * 6 * (size_t)n);
    orc_export_rows(nx, ny, nz, solid, ux, uy, uz, lam, nf, 0.0, 0.0, pinned, diag, rhs, held,
                    nb, coef);
    gather_AT(nx, ny, nz, solid, diag, nb, coef, psi, t);
    free(diag); free(rhs); free(held); free(nb); free(coef);
}

int orc_adjoint(int nx, int ny, int nz, const uint8_t *solid, const double *ux,
                const double *uy, const double *uz, const double *lam, const int8_t *nf,
                double s_in, double s_eq, int pinned, double cfl, double tol, long max_iter,
                int check_every, double *psi, double *out) {
    long n = (long)nx * ny * nz;
    double dt = cfl / orc_max_diag(nx, ny, nz, solid, ux, uy, uz, lam, nf, pinned);
    double *g = (double *)malloc(sizeof(double) * (size_t)n);
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    double *diag = (double *)malloc(sizeof(double) * (size_t)n);
    double *rhs = (double *)malloc(sizeof(double) * (size_t)n);
    uint8_t *held = (uint8_t *)malloc((size_t)n);
    long *nb = (long *)malloc(sizeof(long) * 6 * (size_t)n);
    double *coef = (double *)malloc(sizeof(double) * 6 * (size_t)n);
    orc_export_rows(nx, ny, nz, solid, ux, uy, uz, lam, nf, s_in, s_eq, pinned, diag, rhs, held,
                    nb, coef);
    orc_adjoint_rhs(nx, ny, nz, solid, ux, s_in, s_eq, g);
    double gn = 0.0;
    for (long P = 0; P < n; ++P) gn += g[P] * g[P];
    gn = sqrt(gn);
    memset(psi, 0, sizeof(double) * (size_t)n);
    long it = 0;
    double rel = INFINITY;
    int status = 1;
    if (check_every < 1) check_every = 1;
    while (it < max_iter) {
        gather_AT(nx, ny, nz, solid, diag, nb, coef, psi, t);
        double ss = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : ss)
        for (long P = 0; P < n; ++P) {
            if (held[P]) continue;              /* fibre and pinned cells */
            double r = g[P] - t[P];
            ss += r * r;
            psi[P] += dt * r;
        }
        ++it;
        if (it % check_every == 0) {
            rel = sqrt(ss) / gn;
            if (rel < tol) { status = 0; break; }
        }
    }
    if (pinned) {
        /* held rows are identity rows: psi_P = g_P - (A^T psi)_P without the P term */
        for (long P = 0; P < n; ++P)
            if (!solid[P] && nf[P] > 0) psi[P] = 0.0;
        gather_AT(nx, ny, nz, solid, diag, nb, coef, psi, t);
        for (long P = 0; P < n; ++P)
            if (!solid[P] && nf[P] > 0) psi[P] = g[P] - t[P];
    }
    free(g); free(t); free(diag); free(rhs); free(held); free(nb); free(coef);
    out[0] = (double)it; out[1] = rel;
    return status;
}

/*
 * Gradients from the adjoint state.
 *   dU/dkappa_P = Da * nf_P * psi_P * (s_eq - s_P)   (finite-rate mode; 0 elsewhere)
 *   dU/dln(q)   = sum_P psi_P * Radv_P(s; u)          (u = q u0: advective residual)
 * Returns dU/dln(q); divide by q for dU/dq.
 */
double orc_gradients(int nx, int ny, int nz, const uint8_t *solid, const double *ux,
                     const double *uy, const double *uz, const int8_t *nf, double Da,
                     double s_in, double s_eq, int pinned, const double *s, const double *psi,
                     double *dU_dkappa) {
    prob_t pa = mkprob(nx, ny, nz, solid, ux, uy, uz, NULL, nf, s_in, s_eq, pinned);
    double dq = 0.0;
    row_t r;
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                long P = cidx(&pa, x, y, z);
                if (dU_dkappa) dU_dkappa[P] = 0.0;
                if (solid[P]) continue;
                if (pinned && nf[P] > 0) continue;
                if (dU_dkappa && nf[P] > 0)
                    dU_dkappa[P] = Da * (double)nf[P] * psi[P] * (s_eq - s[P]);
                /* advective residual: the row with every G and lam set to zero */
                double adv = 0.0;
                for (int f = 0; f < 6; ++f) {
                    double w; int cls; long q;
                    face_of(&pa, x, y, z, f, &w, &cls, &q);
                    if (cls == F_INTERIOR) adv += -dmax(w, 0.0) * s[P] - dmin(w, 0.0) * s[q];
                    else if (cls == F_INLET) adv += -dmax(w, 0.0) * s[P] - dmin(w, 0.0) * s_in;
                    else if (cls == F_OUTLET) adv += -w * s[P];
                }
                dq += psi[P] * adv;
            }
    (void)r;
    return dq;
}

/* Rows of A s = b for a sparse assembly: diag[n], rhs[n], held[n], and for face f of
 * cell P nb[6P+f] (neighbour index or -1) and coef[6P+f] = A_P,nb.  Fibre cells get an
 * identity row with rhs 0. */
void orc_export_rows(int nx, int ny, int nz, const uint8_t *solid, const double *ux,
                     const double *uy, const double *uz, const double *lam, const int8_t *nf,
                     double s_in, double s_eq, int pinned, double *diag, double *rhs,
                     uint8_t *held, long *nb, double *coef) {
    prob_t p = mkprob(nx, ny, nz, solid, ux, uy, uz, lam, nf, s_in, s_eq, pinned);
#pragma omp parallel for schedule(static)
    for (long z = 0; z < nz; ++z) {
        row_t r;
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                long P = cidx(&p, x, y, z);
                if (solid[P]) {
                    diag[P] = 1.0; rhs[P] = 0.0; held[P] = 1;
                    for (int f = 0; f < 6; ++f) { nb[6 * P + f] = -1; coef[6 * P + f] = 0.0; }
                    continue;
                }
                row_of(&p, x, y, z, &r);
                diag[P] = r.diag; rhs[P] = r.rhs; held[P] = (uint8_t)r.held;
                for (int f = 0; f < 6; ++f) { nb[6 * P + f] = r.nb[f]; coef[6 * P + f] = r.coef[f]; }
            }
    }
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
