/*
 * FP64 CPU oracle for FDTD leapfrog on a Yee grid (test infrastructure).
 *
 * This file is the plain, slow reference that the GPU path is checked
 * against.  Only the test-suite, the smoke check and the CPU baseline of the
 * benchmark may call it; the product library never links or loads it, and it
 * shares no source with it.
 *
 * What it computes (Sec. III of the paper, restated):
 *  - Ampere and Faraday laws with electric conductivity (Eq. 1-2), reduced to
 *    the 2D polarisation with one out-of-plane E component (Eq. 3-5).  The
 *    paper writes the TE form (Ey; Hx, Hz in the x-z plane); this oracle
 *    uses the identical TMz form (Ez; Hx, Hy) obtained by the relabelling
 *    Ez = -Ey, Hy = Hz, paper-z -> y.  The 3D oracle is the full six
 *    component Yee scheme that the paper says extends directly.
 *  - Centred differences on the staggered grid (Eq. 6) and the leapfrog
 *    update: H at half steps from the curl of E, then E at integer steps from
 *    the curl of H with the lossy factors A-/A+ and dt/(A+ eps) (Eq. 7-9 and
 *    the text after them).  This is the same linear map that Prop. 2 writes
 *    as two message-passing layers with fixed weights.
 *  - A convolutional PML (recursive-convolution auxiliary fields psi with
 *    graded sigma, kappa, alpha) in place of the paper's split-field PML of
 *    Sec. III-C; the paper gives no constants, the profile below takes them
 *    as parameters.
 *  - A soft point source (the paper names Gaussian / Ricker-like pulses but
 *    gives no formula), probes, and the discrete adjoint of the whole step
 *    (reverse-mode of each operation in reverse order) for gradients of a
 *    probe-energy loss with respect to per-cell relative permittivity.
 *
 * Conventions.  Arrays are row-major, last axis contiguous.
 *  2D: idx = i*ny + j.  Cell (i,j) owns Ez at (i,j), Hx at (i,j+1/2),
 *      Hy at (i+1/2,j).
 *  3D: idx = (i*ny + j)*nz + k.  Cell (i,j,k) owns Ex(i+1/2,j,k),
 *      Ey(i,j+1/2,k), Ez(i,j,k+1/2), Hx(i,j+1/2,k+1/2), Hy(i+1/2,j,k+1/2),
 *      Hz(i+1/2,j+1/2,k).
 *  Outer boundary: PEC.  Tangential E on the low planes (index 0) is never
 *  updated (stays at its initial value, zero in every physical run); values
 *  beyond the high end read as zero.
 *  A cell's eps_r / sigma apply to its E components, its mu_r to its H
 *  components.
 * Precision: everything in double.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

/* Built with -DORC_FP32 (liborc32.so) the same code runs in single
 * precision: an FP32 evaluation of the identical update, which the tests
 * use to find the rounding floor that any FP32 implementation of it has.
 * The oracle proper is the default FP64 build. */
#ifdef ORC_FP32
#define double float
#endif

/* CODATA 2018 */
static const double ORC_MU0 = 1.25663706212e-6;
static const double ORC_EPS0 = 8.8541878128e-12;
static const double ORC_PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* Material coefficients (Eq. 7-9):                                         */
/*   s  = sigma dt / (2 eps),  eps = eps0 eps_r                             */
/*   Ca = (1 - s)/(1 + s) = A-/A+,   Cb = (dt/eps)/(1 + s) = dt/(A+ eps)    */
/*   Db = dt/(mu0 mu_r)                                                      */
/* ------------------------------------------------------------------------ */
void orc_coeffs(long ncell, double dt, const double *eps_r, const double *sigma,
                const double *mu_r, double *ca, double *cb, double *db)
{
    for (long c = 0; c < ncell; ++c) {
        double er = eps_r ? eps_r[c] : 1.0;
        double sg = sigma ? sigma[c] : 0.0;
        double mr = mu_r ? mu_r[c] : 1.0;
        double eps = ORC_EPS0 * er;
        double s = sg * dt / (2.0 * eps);
        ca[c] = (1.0 - s) / (1.0 + s);
        cb[c] = (dt / eps) / (1.0 + s);
        db[c] = dt / (ORC_MU0 * mr);
    }
}

/* d Ca / d eps_r and d Cb / d eps_r for the adjoint. */
static void orc_dcoeffs(double er, double sg, double dt, double *dca, double *dcb)
{
    double e = ORC_EPS0 * er;
    double h = 0.5 * sg * dt;
    double den = (e + h) * (e + h);
    *dca = ORC_EPS0 * 2.0 * h / den;
    *dcb = -ORC_EPS0 * dt / den;
}

/* ------------------------------------------------------------------------ */
/* CPML profile along one axis of n cells with d_lo / d_hi absorbing cells  */
/* at the low / high face.  Normalised depth rho in [0,1] (1 at the wall):  */
/* E-type samples at x = i, H-type at x = i + 1/2.                          */
/*   sigma = sigma_max rho^m, kappa = 1 + (kappa_max - 1) rho^m,            */
/*   alpha = alpha_max (1 - rho)^m_alpha (only where rho > 0),              */
/*   b = exp(-(sigma/kappa + alpha) dt/eps0),                               */
/*   c = sigma (b - 1) / (kappa (sigma + kappa alpha))  (0 if sigma = 0).   */
/* sigma_max <= 0 selects 0.8 (m + 1)/(eta0 delta).                         */
/* Output prof[6*n]: bE, cE, ikE (=1/kappa), bH, cH, ikH, each of length n. */
/* ------------------------------------------------------------------------ */
void orc_cpml_axis(int n, int d_lo, int d_hi, double delta, double dt, double m,
                   double sigma_max, double kappa_max, double alpha_max,
                   double m_alpha, double *prof)
{
    double eta0 = sqrt(ORC_MU0 / ORC_EPS0);
    double smax = sigma_max > 0.0 ? sigma_max : 0.8 * (m + 1.0) / (eta0 * delta);
    for (int half = 0; half < 2; ++half) {
        double *b = prof + (half ? 3 * n : 0);
        double *c = b + n;
        double *ik = b + 2 * n;
        for (int i = 0; i < n; ++i) {
            double x = i + (half ? 0.5 : 0.0);
            double rho = 0.0;
            if (d_lo > 0 && x < d_lo) rho = (d_lo - x) / d_lo;
            if (d_hi > 0 && x > n - d_hi) {
                double r2 = (x - (n - d_hi)) / d_hi;
                if (r2 > rho) rho = r2;
            }
            if (rho <= 0.0) {
                b[i] = 1.0;
                c[i] = 0.0;
                ik[i] = 1.0;
                continue;
            }
            double pm = pow(rho, m);
            double sg = smax * pm;
            double kp = 1.0 + (kappa_max - 1.0) * pm;
            double al = alpha_max * pow(1.0 - rho, m_alpha);
            double bb = exp(-(sg / kp + al) * dt / ORC_EPS0);
            b[i] = bb;
            c[i] = sg > 0.0 ? sg * (bb - 1.0) / (kp * (sg + kp * al)) : 0.0;
            ik[i] = 1.0 / kp;
        }
    }
}

/* Source samples out[k] = amp * g((n0 + k + 1) dt), k in [0, count).  The
 * paper names Gaussian, sinusoidal and modulated Gaussian sources (Sec. V-A,
 * V-B) without formulas; these are the readings taken:
 * kind 0 (Gaussian): params {amp, t0, tau}, g = exp(-((t - t0)/tau)^2)
 * kind 1 (Ricker):   params {amp, t0, f},   g = (1 - 2 a) exp(-a), a = (pi f (t - t0))^2
 * kind 3 (sine):     params {amp, f, T},    g = w(t) sin(2 pi f t), where the
 *                    turn-on w rises as sin^2(pi t / 2T) up to t = T, then 1
 * kind 4 (modulated Gaussian): params {amp, t0, tau, f},
 *                    g = exp(-((t - t0)/tau)^2) sin(2 pi f (t - t0)) */
void orc_source(int kind, const double *params, double dt, long n0, long count,
                double *out)
{
    for (long k = 0; k < count; ++k) {
        double t = (double)(n0 + k + 1) * dt;
        double v;
        if (kind == 0) {
            double u = (t - params[1]) / params[2];
            v = exp(-u * u);
        } else if (kind == 1) {
            double a = ORC_PI * params[2] * (t - params[1]);
            a = a * a;
            v = (1.0 - 2.0 * a) * exp(-a);
        } else if (kind == 3) {
            double w = 1.0;
            if (t < params[2]) {
                double h = sin(ORC_PI * t / (2.0 * params[2]));
                w = h * h;
            }
            v = w * sin(2.0 * ORC_PI * params[1] * t);
        } else {
            double s = t - params[1];
            double u = s / params[2];
            v = exp(-u * u) * sin(2.0 * ORC_PI * params[3] * s);
        }
        out[k] = params[0] * v;
    }
}

/* ======================================================================== */
/* 2D TMz                                                                   */
/* ======================================================================== */
typedef struct {
    int nx, ny;
    double dx, dy;
    double *ez, *hx, *hy;
    const double *ca, *cb, *db;
    double *psi_hx, *psi_hy, *psi_ezx, *psi_ezy; /* full grid, zero where unused */
    const double *prof_x, *prof_y;               /* 6*nx and 6*ny (orc_cpml_axis) */
} orc2d_t;

#define P_BE(p, n, i) ((p)[(i)])
#define P_CE(p, n, i) ((p)[(n) + (i)])
#define P_KE(p, n, i) ((p)[2 * (n) + (i)])
#define P_BH(p, n, i) ((p)[3 * (n) + (i)])
#define P_CH(p, n, i) ((p)[4 * (n) + (i)])
#define P_KH(p, n, i) ((p)[5 * (n) + (i)])
/* The CPML auxiliary value psi of a difference along an axis exists only in
 * that axis's absorbing layer: elsewhere b = 1 and c = 0, so a psi that
 * starts at zero stays zero and adds nothing.  The updates below touch psi
 * only where the profile is not (b, c) = (1, 0) and use 0 elsewhere. */
#define IN_LAYER_E(p, n, i) (P_BE(p, n, i) != 1.0 || P_CE(p, n, i) != 0.0)
#define IN_LAYER_H(p, n, i) (P_BH(p, n, i) != 1.0 || P_CH(p, n, i) != 0.0)

/* H layer: messages from the E nodes to Hx, Hy (Eq. 8-9, TMz form).  If
 * brx / bry are given, they receive the brackets that multiply Db (Hx -=
 * Db brx, Hy += Db bry), for the adjoint. */
void orc2d_h_layer_br(const orc2d_t *s, double *brx, double *bry)
{
    const int nx = s->nx, ny = s->ny;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i) {
        for (int j = 0; j < ny; ++j) {
            long c = (long)i * ny + j;
            double e0 = s->ez[c];
            double ey1 = (j + 1 < ny) ? s->ez[c + 1] : 0.0;
            double ex1 = (i + 1 < nx) ? s->ez[c + ny] : 0.0;
            double dey = (ey1 - e0) / s->dy;
            double dex = (ex1 - e0) / s->dx;
            double phx = 0.0, phy = 0.0; /* psi outside the absorbing layer: 0 */
            if (IN_LAYER_H(s->prof_y, ny, j)) {
                s->psi_hx[c] = P_BH(s->prof_y, ny, j) * s->psi_hx[c] + P_CH(s->prof_y, ny, j) * dey;
                phx = s->psi_hx[c];
            }
            const double bx = dey * P_KH(s->prof_y, ny, j) + phx;
            if (brx) brx[c] = bx;
            s->hx[c] -= s->db[c] * bx;
            if (IN_LAYER_H(s->prof_x, nx, i)) {
                s->psi_hy[c] = P_BH(s->prof_x, nx, i) * s->psi_hy[c] + P_CH(s->prof_x, nx, i) * dex;
                phy = s->psi_hy[c];
            }
            const double by = dex * P_KH(s->prof_x, nx, i) + phy;
            if (bry) bry[c] = by;
            s->hy[c] += s->db[c] * by;
        }
    }
}

void orc2d_h_layer(const orc2d_t *s) { orc2d_h_layer_br(s, NULL, NULL); }

/* E layer: messages from Hx, Hy to the Ez nodes (Eq. 7, TMz form).  If curl
 * is given, curl[c] receives the bracket multiplied by Cb (for the adjoint). */
void orc2d_e_layer(const orc2d_t *s, double *curl)
{
    const int nx = s->nx, ny = s->ny;
#pragma omp parallel for schedule(static)
    for (int i = 1; i < nx; ++i) {
        for (int j = 1; j < ny; ++j) {
            long c = (long)i * ny + j;
            double dhy = (s->hy[c] - s->hy[c - ny]) / s->dx;
            double dhx = (s->hx[c] - s->hx[c - 1]) / s->dy;
            double pex = 0.0, pey = 0.0; /* psi outside the absorbing layer: 0 */
            if (IN_LAYER_E(s->prof_x, nx, i)) {
                s->psi_ezx[c] = P_BE(s->prof_x, nx, i) * s->psi_ezx[c] + P_CE(s->prof_x, nx, i) * dhy;
                pex = s->psi_ezx[c];
            }
            if (IN_LAYER_E(s->prof_y, ny, j)) {
                s->psi_ezy[c] = P_BE(s->prof_y, ny, j) * s->psi_ezy[c] + P_CE(s->prof_y, ny, j) * dhx;
                pey = s->psi_ezy[c];
            }
            double br = dhy * P_KE(s->prof_x, nx, i) - dhx * P_KE(s->prof_y, ny, j)
                      + pex - pey;
            if (curl) curl[c] = br;
            s->ez[c] = s->ca[c] * s->ez[c] + s->cb[c] * br;
        }
    }
}

/*
 * Run nsteps leapfrog steps.  Step k (0-based within this call):
 *   H layer, E layer, Ez[c] += src_vals[k] for each of the nsrc source cells
 *   c, rec[p*rec_stride + k] = Ez[probe p].
 * If design != NULL ({i0,i1,j0,j1}), the Ez value before the E layer and
 * the bracket of the E layer at every design cell are stored per step in
 * traj_ez / traj_br ([nsteps][(i1-i0)*(j1-j0)]) for the adjoint, and, if
 * traj_bx / traj_by are given, the brackets of the H layer (Hx -= Db bx,
 * Hy += Db by) likewise.
 */
void orc2d_run_mu(const orc2d_t *s, long nsteps, long nsrc, const long *src_cells, const double *src_vals,
                  int np, const long *probe_idx, double *rec, long rec_stride,
                  const int *design, double *traj_ez, double *traj_br, double *traj_bx, double *traj_by)
{
    const int ny = s->ny;
    long nd = design ? (long)(design[1] - design[0]) * (design[3] - design[2]) : 0;
    double *curl = NULL, *bx = NULL, *by = NULL;
    if (design) curl = (double *)calloc((size_t)s->nx * ny, sizeof(double));
    if (design && traj_bx && traj_by) {
        bx = (double *)calloc((size_t)s->nx * ny, sizeof(double));
        by = (double *)calloc((size_t)s->nx * ny, sizeof(double));
    }
    for (long k = 0; k < nsteps; ++k) {
        orc2d_h_layer_br(s, bx, by);
        if (bx) {
            long q = 0;
            for (int i = design[0]; i < design[1]; ++i)
                for (int j = design[2]; j < design[3]; ++j, ++q) {
                    traj_bx[k * nd + q] = bx[(long)i * ny + j];
                    traj_by[k * nd + q] = by[(long)i * ny + j];
                }
        }
        if (design) {
            long q = 0;
            for (int i = design[0]; i < design[1]; ++i)
                for (int j = design[2]; j < design[3]; ++j)
                    traj_ez[k * nd + q++] = s->ez[(long)i * ny + j];
        }
        orc2d_e_layer(s, curl);
        if (design) {
            long q = 0;
            for (int i = design[0]; i < design[1]; ++i)
                for (int j = design[2]; j < design[3]; ++j)
                    traj_br[k * nd + q++] = curl[(long)i * ny + j];
        }
        for (long q = 0; q < nsrc && src_vals; ++q) s->ez[src_cells[q]] += src_vals[k];
        for (int p = 0; p < np; ++p) rec[(long)p * rec_stride + k] = s->ez[probe_idx[p]];
    }
    free(curl);
    free(bx);
    free(by);
}

void orc2d_run(const orc2d_t *s, long nsteps, long nsrc, const long *src_cells, const double *src_vals,
               int np, const long *probe_idx, double *rec, long rec_stride,
               const int *design, double *traj_ez, double *traj_br)
{
    orc2d_run_mu(s, nsteps, nsrc, src_cells, src_vals, np, probe_idx, rec, rec_stride, design, traj_ez,
                 traj_br, NULL, NULL);
}

/* Adjoint variables: one per forward state variable. */
typedef struct {
    double *ez, *hx, *hy, *psi_hx, *psi_hy, *psi_ezx, *psi_ezy;
} orc2d_adj_t;

/* Transpose of the E layer.  Incoming a->* are the adjoints of the values
 * after the layer; on return they are the adjoints of the values before it.
 * Per E-layer cell with u = Cb * aEz:
 *   aPsiEzx_before = bEx (aPsiEzx + u),   aPsiEzy_before = bEy (aPsiEzy - u)
 *   adjoint of dHy: gy = u ikEx + cEx (aPsiEzx + u)
 *   adjoint of dHx: gx = -u ikEy + cEy (aPsiEzy - u)
 *   aHy[i][j] += gy/dx, aHy[i-1][j] -= gy/dx, aHx[i][j] += gx/dy, aHx[i][j-1] -= gx/dy
 *   aEz_before = Ca aEz
 * Cells the layer does not touch (i = 0 or j = 0) pass their adjoints through. */
static void orc2d_adj_e_layer(const orc2d_t *s, orc2d_adj_t *a, double *gx, double *gy)
{
    const int nx = s->nx, ny = s->ny;
    memset(gx, 0, sizeof(double) * (size_t)nx * ny);
    memset(gy, 0, sizeof(double) * (size_t)nx * ny);
    for (int i = 1; i < nx; ++i) {
        for (int j = 1; j < ny; ++j) {
            long c = (long)i * ny + j;
            double u = s->cb[c] * a->ez[c];
            double px = a->psi_ezx[c] + u;
            double py = a->psi_ezy[c] - u;
            gy[c] = u * P_KE(s->prof_x, nx, i) + P_CE(s->prof_x, nx, i) * px;
            gx[c] = -u * P_KE(s->prof_y, ny, j) + P_CE(s->prof_y, ny, j) * py;
            a->psi_ezx[c] = P_BE(s->prof_x, nx, i) * px;
            a->psi_ezy[c] = P_BE(s->prof_y, ny, j) * py;
            a->ez[c] = s->ca[c] * a->ez[c];
        }
    }
    for (int i = 1; i < nx; ++i) {
        for (int j = 1; j < ny; ++j) {
            long c = (long)i * ny + j;
            a->hy[c] += gy[c] / s->dx;
            a->hy[c - ny] -= gy[c] / s->dx;
            a->hx[c] += gx[c] / s->dy;
            a->hx[c - 1] -= gx[c] / s->dy;
        }
    }
}

/* Transpose of the H layer (the H nodes keep their own adjoint: self weight 1).
 *   Hx: w = aPsiHx - Db aHx;  aPsiHx_before = bHy w;
 *       adjoint of dEy: e = -Db aHx ikHy + cHy w;  aEz[i][j+1] += e/dy, aEz[i][j] -= e/dy
 *   Hy: w = aPsiHy + Db aHy;  aPsiHy_before = bHx w;
 *       adjoint of dEx: e = Db aHy ikHx + cHx w;   aEz[i+1][j] += e/dx, aEz[i][j] -= e/dx */
static void orc2d_adj_h_layer(const orc2d_t *s, orc2d_adj_t *a)
{
    const int nx = s->nx, ny = s->ny;
    for (int i = 0; i < nx; ++i) {
        for (int j = 0; j < ny; ++j) {
            long c = (long)i * ny + j;
            double wx = a->psi_hx[c] - s->db[c] * a->hx[c];
            double ey = -s->db[c] * a->hx[c] * P_KH(s->prof_y, ny, j) + P_CH(s->prof_y, ny, j) * wx;
            a->psi_hx[c] = P_BH(s->prof_y, ny, j) * wx;
            if (j + 1 < ny) a->ez[c + 1] += ey / s->dy;
            a->ez[c] -= ey / s->dy;
            double wy = a->psi_hy[c] + s->db[c] * a->hy[c];
            double ex = s->db[c] * a->hy[c] * P_KH(s->prof_x, nx, i) + P_CH(s->prof_x, nx, i) * wy;
            a->psi_hy[c] = P_BH(s->prof_x, nx, i) * wy;
            if (i + 1 < nx) a->ez[c + ny] += ex / s->dx;
            a->ez[c] -= ex / s->dx;
        }
    }
}

/* One transposed step (E layer^T then H layer^T), exposed for dot-product tests. */
void orc2d_adj_step(const orc2d_t *s, orc2d_adj_t *a)
{
    long n = (long)s->nx * s->ny;
    double *gx = (double *)malloc(sizeof(double) * (size_t)n);
    double *gy = (double *)malloc(sizeof(double) * (size_t)n);
    orc2d_adj_e_layer(s, a, gx, gy);
    orc2d_adj_h_layer(s, a);
    free(gx);
    free(gy);
}

/*
 * Backward sweep for L = sum_p sum_{m in (n0, n1]} Ez^m[p]^2 after a forward
 * run of T steps from state 0 (Ez^m = value after step m-1, m = 1..T).
 * probe_ez[p*T + k] = Ez^{k+1}[p]; traj_* come from orc2d_run with the design
 * box.  grad[(i-i0)*(j1-j0) + (j-j0)] receives dL/d eps_r for each design
 * cell; a (zero on entry) holds the adjoint of the initial state on return.
 */
void orc2d_adjoint_mu(const orc2d_t *s, orc2d_adj_t *a, long T, int np,
                      const long *probe_idx, const double *probe_ez, long n0, long n1,
                      const int *design, const double *traj_ez, const double *traj_br,
                      const double *eps_r, const double *sigma, double dt, double *grad,
                      const double *traj_bx, const double *traj_by, const double *mu_r, double *grad_mu)
{
    const int ny = s->ny;
    long n = (long)s->nx * ny;
    long dj = design[3] - design[2];
    long nd = (long)(design[1] - design[0]) * dj;
    double *gx = (double *)malloc(sizeof(double) * (size_t)n);
    double *gy = (double *)malloc(sizeof(double) * (size_t)n);
    for (long q = 0; q < nd; ++q) grad[q] = 0.0;
    if (grad_mu)
        for (long q = 0; q < nd; ++q) grad_mu[q] = 0.0;
    for (long k = T - 1; k >= 0; --k) {
        /* loss term of Ez^{k+1} (probe recorded after step k) */
        long m = k + 1;
        if (m > n0 && m <= n1)
            for (int p = 0; p < np; ++p) a->ez[probe_idx[p]] += 2.0 * probe_ez[(long)p * T + k];
        /* gradient: Ez_after = Ca Ez_before + Cb * bracket */
        for (int i = design[0]; i < design[1]; ++i) {
            for (int j = design[2]; j < design[3]; ++j) {
                if (i < 1 || j < 1) continue;
                long c = (long)i * ny + j;
                long q = (long)(i - design[0]) * dj + (j - design[2]);
                double dca, dcb;
                orc_dcoeffs(eps_r ? eps_r[c] : 1.0, sigma ? sigma[c] : 0.0, dt, &dca, &dcb);
                grad[q] += a->ez[c] * (dca * traj_ez[k * nd + q] + dcb * traj_br[k * nd + q]);
            }
        }
        orc2d_adj_e_layer(s, a, gx, gy);
        /* gradient with respect to mu_r: Hx -= Db bx and Hy += Db by with
         * Db = dt / (mu0 mu_r), weighted by the adjoints of Hx, Hy after the
         * H layer (they hold them now): dL/dmu_r += (Db / mu_r) (aHx bx - aHy by) */
        if (grad_mu) {
            for (int i = design[0]; i < design[1]; ++i) {
                for (int j = design[2]; j < design[3]; ++j) {
                    long c = (long)i * ny + j;
                    long q = (long)(i - design[0]) * dj + (j - design[2]);
                    double mr = mu_r ? mu_r[c] : 1.0;
                    grad_mu[q] += s->db[c] / mr * (a->hx[c] * traj_bx[k * nd + q] - a->hy[c] * traj_by[k * nd + q]);
                }
            }
        }
        orc2d_adj_h_layer(s, a);
    }
    free(gx);
    free(gy);
}

void orc2d_adjoint(const orc2d_t *s, orc2d_adj_t *a, long T, int np,
                   const long *probe_idx, const double *probe_ez, long n0, long n1,
                   const int *design, const double *traj_ez, const double *traj_br,
                   const double *eps_r, const double *sigma, double dt, double *grad)
{
    orc2d_adjoint_mu(s, a, T, np, probe_idx, probe_ez, n0, n1, design, traj_ez, traj_br, eps_r, sigma, dt,
                     grad, NULL, NULL, NULL, NULL);
}

/* ======================================================================== */
/* 3D Yee                                                                   */
/* ======================================================================== */
typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;
    double *ex, *ey, *ez, *hx, *hy, *hz;
    const double *ca, *cb, *db;
    /* psi_<field><axis>, full grid */
    double *psi_hxy, *psi_hxz, *psi_hyz, *psi_hyx, *psi_hzx, *psi_hzy;
    double *psi_exy, *psi_exz, *psi_eyz, *psi_eyx, *psi_ezx, *psi_ezy;
    const double *prof_x, *prof_y, *prof_z;
} orc3d_t;

void orc3d_h_layer(const orc3d_t *s)
{
    const int nx = s->nx, ny = s->ny, nz = s->nz;
    const long sx = (long)ny * nz, sy = nz;
    const double *px = s->prof_x, *py = s->prof_y, *pz = s->prof_z;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i) {
        const int lx = IN_LAYER_H(px, nx, i);
        for (int j = 0; j < ny; ++j) {
            const int ly = IN_LAYER_H(py, ny, j);
            for (int k = 0; k < nz; ++k) {
                long c = i * sx + j * sy + k;
                double ex0 = s->ex[c], ey0 = s->ey[c], ez0 = s->ez[c];
                double ex_y = (j + 1 < ny) ? s->ex[c + sy] : 0.0;
                double ex_z = (k + 1 < nz) ? s->ex[c + 1] : 0.0;
                double ey_x = (i + 1 < nx) ? s->ey[c + sx] : 0.0;
                double ey_z = (k + 1 < nz) ? s->ey[c + 1] : 0.0;
                double ez_x = (i + 1 < nx) ? s->ez[c + sx] : 0.0;
                double ez_y = (j + 1 < ny) ? s->ez[c + sy] : 0.0;
                double dezdy = (ez_y - ez0) / s->dy, deydz = (ey_z - ey0) / s->dz;
                double dexdz = (ex_z - ex0) / s->dz, dezdx = (ez_x - ez0) / s->dx;
                double deydx = (ey_x - ey0) / s->dx, dexdy = (ex_y - ex0) / s->dy;
                /* psi outside the absorbing layer of its axis: 0 */
                double pxy = 0.0, pxz = 0.0, pyz = 0.0, pyx = 0.0, pzx = 0.0, pzy = 0.0;
                if (lx) {
                    s->psi_hyx[c] = P_BH(px, nx, i) * s->psi_hyx[c] + P_CH(px, nx, i) * dezdx;
                    s->psi_hzx[c] = P_BH(px, nx, i) * s->psi_hzx[c] + P_CH(px, nx, i) * deydx;
                    pyx = s->psi_hyx[c];
                    pzx = s->psi_hzx[c];
                }
                if (ly) {
                    s->psi_hxy[c] = P_BH(py, ny, j) * s->psi_hxy[c] + P_CH(py, ny, j) * dezdy;
                    s->psi_hzy[c] = P_BH(py, ny, j) * s->psi_hzy[c] + P_CH(py, ny, j) * dexdy;
                    pxy = s->psi_hxy[c];
                    pzy = s->psi_hzy[c];
                }
                if (IN_LAYER_H(pz, nz, k)) {
                    s->psi_hxz[c] = P_BH(pz, nz, k) * s->psi_hxz[c] + P_CH(pz, nz, k) * deydz;
                    s->psi_hyz[c] = P_BH(pz, nz, k) * s->psi_hyz[c] + P_CH(pz, nz, k) * dexdz;
                    pxz = s->psi_hxz[c];
                    pyz = s->psi_hyz[c];
                }
                s->hx[c] -= s->db[c] * (dezdy * P_KH(py, ny, j) + pxy
                                        - deydz * P_KH(pz, nz, k) - pxz);
                s->hy[c] -= s->db[c] * (dexdz * P_KH(pz, nz, k) + pyz
                                        - dezdx * P_KH(px, nx, i) - pyx);
                s->hz[c] -= s->db[c] * (deydx * P_KH(px, nx, i) + pzx
                                        - dexdy * P_KH(py, ny, j) - pzy);
            }
        }
    }
}

void orc3d_e_layer(const orc3d_t *s)
{
    const int nx = s->nx, ny = s->ny, nz = s->nz;
    const long sx = (long)ny * nz, sy = nz;
    const double *px = s->prof_x, *py = s->prof_y, *pz = s->prof_z;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i) {
        const int lx = IN_LAYER_E(px, nx, i);
        for (int j = 0; j < ny; ++j) {
            const int ly = IN_LAYER_E(py, ny, j);
            for (int k = 0; k < nz; ++k) {
                long c = i * sx + j * sy + k;
                const int lz = IN_LAYER_E(pz, nz, k);
                /* psi outside the absorbing layer of its axis: 0 */
                if (j >= 1 && k >= 1) {
                    double dhzdy = (s->hz[c] - s->hz[c - sy]) / s->dy;
                    double dhydz = (s->hy[c] - s->hy[c - 1]) / s->dz;
                    double qy = 0.0, qz = 0.0;
                    if (ly) {
                        s->psi_exy[c] = P_BE(py, ny, j) * s->psi_exy[c] + P_CE(py, ny, j) * dhzdy;
                        qy = s->psi_exy[c];
                    }
                    if (lz) {
                        s->psi_exz[c] = P_BE(pz, nz, k) * s->psi_exz[c] + P_CE(pz, nz, k) * dhydz;
                        qz = s->psi_exz[c];
                    }
                    s->ex[c] = s->ca[c] * s->ex[c]
                             + s->cb[c] * (dhzdy * P_KE(py, ny, j) + qy
                                           - dhydz * P_KE(pz, nz, k) - qz);
                }
                if (i >= 1 && k >= 1) {
                    double dhxdz = (s->hx[c] - s->hx[c - 1]) / s->dz;
                    double dhzdx = (s->hz[c] - s->hz[c - sx]) / s->dx;
                    double qz = 0.0, qx = 0.0;
                    if (lz) {
                        s->psi_eyz[c] = P_BE(pz, nz, k) * s->psi_eyz[c] + P_CE(pz, nz, k) * dhxdz;
                        qz = s->psi_eyz[c];
                    }
                    if (lx) {
                        s->psi_eyx[c] = P_BE(px, nx, i) * s->psi_eyx[c] + P_CE(px, nx, i) * dhzdx;
                        qx = s->psi_eyx[c];
                    }
                    s->ey[c] = s->ca[c] * s->ey[c]
                             + s->cb[c] * (dhxdz * P_KE(pz, nz, k) + qz
                                           - dhzdx * P_KE(px, nx, i) - qx);
                }
                if (i >= 1 && j >= 1) {
                    double dhydx = (s->hy[c] - s->hy[c - sx]) / s->dx;
                    double dhxdy = (s->hx[c] - s->hx[c - sy]) / s->dy;
                    double qx = 0.0, qy = 0.0;
                    if (lx) {
                        s->psi_ezx[c] = P_BE(px, nx, i) * s->psi_ezx[c] + P_CE(px, nx, i) * dhydx;
                        qx = s->psi_ezx[c];
                    }
                    if (ly) {
                        s->psi_ezy[c] = P_BE(py, ny, j) * s->psi_ezy[c] + P_CE(py, ny, j) * dhxdy;
                        qy = s->psi_ezy[c];
                    }
                    s->ez[c] = s->ca[c] * s->ez[c]
                             + s->cb[c] * (dhydx * P_KE(px, nx, i) + qx
                                           - dhxdy * P_KE(py, ny, j) - qy);
                }
            }
        }
    }
}

/* Run nsteps 3D steps; src_field / probe_field point at one of the six
 * component arrays of s (the soft source and probes act on that component). */
void orc3d_run(const orc3d_t *s, long nsteps, double *src_field, long nsrc, const long *src_cells,
               const double *src_vals, const double *probe_field, int np,
               const long *probe_idx, double *rec, long rec_stride)
{
    for (long k = 0; k < nsteps; ++k) {
        orc3d_h_layer(s);
        orc3d_e_layer(s);
        for (long q = 0; q < nsrc && src_field && src_vals; ++q) src_field[src_cells[q]] += src_vals[k];
        for (int p = 0; p < np; ++p) rec[(long)p * rec_stride + k] = probe_field[probe_idx[p]];
    }
}
