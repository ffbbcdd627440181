/* Driver of the FP64 oracle for the sanitizer test (test_sanitizers.py):
 * small 2D and 3D runs with CPML on every face, a box source, probes, the
 * design-cell trajectories, the adjoint sweep and single transposed steps,
 * built with AddressSanitizer and UndefinedBehaviorSanitizer.  Exit status
 * 0 and finite results. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int nx, ny;
    double dx, dy;
    double *ez, *hx, *hy;
    const double *ca, *cb, *db;
    double *psi_hx, *psi_hy, *psi_ezx, *psi_ezy;
    const double *prof_x, *prof_y;
} orc2d_t;
typedef struct {
    double *ez, *hx, *hy, *psi_hx, *psi_hy, *psi_ezx, *psi_ezy;
} orc2d_adj_t;
typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;
    double *ex, *ey, *ez, *hx, *hy, *hz;
    const double *ca, *cb, *db;
    double *psi[12];
    const double *prof_x, *prof_y, *prof_z;
} orc3d_t;

void orc_coeffs(long, double, const double *, const double *, const double *, double *, double *, double *);
void orc_cpml_axis(int, int, int, double, double, double, double, double, double, double, double *);
void orc_source(int, const double *, double, long, long, double *);
void orc2d_run(const orc2d_t *, long, long, const long *, const double *, int, const long *, double *, long,
               const int *, double *, double *);
void orc2d_adj_step(const orc2d_t *, orc2d_adj_t *);
void orc2d_adjoint(const orc2d_t *, orc2d_adj_t *, long, int, const long *, const double *, long, long,
                   const int *, const double *, const double *, const double *, const double *, double, double *);
void orc3d_run(const orc3d_t *, long, double *, long, const long *, const double *, const double *, int,
               const long *, double *, long);

static double *zeros(long n) { return (double *)calloc((size_t)n, sizeof(double)); }

static int finite_all(const double *a, long n) {
    for (long q = 0; q < n; ++q)
        if (!isfinite(a[q])) return 0;
    return 1;
}

int main(void) {
    const double c0 = 299792458.0, d = 1e-3, dt = 0.95 * d / (c0 * sqrt(3.0));
    int bad = 0;
    /* ---- 2D: 23 x 19, CPML 4/3/5/2, lossy dielectric, box source ---- */
    {
        const int nx = 23, ny = 19, T = 60;
        const long n = (long)nx * ny;
        double *er = zeros(n), *sg = zeros(n), *mr = zeros(n), *ca = zeros(n), *cb = zeros(n), *db = zeros(n);
        for (long c = 0; c < n; ++c) {
            er[c] = 1.0 + (c % 5);
            sg[c] = 0.001 * (c % 3);
            mr[c] = 1.0 + 0.5 * (c % 2);
        }
        orc_coeffs(n, dt, er, sg, mr, ca, cb, db);
        double *px = zeros(6 * nx), *py = zeros(6 * ny);
        orc_cpml_axis(nx, 4, 3, d, dt, 3.0, 0.0, 2.0, 0.05, 1.0, px);
        orc_cpml_axis(ny, 5, 2, d, dt, 3.0, 0.0, 2.0, 0.05, 1.0, py);
        orc2d_t s = {nx, ny, d, d, zeros(n), zeros(n), zeros(n), ca, cb, db,
                     zeros(n), zeros(n), zeros(n), zeros(n), px, py};
        double par[4] = {1.0, 20 * dt, 1.0 / (12 * dt), 0.0}, src[T];
        orc_source(1, par, dt, 0, T, src);
        long cells[4] = {8 * ny + 9, 8 * ny + 10, 9 * ny + 9, 9 * ny + 10};
        long probes[2] = {5 * ny + 14, 17 * ny + 6};
        double rec[2 * T];
        int design[4] = {10, 14, 6, 11};
        long nd = 4 * 5;
        double *tz = zeros(T * nd), *tb = zeros(T * nd);
        orc2d_run(&s, T, 4, cells, src, 2, probes, rec, T, design, tz, tb);
        bad += !finite_all(s.ez, n) || !finite_all(rec, 2 * T) || !finite_all(tb, T * nd);
        orc2d_adj_t a = {zeros(n), zeros(n), zeros(n), zeros(n), zeros(n), zeros(n), zeros(n)};
        double grad[20];
        orc2d_adjoint(&s, &a, T, 2, probes, rec, T / 2, T, design, tz, tb, er, sg, dt, grad);
        orc2d_adj_step(&s, &a);
        bad += !finite_all(grad, nd) || !finite_all(a.ez, n);
        free(a.ez); free(a.hx); free(a.hy); free(a.psi_hx); free(a.psi_hy); free(a.psi_ezx); free(a.psi_ezy);
        free(s.ez); free(s.hx); free(s.hy); free(s.psi_hx); free(s.psi_hy); free(s.psi_ezx); free(s.psi_ezy);
        free(er); free(sg); free(mr); free(ca); free(cb); free(db); free(px); free(py); free(tz); free(tb);
    }
    /* ---- 3D: 11 x 9 x 13, CPML on every face, Gaussian box source ---- */
    {
        const int nx = 11, ny = 9, nz = 13, T = 30;
        const long n = (long)nx * ny * nz;
        double *er = zeros(n), *ca = zeros(n), *cb = zeros(n), *db = zeros(n);
        for (long c = 0; c < n; ++c) er[c] = 1.0 + (c % 7) * 0.5;
        orc_coeffs(n, dt, er, NULL, NULL, ca, cb, db);
        double *px = zeros(6 * nx), *py = zeros(6 * ny), *pz = zeros(6 * nz);
        orc_cpml_axis(nx, 3, 2, d, dt, 3.0, 0.0, 1.0, 0.0, 1.0, px);
        orc_cpml_axis(ny, 2, 3, d, dt, 3.0, 0.0, 1.0, 0.0, 1.0, py);
        orc_cpml_axis(nz, 4, 1, d, dt, 3.0, 0.0, 1.0, 0.0, 1.0, pz);
        orc3d_t s;
        s.nx = nx; s.ny = ny; s.nz = nz; s.dx = s.dy = s.dz = d;
        s.ex = zeros(n); s.ey = zeros(n); s.ez = zeros(n); s.hx = zeros(n); s.hy = zeros(n); s.hz = zeros(n);
        s.ca = ca; s.cb = cb; s.db = db;
        for (int q = 0; q < 12; ++q) s.psi[q] = zeros(n);
        s.prof_x = px; s.prof_y = py; s.prof_z = pz;
        double par[4] = {1.0, 12 * dt, 3 * dt, 0.0}, src[T];
        orc_source(0, par, dt, 0, T, src);
        long cells[2] = {(5L * ny + 4) * nz + 6, (5L * ny + 4) * nz + 7};
        long probes[1] = {(7L * ny + 2) * nz + 9};
        double rec[T];
        orc3d_run(&s, T, s.ez, 2, cells, src, s.ez, 1, probes, rec, T);
        bad += !finite_all(s.ex, n) || !finite_all(s.hz, n) || !finite_all(rec, T);
        free(s.ex); free(s.ey); free(s.ez); free(s.hx); free(s.hy); free(s.hz);
        for (int q = 0; q < 12; ++q) free(s.psi[q]);
        free(er); free(ca); free(cb); free(db); free(px); free(py); free(pz);
    }
    printf("oracle sanitizer run: %s\n", bad ? "non-finite results" : "ok");
    return bad;
}
