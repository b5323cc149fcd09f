/*
 * sanitize_driver.c -- runs the CPU oracle (bnref.c) from a case file, for builds with the
 * address and undefined-behaviour sanitizers.  TEST INFRASTRUCTURE: only the test-suite builds
 * and runs it; the HIP library never sees it.
 *
 * Case file (little-endian, written by the test):
 *   int32 nx, ny, steps, ncells, has_solid, bc[4], has_bottom
 *   double x0, x1, y0, y1, g, k0, rho0, alpha_liq, alpha_gas, cfl
 *   uint8 solid[nx*ny]            (if has_solid)
 *   double bottom[nx]             (if has_bottom: each column's bottom height)
 *   double q[4*nx*ny]             (state, planes of alpha rho, alpha rho u, alpha rho v, alpha)
 *   int64 cells[ncells]
 * Output file: the state after `steps` CFL steps, then [4][ncells] single-cell updates of that
 * state with its CFL step, then the reconstruction (faces, E-parts, centre, gradients) of every
 * fluid cell listed, then the free-surface heights.  Exit status 0, or the oracle's error code
 * negated (printed on stderr).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct { int32_t nx, ny; double x0, x1, y0, y1; } bnref_grid;
typedef struct {
    double g, k0, rho0, alpha_liq, alpha_gas, cfl;
    int32_t bc[4];
} bnref_params;

int bnref_run(const bnref_grid *, const bnref_params *, const uint8_t *, const double *, double *, int32_t, double *,
              double *);
int bnref_cfl(const bnref_grid *, const bnref_params *, const uint8_t *, const double *, double *, double *);
int bnref_step_cells(const bnref_grid *, const bnref_params *, const uint8_t *, const double *, const double *, double,
                     int64_t, const int64_t *, double *);
int bnref_reconstruct(const bnref_grid *, const bnref_params *, const uint8_t *, const double *, const double *,
                      int32_t, int32_t, double, double *, double *, double *, double *);
int bnref_detector(const bnref_grid *, const bnref_params *, const uint8_t *, const double *, const double *,
                   double *);

static void rd(void *p, size_t size, size_t n, FILE *f)
{
    if (fread(p, size, n, f) != n) {
        fprintf(stderr, "short case file\n");
        exit(2);
    }
}

int main(int argc, char **argv)
{
    int32_t hdr[10];
    double d[10];
    bnref_grid gr;
    bnref_params pa;
    uint8_t *solid = NULL;
    double *bottom = NULL;
    double *q, *out, *y0, t = 0.0, dt = 0.0, lam = 0.0;
    int64_t *cells;
    size_t plane;
    int k, rc;
    FILE *f, *o;
    if (argc != 3) return 2;
    f = fopen(argv[1], "rb");
    if (!f) return 2;
    rd(hdr, sizeof(int32_t), 10, f);
    rd(d, sizeof(double), 10, f);
    gr.nx = hdr[0]; gr.ny = hdr[1];
    gr.x0 = d[0]; gr.x1 = d[1]; gr.y0 = d[2]; gr.y1 = d[3];
    pa.g = d[4]; pa.k0 = d[5]; pa.rho0 = d[6]; pa.alpha_liq = d[7]; pa.alpha_gas = d[8]; pa.cfl = d[9];
    for (k = 0; k < 4; ++k) pa.bc[k] = hdr[5 + k];
    plane = (size_t)gr.nx * gr.ny;
    if (hdr[4]) {
        solid = (uint8_t *)malloc(plane);
        rd(solid, 1, plane, f);
    }
    if (hdr[9]) {
        bottom = (double *)malloc(sizeof(double) * gr.nx);
        rd(bottom, sizeof(double), (size_t)gr.nx, f);
    }
    q = (double *)malloc(sizeof(double) * 4 * plane);
    rd(q, sizeof(double), 4 * plane, f);
    cells = (int64_t *)malloc(sizeof(int64_t) * (hdr[3] > 0 ? hdr[3] : 1));
    rd(cells, sizeof(int64_t), (size_t)hdr[3], f);
    fclose(f);

    out = (double *)malloc(sizeof(double) * 4 * (hdr[3] > 0 ? hdr[3] : 1));
    y0 = (double *)malloc(sizeof(double) * gr.nx);
    o = NULL;
    rc = bnref_run(&gr, &pa, solid, bottom, q, hdr[2], &t, &dt);
    if (!rc) rc = bnref_cfl(&gr, &pa, solid, q, &lam, &dt);
    if (!rc) rc = bnref_step_cells(&gr, &pa, solid, bottom, q, dt, hdr[3], cells, out);
    if (rc) goto done;
    o = fopen(argv[2], "wb");
    if (!o) {
        rc = -100;
        goto done;
    }
    fwrite(q, sizeof(double), 4 * plane, o);
    fwrite(out, sizeof(double), 4 * (size_t)hdr[3], o);
    for (k = 0; k < hdr[3]; ++k) {
        double faces[20], ep[20], centre[5], grad[8];
        int32_t i = (int32_t)(cells[k] % gr.nx), j = (int32_t)(cells[k] / gr.nx);
        if (solid && solid[cells[k]]) continue;
        rc = bnref_reconstruct(&gr, &pa, solid, bottom, q, i, j, dt, faces, ep, centre, grad);
        if (rc < 0) goto done;
        fwrite(faces, sizeof(double), 20, o);
        fwrite(ep, sizeof(double), 20, o);
        fwrite(centre, sizeof(double), 5, o);
        fwrite(grad, sizeof(double), 8, o);
    }
    rc = bnref_detector(&gr, &pa, solid, bottom, q, y0);
    if (!rc) fwrite(y0, sizeof(double), (size_t)gr.nx, o);
done:
    if (o) fclose(o);
    if (rc) fprintf(stderr, "oracle error %d\n", rc);
    free(solid); free(bottom); free(q); free(out); free(cells); free(y0);
    return rc ? (rc < 0 ? -rc : rc) : 0;
}
