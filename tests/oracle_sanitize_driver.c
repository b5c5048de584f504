/* Host driver for an AddressSanitizer + UndefinedBehaviorSanitizer build of
 * the FP64 oracle (oracle/dnnmg_oracle.c, linked in): every exported
 * function on small meshes of every K, with and without the MLP hidden
 * layer, in the FP64 and FP8 network forms, for three steps each, and
 * the paper's network form (both GRU forms) with Crank-Nicolson.  Exits 0
 * if the sanitizers report nothing (they abort on the first report). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int orc_step_prec(int nx, int ny, int K, int H, int Hm, double dt, double nu, unsigned dir,
                  const double *cxy, const double *weights, const double *v, const double *p,
                  double *h, double *uprev, int first, int fp8,
                  double *Pv_out, double *D_out, double *X_out, double *dpatch_out,
                  double *Dbar_out, double *bL_out);
void orc_defect_abs(int nx, int ny, int K, const double *cxy, const double *v, const double *p,
                    const double *uprev, double inv_dt, double nu, double *S);
void orc_qgemm(int M, int N, int Kd, const double *A, const double *B, double *out);
void orc_features(int nx, int ny, const double *cxy, double *feat);
int orc_step_form(int nx, int ny, int K, int H, int Hm, double dt, double nu, double theta, unsigned dir,
                  int form, int reset_after, const double *cxy, const double *weights, const double *v,
                  const double *p, double *h, double *uprev, int first, int fp8,
                  double *Pv_out, double *D_out, double *X_out, double *dpatch_out,
                  double *Dbar_out, double *bL_out);
long orc_paper_weight_count(int K, int H);
int orc_umesh_count(int nc, int ne, const int *elems, int K, int *n_edges, int *n_fine);
int orc_umesh_refine(int nc, int ne, const double *xy, const int *elems, int K, int ncurved, const int *curved,
                     const double *circles, double *fxy, int *pmap);
void orc_u_mask(int ne, int K, const int *elems, const int *pmap, int Fn, int ndir, const int *dir_edges,
                unsigned char *mask);
int orc_u_step(int nc, int ne, const double *xy, const int *elems, int K, int H, int Hm, double dt, double nu,
               const int *pmap, const double *fxy, int Fn, const unsigned char *mask, const double *weights,
               const double *v, const double *p, double *h, double *uprev, int first,
               double *Pv_out, double *D_out, double *X_out, double *dpatch_out, double *Dbar_out, double *bL_out);

static double urand(unsigned long long *s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

int main(void)
{
    unsigned long long seed = 12345;
    const int shapes[][5] = {{3, 2, 1, 8, 0}, {2, 3, 2, 8, 8}, {1, 1, 3, 16, 16}, {4, 1, 1, 8, 8}};
    for (int sh = 0; sh < 4; ++sh) {
        const int nx = shapes[sh][0], ny = shapes[sh][1], K = shapes[sh][2], H = shapes[sh][3], Hm = shapes[sh][4];
        const int n = 1 << K, nf = (n + 1) * (n + 1), nin = 4 * nf + 4, nout = 2 * nf;
        const int P = nx * ny, Nc = (nx + 1) * (ny + 1), Fn = (nx * n + 1) * (ny * n + 1);
        const size_t nw = 3 * (size_t)H * nin + 3 * (size_t)H * H + (Hm ? (size_t)Hm * H + (size_t)nout * Hm : (size_t)nout * H);
        double *cxy = malloc(sizeof(double) * 2 * Nc), *w = malloc(sizeof(double) * nw);
        double *v = malloc(sizeof(double) * 2 * Nc), *p = malloc(sizeof(double) * Nc);
        double *Pv = malloc(sizeof(double) * 2 * Fn), *D = malloc(sizeof(double) * 2 * Fn);
        double *X = malloc(sizeof(double) * (size_t)P * nin), *dp = malloc(sizeof(double) * (size_t)P * nout);
        double *Db = malloc(sizeof(double) * 2 * Fn), *bL = malloc(sizeof(double) * 2 * Nc);
        double *S = malloc(sizeof(double) * 2 * Fn), *feat = malloc(sizeof(double) * 4 * P);
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                const int c = j * (nx + 1) + i;
                const int inner = i > 0 && i < nx && j > 0 && j < ny;
                cxy[2 * c] = 2.2 * i / nx + (inner ? 0.1 * 2.2 / nx * urand(&seed) : 0.0);
                cxy[2 * c + 1] = 0.41 * j / ny + (inner ? 0.1 * 0.41 / ny * urand(&seed) : 0.0);
            }
        for (size_t k = 0; k < nw; ++k) w[k] = 0.3 * urand(&seed);
        orc_features(nx, ny, cxy, feat);
        for (int fp8 = 0; fp8 < 2; ++fp8) {
            double *h = calloc((size_t)P * H, sizeof(double)), *up = calloc(2 * (size_t)Fn, sizeof(double));
            for (int step = 0; step < 3; ++step) {
                for (int c = 0; c < Nc; ++c) {
                    v[2 * c] = urand(&seed); v[2 * c + 1] = urand(&seed); p[c] = 0.1 * urand(&seed);
                }
                if (orc_step_prec(nx, ny, K, H, Hm, 0.01, 1e-3, step == 1 ? 15u : 13u, cxy, w, v, p, h, up,
                                  step == 0, fp8, Pv, D, X, dp, Db, bL) != 0) {
                    fprintf(stderr, "step failed\n");
                    return 1;
                }
            }
            orc_defect_abs(nx, ny, K, cxy, Pv, Pv, up, 100.0, 1e-3, S);
            for (int k = 0; k < 2 * Nc; ++k)
                if (!isfinite(bL[k])) { fprintf(stderr, "non-finite b_L\n"); return 1; }
            free(h);
            free(up);
        }
        {
            /* the paper's network form, Crank-Nicolson, both GRU forms */
            const long npw = orc_paper_weight_count(K, H);
            const int pin = 3 * nf + 24;
            double *pw = malloc(sizeof(double) * npw), *pX = malloc(sizeof(double) * (size_t)P * pin);
            for (long k = 0; k < npw; ++k) pw[k] = 0.3 * urand(&seed);
            for (int ra = 0; ra < 2; ++ra) {
                double *h = calloc((size_t)P * H, sizeof(double)), *up = calloc(2 * (size_t)Fn, sizeof(double));
                for (int step = 0; step < 3; ++step) {
                    for (int c = 0; c < Nc; ++c) {
                        v[2 * c] = urand(&seed); v[2 * c + 1] = urand(&seed); p[c] = 0.1 * urand(&seed);
                    }
                    if (orc_step_form(nx, ny, K, H, 0, 0.01, 1e-3, 0.5, 13u, 1, ra, cxy, pw, v, p, h, up, step == 0, 0,
                                      Pv, D, pX, dp, Db, bL) != 0) {
                        fprintf(stderr, "paper-form step failed\n");
                        return 1;
                    }
                }
                free(h);
                free(up);
            }
            free(pw);
            free(pX);
        }
        double *out = malloc(sizeof(double) * 2 * 3);
        orc_qgemm(1, 3, nin, X, w, out);   /* one row of X (P >= 1), three of W_z (H >= 8) */
        free(out);
        printf("shape %dx%d K=%d H=%d Hm=%d: 3 steps FP64 and FP8, paper form (Crank-Nicolson), error scale, "
               "quantised product\n", nx, ny, K, H, Hm);
        free(cxy); free(w); free(v); free(p); free(Pv); free(D); free(X); free(dp); free(Db); free(bL);
        free(S); free(feat);
    }
    {
        /* an unstructured mesh: 2 x 1 elements, the bottom-left edge on a circle */
        const double xy[12] = {0, 0, 1, 0, 2, 0, 0, 1, 1, 1, 2, 1};
        const int el[8] = {0, 1, 4, 3, 1, 2, 5, 4};
        const int curved[3] = {0, 1, 0}, dirs[4] = {0, 1, 0, 3};
        const double circ[3] = {0.5, 1.0, 1.1180339887498949};
        for (int K = 1; K <= 3; ++K) {
            const int n = 1 << K, nf = (n + 1) * (n + 1), nin = 4 * nf + 4, nout = 2 * nf, H = 8;
            int E, Fn;
            orc_umesh_count(6, 2, el, K, &E, &Fn);
            double *fxy = malloc(sizeof(double) * 2 * Fn), *up = calloc(2 * (size_t)Fn, sizeof(double));
            int *pmap = malloc(sizeof(int) * 2 * nf);
            unsigned char *mask = malloc(Fn);
            orc_umesh_refine(6, 2, xy, el, K, 1, curved, circ, fxy, pmap);
            orc_u_mask(2, K, el, pmap, Fn, 2, dirs, mask);
            const size_t nw = 3 * (size_t)H * nin + 3 * (size_t)H * H + (size_t)nout * H;
            double *w = malloc(sizeof(double) * nw), *h = calloc(2 * (size_t)H, sizeof(double));
            for (size_t k = 0; k < nw; ++k) w[k] = 0.3 * urand(&seed);
            double v[12], p[6], bL[12];
            double *Db = malloc(sizeof(double) * 2 * Fn);
            for (int step = 0; step < 3; ++step) {
                for (int c = 0; c < 6; ++c) { v[2 * c] = urand(&seed); v[2 * c + 1] = urand(&seed); p[c] = urand(&seed); }
                if (orc_u_step(6, 2, xy, el, K, H, 0, 0.01, 1e-3, pmap, fxy, Fn, mask, w, v, p, h, up, step == 0,
                               NULL, NULL, NULL, NULL, Db, bL) != 0) {
                    fprintf(stderr, "unstructured step failed\n");
                    return 1;
                }
            }
            free(fxy); free(up); free(pmap); free(mask); free(w); free(h); free(Db);
        }
        printf("unstructured 2-element mesh with a curved edge, K = 1..3: 3 steps\n");
    }
    return 0;
}
