/*
 * FP64 CPU oracle of the fine-level DNN-MG step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library; both are fed from the
 * seeded input generators.
 *
 * What it computes: the fine-level part of one step of Algorithm 2 of the paper --
 * prolongation of the coarse velocity, the fine Navier-Stokes defect, the
 * per-patch GRU + MLP correction, duplicate averaging, the fine right-hand
 * side and its restriction -- in the implicit-Euler, Q1/Q1 form used by the
 * workloads (readings documented in the design notes: implicit Euler instead
 * of Crank-Nicolson, Q1 instead of Q2, momentum rows only, no biases,
 * reset gate applied before U_h as printed in Eq. (gru)).
 *
 * Everything is plain loops in double precision, in the order the
 * definitions state; no blocking, fusion or reordering.  Loops whose
 * iterations write disjoint outputs (per patch, per fine node) may run on
 * several threads (OpenMP).  The element loops that add into shared nodes
 * run their rows in two passes, even rows then odd rows, so no two threads
 * add into one node and every node receives its contributions in an order
 * that does not depend on the number of threads: results are the same bit
 * for bit on 1 or many threads.
 *
 * Indexing (structured meshes):
 *   coarse node (i,j), 0<=i<=nx, 0<=j<=ny : index j*(nx+1)+i
 *   coarse element / patch (i,j)           : index j*nx+i
 *   n = 2^K; fine node (I,J), 0<=I<=nx*n   : index J*(nx*n+1)+I
 *   patch-local node (a,b), 0<=a,b<=n      : l = b*(n+1)+a  <-> fine (i*n+a, j*n+b)
 * Vector fields are interleaved (x, y) per node.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the parallel loops (1 when built without OpenMP). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- helpers */

static int coarse_node(int nx, int i, int j) { return j * (nx + 1) + i; }
static int fine_node(int nx, int n, int I, int J) { return J * (nx * n + 1) + I; }

/* Bilinear shape functions on [0,1]^2 in the corner order 00, 10, 01, 11. */
static void q1_shape(double s, double t, double N[4])
{
    N[0] = (1.0 - s) * (1.0 - t);
    N[1] = s * (1.0 - t);
    N[2] = (1.0 - s) * t;
    N[3] = s * t;
}

static void q1_shape_ds(double s, double t, double dNs[4], double dNt[4])
{
    (void)s;
    dNs[0] = -(1.0 - t); dNs[1] = (1.0 - t); dNs[2] = -t; dNs[3] = t;
    dNt[0] = -(1.0 - s); dNt[1] = -s;        dNt[2] = (1.0 - s); dNt[3] = s;
}

/* The coarse element that holds fine node I along one axis, and the local
 * offset a in [0, n] inside it.  Nodes on an element edge belong to both
 * neighbours; the left/lower one is taken, except at the last node. */
static void owner(int I, int n, int ne, int *e, int *a)
{
    int i = I / n;
    if (i >= ne) i = ne - 1;
    *e = i;
    *a = I - i * n;
}

/* 2-point Gauss rule on [0,1] (exact for cubics). */
static void gauss2(double g[2])
{
    double d = 0.5 / sqrt(3.0);
    g[0] = 0.5 - d;
    g[1] = 0.5 + d;
}

/* -------------------------------------------------- step 1: fine geometry */
/* Fine node (i*n+a, j*n+b) sits at F_e(a/n, b/n), the bilinear
 * (isoparametric) map of coarse element e; K uniform refinements of the
 * coarse mesh (Sec. 3.4, nested mesh hierarchy). */
void orc_fine_coords(int nx, int ny, int K, const double *cxy, double *fxy)
{
    int n = 1 << K;
    for (int J = 0; J <= ny * n; ++J)
        for (int I = 0; I <= nx * n; ++I) {
            int i, a, j, b;
            owner(I, n, nx, &i, &a);
            owner(J, n, ny, &j, &b);
            double N[4];
            q1_shape((double)a / n, (double)b / n, N);
            int c[4] = {coarse_node(nx, i, j), coarse_node(nx, i + 1, j),
                        coarse_node(nx, i, j + 1), coarse_node(nx, i + 1, j + 1)};
            int f = fine_node(nx, n, I, J);
            for (int d = 0; d < 2; ++d) {
                double x = 0.0;
                for (int k = 0; k < 4; ++k) x += N[k] * cxy[2 * c[k] + d];
                fxy[2 * f + d] = x;
            }
        }
}

/* ---------------------------------------------------- step 2: prolongation */
/* P: interpolation of the coarse Q1 function at the fine nodes (Alg. 2,
 * prolongation; grid transfer of Sec. 3.4).  ncomp values per node. */
void orc_prolong(int nx, int ny, int K, int ncomp, const double *coarse, double *fine)
{
    int n = 1 << K;
#pragma omp parallel for schedule(static)
    for (int J = 0; J <= ny * n; ++J)
        for (int I = 0; I <= nx * n; ++I) {
            int i, a, j, b;
            owner(I, n, nx, &i, &a);
            owner(J, n, ny, &j, &b);
            double N[4];
            q1_shape((double)a / n, (double)b / n, N);
            int c[4] = {coarse_node(nx, i, j), coarse_node(nx, i + 1, j),
                        coarse_node(nx, i, j + 1), coarse_node(nx, i + 1, j + 1)};
            int f = fine_node(nx, n, I, J);
            for (int d = 0; d < ncomp; ++d) {
                double x = 0.0;
                for (int k = 0; k < 4; ++k) x += N[k] * coarse[ncomp * c[k] + d];
                fine[ncomp * f + d] = x;
            }
        }
}

/* --------------------------------------------------- step 10: restriction */
/* R = P^T: the transpose of the prolongation above, applied to a dual
 * (right-hand-side) vector (Alg. 2, restriction). */
void orc_restrict(int nx, int ny, int K, int ncomp, const double *fine, double *coarse)
{
    int n = 1 << K;
    memset(coarse, 0, sizeof(double) * (size_t)ncomp * (nx + 1) * (ny + 1));
    /* a fine row J adds into the coarse rows j and j + 1 of its owner j:
     * owners of one parity never share a coarse row */
    for (int parity = 0; parity < 2; ++parity)
#pragma omp parallel for schedule(static)
    for (int jo = parity; jo < ny; jo += 2)
    for (int J = jo * n; J <= (jo == ny - 1 ? ny * n : jo * n + n - 1); ++J)
        for (int I = 0; I <= nx * n; ++I) {
            int i, a, j, b;
            owner(I, n, nx, &i, &a);
            owner(J, n, ny, &j, &b);
            double N[4];
            q1_shape((double)a / n, (double)b / n, N);
            int c[4] = {coarse_node(nx, i, j), coarse_node(nx, i + 1, j),
                        coarse_node(nx, i, j + 1), coarse_node(nx, i + 1, j + 1)};
            int f = fine_node(nx, n, I, J);
            for (int d = 0; d < ncomp; ++d)
                for (int k = 0; k < 4; ++k) coarse[ncomp * c[k] + d] += N[k] * fine[ncomp * f + d];
        }
}

/* ---------------------------------------------------------- Dirichlet mask */
/* bit0 x=xmin, bit1 x=xmax, bit2 y=ymin, bit3 y=ymax (Eq. boundary: v=v^D
 * on Gamma^D; the do-nothing sides are natural and left free). */
void orc_dirichlet_mask(int nx, int ny, int K, unsigned dir, unsigned char *mask)
{
    int n = 1 << K, NX = nx * n, NY = ny * n;
    for (int J = 0; J <= NY; ++J)
        for (int I = 0; I <= NX; ++I) {
            int m = ((dir & 1u) && I == 0) || ((dir & 2u) && I == NX) ||
                    ((dir & 4u) && J == 0) || ((dir & 8u) && J == NY);
            mask[fine_node(nx, n, I, J)] = (unsigned char)m;
        }
}

/* ------------------------------------------------------ step 3: the defect */
/* D = f - A(Pv, Pp): the momentum rows of the nonlinear residual of
 * Eq. (nonlinearshort) for the prolongated coarse solution, with implicit
 * Euler in place of Crank-Nicolson:
 *   D_a,c = (1/dt)(u_prev - v, phi) - (v.grad v_c, phi) - nu (grad v_c, grad phi)
 *           + (p, d_c phi)
 * assembled element by element over the fine mesh with 2x2 Gauss points on
 * each fine element's own bilinear map, then zeroed at Dirichlet nodes.
 * v, p, u_prev are fine nodal values (2, 1, 2 per node). */
void orc_defect(int nx, int ny, int K, const double *cxy, const double *v, const double *p,
                const double *uprev, double dt, double nu, unsigned dir, double *D)
{
    int n = 1 << K, NX = nx * n, NY = ny * n;
    size_t Fn = (size_t)(NX + 1) * (NY + 1);
    double *fxy = (double *)malloc(sizeof(double) * 2 * Fn);
    unsigned char *mask = (unsigned char *)malloc(Fn);
    orc_fine_coords(nx, ny, K, cxy, fxy);
    orc_dirichlet_mask(nx, ny, K, dir, mask);
    memset(D, 0, sizeof(double) * 2 * Fn);
    double g[2];
    gauss2(g);
    /* element row J adds into node rows J and J + 1: rows of one parity
     * never share a node */
    for (int parity = 0; parity < 2; ++parity)
#pragma omp parallel for schedule(static)
    for (int J = parity; J < NY; J += 2)
        for (int I = 0; I < NX; ++I) {
            int node[4] = {fine_node(nx, n, I, J), fine_node(nx, n, I + 1, J),
                           fine_node(nx, n, I, J + 1), fine_node(nx, n, I + 1, J + 1)};
            for (int qt = 0; qt < 2; ++qt)
                for (int qs = 0; qs < 2; ++qs) {
                    double s = g[qs], t = g[qt], w = 0.25;
                    double N[4], dNs[4], dNt[4];
                    q1_shape(s, t, N);
                    q1_shape_ds(s, t, dNs, dNt);
                    /* Jacobian of the element map x(s,t). */
                    double xs = 0, xt = 0, ys = 0, yt = 0;
                    for (int k = 0; k < 4; ++k) {
                        xs += fxy[2 * node[k]] * dNs[k];
                        xt += fxy[2 * node[k]] * dNt[k];
                        ys += fxy[2 * node[k] + 1] * dNs[k];
                        yt += fxy[2 * node[k] + 1] * dNt[k];
                    }
                    double det = xs * yt - xt * ys;
                    /* Physical gradients: grad N = J^{-T} (dN/ds, dN/dt). */
                    double dNx[4], dNy[4];
                    for (int k = 0; k < 4; ++k) {
                        dNx[k] = (yt * dNs[k] - ys * dNt[k]) / det;
                        dNy[k] = (-xt * dNs[k] + xs * dNt[k]) / det;
                    }
                    double vq[2] = {0, 0}, uq[2] = {0, 0}, pq = 0;
                    double gv[2][2] = {{0, 0}, {0, 0}}; /* gv[c][k] = d v_c / d x_k */
                    for (int k = 0; k < 4; ++k) {
                        for (int c = 0; c < 2; ++c) {
                            vq[c] += N[k] * v[2 * node[k] + c];
                            uq[c] += N[k] * uprev[2 * node[k] + c];
                            gv[c][0] += v[2 * node[k] + c] * dNx[k];
                            gv[c][1] += v[2 * node[k] + c] * dNy[k];
                        }
                        pq += N[k] * p[node[k]];
                    }
                    double conv[2];
                    for (int c = 0; c < 2; ++c) conv[c] = vq[0] * gv[c][0] + vq[1] * gv[c][1];
                    double wd = w * fabs(det);
                    for (int a = 0; a < 4; ++a)
                        for (int c = 0; c < 2; ++c) {
                            double dphi_c = (c == 0) ? dNx[a] : dNy[a];
                            double r = (1.0 / dt) * N[a] * (uq[c] - vq[c])
                                     - N[a] * conv[c]
                                     - nu * (dNx[a] * gv[c][0] + dNy[a] * gv[c][1])
                                     + pq * dphi_c;
                            D[2 * node[a] + c] += wd * r;
                        }
                }
        }
    for (size_t f = 0; f < Fn; ++f)
        if (mask[f]) { D[2 * f] = 0.0; D[2 * f + 1] = 0.0; }
    free(fxy);
    free(mask);
}

/* -------------------------------------------- error scale of the defect */
/* Not part of the step: a scale for judging a floating-point evaluation of
 * orc_defect.  The same element loop, Gauss points and terms, each term in
 * absolute value, and inside each term the sums that form it taken over
 * absolute values: the element map and the velocity written as bilinear
 * polynomials f00 + e_s s + e_t t + e_st s t in the reference coordinates
 * (e_s = f10 - f00, e_t = f01 - f00, e_st = f11 - f10 - f01 + f00), so
 * d/ds f = e_s + e_st t is bounded by |e_s| + |e_st| t, and so on; the
 * interpolated v, u_prev and p from absolute nodal values; the mass term
 * from |u_prev| + |v|.  No Dirichlet masking.
 *
 * An evaluation of D in working precision u that forms the same quantities
 * (in any order, from edge vectors and nodal differences) differs from the
 * exact D at a node by at most a modest multiple of u times this scale (the
 * running-error bound of sums of products), however much the element terms
 * cancel in the node sums.  inv_dt is the 1/dt of that evaluation: 0 for
 * one that leaves the mass term out. */
void orc_defect_abs(int nx, int ny, int K, const double *cxy, const double *v, const double *p,
                    const double *uprev, double inv_dt, double nu, double *S)
{
    int n = 1 << K, NX = nx * n, NY = ny * n;
    size_t Fn = (size_t)(NX + 1) * (NY + 1);
    double *fxy = (double *)malloc(sizeof(double) * 2 * Fn);
    orc_fine_coords(nx, ny, K, cxy, fxy);
    memset(S, 0, sizeof(double) * 2 * Fn);
    double g[2];
    gauss2(g);
    for (int parity = 0; parity < 2; ++parity)
#pragma omp parallel for schedule(static)
    for (int J = parity; J < NY; J += 2)
        for (int I = 0; I < NX; ++I) {
            int node[4] = {fine_node(nx, n, I, J), fine_node(nx, n, I + 1, J),
                           fine_node(nx, n, I, J + 1), fine_node(nx, n, I + 1, J + 1)};
            for (int qt = 0; qt < 2; ++qt)
                for (int qs = 0; qs < 2; ++qs) {
                    double N[4], dNs[4], dNt[4];
                    q1_shape(g[qs], g[qt], N);
                    q1_shape_ds(g[qs], g[qt], dNs, dNt);
                    /* bilinear coefficients of the map (x, y) and of v */
                    double ex[2], et[2], est[2];
                    for (int d = 0; d < 2; ++d) {
                        double f0 = fxy[2 * node[0] + d], f1 = fxy[2 * node[1] + d];
                        double f2 = fxy[2 * node[2] + d], f3 = fxy[2 * node[3] + d];
                        ex[d] = f1 - f0; et[d] = f2 - f0; est[d] = f3 - f1 - f2 + f0;
                    }
                    double s_ = g[qs], t_ = g[qt];
                    double xs = ex[0] + est[0] * t_, xt = et[0] + est[0] * s_;
                    double ys = ex[1] + est[1] * t_, yt = et[1] + est[1] * s_;
                    double axs = fabs(ex[0]) + fabs(est[0]) * t_, axt = fabs(et[0]) + fabs(est[0]) * s_;
                    double ays = fabs(ex[1]) + fabs(est[1]) * t_, ayt = fabs(et[1]) + fabs(est[1]) * s_;
                    double det = fabs(xs * yt - xt * ys);
                    double adx[4], ady[4];   /* |grad N| with the inverse Jacobian taken term by term */
                    for (int k = 0; k < 4; ++k) {
                        adx[k] = (ayt * fabs(dNs[k]) + ays * fabs(dNt[k])) / det;
                        ady[k] = (axt * fabs(dNs[k]) + axs * fabs(dNt[k])) / det;
                    }
                    double av[2] = {0, 0}, au[2] = {0, 0}, ap = 0, ag[2][2];
                    for (int k = 0; k < 4; ++k) {
                        for (int c = 0; c < 2; ++c) {
                            av[c] += N[k] * fabs(v[2 * node[k] + c]);
                            au[c] += N[k] * fabs(uprev[2 * node[k] + c]);
                        }
                        ap += N[k] * fabs(p[node[k]]);
                    }
                    for (int c = 0; c < 2; ++c) {
                        double v0 = v[2 * node[0] + c], v1 = v[2 * node[1] + c];
                        double v2 = v[2 * node[2] + c], v3 = v[2 * node[3] + c];
                        double as = fabs(v1 - v0) + fabs(v3 - v1 - v2 + v0) * t_;   /* |dv/ds| */
                        double at = fabs(v2 - v0) + fabs(v3 - v1 - v2 + v0) * s_;   /* |dv/dt| */
                        ag[c][0] = (ayt * as + ays * at) / det;
                        ag[c][1] = (axt * as + axs * at) / det;
                    }
                    double wd = 0.25 * (axs * ayt + axt * ays);
                    for (int a = 0; a < 4; ++a)
                        for (int c = 0; c < 2; ++c) {
                            double adphi = (c == 0) ? adx[a] : ady[a];
                            double r = inv_dt * N[a] * (au[c] + av[c])
                                     + N[a] * (av[0] * ag[c][0] + av[1] * ag[c][1])
                                     + nu * (adx[a] * ag[c][0] + ady[a] * ag[c][1])
                                     + ap * adphi;
                            S[2 * node[a] + c] += wd * r;
                        }
                }
        }
    free(fxy);
}

/* ---------------------------------------------------- step 9: mass matrix */
/* Mu = M_f u, the consistent fine-level mass matrix (same element loop and
 * quadrature as the defect) applied to a 2-component nodal field. */
void orc_mass_apply(int nx, int ny, int K, const double *cxy, const double *u, double *Mu)
{
    int n = 1 << K, NX = nx * n, NY = ny * n;
    size_t Fn = (size_t)(NX + 1) * (NY + 1);
    double *fxy = (double *)malloc(sizeof(double) * 2 * Fn);
    orc_fine_coords(nx, ny, K, cxy, fxy);
    memset(Mu, 0, sizeof(double) * 2 * Fn);
    double g[2];
    gauss2(g);
    for (int parity = 0; parity < 2; ++parity)
#pragma omp parallel for schedule(static)
    for (int J = parity; J < NY; J += 2)
        for (int I = 0; I < NX; ++I) {
            int node[4] = {fine_node(nx, n, I, J), fine_node(nx, n, I + 1, J),
                           fine_node(nx, n, I, J + 1), fine_node(nx, n, I + 1, J + 1)};
            for (int qt = 0; qt < 2; ++qt)
                for (int qs = 0; qs < 2; ++qs) {
                    double s = g[qs], t = g[qt], w = 0.25;
                    double N[4], dNs[4], dNt[4];
                    q1_shape(s, t, N);
                    q1_shape_ds(s, t, dNs, dNt);
                    double xs = 0, xt = 0, ys = 0, yt = 0;
                    for (int k = 0; k < 4; ++k) {
                        xs += fxy[2 * node[k]] * dNs[k];
                        xt += fxy[2 * node[k]] * dNt[k];
                        ys += fxy[2 * node[k] + 1] * dNs[k];
                        yt += fxy[2 * node[k] + 1] * dNt[k];
                    }
                    double wd = w * fabs(xs * yt - xt * ys);
                    double uq[2] = {0, 0};
                    for (int k = 0; k < 4; ++k)
                        for (int c = 0; c < 2; ++c) uq[c] += N[k] * u[2 * node[k] + c];
                    for (int a = 0; a < 4; ++a)
                        for (int c = 0; c < 2; ++c) Mu[2 * node[a] + c] += wd * N[a] * uq[c];
                }
        }
    free(fxy);
}

/* ------------------------------------------------ step 4: patch features */
/* Geometry inputs per patch (Sec. 4.2 uses edge lengths, aspect ratios and
 * angles; the workloads use hx, hy, aspect = hx/hy and the exact area). */
void orc_features(int nx, int ny, const double *cxy, double *feat)
{
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const double *c00 = cxy + 2 * coarse_node(nx, i, j);
            const double *c10 = cxy + 2 * coarse_node(nx, i + 1, j);
            const double *c01 = cxy + 2 * coarse_node(nx, i, j + 1);
            const double *c11 = cxy + 2 * coarse_node(nx, i + 1, j + 1);
            double hx = 0.5 * (hypot(c10[0] - c00[0], c10[1] - c00[1]) +
                               hypot(c11[0] - c01[0], c11[1] - c01[1]));
            double hy = 0.5 * (hypot(c01[0] - c00[0], c01[1] - c00[1]) +
                               hypot(c11[0] - c10[0], c11[1] - c10[1]));
            double d1x = c11[0] - c00[0], d1y = c11[1] - c00[1];
            double d2x = c01[0] - c10[0], d2y = c01[1] - c10[1];
            double area = 0.5 * fabs(d1x * d2y - d1y * d2x);
            double *f = feat + 4 * (size_t)(j * nx + i);
            f[0] = hx; f[1] = hy; f[2] = hx / hy; f[3] = area;
        }
}

/* ------------------------------------------------ step 5: network inputs */
/* x_e = [Pv at the patch nodes (x,y interleaved, patch-local lexicographic
 * order, x fastest); D at the same nodes; hx, hy, aspect, area]. */
void orc_gather_input(int nx, int ny, int K, const double *pv, const double *D,
                      const double *feat, double *X)
{
    int n = 1 << K, nf = (n + 1) * (n + 1), nin = 4 * nf + 4;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t e = (size_t)j * nx + i;
            double *x = X + e * nin;
            for (int b = 0; b <= n; ++b)
                for (int a = 0; a <= n; ++a) {
                    int l = b * (n + 1) + a;
                    int f = fine_node(nx, n, i * n + a, j * n + b);
                    x[2 * l] = pv[2 * f];
                    x[2 * l + 1] = pv[2 * f + 1];
                    x[2 * nf + 2 * l] = D[2 * f];
                    x[2 * nf + 2 * l + 1] = D[2 * f + 1];
                }
            for (int k = 0; k < 4; ++k) x[4 * nf + k] = feat[4 * e + k];
        }
}

/* ---------------------------------------------------------- step 6: GRU */
/* Eq. (gru) with no biases:
 *   z = sigma(W_z x + U_z h), r = sigma(W_r x + U_r h),
 *   h' = z*h + (1-z)*tanh(W_h x + U_h (r*h)),
 * sigma the logistic function.  W: H x nin each, U: H x H each. */
static double logistic(double t) { return 1.0 / (1.0 + exp(-t)); }

void orc_gru(int P, int nin, int H, const double *Wz, const double *Wr, const double *Wh,
             const double *Uz, const double *Ur, const double *Uh,
             const double *X, const double *h, double *hout)
{
#pragma omp parallel
    {
    double *z = (double *)malloc(sizeof(double) * H);
    double *rh = (double *)malloc(sizeof(double) * H);
#pragma omp for schedule(static)
    for (int e = 0; e < P; ++e) {
        const double *x = X + (size_t)e * nin;
        const double *he = h + (size_t)e * H;
        for (int k = 0; k < H; ++k) {
            double az = 0.0, ar = 0.0;
            for (int i = 0; i < nin; ++i) {
                az += Wz[(size_t)k * nin + i] * x[i];
                ar += Wr[(size_t)k * nin + i] * x[i];
            }
            for (int m = 0; m < H; ++m) {
                az += Uz[(size_t)k * H + m] * he[m];
                ar += Ur[(size_t)k * H + m] * he[m];
            }
            z[k] = logistic(az);
            rh[k] = logistic(ar) * he[k];
        }
        for (int k = 0; k < H; ++k) {
            double ah = 0.0;
            for (int i = 0; i < nin; ++i) ah += Wh[(size_t)k * nin + i] * x[i];
            for (int m = 0; m < H; ++m) ah += Uh[(size_t)k * H + m] * rh[m];
            hout[(size_t)e * H + k] = z[k] * he[k] + (1.0 - z[k]) * tanh(ah);
        }
    }
    free(z);
    free(rh);
    }
}

/* ---------------------------------------------------------- step 7: MLP */
/* d = M2 max(0, M1 h) (Hm > 0) or d = M h (Hm == 0); no biases. */
void orc_mlp(int P, int H, int Hm, int nout, const double *M1, const double *M2,
             const double *h, double *d)
{
#pragma omp parallel
    {
    double *a = (double *)malloc(sizeof(double) * (Hm > 0 ? Hm : 1));
#pragma omp for schedule(static)
    for (int e = 0; e < P; ++e) {
        const double *he = h + (size_t)e * H;
        double *de = d + (size_t)e * nout;
        if (Hm > 0) {
            for (int k = 0; k < Hm; ++k) {
                double s = 0.0;
                for (int m = 0; m < H; ++m) s += M1[(size_t)k * H + m] * he[m];
                a[k] = s > 0.0 ? s : 0.0;
            }
            for (int o = 0; o < nout; ++o) {
                double s = 0.0;
                for (int k = 0; k < Hm; ++k) s += M2[(size_t)o * Hm + k] * a[k];
                de[o] = s;
            }
        } else {
            for (int o = 0; o < nout; ++o) {
                double s = 0.0;
                for (int m = 0; m < H; ++m) s += M1[(size_t)o * H + m] * he[m];
                de[o] = s;
            }
        }
    }
    free(a);
    }
}

/* ------------------------------------- steps 6-7 with FP8 E4M3 operands */
/* The precision form with 8-bit operands (not part of the paper, which runs
 * its network in FP32): every product of the GRU and the MLP takes both
 * operands as OCP FP8 E4M3 codes with one FP32 scale per row, and
 * accumulates exactly; everything else is as in orc_gru / orc_mlp.
 *
 * E4M3 (OCP 8-bit floating point, "E4M3FN"): sign, 4 exponent bits with
 * bias 7, 3 mantissa bits; exponent field 0 holds subnormals m/8 * 2^-6;
 * there are no infinities, S.1111.111 is NaN, so the largest finite value
 * is 1.75 * 2^8 = 448. */
double orc_e4m3_decode(unsigned code)
{
    const unsigned e = (code >> 3) & 15u, m = code & 7u;
    const double sign = (code & 0x80u) ? -1.0 : 1.0;
    if (e == 15u && m == 7u) return NAN;
    if (e == 0u) return sign * ldexp((double)m / 8.0, -6);
    return sign * ldexp(1.0 + (double)m / 8.0, (int)e - 7);
}

/* Nearest E4M3 value of x, ties to the even code; magnitudes above 448
 * saturate to 448 (the scaled operands never exceed it by more than an FP32
 * rounding); NaN gives the NaN code. */
unsigned orc_e4m3_encode(float x)
{
    if (isnan(x)) return 0x7Fu;
    const unsigned sign = signbit(x) ? 0x80u : 0u;
    const double a = fabs((double)x);
    if (a >= 448.0) return sign | 0x7Eu;
    if (a < ldexp(1.0, -6)) {                       /* subnormal range: steps of 2^-9 */
        const double m = rint(a * 512.0);           /* rint: nearest, ties to even */
        return sign | (unsigned)m;                   /* m == 8 is the smallest normal */
    }
    int e;
    (void)frexp(a, &e);                             /* a = f 2^e, f in [0.5, 1) */
    e -= 1;                                         /* a = (1 + t) 2^e, t in [0, 1) */
    double m = rint((ldexp(a, -e) - 1.0) * 8.0);
    if (m == 8.0) { m = 0.0; e += 1; }
    const unsigned code = ((unsigned)(e + 7) << 3) | (unsigned)m;
    return sign | (code > 0x7Eu ? 0x7Eu : code);
}

/* Per-row quantisation of a rows x cols matrix of FP32 values, in FP32:
 *   m = max(max_k |a_k|, 448 * 2^-64), r = 448 / m, s = m / 448,
 *   q_k = e4m3(a_k * r);  a_k ~ s * dec(q_k).
 * The floor keeps 1/s finite for an all-zero row. */
void orc_quantize_rows(int rows, int cols, const float *a, unsigned char *q, float *s)
{
    const float floor_m = 448.0f * 0x1p-64f;
    for (int i = 0; i < rows; ++i) {
        const float *ai = a + (size_t)i * cols;
        float m = floor_m;
        for (int k = 0; k < cols; ++k) {
            const float v = fabsf(ai[k]);
            if (v > m) m = v;
        }
        const float r = 448.0f / m;
        s[i] = m / 448.0f;
        for (int k = 0; k < cols; ++k) q[(size_t)i * cols + k] = (unsigned char)orc_e4m3_encode(ai[k] * r);
    }
}

/* One quantised operand row: codes and scale of x (rounded to FP32 first). */
static void quant_row(int n, const double *x, unsigned char *q, float *s)
{
    float *xf = (float *)malloc(sizeof(float) * (n > 0 ? n : 1));
    for (int k = 0; k < n; ++k) xf[k] = (float)x[k];
    orc_quantize_rows(1, n, xf, q, s);
    free(xf);
}

/* Weights, one scale per output row of the product that uses them. */
static void quant_matrix(int rows, int cols, const double *w, unsigned char *q, float *s)
{
    for (int i = 0; i < rows; ++i) quant_row(cols, w + (size_t)i * cols, q + (size_t)i * cols, s + i);
}

static double qdot(int n, const unsigned char *a, const unsigned char *b)
{
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc += orc_e4m3_decode(a[k]) * orc_e4m3_decode(b[k]);
    return acc;
}

/* Quantised product: out[i][j] = s_a[i] s_b[j] sum_k dec(qa[i][k]) dec(qb[j][k]),
 * each row of A and of B quantised with its own scale (orc_quantize_rows). */
void orc_qgemm(int M, int N, int Kd, const double *A, const double *B, double *out)
{
    unsigned char *qa = (unsigned char *)malloc((size_t)M * Kd + 1), *qb = (unsigned char *)malloc((size_t)N * Kd + 1);
    float *sa = (float *)malloc(sizeof(float) * (M + 1)), *sb = (float *)malloc(sizeof(float) * (N + 1));
    quant_matrix(M, Kd, A, qa, sa);
    quant_matrix(N, Kd, B, qb, sb);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < N; ++j)
            out[(size_t)i * N + j] = (double)sa[i] * (double)sb[j] * qdot(Kd, qa + (size_t)i * Kd, qb + (size_t)j * Kd);
    free(qa); free(qb); free(sa); free(sb);
}

/* GRU with FP8 operands.  The products and their operands:
 *   gates z, r: [W_g | U_g] (one scale per row over both blocks) times x and
 *     h, which are quantised separately (the network input x with its own
 *     per-patch scale, the state h with another);
 *   candidate:  W_h x (row scales of W_h) and U_h (r*h) (row scales of U_h,
 *     per-patch scale of r*h). */
void orc_gru_fp8(int P, int nin, int H, const double *Wz, const double *Wr, const double *Wh,
                 const double *Uz, const double *Ur, const double *Uh,
                 const double *X, const double *h, double *hout)
{
    const int nb = nin + H;
    unsigned char *qB[3], *qUh = (unsigned char *)malloc((size_t)H * H);
    float *sB[3], *sUh = (float *)malloc(sizeof(float) * H);
    const double *Wg[3] = {Wz, Wr, Wh}, *Ug[3] = {Uz, Ur, NULL};
    double *row = (double *)malloc(sizeof(double) * nb);
    for (int g = 0; g < 3; ++g) {
        qB[g] = (unsigned char *)malloc((size_t)H * nb);
        sB[g] = (float *)malloc(sizeof(float) * H);
        for (int k = 0; k < H; ++k) {
            for (int i = 0; i < nin; ++i) row[i] = Wg[g][(size_t)k * nin + i];
            for (int m = 0; m < H; ++m) row[nin + m] = Ug[g] ? Ug[g][(size_t)k * H + m] : 0.0;
            quant_row(nb, row, qB[g] + (size_t)k * nb, sB[g] + k);
        }
    }
    quant_matrix(H, H, Uh, qUh, sUh);
#pragma omp parallel
    {
    unsigned char *qx = (unsigned char *)malloc(nin), *qh = (unsigned char *)malloc(H), *qrh = (unsigned char *)malloc(H);
    double *z = (double *)malloc(sizeof(double) * H), *rh = (double *)malloc(sizeof(double) * H);
#pragma omp for schedule(static)
    for (int e = 0; e < P; ++e) {
        const double *he = h + (size_t)e * H;
        float sx, sh, srh;
        quant_row(nin, X + (size_t)e * nin, qx, &sx);
        quant_row(H, he, qh, &sh);
        for (int k = 0; k < H; ++k) {
            double a[2];
            for (int g = 0; g < 2; ++g) {
                const unsigned char *b = qB[g] + (size_t)k * nb;
                a[g] = (double)sB[g][k] * ((double)sx * qdot(nin, qx, b) + (double)sh * qdot(H, qh, b + nin));
            }
            z[k] = logistic(a[0]);
            rh[k] = logistic(a[1]) * he[k];
        }
        quant_row(H, rh, qrh, &srh);
        for (int k = 0; k < H; ++k) {
            const double ah = (double)sB[2][k] * (double)sx * qdot(nin, qx, qB[2] + (size_t)k * nb) +
                              (double)sUh[k] * (double)srh * qdot(H, qrh, qUh + (size_t)k * H);
            hout[(size_t)e * H + k] = z[k] * he[k] + (1.0 - z[k]) * tanh(ah);
        }
    }
    free(qx); free(qh); free(qrh); free(z); free(rh);
    }
    for (int g = 0; g < 3; ++g) { free(qB[g]); free(sB[g]); }
    free(qUh); free(sUh); free(row);
}

/* MLP with FP8 operands: each layer quantises its input per patch and its
 * weights per output row. */
void orc_mlp_fp8(int P, int H, int Hm, int nout, const double *M1, const double *M2,
                 const double *h, double *d)
{
    const int n1 = Hm > 0 ? Hm : nout;
    unsigned char *q1 = (unsigned char *)malloc((size_t)n1 * H), *q2 = (unsigned char *)malloc((size_t)nout * (Hm > 0 ? Hm : 1));
    float *s1 = (float *)malloc(sizeof(float) * n1), *s2 = (float *)malloc(sizeof(float) * nout);
    quant_matrix(n1, H, M1, q1, s1);
    if (Hm > 0) quant_matrix(nout, Hm, M2, q2, s2);
#pragma omp parallel
    {
    unsigned char *qh = (unsigned char *)malloc(H), *qa = (unsigned char *)malloc(Hm > 0 ? Hm : 1);
    double *a = (double *)malloc(sizeof(double) * (Hm > 0 ? Hm : 1));
#pragma omp for schedule(static)
    for (int e = 0; e < P; ++e) {
        float sh, sa;
        double *de = d + (size_t)e * nout;
        quant_row(H, h + (size_t)e * H, qh, &sh);
        if (Hm > 0) {
            for (int k = 0; k < Hm; ++k) {
                const double t = (double)s1[k] * (double)sh * qdot(H, qh, q1 + (size_t)k * H);
                a[k] = t > 0.0 ? t : 0.0;
            }
            quant_row(Hm, a, qa, &sa);
            for (int o = 0; o < nout; ++o) de[o] = (double)s2[o] * (double)sa * qdot(Hm, qa, q2 + (size_t)o * Hm);
        } else {
            for (int o = 0; o < nout; ++o) de[o] = (double)s1[o] * (double)sh * qdot(H, qh, q1 + (size_t)o * H);
        }
    }
    free(qh); free(qa); free(a);
    }
    free(q1); free(q2); free(s1); free(s2);
}

/* ---------------------------------------------------- step 8: averaging */
/* Duplicate predictions at fine nodes shared by adjacent patches are
 * averaged (Sec. 4.2, patch-based network); the mean over the 1, 2 or 4
 * patches that contain the node, then zero at Dirichlet nodes. */
void orc_average(int nx, int ny, int K, const double *dpatch, unsigned dir, double *Dbar)
{
    int n = 1 << K, NX = nx * n, NY = ny * n, nf = (n + 1) * (n + 1);
    size_t Fn = (size_t)(NX + 1) * (NY + 1);
    unsigned char *mask = (unsigned char *)malloc(Fn);
    orc_dirichlet_mask(nx, ny, K, dir, mask);
#pragma omp parallel for schedule(static)
    for (int J = 0; J <= NY; ++J)
        for (int I = 0; I <= NX; ++I) {
            double s[2] = {0, 0};
            int cnt = 0;
            /* only patches J/n-1 and J/n (resp. I/n-1, I/n) can contain the
             * node; the containment test below decides. */
            for (int pj = J / n - 1; pj <= J / n; ++pj) {
                if (pj < 0 || pj >= ny || J < pj * n || J > pj * n + n) continue;
                for (int pi = I / n - 1; pi <= I / n; ++pi) {
                    if (pi < 0 || pi >= nx || I < pi * n || I > pi * n + n) continue;
                    int l = (J - pj * n) * (n + 1) + (I - pi * n);
                    const double *de = dpatch + ((size_t)pj * nx + pi) * 2 * nf;
                    s[0] += de[2 * l];
                    s[1] += de[2 * l + 1];
                    ++cnt;
                }
            }
            size_t f = (size_t)fine_node(nx, n, I, J);
            Dbar[2 * f] = mask[f] ? 0.0 : s[0] / cnt;
            Dbar[2 * f + 1] = mask[f] ? 0.0 : s[1] / cnt;
        }
    free(mask);
}

/* -------------------------------------------- steps 9-10 as one operation */
/* b_L = R (1/dt) M_f u_corr with u_corr = P v + Dbar (Alg. 2, right-hand
 * side and restriction, implicit-Euler right-hand side, no body force).  v is the coarse
 * velocity, Dbar the fine correction. */
void orc_rhs_restrict(int nx, int ny, int K, const double *cxy, const double *v,
                      const double *Dbar, double dt, double *bL)
{
    int n = 1 << K;
    size_t Fn = (size_t)(nx * n + 1) * (ny * n + 1);
    double *u = (double *)malloc(sizeof(double) * 2 * Fn);
    double *bf = (double *)malloc(sizeof(double) * 2 * Fn);
    orc_prolong(nx, ny, K, 2, v, u);
    for (size_t f = 0; f < 2 * Fn; ++f) u[f] += Dbar[f];
    orc_mass_apply(nx, ny, K, cxy, u, bf);
    for (size_t f = 0; f < 2 * Fn; ++f) bf[f] *= 1.0 / dt;
    orc_restrict(nx, ny, K, 2, bf, bL);
    free(u);
    free(bf);
}

/* ------------------------------------- theta scheme (Crank-Nicolson: 1/2) */
/* T(w) = C(w) w + nu K w: the convection and diffusion rows of the
 * momentum operator applied to a fine nodal field w (2 per node), with the
 * defect's element loop and quadrature, unmasked.  The time scheme of
 * Eq. (4cranknicholson3) weights them by 1/2 at the new and the old time
 * level; with a general weight theta (1 = implicit Euler, 1/2 = the paper's
 * Crank-Nicolson) the step's two operators are
 *   D = (1/dt) M (u_prev - v) - theta T(v) - (1 - theta) T(u_prev) + B^T p,
 *   b = (1/dt) M u_corr - (1 - theta) T(u_corr)            (no body force). */
void orc_transport_apply(int nx, int ny, int K, const double *cxy, const double *w, double nu, double *T)
{
    int n = 1 << K, NX = nx * n, NY = ny * n;
    size_t Fn = (size_t)(NX + 1) * (NY + 1);
    double *fxy = (double *)malloc(sizeof(double) * 2 * Fn);
    orc_fine_coords(nx, ny, K, cxy, fxy);
    memset(T, 0, sizeof(double) * 2 * Fn);
    double g[2];
    gauss2(g);
    for (int parity = 0; parity < 2; ++parity)
#pragma omp parallel for schedule(static)
    for (int J = parity; J < NY; J += 2)
        for (int I = 0; I < NX; ++I) {
            int node[4] = {fine_node(nx, n, I, J), fine_node(nx, n, I + 1, J),
                           fine_node(nx, n, I, J + 1), fine_node(nx, n, I + 1, J + 1)};
            for (int qt = 0; qt < 2; ++qt)
                for (int qs = 0; qs < 2; ++qs) {
                    double N[4], dNs[4], dNt[4];
                    q1_shape(g[qs], g[qt], N);
                    q1_shape_ds(g[qs], g[qt], dNs, dNt);
                    double xs = 0, xt = 0, ys = 0, yt = 0;
                    for (int k = 0; k < 4; ++k) {
                        xs += fxy[2 * node[k]] * dNs[k];
                        xt += fxy[2 * node[k]] * dNt[k];
                        ys += fxy[2 * node[k] + 1] * dNs[k];
                        yt += fxy[2 * node[k] + 1] * dNt[k];
                    }
                    double det = xs * yt - xt * ys;
                    double dNx[4], dNy[4];
                    for (int k = 0; k < 4; ++k) {
                        dNx[k] = (yt * dNs[k] - ys * dNt[k]) / det;
                        dNy[k] = (-xt * dNs[k] + xs * dNt[k]) / det;
                    }
                    double wq[2] = {0, 0}, gw[2][2] = {{0, 0}, {0, 0}};
                    for (int k = 0; k < 4; ++k)
                        for (int c = 0; c < 2; ++c) {
                            wq[c] += N[k] * w[2 * node[k] + c];
                            gw[c][0] += w[2 * node[k] + c] * dNx[k];
                            gw[c][1] += w[2 * node[k] + c] * dNy[k];
                        }
                    double wd = 0.25 * fabs(det);
                    for (int a = 0; a < 4; ++a)
                        for (int c = 0; c < 2; ++c) {
                            double conv = wq[0] * gw[c][0] + wq[1] * gw[c][1];
                            double r = N[a] * conv + nu * (dNx[a] * gw[c][0] + dNy[a] * gw[c][1]);
                            T[2 * node[a] + c] += wd * r;
                        }
                }
        }
    free(fxy);
}

/* The defect of the theta scheme: the implicit-Euler defect (theta = 1)
 * plus (1 - theta) (T(v) - T(u_prev)), masked at Dirichlet nodes. */
void orc_defect_theta(int nx, int ny, int K, const double *cxy, const double *v, const double *p,
                      const double *uprev, double dt, double nu, double theta, unsigned dir, double *D)
{
    int n = 1 << K;
    size_t Fn = (size_t)(nx * n + 1) * (ny * n + 1);
    orc_defect(nx, ny, K, cxy, v, p, uprev, dt, nu, dir, D);
    if (theta == 1.0) return;
    double *Tv = (double *)malloc(sizeof(double) * 2 * Fn);
    double *Tu = (double *)malloc(sizeof(double) * 2 * Fn);
    unsigned char *mask = (unsigned char *)malloc(Fn);
    orc_transport_apply(nx, ny, K, cxy, v, nu, Tv);
    orc_transport_apply(nx, ny, K, cxy, uprev, nu, Tu);
    orc_dirichlet_mask(nx, ny, K, dir, mask);
    for (size_t f = 0; f < Fn; ++f)
        for (int c = 0; c < 2; ++c)
            D[2 * f + c] = mask[f] ? 0.0 : D[2 * f + c] + (1.0 - theta) * (Tv[2 * f + c] - Tu[2 * f + c]);
    free(Tv);
    free(Tu);
    free(mask);
}

/* b_L = R [(1/dt) M_f u_corr - (1 - theta) T(u_corr)], u_corr = P v + Dbar. */
void orc_rhs_restrict_theta(int nx, int ny, int K, const double *cxy, const double *v, const double *Dbar,
                            double dt, double nu, double theta, double *bL)
{
    orc_rhs_restrict(nx, ny, K, cxy, v, Dbar, dt, bL);
    if (theta == 1.0) return;
    int n = 1 << K;
    size_t Fn = (size_t)(nx * n + 1) * (ny * n + 1), Nc = (size_t)(nx + 1) * (ny + 1);
    double *u = (double *)malloc(sizeof(double) * 2 * Fn);
    double *T = (double *)malloc(sizeof(double) * 2 * Fn);
    double *RT = (double *)malloc(sizeof(double) * 2 * Nc);
    orc_prolong(nx, ny, K, 2, v, u);
    for (size_t f = 0; f < 2 * Fn; ++f) u[f] += Dbar[f];
    orc_transport_apply(nx, ny, K, cxy, u, nu, T);
    orc_restrict(nx, ny, K, 2, T, RT);
    for (size_t c = 0; c < 2 * Nc; ++c) bL[c] -= (1.0 - theta) * RT[c];
    free(u);
    free(T);
    free(RT);
}

/* ----------------------------------- the paper's network form (Sec. 4.2) */
/* The inputs and the head of the network as the paper describes them, in
 * place of the workloads' [P v, D, hx, hy, aspect, area] and MLP:
 *   inputs (3 nf + 24 per patch; 51 at K = 1, 99 at K = 2): the residual of
 *   the prolongated solution at the patch's fine nodes, momentum rows (the
 *   defect D, x, y interleaved) then continuity rows; the coarse velocity at
 *   the four corners; a Peclet number per corner; twelve geometry values;
 *   head: a fully connected layer H -> nout, two convolutional blocks on its
 *   output and a final length-1 convolution. */

/* Continuity rows of the residual of the prolongated velocity: the
 * divergence part -(div Pv, xi_a), assembled like the defect over the fine
 * elements with 2x2 Gauss points on their own bilinear maps.  The pressure
 * stabilisation of the continuity equation is not part of this input
 * (reading), and no row is masked (the pressure has no Dirichlet values). */
void orc_continuity_rows(int nx, int ny, int K, const double *cxy, const double *v, double *Rp)
{
    int n = 1 << K, NX = nx * n, NY = ny * n;
    size_t Fn = (size_t)(NX + 1) * (NY + 1);
    double *fxy = (double *)malloc(sizeof(double) * 2 * Fn);
    orc_fine_coords(nx, ny, K, cxy, fxy);
    memset(Rp, 0, sizeof(double) * Fn);
    double g[2];
    gauss2(g);
    for (int parity = 0; parity < 2; ++parity)
#pragma omp parallel for schedule(static)
    for (int J = parity; J < NY; J += 2)
        for (int I = 0; I < NX; ++I) {
            int node[4] = {fine_node(nx, n, I, J), fine_node(nx, n, I + 1, J),
                           fine_node(nx, n, I, J + 1), fine_node(nx, n, I + 1, J + 1)};
            for (int qt = 0; qt < 2; ++qt)
                for (int qs = 0; qs < 2; ++qs) {
                    double N[4], dNs[4], dNt[4];
                    q1_shape(g[qs], g[qt], N);
                    q1_shape_ds(g[qs], g[qt], dNs, dNt);
                    double xs = 0, xt = 0, ys = 0, yt = 0;
                    for (int k = 0; k < 4; ++k) {
                        xs += fxy[2 * node[k]] * dNs[k];
                        xt += fxy[2 * node[k]] * dNt[k];
                        ys += fxy[2 * node[k] + 1] * dNs[k];
                        yt += fxy[2 * node[k] + 1] * dNt[k];
                    }
                    double det = xs * yt - xt * ys;
                    double div = 0.0;
                    for (int k = 0; k < 4; ++k)
                        div += v[2 * node[k]] * (yt * dNs[k] - ys * dNt[k]) / det +
                               v[2 * node[k] + 1] * (-xt * dNs[k] + xs * dNt[k]) / det;
                    double wd = 0.25 * fabs(det);
                    for (int a = 0; a < 4; ++a) Rp[node[a]] -= wd * div * N[a];
                }
        }
    free(fxy);
}

/* Twelve geometry values per patch (its coarse element with corners
 * c00, c10, c11, c01 counter-clockwise):
 *   edge lengths  h = (|c10 - c00|, |c11 - c10|, |c11 - c01|, |c01 - c00|)
 *                     (bottom, right, top, left);
 *   aspect ratios (h0 / h1, h2 / h3, h0 / h2, h1 / h3): two pairs of
 *                     neighbouring edges, then the two pairs of opposite ones;
 *   angles        the interior angles at c00, c10, c11, c01 (radians).
 * (The paper names these three groups of four; the order and the pairing
 * are a reading.) */
static double corner_angle(const double *o, const double *a, const double *b)
{
    double ux = a[0] - o[0], uy = a[1] - o[1], wx = b[0] - o[0], wy = b[1] - o[1];
    return atan2(fabs(ux * wy - uy * wx), ux * wx + uy * wy);
}

void orc_paper_geometry(int nx, int ny, const double *cxy, double *G)
{
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const double *c00 = cxy + 2 * coarse_node(nx, i, j);
            const double *c10 = cxy + 2 * coarse_node(nx, i + 1, j);
            const double *c01 = cxy + 2 * coarse_node(nx, i, j + 1);
            const double *c11 = cxy + 2 * coarse_node(nx, i + 1, j + 1);
            double h0 = hypot(c10[0] - c00[0], c10[1] - c00[1]);
            double h1 = hypot(c11[0] - c10[0], c11[1] - c10[1]);
            double h2 = hypot(c11[0] - c01[0], c11[1] - c01[1]);
            double h3 = hypot(c01[0] - c00[0], c01[1] - c00[1]);
            double *o = G + 12 * (size_t)(j * nx + i);
            o[0] = h0; o[1] = h1; o[2] = h2; o[3] = h3;
            o[4] = h0 / h1; o[5] = h2 / h3; o[6] = h0 / h2; o[7] = h1 / h3;
            o[8] = corner_angle(c00, c10, c01);
            o[9] = corner_angle(c10, c11, c00);
            o[10] = corner_angle(c11, c01, c10);
            o[11] = corner_angle(c01, c00, c11);
        }
}

/* Peclet numbers Pe = q |v| / nu at the four corners of each patch (order
 * 00, 10, 01, 11), q the patch size, read as the square root of the coarse
 * element's area; v the coarse velocity (Euclidean norm). */
void orc_peclet(int nx, int ny, const double *cxy, const double *v, double nu, double *Pe)
{
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int c[4] = {coarse_node(nx, i, j), coarse_node(nx, i + 1, j), coarse_node(nx, i, j + 1),
                        coarse_node(nx, i + 1, j + 1)};
            const double *c00 = cxy + 2 * c[0], *c10 = cxy + 2 * c[1], *c01 = cxy + 2 * c[2], *c11 = cxy + 2 * c[3];
            double d1x = c11[0] - c00[0], d1y = c11[1] - c00[1];
            double d2x = c01[0] - c10[0], d2y = c01[1] - c10[1];
            double q = sqrt(0.5 * fabs(d1x * d2y - d1y * d2x));
            for (int k = 0; k < 4; ++k)
                Pe[4 * (size_t)(j * nx + i) + k] = q * hypot(v[2 * c[k]], v[2 * c[k] + 1]) / nu;
        }
}

/* x_e = [D at the patch nodes (x, y interleaved, x fastest), the continuity
 * rows at the same nodes, v at the corners 00, 10, 01, 11 (x, y), Pe at the
 * corners, the twelve geometry values]: 3 nf + 24 values. */
void orc_gather_input_paper(int nx, int ny, int K, const double *D, const double *Rp, const double *v,
                            const double *Pe, const double *G, double *X)
{
    int n = 1 << K, nf = (n + 1) * (n + 1), nin = 3 * nf + 24;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t e = (size_t)j * nx + i;
            double *x = X + e * nin;
            for (int b = 0; b <= n; ++b)
                for (int a = 0; a <= n; ++a) {
                    int l = b * (n + 1) + a;
                    int f = fine_node(nx, n, i * n + a, j * n + b);
                    x[2 * l] = D[2 * f];
                    x[2 * l + 1] = D[2 * f + 1];
                    x[2 * nf + l] = Rp[f];
                }
            int c[4] = {coarse_node(nx, i, j), coarse_node(nx, i + 1, j), coarse_node(nx, i, j + 1),
                        coarse_node(nx, i + 1, j + 1)};
            for (int k = 0; k < 4; ++k) {
                x[3 * nf + 2 * k] = v[2 * c[k]];
                x[3 * nf + 2 * k + 1] = v[2 * c[k] + 1];
                x[3 * nf + 8 + k] = Pe[4 * e + k];
            }
            for (int k = 0; k < 12; ++k) x[3 * nf + 12 + k] = G[12 * e + k];
        }
}

/* The GRU of Eq. (gru) (reset_after = 0: the reset gate multiplies h before
 * U_h, as printed) or with the reset gate applied after U_h,
 *   h' = z*h + (1-z)*tanh(W_h x + r * (U_h h))   (reset_after = 1),
 * the form of the common library GRU cell the paper's implementation used. */
void orc_gru_form(int P, int nin, int H, const double *Wz, const double *Wr, const double *Wh,
                  const double *Uz, const double *Ur, const double *Uh,
                  const double *X, const double *h, int reset_after, double *hout)
{
    if (!reset_after) {
        orc_gru(P, nin, H, Wz, Wr, Wh, Uz, Ur, Uh, X, h, hout);
        return;
    }
#pragma omp parallel
    {
    double *z = (double *)malloc(sizeof(double) * H);
    double *r = (double *)malloc(sizeof(double) * H);
#pragma omp for schedule(static)
    for (int e = 0; e < P; ++e) {
        const double *x = X + (size_t)e * nin;
        const double *he = h + (size_t)e * H;
        for (int k = 0; k < H; ++k) {
            double az = 0.0, ar = 0.0;
            for (int i = 0; i < nin; ++i) {
                az += Wz[(size_t)k * nin + i] * x[i];
                ar += Wr[(size_t)k * nin + i] * x[i];
            }
            for (int m = 0; m < H; ++m) {
                az += Uz[(size_t)k * H + m] * he[m];
                ar += Ur[(size_t)k * H + m] * he[m];
            }
            z[k] = logistic(az);
            r[k] = logistic(ar);
        }
        for (int k = 0; k < H; ++k) {
            double wx = 0.0, uh = 0.0;
            for (int i = 0; i < nin; ++i) wx += Wh[(size_t)k * nin + i] * x[i];
            for (int m = 0; m < H; ++m) uh += Uh[(size_t)k * H + m] * he[m];
            hout[(size_t)e * H + k] = z[k] * he[k] + (1.0 - z[k]) * tanh(wx + r[k] * uh);
        }
    }
    free(z);
    free(r);
    }
}

/* A convolutional block: a convolution with 4 filters of 3 x 3 taps (zero
 * padding 1, stride 1) from one channel to 4, then the transposed
 * convolution with the same weights from 4 channels back to one (the
 * block's second layer is the first one transposed; 36 weights).  The
 * image is rows x cols, row-major; W[f][dr][dc] for offsets dr, dc in -1..1. */
static void conv_block(int rows, int cols, const double *W, const double *in, double *out)
{
    double *z = (double *)malloc(sizeof(double) * 4 * rows * cols);
    for (int f = 0; f < 4; ++f)
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c) {
                double s = 0.0;
                for (int dr = -1; dr <= 1; ++dr)
                    for (int dc = -1; dc <= 1; ++dc) {
                        int rr = r + dr, cc = c + dc;
                        if (rr >= 0 && rr < rows && cc >= 0 && cc < cols)
                            s += W[9 * f + 3 * (dr + 1) + (dc + 1)] * in[rr * cols + cc];
                    }
                z[(f * rows + r) * cols + c] = s;
            }
    /* the adjoint: out[r][c] = sum_f sum_{dr,dc} W[f][dr][dc] z_f[r - dr][c - dc] */
    for (int r = 0; r < rows; ++r)
        for (int c = 0; c < cols; ++c) {
            double s = 0.0;
            for (int f = 0; f < 4; ++f)
                for (int dr = -1; dr <= 1; ++dr)
                    for (int dc = -1; dc <= 1; ++dc) {
                        int rr = r - dr, cc = c - dc;
                        if (rr >= 0 && rr < rows && cc >= 0 && cc < cols)
                            s += W[9 * f + 3 * (dr + 1) + (dc + 1)] * z[(f * rows + rr) * cols + cc];
                    }
            out[r * cols + c] = s;
        }
    free(z);
}

/* The paper's head on the GRU state h' (no biases, no activations stated):
 *   y = M h'                                       (fully connected, nout x H)
 *   a = V(y): the vertex block, on y as a 2 x nf image (component rows,
 *             patch nodes in the input's order as columns): its 3 x 3
 *             taps join the two components of a node and of the nodes
 *             beside it in that order;
 *   b = S(y): the spatial block, on each component as an (n+1) x (n+1)
 *             image of the patch's nodes;
 *   d = wf * (a + b)                               (the final length-1
 *             convolution: the two blocks' single filters summed, each
 *             output entry weighted; nout weights).
 * (Reading of the architecture figure and the parameter counts: the 90
 * parameters beside the GRU and the dense layer are 36 + 36 + 18 at K = 1.) */
void orc_conv_head(int P, int K, int H, const double *M, const double *WV, const double *WS, const double *wf,
                   const double *h, double *d)
{
    int n = 1 << K, nf = (n + 1) * (n + 1), nout = 2 * nf;
#pragma omp parallel
    {
    double *y = (double *)malloc(sizeof(double) * nout);
    double *a = (double *)malloc(sizeof(double) * nout);
    double *comp = (double *)malloc(sizeof(double) * nf);
    double *bc = (double *)malloc(sizeof(double) * nf);
    double *img = (double *)malloc(sizeof(double) * nout);
#pragma omp for schedule(static)
    for (int e = 0; e < P; ++e) {
        const double *he = h + (size_t)e * H;
        for (int o = 0; o < nout; ++o) {
            double s = 0.0;
            for (int m = 0; m < H; ++m) s += M[(size_t)o * H + m] * he[m];
            y[o] = s;
        }
        /* vertex block: image row c = component, column l = node */
        for (int c = 0; c < 2; ++c)
            for (int l = 0; l < nf; ++l) img[c * nf + l] = y[2 * l + c];
        conv_block(2, nf, WV, img, a);
        double *de = d + (size_t)e * nout;
        for (int c = 0; c < 2; ++c)
            for (int l = 0; l < nf; ++l) de[2 * l + c] = a[c * nf + l];
        /* spatial block, per component */
        for (int c = 0; c < 2; ++c) {
            for (int l = 0; l < nf; ++l) comp[l] = y[2 * l + c];
            conv_block(n + 1, n + 1, WS, comp, bc);
            for (int l = 0; l < nf; ++l) de[2 * l + c] += bc[l];
        }
        for (int o = 0; o < nout; ++o) de[o] *= wf[o];
    }
    free(y); free(a); free(comp); free(bc); free(img);
    }
}

/* Weights of the paper's form: W_z, W_r, W_h (H x (3 nf + 24)), U_z, U_r,
 * U_h (H x H), M (nout x H), the vertex block's 36, the spatial block's 36,
 * the final layer's nout. */
long orc_paper_weight_count(int K, int H)
{
    int n = 1 << K, nf = (n + 1) * (n + 1), nin = 3 * nf + 24, nout = 2 * nf;
    return 3L * H * (nin + H) + (long)nout * H + 36 + 36 + nout;
}

/* ------------------------------------------ unstructured quadrilateral meshes */
/* A coarse mesh of quadrilaterals given by node coordinates and, per element,
 * its four nodes v0, v1, v2, v3 counter-clockwise (reference corners (0,0),
 * (1,0), (1,1), (0,1)); edges may lie on circles (isoparametric refinement).
 * Each element is refined into n x n fine elements, n = 2^K (one patch per
 * coarse element).  Fine nodes are numbered
 *   0 .. Nc-1                  the coarse nodes;
 *   Nc + k (n-1) + (t-1)       the n-1 inner nodes of coarse edge k, t = 1..n-1
 *                              counted from the edge's lower-numbered node;
 *                              edges numbered in order of first appearance over
 *                              the elements, local edges in the order
 *                              (v0,v1), (v1,v2), (v3,v2), (v0,v3);
 *   Nc + E (n-1) + e (n-1)^2 + (b-1)(n-1) + (a-1)
 *                              the inner nodes (a, b) of element e.
 * pmap[e nf + b (n+1) + a] is the fine node at reference point (a/n, b/n) of
 * element e (patch-local order as in the structured form). */

/* Edges: an open-addressing table of node pairs (lo, hi) -> edge index. */
typedef struct { int *key; int cap; } edge_table;

static int edge_find_or_add(edge_table *t, int a, int b, int *next)
{
    int lo = a < b ? a : b, hi = a < b ? b : a;
    unsigned long long h = ((unsigned long long)(unsigned)lo * 2654435761ULL) ^ ((unsigned long long)(unsigned)hi * 40503ULL);
    int i = (int)(h % (unsigned long long)t->cap);
    for (;;) {
        if (t->key[3 * i] < 0) {
            t->key[3 * i] = lo; t->key[3 * i + 1] = hi; t->key[3 * i + 2] = (*next)++;
            return t->key[3 * i + 2];
        }
        if (t->key[3 * i] == lo && t->key[3 * i + 1] == hi) return t->key[3 * i + 2];
        i = (i + 1) % t->cap;
    }
}

/* Edge index of each element's four local edges (ne x 4); returns E. */
static int umesh_edges(int ne, const int *elems, int *eidx)
{
    edge_table t;
    t.cap = 8 * ne + 16;
    t.key = (int *)malloc(sizeof(int) * 3 * t.cap);
    for (int i = 0; i < 3 * t.cap; ++i) t.key[i] = -1;
    int next = 0;
    for (int e = 0; e < ne; ++e) {
        const int *v = elems + 4 * e;
        const int ends[4][2] = {{v[0], v[1]}, {v[1], v[2]}, {v[3], v[2]}, {v[0], v[3]}};
        for (int k = 0; k < 4; ++k) eidx[4 * e + k] = edge_find_or_add(&t, ends[k][0], ends[k][1], &next);
    }
    free(t.key);
    return next;
}

/* Number of edges and of fine nodes. */
int orc_umesh_count(int nc, int ne, const int *elems, int K, int *n_edges, int *n_fine)
{
    int n = 1 << K;
    int *eidx = (int *)malloc(sizeof(int) * 4 * ne);
    int E = umesh_edges(ne, elems, eidx);
    free(eidx);
    *n_edges = E;
    *n_fine = nc + E * (n - 1) + ne * (n - 1) * (n - 1);
    return 0;
}

/* The curve of an element edge from node a to node b at parameter s in
 * [0, 1]: the straight segment, or the circular arc between them (angle
 * linear in s) when the edge is listed as curved. */
static int curve_of(int a, int b, int ncurved, const int *curved)
{
    for (int k = 0; k < ncurved; ++k)
        if ((curved[3 * k] == a && curved[3 * k + 1] == b) || (curved[3 * k] == b && curved[3 * k + 1] == a))
            return curved[3 * k + 2];
    return -1;
}

static void edge_point(const double *xy, int a, int b, double s, int circ, const double *circles, double *out)
{
    const double *A = xy + 2 * a, *B = xy + 2 * b;
    if (circ < 0) {
        out[0] = (1.0 - s) * A[0] + s * B[0];
        out[1] = (1.0 - s) * A[1] + s * B[1];
        return;
    }
    const double cx = circles[3 * circ], cy = circles[3 * circ + 1], r = circles[3 * circ + 2];
    double ta = atan2(A[1] - cy, A[0] - cx), tb = atan2(B[1] - cy, B[0] - cx);
    double d = tb - ta;
    const double pi = 3.14159265358979323846;
    while (d > pi) d -= 2.0 * pi;
    while (d < -pi) d += 2.0 * pi;
    out[0] = cx + r * cos(ta + s * d);
    out[1] = cy + r * sin(ta + s * d);
}

/* Fine node coordinates (Fn x 2) and the patch maps (ne x nf).  Edge nodes
 * sit on the edge's curve at parameter t/n from its lower-numbered node;
 * inner nodes at F_e(a/n, b/n), F_e the transfinite (Gordon-Hall) map of the
 * element's four edge curves (the bilinear map when all four are straight). */
int orc_umesh_refine(int nc, int ne, const double *xy, const int *elems, int K, int ncurved, const int *curved,
                     const double *circles, double *fxy, int *pmap)
{
    int n = 1 << K, nf = (n + 1) * (n + 1);
    int *eidx = (int *)malloc(sizeof(int) * 4 * ne);
    int E = umesh_edges(ne, elems, eidx);
    int base_in = nc + E * (n - 1);
    for (int i = 0; i < nc; ++i) { fxy[2 * i] = xy[2 * i]; fxy[2 * i + 1] = xy[2 * i + 1]; }
    for (int e = 0; e < ne; ++e) {
        const int *v = elems + 4 * e;
        const int ends[4][2] = {{v[0], v[1]}, {v[1], v[2]}, {v[3], v[2]}, {v[0], v[3]}};
        int circ[4];
        for (int k = 0; k < 4; ++k) circ[k] = curve_of(ends[k][0], ends[k][1], ncurved, curved);
        for (int b = 0; b <= n; ++b)
            for (int a = 0; a <= n; ++a) {
                int l = b * (n + 1) + a, f;
                double xi = (double)a / n, eta = (double)b / n;
                int edge = -1, along = 0;            /* local edge and the index along it from its first end */
                if (b == 0 && a > 0 && a < n) { edge = 0; along = a; }
                else if (a == n && b > 0 && b < n) { edge = 1; along = b; }
                else if (b == n && a > 0 && a < n) { edge = 2; along = a; }
                else if (a == 0 && b > 0 && b < n) { edge = 3; along = b; }
                if (a == 0 && b == 0) f = v[0];
                else if (a == n && b == 0) f = v[1];
                else if (a == n && b == n) f = v[2];
                else if (a == 0 && b == n) f = v[3];
                else if (edge >= 0) {
                    int p = ends[edge][0], q = ends[edge][1];
                    int t = p < q ? along : n - along;          /* from the lower-numbered node */
                    f = nc + eidx[4 * e + edge] * (n - 1) + (t - 1);
                    int lo = p < q ? p : q, hi = p < q ? q : p;
                    edge_point(xy, lo, hi, (double)t / n, circ[edge], circles, fxy + 2 * f);
                } else {
                    f = base_in + e * (n - 1) * (n - 1) + (b - 1) * (n - 1) + (a - 1);
                    /* transfinite map: edge curves blended, minus the bilinear corner part */
                    double Bp[2], Tp[2], Lp[2], Rp[2];
                    edge_point(xy, v[0], v[1], xi, circ[0], circles, Bp);
                    edge_point(xy, v[3], v[2], xi, circ[2], circles, Tp);
                    edge_point(xy, v[0], v[3], eta, circ[3], circles, Lp);
                    edge_point(xy, v[1], v[2], eta, circ[1], circles, Rp);
                    for (int c = 0; c < 2; ++c) {
                        double bil = (1 - xi) * (1 - eta) * xy[2 * v[0] + c] + xi * (1 - eta) * xy[2 * v[1] + c] +
                                     xi * eta * xy[2 * v[2] + c] + (1 - xi) * eta * xy[2 * v[3] + c];
                        fxy[2 * f + c] = (1 - eta) * Bp[c] + eta * Tp[c] + (1 - xi) * Lp[c] + xi * Rp[c] - bil;
                    }
                }
                pmap[(size_t)e * nf + l] = f;
            }
    }
    free(eidx);
    return 0;
}

/* P: fine node f takes the bilinear interpolation (in reference
 * coordinates) of the corner values of the first element containing it. */
static void umesh_first(int ne, int K, const int *pmap, int Fn, int *first)
{
    int nf = ((1 << K) + 1) * ((1 << K) + 1);
    for (int f = 0; f < Fn; ++f) first[f] = -1;
    for (int e = 0; e < ne; ++e)
        for (int l = 0; l < nf; ++l)
            if (first[pmap[(size_t)e * nf + l]] < 0) first[pmap[(size_t)e * nf + l]] = e * nf + l;
}

static void umesh_hats(int K, int l, double N[4])   /* corner order v0, v1, v2, v3 */
{
    int n = 1 << K, a = l % (n + 1), b = l / (n + 1);
    double s = (double)a / n, t = (double)b / n;
    N[0] = (1 - s) * (1 - t); N[1] = s * (1 - t); N[2] = s * t; N[3] = (1 - s) * t;
}

void orc_u_prolong(int ne, int K, const int *elems, const int *pmap, int Fn, int ncomp, const double *coarse,
                   double *fine)
{
    int nf = ((1 << K) + 1) * ((1 << K) + 1);
    int *first = (int *)malloc(sizeof(int) * Fn);
    umesh_first(ne, K, pmap, Fn, first);
    for (int f = 0; f < Fn; ++f) {
        int e = first[f] / nf, l = first[f] % nf;
        double N[4];
        umesh_hats(K, l, N);
        for (int c = 0; c < ncomp; ++c) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += N[k] * coarse[ncomp * elems[4 * e + k] + c];
            fine[ncomp * f + c] = s;
        }
    }
    free(first);
}

/* R = P^T. */
void orc_u_restrict(int nc, int ne, int K, const int *elems, const int *pmap, int Fn, int ncomp, const double *fine,
                    double *coarse)
{
    int nf = ((1 << K) + 1) * ((1 << K) + 1);
    int *first = (int *)malloc(sizeof(int) * Fn);
    umesh_first(ne, K, pmap, Fn, first);
    memset(coarse, 0, sizeof(double) * ncomp * nc);
    for (int f = 0; f < Fn; ++f) {
        int e = first[f] / nf, l = first[f] % nf;
        double N[4];
        umesh_hats(K, l, N);
        for (int k = 0; k < 4; ++k)
            for (int c = 0; c < ncomp; ++c) coarse[ncomp * elems[4 * e + k] + c] += N[k] * fine[ncomp * f + c];
    }
    free(first);
}

/* Dirichlet mask: fine nodes on the listed coarse edges (node pairs), ends
 * included. */
void orc_u_mask(int ne, int K, const int *elems, const int *pmap, int Fn, int ndir, const int *dir_edges,
                unsigned char *mask)
{
    int n = 1 << K, nf = (n + 1) * (n + 1);
    memset(mask, 0, Fn);
    for (int e = 0; e < ne; ++e) {
        const int *v = elems + 4 * e;
        const int ends[4][2] = {{v[0], v[1]}, {v[1], v[2]}, {v[3], v[2]}, {v[0], v[3]}};
        for (int k = 0; k < 4; ++k) {
            int on = 0;
            for (int d = 0; d < ndir; ++d)
                if ((dir_edges[2 * d] == ends[k][0] && dir_edges[2 * d + 1] == ends[k][1]) ||
                    (dir_edges[2 * d] == ends[k][1] && dir_edges[2 * d + 1] == ends[k][0])) on = 1;
            if (!on) continue;
            for (int t = 0; t <= n; ++t) {
                int a = k == 0 || k == 2 ? t : (k == 1 ? n : 0);
                int b = k == 1 || k == 3 ? t : (k == 2 ? n : 0);
                mask[pmap[(size_t)e * nf + b * (n + 1) + a]] = 1;
            }
        }
    }
}

/* The fine elements of the refined mesh: element (e, a, b) has the fine
 * nodes of patch-local (a,b), (a+1,b), (a,b+1), (a+1,b+1) (corner order 00,
 * 10, 01, 11 of q1_shape). */
static void ufine_nodes(int K, const int *pmap, int e, int a, int b, int node[4])
{
    int n = 1 << K, nf = (n + 1) * (n + 1);
    const int *pm = pmap + (size_t)e * nf;
    node[0] = pm[b * (n + 1) + a]; node[1] = pm[b * (n + 1) + a + 1];
    node[2] = pm[(b + 1) * (n + 1) + a]; node[3] = pm[(b + 1) * (n + 1) + a + 1];
}

/* The defect of orc_defect on the refined unstructured mesh (same element
 * terms and quadrature on every fine element), masked. */
void orc_u_defect(int ne, int K, const int *pmap, const double *fxy, int Fn, const double *v, const double *p,
                  const double *uprev, double dt, double nu, const unsigned char *mask, double *D)
{
    int n = 1 << K;
    memset(D, 0, sizeof(double) * 2 * Fn);
    double g[2];
    gauss2(g);
    for (int e = 0; e < ne; ++e)
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
                int node[4];
                ufine_nodes(K, pmap, e, a, b, node);
                for (int qt = 0; qt < 2; ++qt)
                    for (int qs = 0; qs < 2; ++qs) {
                        double N[4], dNs[4], dNt[4];
                        q1_shape(g[qs], g[qt], N);
                        q1_shape_ds(g[qs], g[qt], dNs, dNt);
                        double xs = 0, xt = 0, ys = 0, yt = 0;
                        for (int k = 0; k < 4; ++k) {
                            xs += fxy[2 * node[k]] * dNs[k];
                            xt += fxy[2 * node[k]] * dNt[k];
                            ys += fxy[2 * node[k] + 1] * dNs[k];
                            yt += fxy[2 * node[k] + 1] * dNt[k];
                        }
                        double det = xs * yt - xt * ys;
                        double dNx[4], dNy[4];
                        for (int k = 0; k < 4; ++k) {
                            dNx[k] = (yt * dNs[k] - ys * dNt[k]) / det;
                            dNy[k] = (-xt * dNs[k] + xs * dNt[k]) / det;
                        }
                        double vq[2] = {0, 0}, uq[2] = {0, 0}, pq = 0, gv[2][2] = {{0, 0}, {0, 0}};
                        for (int k = 0; k < 4; ++k) {
                            for (int c = 0; c < 2; ++c) {
                                vq[c] += N[k] * v[2 * node[k] + c];
                                uq[c] += N[k] * uprev[2 * node[k] + c];
                                gv[c][0] += v[2 * node[k] + c] * dNx[k];
                                gv[c][1] += v[2 * node[k] + c] * dNy[k];
                            }
                            pq += N[k] * p[node[k]];
                        }
                        double wd = 0.25 * fabs(det);
                        for (int k = 0; k < 4; ++k)
                            for (int c = 0; c < 2; ++c) {
                                double conv = vq[0] * gv[c][0] + vq[1] * gv[c][1];
                                double dphi = c == 0 ? dNx[k] : dNy[k];
                                D[2 * node[k] + c] += wd * ((1.0 / dt) * N[k] * (uq[c] - vq[c]) - N[k] * conv -
                                                            nu * (dNx[k] * gv[c][0] + dNy[k] * gv[c][1]) + pq * dphi);
                            }
                    }
            }
    for (int f = 0; f < Fn; ++f)
        if (mask[f]) { D[2 * f] = 0.0; D[2 * f + 1] = 0.0; }
}

/* M_f u on the refined unstructured mesh. */
void orc_u_mass_apply(int ne, int K, const int *pmap, const double *fxy, int Fn, const double *u, double *Mu)
{
    int n = 1 << K;
    memset(Mu, 0, sizeof(double) * 2 * Fn);
    double g[2];
    gauss2(g);
    for (int e = 0; e < ne; ++e)
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
                int node[4];
                ufine_nodes(K, pmap, e, a, b, node);
                for (int qt = 0; qt < 2; ++qt)
                    for (int qs = 0; qs < 2; ++qs) {
                        double N[4], dNs[4], dNt[4];
                        q1_shape(g[qs], g[qt], N);
                        q1_shape_ds(g[qs], g[qt], dNs, dNt);
                        double xs = 0, xt = 0, ys = 0, yt = 0;
                        for (int k = 0; k < 4; ++k) {
                            xs += fxy[2 * node[k]] * dNs[k];
                            xt += fxy[2 * node[k]] * dNt[k];
                            ys += fxy[2 * node[k] + 1] * dNs[k];
                            yt += fxy[2 * node[k] + 1] * dNt[k];
                        }
                        double wd = 0.25 * fabs(xs * yt - xt * ys), uq[2] = {0, 0};
                        for (int k = 0; k < 4; ++k)
                            for (int c = 0; c < 2; ++c) uq[c] += N[k] * u[2 * node[k] + c];
                        for (int k = 0; k < 4; ++k)
                            for (int c = 0; c < 2; ++c) Mu[2 * node[k] + c] += wd * N[k] * uq[c];
                    }
            }
}

/* Patch features of orc_features from each element's four corners (v0..v3
 * counter-clockwise): hx the mean of the edges (v0,v1), (v3,v2), hy of
 * (v0,v3), (v1,v2), their ratio, and the area of the straight quadrilateral. */
void orc_u_features(int ne, const double *xy, const int *elems, double *feat)
{
    for (int e = 0; e < ne; ++e) {
        const double *c0 = xy + 2 * elems[4 * e], *c1 = xy + 2 * elems[4 * e + 1];
        const double *c2 = xy + 2 * elems[4 * e + 2], *c3 = xy + 2 * elems[4 * e + 3];
        double hx = 0.5 * (hypot(c1[0] - c0[0], c1[1] - c0[1]) + hypot(c2[0] - c3[0], c2[1] - c3[1]));
        double hy = 0.5 * (hypot(c3[0] - c0[0], c3[1] - c0[1]) + hypot(c2[0] - c1[0], c2[1] - c1[1]));
        double d1x = c2[0] - c0[0], d1y = c2[1] - c0[1], d2x = c3[0] - c1[0], d2y = c3[1] - c1[1];
        double *f = feat + 4 * (size_t)e;
        f[0] = hx; f[1] = hy; f[2] = hx / hy; f[3] = 0.5 * fabs(d1x * d2y - d1y * d2x);
    }
}

/* Network input rows as orc_gather_input, through the patch maps. */
void orc_u_gather_input(int ne, int K, const int *pmap, const double *pv, const double *D, const double *feat,
                        double *X)
{
    int n = 1 << K, nf = (n + 1) * (n + 1), nin = 4 * nf + 4;
    for (int e = 0; e < ne; ++e) {
        double *x = X + (size_t)e * nin;
        for (int l = 0; l < nf; ++l) {
            int f = pmap[(size_t)e * nf + l];
            x[2 * l] = pv[2 * f]; x[2 * l + 1] = pv[2 * f + 1];
            x[2 * nf + 2 * l] = D[2 * f]; x[2 * nf + 2 * l + 1] = D[2 * f + 1];
        }
        for (int k = 0; k < 4; ++k) x[4 * nf + k] = feat[4 * (size_t)e + k];
    }
}

/* Duplicate averaging: the mean of the outputs of every patch that holds
 * the fine node (summed in patch order), zero at masked nodes. */
void orc_u_average(int ne, int K, const int *pmap, int Fn, const double *dpatch, const unsigned char *mask,
                   double *Dbar)
{
    int nf = ((1 << K) + 1) * ((1 << K) + 1);
    int *cnt = (int *)calloc(Fn, sizeof(int));
    memset(Dbar, 0, sizeof(double) * 2 * Fn);
    for (int e = 0; e < ne; ++e)
        for (int l = 0; l < nf; ++l) {
            int f = pmap[(size_t)e * nf + l];
            Dbar[2 * f] += dpatch[((size_t)e * nf + l) * 2];
            Dbar[2 * f + 1] += dpatch[((size_t)e * nf + l) * 2 + 1];
            cnt[f]++;
        }
    for (int f = 0; f < Fn; ++f) {
        if (mask[f] || cnt[f] == 0) { Dbar[2 * f] = 0.0; Dbar[2 * f + 1] = 0.0; continue; }
        Dbar[2 * f] /= cnt[f];
        Dbar[2 * f + 1] /= cnt[f];
    }
    free(cnt);
}

/* b_L = R (1/dt) M_f (P v + Dbar) on the unstructured mesh. */
void orc_u_rhs_restrict(int nc, int ne, int K, const int *elems, const int *pmap, const double *fxy, int Fn,
                        const double *v, const double *Dbar, double dt, double *bL)
{
    double *u = (double *)malloc(sizeof(double) * 2 * Fn), *Mu = (double *)malloc(sizeof(double) * 2 * Fn);
    orc_u_prolong(ne, K, elems, pmap, Fn, 2, v, u);
    for (int f = 0; f < 2 * Fn; ++f) u[f] += Dbar[f];
    orc_u_mass_apply(ne, K, pmap, fxy, Fn, u, Mu);
    for (int f = 0; f < 2 * Fn; ++f) Mu[f] /= dt;
    orc_u_restrict(nc, ne, K, elems, pmap, Fn, 2, Mu, bL);
    free(u);
    free(Mu);
}

/* One fine step (the fine part of Alg. 2; implicit Euler, the workloads' network)
 * on the refined unstructured mesh: orc_step with the mesh's own prolongation,
 * defect, patch inputs, averaging and rhs.  State h (ne x H), uprev (Fn x 2);
 * optional outputs as orc_step (D, X, dpatch, Dbar over the fine nodes,
 * bL over the coarse nodes). */
int orc_u_step(int nc, int ne, const double *xy, const int *elems, int K, int H, int Hm, double dt, double nu,
               const int *pmap, const double *fxy, int Fn, const unsigned char *mask, const double *weights,
               const double *v, const double *p, double *h, double *uprev, int first,
               double *Pv_out, double *D_out, double *X_out, double *dpatch_out, double *Dbar_out, double *bL_out)
{
    int n = 1 << K, nf = (n + 1) * (n + 1), nout = 2 * nf, nin = 4 * nf + 4, P = ne;
    const double *Wz = weights, *Wr = Wz + (size_t)H * nin, *Wh = Wr + (size_t)H * nin;
    const double *Uz = Wh + (size_t)H * nin, *Ur = Uz + (size_t)H * H, *Uh = Ur + (size_t)H * H;
    const double *M1 = Uh + (size_t)H * H, *M2 = Hm > 0 ? M1 + (size_t)Hm * H : NULL;
    double *Pv = (double *)malloc(sizeof(double) * 2 * Fn), *Pp = (double *)malloc(sizeof(double) * Fn);
    double *D = (double *)malloc(sizeof(double) * 2 * Fn), *feat = (double *)malloc(sizeof(double) * 4 * P);
    double *X = (double *)malloc(sizeof(double) * (size_t)P * nin), *hn = (double *)malloc(sizeof(double) * (size_t)P * H);
    double *dp = (double *)malloc(sizeof(double) * (size_t)P * nout), *Dbar = (double *)malloc(sizeof(double) * 2 * Fn);
    double *bL = (double *)malloc(sizeof(double) * 2 * nc);
    if (!Pv || !Pp || !D || !feat || !X || !hn || !dp || !Dbar || !bL) return -2;
    orc_u_prolong(ne, K, elems, pmap, Fn, 2, v, Pv);
    orc_u_prolong(ne, K, elems, pmap, Fn, 1, p, Pp);
    if (first) memcpy(uprev, Pv, sizeof(double) * 2 * Fn);
    orc_u_defect(ne, K, pmap, fxy, Fn, Pv, Pp, uprev, dt, nu, mask, D);
    orc_u_features(ne, xy, elems, feat);
    orc_u_gather_input(ne, K, pmap, Pv, D, feat, X);
    orc_gru(P, nin, H, Wz, Wr, Wh, Uz, Ur, Uh, X, h, hn);
    orc_mlp(P, H, Hm, nout, M1, M2, hn, dp);
    orc_u_average(ne, K, pmap, Fn, dp, mask, Dbar);
    orc_u_rhs_restrict(nc, ne, K, elems, pmap, fxy, Fn, v, Dbar, dt, bL);
    memcpy(h, hn, sizeof(double) * (size_t)P * H);
    for (int f = 0; f < 2 * Fn; ++f) uprev[f] = Pv[f] + Dbar[f];
    if (Pv_out) memcpy(Pv_out, Pv, sizeof(double) * 2 * Fn);
    if (D_out) memcpy(D_out, D, sizeof(double) * 2 * Fn);
    if (X_out) memcpy(X_out, X, sizeof(double) * (size_t)P * nin);
    if (dpatch_out) memcpy(dpatch_out, dp, sizeof(double) * (size_t)P * nout);
    if (Dbar_out) memcpy(Dbar_out, Dbar, sizeof(double) * 2 * Fn);
    if (bL_out) memcpy(bL_out, bL, sizeof(double) * 2 * nc);
    free(Pv); free(Pp); free(D); free(feat); free(X); free(hn); free(dp); free(Dbar); free(bL);
    return 0;
}

/* ---------------------------------------------------------- the full step */
/* One DNN-MG fine step (the fine part of Alg. 2) for given coarse v, p, with the
 * time scheme's weight theta (1: implicit Euler; 1/2: Crank-Nicolson as in
 * Eq. (4cranknicholson3); see orc_defect_theta, orc_rhs_restrict_theta).
 * form 0: the workloads' network, inputs [P v, D, hx, hy, aspect, area] and
 *   weights W_z, W_r, W_h (H x nin), U_z, U_r, U_h (H x H), then M1 (Hm x H)
 *   and M2 (nout x Hm), or M (nout x H) when Hm == 0;
 * form 1: the paper's network (inputs of orc_gather_input_paper, head of
 *   orc_conv_head; weights as orc_paper_weight_count lists; Hm unused).
 * reset_after selects the GRU form (orc_gru_form).
 * fp8 != 0 takes the network products with FP8 E4M3 operands (form 0 with
 * reset_after = 0 only: orc_gru_fp8, orc_mlp_fp8).
 * State in/out: h (P x H), uprev (Fn x 2).  When first != 0 the previous
 * corrected velocity is taken as P v of this step (no right-hand side from
 * an earlier step exists yet), so the mass term of the defect vanishes.
 * Optional outputs (NULL to skip): Pv (Fn x 2), D (Fn x 2), X (P x nin),
 * dpatch (P x nout), Dbar (Fn x 2), bL ((nx+1)(ny+1) x 2).
 * Returns 0, -1 for an unsupported combination, -2 when out of memory. */
int orc_step_form(int nx, int ny, int K, int H, int Hm, double dt, double nu, double theta, unsigned dir,
                  int form, int reset_after, const double *cxy, const double *weights, const double *v,
                  const double *p, double *h, double *uprev, int first, int fp8,
                  double *Pv_out, double *D_out, double *X_out, double *dpatch_out,
                  double *Dbar_out, double *bL_out)
{
    int n = 1 << K, nf = (n + 1) * (n + 1), nout = 2 * nf;
    int nin = form ? 3 * nf + 24 : 4 * nf + 4;
    int P = nx * ny;
    if (fp8 && (form || reset_after)) return -1;
    size_t Fn = (size_t)(nx * n + 1) * (ny * n + 1);
    size_t Nc = (size_t)(nx + 1) * (ny + 1);
    const double *Wz = weights, *Wr = Wz + (size_t)H * nin, *Wh = Wr + (size_t)H * nin;
    const double *Uz = Wh + (size_t)H * nin, *Ur = Uz + (size_t)H * H, *Uh = Ur + (size_t)H * H;
    const double *M1 = Uh + (size_t)H * H;
    const double *M2 = (!form && Hm > 0) ? M1 + (size_t)Hm * H : NULL;
    const double *WV = M1 + (size_t)nout * H, *WS = WV + 36, *wf = WS + 36;   /* form 1 */

    double *Pv = (double *)malloc(sizeof(double) * 2 * Fn);
    double *Pp = (double *)malloc(sizeof(double) * Fn);
    double *D = (double *)malloc(sizeof(double) * 2 * Fn);
    double *feat = (double *)malloc(sizeof(double) * 12 * P);
    double *X = (double *)malloc(sizeof(double) * (size_t)P * nin);
    double *hn = (double *)malloc(sizeof(double) * (size_t)P * H);
    double *dp = (double *)malloc(sizeof(double) * (size_t)P * nout);
    double *Dbar = (double *)malloc(sizeof(double) * 2 * Fn);
    double *bL = (double *)malloc(sizeof(double) * 2 * Nc);
    double *Rp = form ? (double *)malloc(sizeof(double) * Fn) : NULL;
    double *Pe = form ? (double *)malloc(sizeof(double) * 4 * P) : NULL;
    if (!Pv || !Pp || !D || !feat || !X || !hn || !dp || !Dbar || !bL || (form && (!Rp || !Pe))) return -2;

    orc_prolong(nx, ny, K, 2, v, Pv);
    orc_prolong(nx, ny, K, 1, p, Pp);
    if (first) memcpy(uprev, Pv, sizeof(double) * 2 * Fn);
    orc_defect_theta(nx, ny, K, cxy, Pv, Pp, uprev, dt, nu, theta, dir, D);
    if (form) {
        orc_continuity_rows(nx, ny, K, cxy, Pv, Rp);
        orc_peclet(nx, ny, cxy, v, nu, Pe);
        orc_paper_geometry(nx, ny, cxy, feat);
        orc_gather_input_paper(nx, ny, K, D, Rp, v, Pe, feat, X);
    } else {
        orc_features(nx, ny, cxy, feat);
        orc_gather_input(nx, ny, K, Pv, D, feat, X);
    }
    if (fp8) {
        orc_gru_fp8(P, nin, H, Wz, Wr, Wh, Uz, Ur, Uh, X, h, hn);
        orc_mlp_fp8(P, H, Hm, nout, M1, M2, hn, dp);
    } else {
        orc_gru_form(P, nin, H, Wz, Wr, Wh, Uz, Ur, Uh, X, h, reset_after, hn);
        if (form) orc_conv_head(P, K, H, M1, WV, WS, wf, hn, dp);
        else orc_mlp(P, H, Hm, nout, M1, M2, hn, dp);
    }
    orc_average(nx, ny, K, dp, dir, Dbar);
    orc_rhs_restrict_theta(nx, ny, K, cxy, v, Dbar, dt, nu, theta, bL);

    /* state update: h <- h', u_prev <- u_corr = P v + Dbar */
    memcpy(h, hn, sizeof(double) * (size_t)P * H);
    for (size_t f = 0; f < 2 * Fn; ++f) uprev[f] = Pv[f] + Dbar[f];

    if (Pv_out) memcpy(Pv_out, Pv, sizeof(double) * 2 * Fn);
    if (D_out) memcpy(D_out, D, sizeof(double) * 2 * Fn);
    if (X_out) memcpy(X_out, X, sizeof(double) * (size_t)P * nin);
    if (dpatch_out) memcpy(dpatch_out, dp, sizeof(double) * (size_t)P * nout);
    if (Dbar_out) memcpy(Dbar_out, Dbar, sizeof(double) * 2 * Fn);
    if (bL_out) memcpy(bL_out, bL, sizeof(double) * 2 * Nc);
    free(Pv); free(Pp); free(D); free(feat); free(X); free(hn); free(dp); free(Dbar); free(bL);
    free(Rp); free(Pe);
    return 0;
}

/* orc_step_form with the workloads' network (form 0, reset gate as printed). */
int orc_step_theta(int nx, int ny, int K, int H, int Hm, double dt, double nu, double theta, unsigned dir,
                   const double *cxy, const double *weights, const double *v, const double *p,
                   double *h, double *uprev, int first, int fp8,
                   double *Pv_out, double *D_out, double *X_out, double *dpatch_out,
                   double *Dbar_out, double *bL_out)
{
    return orc_step_form(nx, ny, K, H, Hm, dt, nu, theta, dir, 0, 0, cxy, weights, v, p, h, uprev, first, fp8,
                         Pv_out, D_out, X_out, dpatch_out, Dbar_out, bL_out);
}

/* orc_step_theta with implicit Euler (theta = 1). */
int orc_step_prec(int nx, int ny, int K, int H, int Hm, double dt, double nu, unsigned dir,
                  const double *cxy, const double *weights, const double *v, const double *p,
                  double *h, double *uprev, int first, int fp8,
                  double *Pv_out, double *D_out, double *X_out, double *dpatch_out,
                  double *Dbar_out, double *bL_out)
{
    return orc_step_theta(nx, ny, K, H, Hm, dt, nu, 1.0, dir, cxy, weights, v, p, h, uprev, first, fp8,
                          Pv_out, D_out, X_out, dpatch_out, Dbar_out, bL_out);
}

/* orc_step_prec with FP64 network products. */
int orc_step(int nx, int ny, int K, int H, int Hm, double dt, double nu, unsigned dir,
             const double *cxy, const double *weights, const double *v, const double *p,
             double *h, double *uprev, int first,
             double *Pv_out, double *D_out, double *X_out, double *dpatch_out,
             double *Dbar_out, double *bL_out)
{
    return orc_step_prec(nx, ny, K, H, Hm, dt, nu, dir, cxy, weights, v, p, h, uprev, first, 0,
                         Pv_out, D_out, X_out, dpatch_out, Dbar_out, bL_out);
}
