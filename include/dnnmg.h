/*
 * dnnmg.h -- C ABI of the fine-level DNN-MG step on AMD Instinct MI355X (gfx950).
 *
 * The library performs, for one or many flows, the work that DNN-MG does in
 * place of fine-level multigrid at every time step (Margenberg, Hartmann,
 * Lessig, Richter, arXiv 2008.11520, the fine-level part of Algorithm 2; Sec. 4.1):
 *   1. prolongation of the coarse (level L) velocity and pressure to level L+K,
 *   2. element-wise assembly of the fine Navier-Stokes defect (momentum rows of
 *      the nonlinear residual of Eq. (nonlinearshort), implicit-Euler form),
 *   3. the per-patch GRU (Eq. (gru), no biases, Sec. 5.2) and MLP head that
 *      predict a velocity correction, averaged where patches share fine nodes
 *      (Sec. 4.2),
 *   4. the fine right-hand side (1/dt) M_f (P v + d) and its restriction
 *      R = P^T to level L, accumulated in FP64.
 * A patch is one coarse element (Sec. 5.2); n = 2^K fine elements per coarse
 * element and direction.
 *
 * Meshes are structured: coarse node (i,j), 0<=i<=nx, 0<=j<=ny has index
 * j*(nx+1)+i; fine node (I,J), 0<=I<=nx*n has index J*(nx*n+1)+I.  Vector
 * fields are interleaved (x,y) per node.  Coarse elements may be general
 * (positively oriented) quadrilaterals; fine levels come from uniform
 * bilinear refinement.
 *
 * Conventions for every entry point:
 *  - Ownership: the caller owns every pointer it passes; device pointers must
 *    stay valid until the work enqueued on the stream has completed.  The
 *    library owns the per-flow state (GRU hidden state h, previous corrected
 *    velocity), its workspace and the packed weights.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 *    stream).  Step calls only enqueue work: no host synchronisation and no
 *    device allocation happen after dnnmg_create.
 *  - Errors: arguments are validated on the host before anything is enqueued;
 *    on failure nothing is enqueued, the context is unchanged and a negative
 *    status is returned (the message is in dnnmg_last_error()).  Calls never
 *    abort.  A device error raised by enqueued work is reported as
 *    DNNMG_EDEVICE by the call that observes it.
 *  - Threads: a context must not be used from two threads at once;
 *    dnnmg_last_error() is per thread.
 */
#ifndef DNNMG_H
#define DNNMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dnnmg_ctx dnnmg_ctx;     /* one flow: mesh, state, workspace   */
typedef struct dnnmg_batch dnnmg_batch; /* descriptor table for batched steps */

enum {
    DNNMG_OK = 0,
    DNNMG_EINVAL = -1,       /* bad argument (NULL, out of range, size mismatch) */
    DNNMG_ENOMEM = -2,       /* device allocation failed (create only)           */
    DNNMG_EDEVICE = -3,      /* HIP runtime or kernel error                      */
    DNNMG_ESTATE = -4,       /* call out of order (e.g. restrict before a step)  */
    DNNMG_EUNSUPPORTED = -5  /* valid but not built (e.g. an H without kernels)  */
};

/* Operand precision of the GRU/MLP products (accumulation is always FP32;
 * prolongation and defect are FP32; rhs and restriction are FP64).
 * BF16: operands rounded to nearest even.  FP8_E4M3: OCP E4M3 operands, each
 * with one FP32 scale per row: weights per output row (at create), the
 * network input, the state h, r*h, h' and the MLP hidden layer per patch
 * (scale m / 448 with m the row's largest magnitude, floored at 448 * 2^-64;
 * codes round x * 448 / m to nearest even).  The network input and the state
 * carry separate scales in the gate products. */
enum { DNNMG_FP32 = 0, DNNMG_BF16 = 1, DNNMG_FP8_E4M3 = 2 };

/* Configuration flags.  DNNMG_F_UNFUSED: where the library would run the
 * defect, the network input, the GRU and the MLP as one launch (K = 2, BF16
 * operands, H = 64, Hm 0 or 64; the network input then stays on chip, and
 * the launch also averages the duplicate outputs at every fine node inside
 * its tile, so the per-patch outputs stay on chip too), run them as separate
 * launches through HBM buffers instead.  Both forms do the same arithmetic in
 * the same order, so their results are bitwise equal. */
enum { DNNMG_F_UNFUSED = 1 };

/* DNNMG_F_PATCH_OUTPUTS: the one-launch step also stores the per-patch
 * network outputs for dnnmg_patch_output (the other forms always store them:
 * their averaging reads them back).  Results are the same with or without it. */
enum { DNNMG_F_PATCH_OUTPUTS = 32 };

/* DNNMG_F_NANCHECK: the step's kernels also record whether any value of the
 * averaged correction d (bit DNNMG_NONFINITE_CORRECTION) or of the restricted
 * right-hand side b^L (bit DNNMG_NONFINITE_RHS, set by dnnmg_restrict_rhs and
 * the batched gather) was NaN or infinite, in a device flag of the context
 * that dnnmg_nonfinite reads.  Results are the same with or without it.
 * The state h is not watched: with an MLP hidden layer, max(0, s) maps a NaN
 * hidden value to zero (here and in the FP64 definition), so a non-finite
 * state can leave the correction finite. */
enum { DNNMG_F_NANCHECK = 2 };
enum { DNNMG_NONFINITE_CORRECTION = 1, DNNMG_NONFINITE_RHS = 2 };

/* DNNMG_F_CRANK_NICOLSON: the Crank-Nicolson time scheme of
 * Eq. (4cranknicholson3) (no body force) instead of implicit Euler.  With
 * T(w) = C(w) w + nu K w the convection and diffusion rows, the step's defect
 * becomes
 *   D = (1/dt) M (u_prev - P v) - (1/2) T(P v) - (1/2) T(u_prev) + B^T P p
 * and its right-hand side
 *   b^L = R [ (1/dt) M u_corr - (1/2) T(u_corr) ],  u_corr = P v + d,
 * the explicit term formed in FP64 like the mass term.  On the first step
 * u_prev = P v (as with implicit Euler).  Such contexts always run the
 * separate-launch form, step alone (dnnmg_step_batch rejects them) and use
 * the same weights and state layout; dnnmg_defect and dnnmg_rhs_restrict
 * follow the context's scheme, dnnmg_rhs_restrict_noalloc is implicit Euler. */
enum { DNNMG_F_CRANK_NICOLSON = 4 };

/* DNNMG_F_PAPER_NET: the network of the paper (Sec. 4.2, the architecture
 * figure, Sec. 5.2) instead of the workloads' MLP form.
 * Inputs per patch, 3 nf + 24 values (51 at K = 1, 99 at K = 2), nf = (n+1)^2:
 *   the residual of the prolongated solution at the patch's fine nodes,
 *   momentum rows (the defect D, x and y interleaved, x-fastest node order),
 *   then continuity rows -(div P v, xi) (without the pressure
 *   stabilisation); the coarse velocity at the corners 00, 10, 01, 11 (x, y);
 *   a Peclet number q |v| / nu per corner, q the square root of the patch
 *   area; twelve geometry values: edge lengths (bottom, right, top, left),
 *   ratios h0/h1, h2/h3, h0/h2, h1/h3, interior angles at 00, 10, 11, 01.
 * Head: y = M h' (nout x H), then two convolutional blocks of 4 filters with
 *   3 x 3 taps, each a convolution and its transpose with the same weights
 *   (zero padding 1): the vertex block on y as a 2 x nf image (component,
 *   node), the spatial block on each component's (n+1) x (n+1) node grid;
 *   the output is wf * (vertex + spatial), one weight per output entry.
 * Weights (float, in this order): W_z, W_r, W_h (H x (3 nf + 24) each),
 *   U_z, U_r, U_h (H x H), M (nout x H), the vertex block's 36 (filter,
 *   row offset -1..1, column offset -1..1), the spatial block's 36, wf (nout):
 *   8634 values at K = 1, H = 32.  The head is linear, so the library folds
 *   it into one nout x H matrix at create time (in FP64).
 * Requires Hm = 0, nu > 0 and FP32 or BF16 operands; such contexts step
 * alone (dnnmg_step_batch rejects them) and run the separate-launch form. */
enum { DNNMG_F_PAPER_NET = 8 };

/* DNNMG_F_GRU_RESET_AFTER: the GRU candidate tanh(W_h x + r * (U_h h)) (the
 * reset gate applied after U_h, as common library GRU cells do) instead of
 * tanh(W_h x + U_h (r * h)) of Eq. (gru).  FP32 or BF16 operands. */
enum { DNNMG_F_GRU_RESET_AFTER = 16 };

/* Dirichlet sides (Eq. (boundary)); other sides are do-nothing outflow. */
enum { DNNMG_DIR_XMIN = 1, DNNMG_DIR_XMAX = 2, DNNMG_DIR_YMIN = 4, DNNMG_DIR_YMAX = 8 };

typedef struct {
    int nx, ny;          /* coarse elements per direction, >= 1; patches = nx*ny    */
    int K;               /* levels bridged, 1..3; n = 2^K                           */
    int H;               /* GRU hidden size: 32, 64, 96 (FP32, BF16) or 128          */
    int Hm;              /* MLP hidden width: 0 (single linear H -> N_out), or a
                            multiple of 32 up to 256                                 */
    double dt;           /* time step (> 0)                                          */
    double nu;           /* viscosity (>= 0)                                         */
    int precision;       /* DNNMG_FP32 / DNNMG_BF16 / DNNMG_FP8_E4M3                 */
    unsigned dirichlet;  /* DNNMG_DIR_* bits                                         */
    unsigned flags;      /* 0, or DNNMG_F_UNFUSED | DNNMG_F_NANCHECK |
                            DNNMG_F_CRANK_NICOLSON | DNNMG_F_PAPER_NET |
                            DNNMG_F_GRU_RESET_AFTER | DNNMG_F_PATCH_OUTPUTS          */
} dnnmg_config;

/* Network sizes: N_in = 4 (n+1)^2 + 4 (prolongated velocity and defect at the
 * (n+1)^2 patch nodes, then hx, hy, hx/hy, area), N_out = 2 (n+1)^2.
 * Weight count = 3 H N_in + 3 H H + (Hm > 0 ? Hm H + N_out Hm : N_out H). */
size_t dnnmg_weight_count(const dnnmg_config *cfg);

/* Device bytes one context of this configuration allocates (state, workspace
 * and its own packed weights); 0 if cfg is invalid.  For admission control. */
size_t dnnmg_workspace_bytes(const dnnmg_config *cfg);

/* Create a flow.
 * coarse_xy_host: host, (ny+1)(nx+1) x 2 doubles, node-major, coordinates of
 *   the coarse nodes; every element must be positively oriented.
 * weights_host: host FP32, dnnmg_weight_count(cfg) values in the order
 *   W_z, W_r, W_h (H x N_in each), U_z, U_r, U_h (H x H each), then M1 (Hm x H)
 *   and M2 (N_out x Hm), or M (N_out x H) when Hm == 0; row-major (out x in),
 *   y = W x, no biases (Sec. 5.2).  Copied and packed (BF16, or FP8 E4M3 with
 *   one FP32 scale per output row) at create.
 * The GRU state starts at h = 0.  Allocates all device memory of the flow.
 * Enqueues uploads on `stream` and synchronises it before returning. */
int dnnmg_create(const dnnmg_config *cfg, const double *coarse_xy_host,
                 const float *weights_host, size_t n_weights,
                 void *stream, dnnmg_ctx **out);

/* Create a flow that shares the packed weights of `model` (same K, H, Hm and
 * precision required); flows created this way can be stepped together by
 * dnnmg_step_batch.  The shared weights live until the last user is destroyed. */
int dnnmg_create_shared(const dnnmg_config *cfg, const double *coarse_xy_host,
                        const dnnmg_ctx *model, void *stream, dnnmg_ctx **out);

/* One fine DNN-MG step (Alg. 2: prolongation, network correction, corrected
 * velocity).
 * v_coarse_dev: device, (ny+1)(nx+1) x 2 FP32 coarse velocity v_n^L.
 * p_coarse_dev: device, (ny+1)(nx+1) FP32 coarse pressure, or NULL (= 0).
 * d_fine_dev:   device, optional (NULL to skip), Fn x 2 FP32: the averaged,
 *   Dirichlet-masked correction d_n^{L+1} at the fine nodes.
 * Updates h and the stored corrected velocity P v + d, and prepares the
 * restricted right-hand side for dnnmg_restrict_rhs.  On the first step of a
 * context the previous corrected velocity is taken as P v of this step. */
int dnnmg_step(dnnmg_ctx *ctx, const float *v_coarse_dev, const float *p_coarse_dev,
               float *d_fine_dev, void *stream);

/* Restricted right-hand side of the most recent step (Alg. 2, restriction):
 * b_coarse_dev: device, (ny+1)(nx+1) x 2 doubles,
 *   b^L = P^T (1/dt) M_f (P v + d), accumulated in FP64 from the stored FP32
 *   corrected velocity P v + d (the state the next step reads; implicit
 *   Euler), or from P v and d (Crank-Nicolson).
 * DNNMG_ESTATE before the first step.  May be called more than once. */
int dnnmg_restrict_rhs(dnnmg_ctx *ctx, double *b_coarse_dev, void *stream);

/* Batched steps (serving form).  A batch object owns one device table of up to
 * max_flows flow descriptors and double-buffered pinned staging for it.  Use a
 * batch object from one stream only: table uploads and launches are ordered
 * on that stream. */
int dnnmg_batch_create(int max_flows, dnnmg_batch **out);
int dnnmg_batch_destroy(dnnmg_batch *b);

/* Describe the next step of nflows flows (all sharing one weight set, see
 * dnnmg_create_shared): v[f], p[f] (may be NULL) and d_out[f] (may be NULL) as
 * in dnnmg_step; d_out itself may be NULL.  b_out (may be NULL) gives each
 * flow's restricted rhs output, (ny+1)(nx+1) x 2 doubles, so that the batched
 * launch also performs the restriction.  Uploads the table with an async copy
 * from pinned memory (waiting, if needed, for the upload two calls back to
 * finish) and advances each context's step counter. */
int dnnmg_batch_prepare(dnnmg_batch *b, dnnmg_ctx *const *ctxs, int nflows,
                        const float *const *v, const float *const *p, float *const *d_out,
                        double *const *b_out, void *stream);

/* Launch the prepared step: one launch per kernel stage over all flows.  With
 * use_graph != 0 the launch sequence is captured into a hipGraph and replayed.
 * Its kernels read every per-flow argument and the tile counts from the device
 * table at run time: most stride over the listed tiles from a fixed grid; the
 * one-launch tiles (K = 2, BF16, H = 64) and the rhs after them take one tile
 * per block from a grid captured with room to spare (blocks past the tiles
 * return).  So one capture serves many memberships: the graph is captured
 * again when K, the precision, whether b_out is given, the weight set, or
 * whether every flow has the one-launch step's tile frame changes, or when a
 * membership has more one-launch tiles than the captured grid.  stream must
 * then be a non-default stream.  Results equal dnnmg_step on each context, bit
 * for bit.  DNNMG_ESTATE if nothing was prepared. */
int dnnmg_batch_launch(dnnmg_batch *b, int use_graph, void *stream);

/* Number of graph captures this batch object has made (-1 for NULL). */
int dnnmg_batch_captures(const dnnmg_batch *b);

/* dnnmg_batch_prepare (without b_out) followed by an eager dnnmg_batch_launch. */
int dnnmg_step_batch(dnnmg_batch *b, dnnmg_ctx *const *ctxs, int nflows,
                     const float *const *v, const float *const *p, float *const *d_out,
                     void *stream);

int dnnmg_destroy(dnnmg_ctx *ctx);

/* ------------------------------------------------ unstructured meshes
 * A coarse mesh of quadrilaterals with explicit connectivity (the paper's
 * meshes, Sec. 3.1 and the obstacle geometries of the numerical examples):
 * node coordinates, four nodes per element counter-clockwise (v0, v1, v2, v3
 * at the reference corners (0,0), (1,0), (1,1), (0,1)), the boundary edges
 * with Dirichlet values (node pairs; other boundary edges are do-nothing
 * outflow), circles (cx, cy, r) and the edges lying on them (node a, node b,
 * circle index; both nodes on the circle).  All arrays are host memory owned
 * by the caller.  Elements next to each other must be oriented alike; every
 * fine element must be positively oriented.
 * Refinement: each element into n x n fine elements (one patch per element).
 * Fine nodes on a curved edge lie on its arc (angle linear along the edge);
 * element interiors follow the transfinite (Gordon-Hall) map of the four edge
 * curves, so the fine mesh is the isoparametric refinement.  Fine node
 * numbering (d_fine_dev, the u_prev state):
 *   0 .. Nc-1                    the coarse nodes;
 *   Nc + k (n-1) + t - 1         the inner nodes of edge k, t = 1 .. n-1 from
 *                                its lower-numbered node; edges numbered in
 *                                order of first appearance over the elements,
 *                                local edges (v0,v1), (v1,v2), (v3,v2), (v0,v3);
 *   Nc + E (n-1) + e (n-1)^2 + (b-1)(n-1) + a - 1
 *                                the inner node (a, b) of element e.
 * The step is the structured one's (the fine part of Alg. 2; implicit Euler, the
 * workloads' network) with the mesh's own operators: P v at a fine node is the
 * bilinear interpolation, in the reference coordinates of the first element
 * that holds it, of that element's corner values; the defect and the mass
 * matrix are assembled over the fine elements (2 x 2 Gauss points on each
 * fine element's own bilinear map); a node's correction is the mean of the
 * outputs of every patch that holds it; R = P^T.  Patch-local node order and the
 * network input are those of the structured form, the features taken from
 * each element's four corners (hx the mean of edges (v0,v1), (v3,v2); hy of
 * (v0,v3), (v1,v2); hx / hy; the straight quadrilateral's area). */
typedef struct {
    int n_nodes, n_elems;
    const double *xy;              /* n_nodes x 2                                */
    const int *elems;              /* n_elems x 4                                */
    int n_dirichlet;
    const int *dirichlet_edges;    /* n_dirichlet x 2 (or NULL when 0)           */
    int n_circles;
    const double *circles;         /* n_circles x 3 (or NULL when 0)             */
    int n_curved;
    const int *curved_edges;       /* n_curved x 3 (or NULL when 0)              */
} dnnmg_umesh;

/* Edge and fine node counts of `mesh` refined K times (host only; validates
 * the mesh: DNNMG_EINVAL with the reason in dnnmg_last_error). */
int dnnmg_umesh_counts(const dnnmg_umesh *mesh, int K, int *n_edges, int *n_fine_nodes);

/* A flow on an unstructured mesh.  cfg supplies K, H, Hm, dt, nu, precision
 * (FP32 or BF16) and flags (DNNMG_F_NANCHECK, DNNMG_F_GRU_RESET_AFTER);
 * cfg->nx, ny and dirichlet are not used.  Weights as dnnmg_create.  The
 * context then takes dnnmg_step (v: n_nodes x 2, p: n_nodes, d: Fn x 2),
 * dnnmg_restrict_rhs (b: n_nodes x 2), dnnmg_prolong, dnnmg_defect,
 * dnnmg_rhs_restrict (fine arrays in the numbering above), dnnmg_get_state /
 * dnnmg_set_state (u_prev Fn x 2), dnnmg_patch_output, dnnmg_nonfinite and
 * the profiling calls; it steps alone (dnnmg_step_batch rejects it). */
int dnnmg_create_umesh(const dnnmg_config *cfg, const dnnmg_umesh *mesh, const float *weights_host,
                       size_t n_weights, void *stream, dnnmg_ctx **out);

/* ---------------------------------------------------------------------
 * Device arena (serving form: flows admitted and retired while others run).
 * One hipMalloc of `bytes` and a pinned staging ring of `staging_bytes` when
 * the arena is made; contexts made in it take their workspace from it (first
 * fit) and return it when destroyed, so dnnmg_create_in_arena and
 * dnnmg_destroy of such a context neither allocate, free nor synchronise a
 * stream (the coarse coordinates travel through the staging ring with an
 * asynchronous copy; the mesh orientation is checked on the host).  A freed
 * block is reused by later contexts, whose set-up is enqueued on their
 * creation stream: on one stream it follows the destroyed context's work;
 * across streams, wait for that work before destroying.  Not thread-safe.
 * ------------------------------------------------------------------- */
typedef struct dnnmg_arena dnnmg_arena;
int dnnmg_arena_create(size_t bytes, size_t staging_bytes, dnnmg_arena **out);
/* DNNMG_ESTATE while contexts still use the arena. */
int dnnmg_arena_destroy(dnnmg_arena *arena);
/* Bytes a context of this configuration takes from an arena (its weights
 * are the model's); 0 if cfg is invalid. */
size_t dnnmg_arena_block_bytes(const dnnmg_config *cfg);
/* Bytes in use, and the largest free block. */
int dnnmg_arena_usage(const dnnmg_arena *arena, size_t *used, size_t *largest_free);
/* Copy `bytes` from host memory to device memory through the arena's pinned
 * staging ring, asynchronously on `stream` (the host buffer may be reused at
 * once; nothing waits for the stream unless the ring is full).  DNNMG_EINVAL
 * if bytes exceed the ring. */
int dnnmg_arena_upload(dnnmg_arena *arena, void *dst_dev, const void *src_host, size_t bytes, void *stream);
/* dnnmg_create_shared with the workspace taken from `arena`.  DNNMG_ENOMEM if
 * no free block is large enough (nothing is changed); DNNMG_EINVAL for the
 * cases of dnnmg_create_shared, and if the coordinates exceed the staging
 * ring.  No host synchronisation. */
int dnnmg_create_in_arena(dnnmg_arena *arena, const dnnmg_config *cfg, const double *coarse_xy_host,
                          const dnnmg_ctx *model, void *stream, dnnmg_ctx **out);

/* Last error message of the calling thread ("" if none). */
const char *dnnmg_last_error(void);

/* ---------------------------------------------------------------------
 * Stage entry points: the same kernels as dnnmg_step, one stage at a time,
 * for per-output verification.  None of them changes the flow's state.
 * ------------------------------------------------------------------- */

/* Prolongation (Alg. 2, its first fine step): pv_out Fn x 2 and pp_out Fn (either may be
 * NULL) from the coarse v (and p, NULL = 0). */
int dnnmg_prolong(dnnmg_ctx *ctx, const float *v_coarse_dev, const float *p_coarse_dev,
                  float *pv_out_dev, float *pp_out_dev, void *stream);

/* Fine defect of P(v, p) against the stored previous corrected velocity
 * (P v itself before the first step), Dirichlet-masked: D_out Fn x 2 FP32. */
int dnnmg_defect(dnnmg_ctx *ctx, const float *v_coarse_dev, const float *p_coarse_dev,
                 float *D_out_dev, void *stream);

/* Right-hand side and restriction alone (Alg. 2, its last two steps) for a given fine
 * correction: b_out = P^T (1/dt) M_f (P v + dbar), FP64.  dbar_dev Fn x 2. */
int dnnmg_rhs_restrict(dnnmg_ctx *ctx, const float *v_coarse_dev, const float *dbar_dev,
                       double *b_out_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * dnnmg_rhs_restrict without a context.  b_out = P^T (1/dt) M_f (P v + dbar)
 * in FP64 for the structured nx x ny coarse mesh coarse_xy_dev (device,
 * (ny+1)(nx+1) x 2 doubles, positively oriented elements: not checked here),
 * with v_coarse_dev (ny+1)(nx+1) x 2 FP32, dbar_dev Fn x 2 FP32 and b_out_dev
 * (ny+1)(nx+1) x 2 doubles, all device pointers owned by the caller.  The
 * same kernels as dnnmg_rhs_restrict, and moment tables formed on the device
 * by the same formula as at create, so the same result bit for bit.
 * Allocates nothing: the kernels' scratch (map coefficients, FP64 corner
 * partial sums, moment tables) is one static device array of
 * dnnmg_noalloc_scratch_bytes() bytes (about 34 MiB) per GPU, held until the
 * process ends, which limits nx * ny to DNNMG_NOALLOC_MAX_PATCHES
 * (DNNMG_EINVAL beyond).  Every call on a GPU uses that GPU's one array:
 * calls that overlap on one GPU (other streams, other threads) race; calls
 * ordered on one stream do not.  Graph-capturable (kernel launches only). */
enum { DNNMG_NOALLOC_MAX_PATCHES = 1 << 18 };
size_t dnnmg_noalloc_scratch_bytes(void);
int dnnmg_rhs_restrict_noalloc(int nx, int ny, int K, double dt, const double *coarse_xy_dev,
                               const float *v_coarse_dev, const float *dbar_dev, double *b_out_dev,
                               void *stream);

/* Copy the state out (h: P x H FP32, uprev: Fn x 2 FP32; either may be NULL)
 * or in (then `steps` sets the step counter; 0 means "before the first step"). */
int dnnmg_get_state(dnnmg_ctx *ctx, float *h_out_dev, float *uprev_out_dev, void *stream);
int dnnmg_set_state(dnnmg_ctx *ctx, const float *h_in_dev, const float *uprev_in_dev,
                    long long steps, void *stream);

/* Non-finite check (DNNMG_F_NANCHECK; failure detection: a flow whose
 * correction or right-hand side has diverged is caught before the coarse
 * solver consumes it or its state is stepped again):
 * waits for the work enqueued on `stream` (a host synchronisation, so not for
 * use under graph capture), then stores in *flags_out the DNNMG_NONFINITE_*
 * bits recorded since the context was created or last cleared, and clears
 * them if `clear` is nonzero.  DNNMG_ESTATE if the context was created
 * without the flag; DNNMG_EINVAL for NULL arguments. */
int dnnmg_nonfinite(dnnmg_ctx *ctx, int clear, int *flags_out, void *stream);

/* Per-patch network output of the most recent step, before averaging:
 * d_out P x N_out FP32.  DNNMG_ESTATE before the first step, and after a
 * one-launch step of a context created without DNNMG_F_PATCH_OUTPUTS. */
int dnnmg_patch_output(dnnmg_ctx *ctx, float *d_out_dev, void *stream);

long long dnnmg_step_count(const dnnmg_ctx *ctx);

/* The FP8 form's activation quantiser alone (the rule under DNNMG_FP8_E4M3
 * above): a_dev rows x cols FP32, row-major, finite values -> q_dev rows x
 * cols E4M3 codes and scale_dev rows FP32 scales, so a ~ scale * value(q).
 * Device pointers, caller-owned.  DNNMG_EINVAL for NULL pointers or
 * rows, cols < 1. */
int dnnmg_quantize_e4m3(const float *a_dev, int rows, int cols, unsigned char *q_dev, float *scale_dev,
                        void *stream);

/* ---------------------------------------------------------------------
 * Kernel timing for benchmarks.  While enabled, dnnmg_step and
 * dnnmg_restrict_rhs record HIP events on their stream around each kernel
 * stage: 0 = prolongation + defect + network input, 1 = GRU + MLP,
 * 2 = averaging + FP64 rhs, 3 = restriction gather.  Up to max_steps steps
 * are recorded (later ones are not timed).  Enabling creates the events (no
 * device memory); max_steps = 0 disables and releases them.
 * dnnmg_profile_read waits for the recorded events and returns, per stage,
 * the summed milliseconds and the number of timed launches, then clears.
 * ------------------------------------------------------------------- */
enum { DNNMG_STAGES = 4 };
int dnnmg_profile_enable(dnnmg_ctx *ctx, int max_steps);
int dnnmg_profile_read(dnnmg_ctx *ctx, double *ms_per_stage, int *launches_per_stage);

#ifdef __cplusplus
}
#endif

#endif /* DNNMG_H */
