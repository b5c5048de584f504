// Internal interfaces between the C ABI (api.cpp) and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dnnmg {

constexpr int kThreads = 256;     // every kernel: 4 wave64s per workgroup
constexpr int kTileFine = 32;     // defect tile: 32 x 32 fine elements
constexpr int kRhsFine = 32;      // averaging / rhs tile: 32 x 32 fine elements
constexpr int kNetRows = 64;      // GRU/MLP: patches per workgroup
constexpr int kMaxBatch = 256;    // flows per batched launch

// Per-flow arguments of one step.  Passed by value for a single flow, or read
// from a device table for a batch.
struct FlowArgs {
    int nx, ny;
    unsigned dirichlet;
    int xfmt;              // network input storage: 0 FP32, 1 BF16, 2 FP8 E4M3 with per-patch scales
    float inv_dt, nu;
    double inv_dt64;
    const float *v;        // (ny+1)(nx+1) x 2
    const float *p;        // (ny+1)(nx+1) or nullptr
    const float *geo;      // per coarse element: ex, ey, exy (2 floats each)
    const double *geo64;   // per coarse element: d0, d1, d2, (pad): det of the map
    const float *feat;     // P x 4
    int *first_flag;       // device: nonzero before the first step (then u_prev := P v)
    float *h;              // P x H
    float *uprev;          // (NY+1) rows of upitch nodes x 2 (the first NX+1 nodes of a row used)
    int upitch;            // nodes per u_prev row: NX+1 rounded up to 16 (128-byte rows)
    float *X;              // network input, the step writes it: P x nin FP32 or BF16, or for FP8
                           // P rows of xstride(nin) E4M3 codes (zero beyond nin)
    float *sx;             // FP8: per-patch scale of X
    float *dpatch;         // P x nout
    double *part;          // 4 x P x 2: per-patch rhs contribution, one plane per corner
    float *dbar_out;       // optional Fn x 2
    float *D;              // stage only: Fn x 2 defect at the fine nodes
    const float *dbar_in;  // stage: given fine correction (rhs/restrict alone)
    double *bL;            // restricted rhs output (gather)
    int *nonfinite;        // non-finite check (or nullptr): bit 0 correction, bit 1 restricted rhs
    // time scheme: theta = 1 implicit Euler, 1/2 Crank-Nicolson (then map64
    // holds the coarse maps in FP64 and nu64 the viscosity for the rhs)
    int xform = 0;                   // network input form (NetArgs::xform)
    const float *geo12 = nullptr;    // xform 1: per patch the twelve geometry inputs
    float theta = 1.0f;
    double nu64 = 0.0;
    const double *map64 = nullptr;   // per coarse element: ex, ey, exy (x, y each), 2 pad
    // one-launch K = 2 step (single flow): the tile frame it hands to the rhs
    // (frame.h; nullptr: it stores the per-patch outputs instead), and
    // whether it also stores them (keep_dpatch)
    float *frame = nullptr;
    int keep_dpatch = 1;
};

// Shared network description.
struct NetArgs {
    int K, H, Hm, nin, nout, prec;
    int kc1;               // k-chunks of phase 1 ([x | h])
    const void *B1;        // phase 1 fragments: gates z, r, h over [x | h]
    const void *B2;        // U_h fragments
    const void *B3;        // M1 (or M when Hm == 0)
    const void *B4;        // M2
    const float *s1, *s2, *s3, *s4;  // FP8: per-output-row weight scales
    int xform = 0;         // network input: 0 [P v, D, 4 features]; 1 the paper's (3 nf + 24, padded to nin)
    int reset_after = 0;   // GRU candidate tanh(W_h x + r * (U_h h)) instead of U_h (r * h)
};

// Moment tables for the FP64 right-hand side (exact integrals on the
// reference square; see rhs.hip).
struct RhsTables {
    const double *A;       // 2 x 2 x (n+1): A[m][p][a] = int_0^1 L_p(x) hat_a(x) x^m dx
    const double *M;       // 3 x 4 x 4    : int N_c N_c' {1, xi, eta} on the reference square
};

// Exact moment tables on the reference square (see rhs.hip), host and
// device (the allocation-free entry point forms them on the device):
//   int N_c phi_l m_k = A[mx_k][cx][a] A[my_k][cy][b]  (l = (a,b), c = (cx,cy)),
//   M[k][c][c'] = int N_c N_c' m_k,  m = {1, xi, eta}.
// Each factor is a 1D integral of a piecewise cubic, done with two Gauss
// points per fine interval (exact).  A: 2 x 2 x (n+1), M: 3 x 4 x 4.
__host__ __device__ constexpr int moment_a_size(int K) { return 4 * ((1 << K) + 1); }
constexpr int kMomentMSize = 3 * 4 * 4;
__host__ __device__ inline void fill_moment_tables(int K, double *A, double *M)
{
#pragma clang fp contract(off)   // plain products and sums: host and device round alike
    const int n = 1 << K;
    const double r = 0.28867513459481288225;   // 1 / (2 sqrt 3)
    const double gp[2] = {0.5 - r, 0.5 + r};
    for (int i = 0; i < moment_a_size(K); ++i) A[i] = 0.0;
    double C[2][2][2] = {};
    for (int iv = 0; iv < n; ++iv)
        for (int g = 0; g < 2; ++g) {
            const double x = (iv + gp[g]) / n, w = 0.5 / n;
            const double L[2] = {1.0 - x, x};
            for (int m = 0; m < 2; ++m)
                for (int p = 0; p < 2; ++p) {
                    const double xm = m ? x : 1.0;
                    for (int a = 0; a <= n; ++a) {
                        double hat = 1.0 - fabs(n * x - a);
                        hat = hat > 0.0 ? hat : 0.0;
                        A[(m * 2 + p) * (n + 1) + a] += w * L[p] * hat * xm;
                    }
                    for (int q = 0; q < 2; ++q) C[m][p][q] += w * L[p] * L[q] * xm;
                }
        }
    const int mx[3] = {0, 1, 0}, my[3] = {0, 0, 1};   // which direction carries xi / eta
    for (int k = 0; k < 3; ++k)
        for (int c = 0; c < 4; ++c) {
            const int cx = c & 1, cy = c >> 1;
            for (int cc = 0; cc < 4; ++cc)
                M[(k * 4 + c) * 4 + cc] = C[mx[k]][cx][cc & 1] * C[my[k]][cy][cc >> 1];
        }
}
// The same tables formed on the device (one thread), for callers without a
// context.
hipError_t launch_moment_tables(int K, double *A, double *M, hipStream_t s);

// Device table for batched launches: per kernel kind, a block prefix over
// flows, then the flows.
enum { kKindDefect = 0, kKindNet = 1, kKindRhs = 2, kKindGather = 3, kKinds = 4 };
struct BatchTable {
    int nflows;
    int pad[3];
    int prefix[kKinds][kMaxBatch + 1];
    FlowArgs flows[kMaxBatch];
};

// FP8 E4M3 operands.  Row stride (bytes) of the FP8 network input: nin
// rounded up to the 32-wide k-chunk, so the input and the state occupy
// separate chunks (they carry separate scales).
__host__ __device__ constexpr int xstride_fp8(int nin) { return (nin + 31) / 32 * 32; }
// Smallest row maximum a scale is computed from (keeps 448 / m finite).
constexpr float kFp8MinMax = 448.0f * 0x1p-64f;
// BF16 gate weights are packed pre-multiplied by -log2(e) (z, r) and
// 2 log2(e) (W_h, U_h): the kernels then form the GRU's exponentials as 2^x.
constexpr float kLog2e = 1.44269504088896340736f;


// Arguments of the unstructured-mesh step (umesh.hip).  Patch e is coarse
// element e (corners v0..v3 counter-clockwise, reference corners (0,0),
// (1,0), (1,1), (0,1)); its (n+1)^2 fine nodes, patch-local l = b (n+1) + a,
// are fine nodes pmap[e nf + l] at fine coordinates rel[...] relative to v0.
// node_ptr/node_occ: for each fine node the (patch nf + l) that hold it, in
// patch order; cnode_ptr/cnode_occ: for each coarse node the (patch 4 + corner).
struct UArgs {
    int K, P, Fn, Nc, nin, xfmt;
    float inv_dt, nu;
    double inv_dt64;
    const float *v, *p;              // coarse fields (Nc x 2, Nc)
    const int *corners;              // P x 4
    const int *pmap;                 // P x nf
    const float *rel;                // P x nf x 2 (FP32: fine coordinates relative to v0)
    const double *dgeo;              // P x 4: d0, d1, d2 of det J (straight patches: exact moments)
    const int *cidx;                 // P: row of W and M4 of a patch with a curved edge, or -1
    const double *W;                 // rows x 4 x nf: hat-weighted mass rows (curved patches)
    const double *M4;                // rows x 4 x 4: the same applied to P v (corner values)
    RhsTables tab;                   // the moment tables (straight patches)
    const float *feat;               // P x 4
    const unsigned char *mask;       // Fn: Dirichlet nodes
    const int *node_ptr, *node_occ;  // Fn + 1, P nf
    const int *cnode_ptr, *cnode_occ;// Nc + 1, 4 P
    int *first_flag;                 // nonzero before the first step (then u_prev := P v)
    float *uprev;                    // Fn x 2
    float *dloc;                     // P x nf x 2: each patch's element contributions to its nodes
    float *D;                        // Fn x 2: the assembled defect, then (step) the averaged correction
    void *X;                         // P x nin network input (FP32 or BF16)
    const float *dpatch;             // P x nout
    double *part;                    // P x 4 x 2: the patches' rhs shares at their corners
    double *bL;                      // Nc x 2
    float *dbar_out;                 // optional Fn x 2
    const float *dbar_in;            // stage: given correction
    float *pv_out, *pp_out;          // prolongation stage
    int *nonfinite;                  // non-finite check (or nullptr)
};

hipError_t launch_udefect(const UArgs &u, float *D_out, hipStream_t s);          // contributions, and D_out (if given)
hipError_t launch_uinput(const UArgs &u, hipStream_t s);                         // network input rows
hipError_t launch_uaverage(const UArgs &u, hipStream_t s);                       // averaging, state, correction
hipError_t launch_urhs(const UArgs &u, const float *dbar, hipStream_t s);       // FP64 rhs shares per patch
hipError_t launch_ugather(const UArgs &u, hipStream_t s);                        // b_L at the coarse nodes
hipError_t launch_uprolong(const UArgs &u, hipStream_t s);                       // P v, P p at the fine nodes

// Blocks each kernel kind needs for one flow.
int blocks_for(int kind, int nx, int ny, int K);

// Launchers (return hipError_t of the launch).
// map64 (or nullptr): the FP64 map vectors the Crank-Nicolson rhs needs;
// geo12 (or nullptr): the paper-form network's twelve geometry inputs.
hipError_t launch_geometry(const double *cxy, int nx, int ny, float *geo, double *geo64, double *map64,
                           float *feat, float *geo12, int *bad, hipStream_t s);
hipError_t launch_prolong(const FlowArgs &f, int K, float *pv, float *pp, hipStream_t s);
// f.theta != 1 (Crank-Nicolson) takes the theta-weighted element residuals;
// single flow only (bt must be null then).
hipError_t launch_defect(const FlowArgs &f, const BatchTable *bt, int nblocks, int K, int xfmt, hipStream_t s);
// Defect + GRU + MLP in one launch (K = 2, BF16 operands, H = 64, Hm 0 or 64):
// the network input never leaves LDS.  fused_step tells whether it applies.
bool fused_step(const NetArgs &net);
hipError_t launch_defect_net(const FlowArgs &f, const BatchTable *bt, int nblocks, const NetArgs &net, hipStream_t s);
// FP8 activation quantiser (stage entry point): rows x cols FP32 -> codes, scales.
hipError_t launch_quantize(const float *a, int rows, int cols, uint8_t *q, float *s, hipStream_t st);
hipError_t launch_net(const FlowArgs &f, const BatchTable *bt, int nblocks, const NetArgs &net,
                      hipStream_t s);
// Blocks of the network launch (persistent kernels use fewer than row tiles).
int net_blocks(const NetArgs &net, int row_tiles);
// f.theta != 1 adds the explicit transport term -(1 - theta) R T(u) (single flow).
hipError_t launch_rhs(const FlowArgs &f, const BatchTable *bt, int nblocks, int K,
                      const RhsTables &tab, int from_patches, hipStream_t s);
hipError_t launch_gather(const FlowArgs &f, const BatchTable *bt, int nblocks, hipStream_t s);

// Workgroups are handed to the chip's eight XCDs in turn (workgroup b to XCD
// b mod 8), and each XCD has its own L2.  Tile order for the kernels whose
// tiles read their neighbours' edge data: XCD x takes a contiguous run of the n
// tiles, so neighbouring tiles meet in one L2.  A bijection of [0, n), so any
// other dispatch order only costs locality.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    constexpr int X = 8;
    const int q = n / X, r = n % X, x = b % X;
    return x * q + min(x, r) + b / X;
}

// Find the flow and the flow-local block of a block of a batched launch.
__device__ inline const FlowArgs *batch_flow(const BatchTable *bt, int kind, int &blk)
{
    int lo = 0, hi = bt->nflows - 1;
    const int *pre = bt->prefix[kind];
    while (lo < hi) {                      // last flow with prefix <= blk
        int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= blk) lo = mid; else hi = mid - 1;
    }
    blk -= pre[lo];
    return &bt->flows[lo];
}

}  // namespace dnnmg
