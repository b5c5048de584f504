// C ABI of the fine-level DNN-MG step (declared in include/dnnmg.h).
//
// Host side only: argument validation, device memory layout, weight packing
// into MFMA fragments, exact moment tables for the FP64 right-hand side, and
// kernel launches.  All per-step arithmetic runs in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "arena.h"
#include "dnnmg.h"
#include "frame.h"
#include "internal.h"
#include "umesh_build.h"

using namespace dnnmg;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_OR_FAIL(expr)                                                                       \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(DNNMG_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

extern "C" const char *dnnmg_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------- sizes
namespace {

struct Sizes {
    int n, nf, nin, nout, P, Fn, Nc;
    int nin_true;  // inputs per patch: 4 nf + 4, or 3 nf + 24 in the paper's form (nin pads it to 8)
    int upitch;   // nodes per row of the u_prev state: NX+1 rounded up to 16, so
                  // that rows (and the defect/rhs tiles' 32-node runs) start on
                  // 128-byte lines and tiles do not share lines of it
    size_t Fu;    // nodes of the u_prev state, (NY+1) upitch
};

Sizes sizes_of(const dnnmg_config &c)
{
    Sizes s;
    s.n = 1 << c.K;
    s.nf = (s.n + 1) * (s.n + 1);
    const bool paper = (c.flags & DNNMG_F_PAPER_NET) != 0u;
    s.nin_true = paper ? 3 * s.nf + 24 : 4 * s.nf + 4;
    s.nin = paper ? (s.nin_true + 7) / 8 * 8 : s.nin_true;
    s.nout = 2 * s.nf;
    s.P = c.nx * c.ny;
    s.Fn = (c.nx * s.n + 1) * (c.ny * s.n + 1);
    s.Nc = (c.nx + 1) * (c.ny + 1);
    s.upitch = (c.nx * s.n + 1 + 15) / 16 * 16;
    s.Fu = (size_t)s.upitch * (c.ny * s.n + 1);
    return s;
}

// Configuration flags that change the network (weights are shared only
// between contexts that agree on them).
constexpr unsigned kNetFlags = DNNMG_F_PAPER_NET | DNNMG_F_GRU_RESET_AFTER;

int kchunk(int prec) { return prec == DNNMG_FP32 ? 16 : 32; }
int kquad(int prec) { return prec == DNNMG_FP32 ? 4 : 8; }
int elem_bytes(int prec) { return prec == DNNMG_FP32 ? 4 : (prec == DNNMG_BF16 ? 2 : 1); }

int check_config(const dnnmg_config *c)
{
    if (!c) return fail(DNNMG_EINVAL, "config is NULL");
    if (c->nx < 1 || c->ny < 1) return fail(DNNMG_EINVAL, "nx, ny must be >= 1 (got %d, %d)", c->nx, c->ny);
    if (c->K < 1 || c->K > 3) return fail(DNNMG_EINVAL, "K must be 1, 2 or 3 (got %d)", c->K);
    if (!(c->dt > 0.0) || !std::isfinite(c->dt)) return fail(DNNMG_EINVAL, "dt must be > 0");
    if (!(c->nu >= 0.0) || !std::isfinite(c->nu)) return fail(DNNMG_EINVAL, "nu must be >= 0");
    if (c->precision < DNNMG_FP32 || c->precision > DNNMG_FP8_E4M3)
        return fail(DNNMG_EINVAL, "precision %d unknown", c->precision);
    if (c->dirichlet > 15u) return fail(DNNMG_EINVAL, "dirichlet flags 0x%x out of range", c->dirichlet);
    if ((c->flags & ~(unsigned)(DNNMG_F_UNFUSED | DNNMG_F_NANCHECK | DNNMG_F_CRANK_NICOLSON | DNNMG_F_PAPER_NET |
                                DNNMG_F_GRU_RESET_AFTER | DNNMG_F_PATCH_OUTPUTS)) != 0u)
        return fail(DNNMG_EINVAL, "unknown flags 0x%x", c->flags);
    if ((c->flags & (DNNMG_F_PAPER_NET | DNNMG_F_GRU_RESET_AFTER)) && c->precision == DNNMG_FP8_E4M3)
        return fail(DNNMG_EUNSUPPORTED, "DNNMG_F_PAPER_NET and DNNMG_F_GRU_RESET_AFTER run FP32 or BF16 operands");
    if ((c->flags & DNNMG_F_PAPER_NET) && c->Hm != 0)
        return fail(DNNMG_EINVAL, "the paper's network has no MLP hidden layer (Hm must be 0)");
    if ((c->flags & DNNMG_F_PAPER_NET) && !(c->nu > 0.0))
        return fail(DNNMG_EINVAL, "the paper's network input (Peclet numbers) needs nu > 0");
    if (c->H <= 0 || c->Hm < 0) return fail(DNNMG_EINVAL, "H must be > 0 and Hm >= 0");
    if (c->H != 32 && c->H != 64 && c->H != 96 && c->H != 128)
        return fail(DNNMG_EUNSUPPORTED, "H = %d has no kernels (32, 64, 96, 128)", c->H);
    if (c->H == 96 && c->precision == DNNMG_FP8_E4M3)
        return fail(DNNMG_EUNSUPPORTED, "H = 96 runs FP32 or BF16 operands");
    if (c->Hm != 0 && (c->Hm % 32 != 0 || c->Hm > 256))
        return fail(DNNMG_EUNSUPPORTED, "Hm = %d unsupported (0 or a multiple of 32 up to 256)", c->Hm);
    const double n = double(1 << c->K);
    const double fn = (c->nx * n + 1.0) * (c->ny * n + 1.0);
    if (fn > 2.0e9 || double(c->nx) * c->ny * (4.0 * (n + 1) * (n + 1) + 4) > 4.0e9)
        return fail(DNNMG_EINVAL, "mesh too large for one context");
    // a tile's rows of the state (35 rows of the padded fine row) are
    // addressed with 32-bit offsets
    if ((c->nx * n + 16.0) * 36.0 > 2.0e9)
        return fail(DNNMG_EINVAL, "mesh too wide for one context (nx * 2^K must stay below 5.5e7)");
    return DNNMG_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Device layout of one context's workspace.
struct Layout {
    size_t geo, geo64, map64, geo12, feat, h, uprev, X, sx, dpatch, frame, part, part2, cxy, flag, bad, nonfinite,
        total;
    size_t frame_bytes;
};

// Whether a structured context's single-flow step runs as one launch
// (defect, network input, GRU and MLP; then the duplicate averaging of the
// tile's inner nodes too, and the tile frame goes to the rhs kernel).
bool one_launch(const dnnmg_config &c)
{
    return c.K == 2 && c.H == 64 && (c.Hm == 0 || c.Hm == 64) && c.precision == DNNMG_BF16 &&
           !(c.flags & (DNNMG_F_UNFUSED | DNNMG_F_CRANK_NICOLSON | DNNMG_F_PAPER_NET | DNNMG_F_GRU_RESET_AFTER));
}

Layout layout_of(const dnnmg_config &c, bool structured = true)
{
    Sizes s = sizes_of(c);
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += align256(bytes); return r; };
    L.geo = take(sizeof(float) * 6 * s.P);
    L.geo64 = take(sizeof(double) * 4 * s.P);
    L.map64 = take((c.flags & DNNMG_F_CRANK_NICOLSON) ? sizeof(double) * 8 * s.P : 0);
    L.geo12 = take((c.flags & DNNMG_F_PAPER_NET) ? sizeof(float) * 12 * s.P : 0);
    L.feat = take(sizeof(float) * 4 * s.P);
    L.h = take(sizeof(float) * (size_t)s.P * c.H);
    L.uprev = take(sizeof(float) * 2 * s.Fu);
    if (c.precision == DNNMG_FP8_E4M3) {
        L.X = take((size_t)s.P * xstride_fp8(s.nin));
        L.sx = take(sizeof(float) * (size_t)s.P);
    } else {
        L.X = take((c.precision == DNNMG_BF16 ? 2 : 4) * (size_t)s.P * s.nin);
        L.sx = L.X;
    }
    L.dpatch = take(sizeof(float) * (size_t)s.P * s.nout);
    {
        typedef TileFrame<2> FR;
        const size_t tiles = (size_t)((c.nx + FR::TP - 1) / FR::TP) * ((c.ny + FR::TP - 1) / FR::TP);
        L.frame_bytes = structured && one_launch(c) ? sizeof(float) * 2 * FR::SIZE * tiles : 0;
        L.frame = take(L.frame_bytes);
    }
    L.part = take(sizeof(double) * 8 * (size_t)s.P);
    L.part2 = take(sizeof(double) * 8 * (size_t)s.P);
    L.cxy = take(sizeof(double) * 2 * (size_t)s.Nc);
    L.flag = take(sizeof(int));
    L.bad = take(sizeof(int));
    L.nonfinite = take(sizeof(int));
    L.total = o;
    return L;
}

// -------------------------------------------------------- weight packing
// Fragment layout: [tile ot][chunk kc][lane][e], value M[j][k] with
// j = 16 ot + lane % 16, k = kc KC + (lane / 16) KQ + e (zero outside).
uint16_t bf16_rne(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// OCP FP8 E4M3 code of x, round to nearest even on the bit pattern;
// magnitudes above 448 saturate.
uint8_t e4m3_rne(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    const uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
    const uint32_t a = u & 0x7fffffffu;
    if (a > 0x7f800000u) return sign | 0x7f;              // NaN
    if (a >= 0x43e00000u) return sign | 0x7e;             // >= 448
    int e = (int)(a >> 23) - 127;
    if (e < -6) {                                         // E4M3 subnormal: multiples of 2^-9
        const float t = std::fabs(x) * 512.0f;            // exact
        return sign | (uint8_t)std::nearbyint(t);         // ties to even (default rounding mode)
    }
    uint32_t keep = (a >> 20) & 7u;
    const uint32_t rest = a & 0xfffffu;
    if (rest > 0x80000u || (rest == 0x80000u && (keep & 1u))) ++keep;
    if (keep == 8u) { keep = 0; ++e; }
    if (e > 8 || (e == 8 && keep > 6u)) return sign | 0x7e;
    return sign | (uint8_t)(((e + 7) << 3) | (int)keep);
}

// Per-row FP8 scale of a weight row: m = max(max |w|, floor), codes of
// w * (448 / m), scale m / 448 (all in FP32, as for the activations).
void fp8_rows(std::vector<float> &M, int rows, int cols, std::vector<float> &scale)
{
    scale.assign(rows, 1.0f);
    for (int j = 0; j < rows; ++j) {
        float m = kFp8MinMax;
        for (int k = 0; k < cols; ++k) m = std::max(m, std::fabs(M[(size_t)j * cols + k]));
        const float r = 448.0f / m;
        scale[j] = m / 448.0f;
        for (int k = 0; k < cols; ++k) M[(size_t)j * cols + k] *= r;
    }
}

void pack_matrix(std::vector<unsigned char> &out, const std::vector<float> &M, int rows, int cols, int tiles,
                 int chunks, int prec)
{
    const int KC = kchunk(prec), KQ = kquad(prec), eb = elem_bytes(prec);
    size_t base = out.size();
    out.resize(base + (size_t)tiles * chunks * 64 * KQ * eb, 0);
    for (int ot = 0; ot < tiles; ++ot)
        for (int kc = 0; kc < chunks; ++kc)
            for (int lane = 0; lane < 64; ++lane)
                for (int e = 0; e < KQ; ++e) {
                    int j = 16 * ot + lane % 16, k = kc * KC + (lane / 16) * KQ + e;
                    float v = (j < rows && k < cols) ? M[(size_t)j * cols + k] : 0.0f;
                    size_t idx = base + ((((size_t)ot * chunks + kc) * 64 + lane) * KQ + e) * eb;
                    if (prec == DNNMG_FP32) std::memcpy(&out[idx], &v, 4);
                    else if (prec == DNNMG_FP8_E4M3) out[idx] = e4m3_rne(v);   // v already scaled
                    else { uint16_t b = bf16_rne(v); std::memcpy(&out[idx], &b, 2); }
                }
}

}  // namespace

// Shared, reference-counted packed weights.
struct Weights {
    std::atomic<int> refs{1};
    void *dev = nullptr;
    size_t bytes = 0;
    int K = 0, H = 0, Hm = 0, prec = 0;
    unsigned netflags = 0;   // the configuration flags that shape the network (kNetFlags)
    NetArgs net{};
    RhsTables tab{};       // moment tables (depend on K only), inside dev
};

// Event ring for per-stage kernel timing (benchmarks only).
struct Profile {
    int max_steps = 0;
    std::vector<hipEvent_t> ev;        // per step: 4 events (defect start .. rhs end)
    std::vector<hipEvent_t> evg;       // per restrict call: 2 events
    int steps = 0, gathers = 0;
};
static void profile_release(Profile &pr);

struct dnnmg_arena;

// The refined unstructured mesh on the device (contexts made by
// dnnmg_create_umesh): one allocation holding the gather lists, patch maps,
// fine coordinates and the per-fine-node buffers.
struct UMeshDev {
    int nc = 0, ne = 0, E = 0, Fn = 0;
    unsigned char *dev = nullptr;
    int *corners = nullptr, *pmap = nullptr, *node_ptr = nullptr, *node_occ = nullptr;
    int *cnode_ptr = nullptr, *cnode_occ = nullptr;
    float *rel = nullptr;
    double *dgeo = nullptr, *W = nullptr, *M4 = nullptr;
    int *cidx = nullptr;
    float *feat = nullptr, *uprev = nullptr, *dloc = nullptr, *D = nullptr;
    unsigned char *mask = nullptr;
};

struct dnnmg_ctx {
    dnnmg_config cfg;
    Profile prof;
    Sizes s;
    Layout L;
    unsigned char *ws = nullptr;
    Weights *w = nullptr;
    long long steps = 0;
    bool dpatch_kept = true;        // the last step stored its per-patch outputs
    int device = 0;
    dnnmg_arena *arena = nullptr;   // the workspace is a block of this arena (not hipMalloc'd)
    UMeshDev *um = nullptr;         // unstructured mesh (dnnmg_create_umesh), else structured

    float *geo() const { return (float *)(ws + L.geo); }
    double *geo64() const { return (double *)(ws + L.geo64); }
    double *map64() const { return (cfg.flags & DNNMG_F_CRANK_NICOLSON) ? (double *)(ws + L.map64) : nullptr; }
    float *geo12() const { return (cfg.flags & DNNMG_F_PAPER_NET) ? (float *)(ws + L.geo12) : nullptr; }
    float *feat() const { return (float *)(ws + L.feat); }
    float *h() const { return (float *)(ws + L.h); }
    float *uprev() const { return (float *)(ws + L.uprev); }
    float *X() const { return (float *)(ws + L.X); }
    float *sx() const { return cfg.precision == DNNMG_FP8_E4M3 ? (float *)(ws + L.sx) : nullptr; }
    float *dpatch() const { return (float *)(ws + L.dpatch); }
    float *frame() const { return L.frame_bytes ? (float *)(ws + L.frame) : nullptr; }
    double *part() const { return (double *)(ws + L.part); }
    int *first_flag() const { return (int *)(ws + L.flag); }
    RhsTables tables() const { return w->tab; }
};

struct dnnmg_batch {
    int max_flows = 0;
    BatchTable *dev = nullptr;                  // the one device table every launch reads
    BatchTable *host[2] = {nullptr, nullptr};   // pinned staging, double-buffered
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool used[2] = {false, false};
    int slot = 0;
    // what the last prepare uploaded
    bool prepared = false;
    int nflows = 0, K = 0, xfmt = 0, gather = 0;
    int frame = 0;                              // the one-launch tiles hand over in their tile frames
    int totals[kKinds] = {0, 0, 0, 0};
    NetArgs net{};
    RhsTables tab{};
    int cap = 0;                                // grid of every batched launch in a graph
    // grid of the one-tile-per-block launches (the one-launch tiles and the
    // rhs after them) in the captured graph: at least their tiles, grown
    // (and the graph captured again) when a membership has more
    int tile_grid = 0;
    // captured launch sequence.  Every per-flow argument and the tile counts
    // are read from `dev` at run time, so a graph stays valid while K, the X
    // type, the gather and the shared weight set are unchanged, whichever
    // flows fill the table.
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_K = -1, graph_xfmt = -1, graph_gather = -1, graph_frame = -1;
    NetArgs graph_net{};
    RhsTables graph_tab{};
    int captures = 0;
};

namespace {

size_t weight_count(const dnnmg_config &c)
{
    Sizes s = sizes_of(c);
    if (c.flags & DNNMG_F_PAPER_NET)   // GRU, FC, two convolutional blocks of 36, the last layer
        return 3 * (size_t)c.H * (s.nin_true + c.H) + (size_t)s.nout * c.H + 36 + 36 + s.nout;
    size_t n = 3 * (size_t)c.H * s.nin + 3 * (size_t)c.H * c.H;
    n += c.Hm > 0 ? (size_t)c.Hm * c.H + (size_t)s.nout * c.Hm : (size_t)s.nout * c.H;
    return n;
}

void moment_tables(int K, std::vector<double> &A1, std::vector<double> &M);

// B = sum_f C_f^T C_f for a block of 4 filters of 3 x 3 taps (W[f][dr][dc],
// offsets -1..1) on a rows x cols image (row-major, zero padding): C_f is the
// convolution, its transpose the block's second layer.  Dense, FP64.
std::vector<double> conv_block_matrix(int rows, int cols, const float *W)
{
    const int m = rows * cols;
    std::vector<double> C((size_t)m * m), B((size_t)m * m, 0.0);
    for (int f = 0; f < 4; ++f) {
        std::fill(C.begin(), C.end(), 0.0);
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c)
                for (int dr = -1; dr <= 1; ++dr)
                    for (int dc = -1; dc <= 1; ++dc) {
                        const int rr = r + dr, cc = c + dc;
                        if (rr < 0 || rr >= rows || cc < 0 || cc >= cols) continue;
                        C[(size_t)(r * cols + c) * m + rr * cols + cc] += W[9 * f + 3 * (dr + 1) + (dc + 1)];
                    }
        for (int i = 0; i < m; ++i)
            for (int k = 0; k < m; ++k) {
                const double cki = C[(size_t)k * m + i];
                if (cki == 0.0) continue;
                for (int j = 0; j < m; ++j) B[(size_t)i * m + j] += cki * C[(size_t)k * m + j];
            }
    }
    return B;
}

// The paper's network weights (W_g: H x nin_true, U_g, M: nout x H, the
// vertex and spatial convolution blocks, the last layer's nout weights) in
// the standard layout: W_g padded with zero columns to nin, and the head,
// which is linear (a dense layer, two blocks W^T W, the weighted sum), folded
// into one nout x H matrix  diag(wf) (B_vertex + B_spatial) M  in FP64.  The
// vertex block acts on the 2 x nf image (component, node), the spatial block
// on each component's (n+1) x (n+1) node grid.
std::vector<float> fold_paper_weights(const dnnmg_config &c, const float *w)
{
    const Sizes s = sizes_of(c);
    const int H = c.H, nt = s.nin_true, nin = s.nin, nout = s.nout, nf = s.nf, n1 = s.n + 1;
    std::vector<float> out((size_t)3 * H * nin + 3 * (size_t)H * H + (size_t)nout * H, 0.0f);
    for (int g = 0; g < 3; ++g)
        for (int j = 0; j < H; ++j)
            for (int k = 0; k < nt; ++k)
                out[((size_t)g * H + j) * nin + k] = w[((size_t)g * H + j) * nt + k];
    const float *U = w + 3 * (size_t)H * nt;
    std::copy(U, U + 3 * (size_t)H * H, out.begin() + 3 * (size_t)H * nin);
    const float *M = U + 3 * (size_t)H * H, *WV = M + (size_t)nout * H, *WS = WV + 36, *wf = WS + 36;
    // block operators on the output vector y (entry 2 l + comp)
    std::vector<double> B((size_t)nout * nout, 0.0);
    const std::vector<double> BV = conv_block_matrix(2, nf, WV);   // image index comp * nf + l
    for (int ci = 0; ci < 2; ++ci)
        for (int li = 0; li < nf; ++li)
            for (int cj = 0; cj < 2; ++cj)
                for (int lj = 0; lj < nf; ++lj)
                    B[(size_t)(2 * li + ci) * nout + 2 * lj + cj] += BV[(size_t)(ci * nf + li) * 2 * nf + cj * nf + lj];
    const std::vector<double> BS = conv_block_matrix(n1, n1, WS);  // image index l
    for (int comp = 0; comp < 2; ++comp)
        for (int li = 0; li < nf; ++li)
            for (int lj = 0; lj < nf; ++lj)
                B[(size_t)(2 * li + comp) * nout + 2 * lj + comp] += BS[(size_t)li * nf + lj];
    float *Mf = out.data() + 3 * (size_t)H * nin + 3 * (size_t)H * H;
    for (int o = 0; o < nout; ++o)
        for (int m = 0; m < H; ++m) {
            double acc = 0.0;
            for (int i = 0; i < nout; ++i) acc += B[(size_t)o * nout + i] * (double)M[(size_t)i * H + m];
            Mf[(size_t)o * H + m] = (float)((double)wf[o] * acc);
        }
    return out;
}

// Pack host FP32 weights into the four fragment arrays the network kernel reads.
int build_weights(const dnnmg_config &c, const float *w, hipStream_t st, Weights **out)
{
    std::vector<float> folded;
    if (c.flags & DNNMG_F_PAPER_NET) {
        folded = fold_paper_weights(c, w);
        w = folded.data();
    }
    Sizes s = sizes_of(c);
    const int H = c.H, Hm = c.Hm, prec = c.precision, KC = kchunk(prec);
    const int nin = s.nin, nout = s.nout, HT = H / 16;
    const bool fp8 = prec == DNNMG_FP8_E4M3;
    // phase-1 columns: [x | h]; FP8 pads the input to whole k-chunks so that
    // the input and the state (separately scaled) never share a chunk
    const int xw = fp8 ? xstride_fp8(nin) : nin;
    const int kc1 = (xw + H + KC - 1) / KC;
    const float *Wg[3] = {w, w + (size_t)H * nin, w + 2 * (size_t)H * nin};
    const float *Ug[3] = {w + 3 * (size_t)H * nin, w + 3 * (size_t)H * nin + (size_t)H * H,
                          w + 3 * (size_t)H * nin + 2 * (size_t)H * H};
    const float *M1 = w + 3 * (size_t)H * nin + 3 * (size_t)H * H;
    const float *M2 = Hm > 0 ? M1 + (size_t)Hm * H : nullptr;

    std::vector<unsigned char> buf;
    std::vector<float> scales[4], sc;          // FP8: per-output-row weight scales
    // FP8 matrices are scaled per row before packing
    auto pack = [&](std::vector<float> A, int rows, int cols, int tiles, int chunks, int which) {
        if (fp8) {
            fp8_rows(A, rows, cols, sc);
            scales[which].insert(scales[which].end(), sc.begin(), sc.end());
        }
        pack_matrix(buf, A, rows, cols, tiles, chunks, prec);
    };
    // BF16: gate rows pre-multiplied by -log2(e) (z, r) and 2 log2(e) (the
    // candidate's W_h and U_h), so that the kernels' exponentials are 2^x
    const bool l2 = prec == DNNMG_BF16;
    const float gs[3] = {l2 ? -kLog2e : 1.0f, l2 ? -kLog2e : 1.0f, l2 ? 2.0f * kLog2e : 1.0f};
    size_t off[4];
    off[0] = 0;
    for (int g = 0; g < 3; ++g) {   // [W_g | U_g], the U_h block is applied in phase 2
        std::vector<float> A((size_t)H * (xw + H), 0.0f);
        for (int j = 0; j < H; ++j) {
            for (int k = 0; k < nin; ++k) A[(size_t)j * (xw + H) + k] = gs[g] * Wg[g][(size_t)j * nin + k];
            if (g < 2)
                for (int k = 0; k < H; ++k) A[(size_t)j * (xw + H) + xw + k] = gs[g] * Ug[g][(size_t)j * H + k];
        }
        pack(A, H, xw + H, HT, kc1, 0);
    }
    buf.resize(align256(buf.size()));
    off[1] = buf.size();
    {
        std::vector<float> Uh(Ug[2], Ug[2] + (size_t)H * H);
        for (float &x : Uh) x *= gs[2];
        pack(Uh, H, H, HT, H / KC, 1);
    }
    buf.resize(align256(buf.size()));
    off[2] = buf.size();
    if (Hm > 0) {
        pack(std::vector<float>(M1, M1 + (size_t)Hm * H), Hm, H, Hm / 16, H / KC, 2);
        buf.resize(align256(buf.size()));
        off[3] = buf.size();
        pack(std::vector<float>(M2, M2 + (size_t)nout * Hm), nout, Hm, (nout + 15) / 16, Hm / KC, 3);
    } else {
        pack(std::vector<float>(M1, M1 + (size_t)nout * H), nout, H, (nout + 15) / 16, H / KC, 2);
        buf.resize(align256(buf.size()));
        off[3] = buf.size();
    }
    size_t offS[4] = {0, 0, 0, 0};
    for (int i = 0; i < 4 && fp8; ++i) {
        buf.resize(align256(buf.size()));
        offS[i] = buf.size();
        buf.resize(offS[i] + align256(sizeof(float) * std::max<size_t>(scales[i].size(), 1)));
        if (!scales[i].empty()) std::memcpy(&buf[offS[i]], scales[i].data(), sizeof(float) * scales[i].size());
    }
    // moment tables of the FP64 right-hand side, shared by every flow of the model
    std::vector<double> A1, Mt;
    moment_tables(c.K, A1, Mt);
    buf.resize(align256(buf.size()));
    const size_t offA = buf.size();
    buf.resize(offA + align256(sizeof(double) * A1.size()));
    std::memcpy(&buf[offA], A1.data(), sizeof(double) * A1.size());
    const size_t offM = buf.size();
    buf.resize(offM + align256(sizeof(double) * Mt.size()));
    std::memcpy(&buf[offM], Mt.data(), sizeof(double) * Mt.size());
    buf.resize(align256(buf.size()) + 256);

    Weights *W = new Weights();
    W->bytes = buf.size();
    if (hipMalloc(&W->dev, W->bytes) != hipSuccess) {
        delete W;
        (void)hipGetLastError();
        return fail(DNNMG_ENOMEM, "hipMalloc of %zu weight bytes failed", buf.size());
    }
    hipError_t e = hipMemcpyAsync(W->dev, buf.data(), buf.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(W->dev);
        delete W;
        return fail(DNNMG_EDEVICE, "weight upload: %s", hipGetErrorString(e));
    }
    W->K = c.K; W->H = H; W->Hm = Hm; W->prec = prec;
    W->netflags = c.flags & kNetFlags;
    unsigned char *d = (unsigned char *)W->dev;
    W->net = NetArgs{c.K, H, Hm, nin, nout, prec, kc1, d + off[0], d + off[1], d + off[2], d + off[3],
                     nullptr, nullptr, nullptr, nullptr};
    W->net.xform = (c.flags & DNNMG_F_PAPER_NET) ? 1 : 0;
    W->net.reset_after = (c.flags & DNNMG_F_GRU_RESET_AFTER) ? 1 : 0;
    if (fp8) {
        W->net.s1 = (const float *)(d + offS[0]);
        W->net.s2 = (const float *)(d + offS[1]);
        W->net.s3 = (const float *)(d + offS[2]);
        W->net.s4 = (const float *)(d + offS[3]);
    }
    W->tab = RhsTables{(const double *)(d + offA), (const double *)(d + offM)};
    *out = W;
    return DNNMG_OK;
}

size_t weight_bytes_estimate(const dnnmg_config &c)
{
    Sizes s = sizes_of(c);
    const int KC = kchunk(c.precision), KQ = kquad(c.precision), eb = elem_bytes(c.precision);
    auto frag = [&](int rows, int cols) {
        return align256((size_t)((rows + 15) / 16) * ((cols + KC - 1) / KC) * 64 * KQ * eb);
    };
    const bool fp8 = c.precision == DNNMG_FP8_E4M3;
    const int xw = fp8 ? xstride_fp8(s.nin) : s.nin;
    size_t b = 3 * (size_t)((c.H / 16) * ((xw + c.H + KC - 1) / KC) * 64 * KQ * eb);
    b = align256(b) + frag(c.H, c.H);
    b += c.Hm > 0 ? frag(c.Hm, c.H) + frag(s.nout, c.Hm) : frag(s.nout, c.H);
    if (fp8)
        b += align256(sizeof(float) * 3 * c.H) + align256(sizeof(float) * c.H) +
             align256(sizeof(float) * (c.Hm > 0 ? c.Hm : s.nout)) + align256(sizeof(float) * (c.Hm > 0 ? s.nout : 1));
    b = align256(b) + align256(sizeof(double) * 4 * (s.n + 1)) + align256(sizeof(double) * 48);
    return b + 256;
}

void release_weights(Weights *w)
{
    if (w && --w->refs == 0) {
        (void)hipFree(w->dev);
        delete w;
    }
}

void moment_tables(int K, std::vector<double> &A1, std::vector<double> &M)
{
    A1.assign(moment_a_size(K), 0.0);
    M.assign(kMomentMSize, 0.0);
    fill_moment_tables(K, A1.data(), M.data());
}

FlowArgs flow_args(const dnnmg_ctx *c, const float *v, const float *p)
{
    FlowArgs f{};
    f.nx = c->cfg.nx;
    f.ny = c->cfg.ny;
    f.dirichlet = c->cfg.dirichlet;
    f.first_flag = c->first_flag();
    f.inv_dt = (float)(1.0 / c->cfg.dt);
    f.nu = (float)c->cfg.nu;
    f.inv_dt64 = 1.0 / c->cfg.dt;
    f.v = v;
    f.p = p;
    f.geo = c->geo();
    f.geo64 = c->geo64();
    f.feat = c->feat();
    f.h = c->h();
    f.uprev = c->uprev();
    f.upitch = c->s.upitch;
    f.X = c->X();
    f.xfmt = c->cfg.precision;
    f.sx = c->sx();
    f.dpatch = c->dpatch();
    f.part = c->part();
    f.nonfinite = (c->cfg.flags & DNNMG_F_NANCHECK) ? (int *)(c->ws + c->L.nonfinite) : nullptr;
    if (c->cfg.flags & DNNMG_F_PAPER_NET) {
        f.xform = 1;
        f.geo12 = c->geo12();
    }
    if (c->cfg.flags & DNNMG_F_CRANK_NICOLSON) {
        f.theta = 0.5f;
        f.nu64 = c->cfg.nu;
        f.map64 = c->map64();
    }
    return f;
}

int create_common(const dnnmg_config *cfg, const double *cxy, const float *weights, size_t nw, Weights *shared,
                  void *stream, dnnmg_ctx **out)
{
    if (!out) return fail(DNNMG_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_config(cfg);
    if (rc) return rc;
    if (!cxy) return fail(DNNMG_EINVAL, "coarse_xy_host is NULL");
    for (size_t i = 0; i < 2 * (size_t)(cfg->nx + 1) * (cfg->ny + 1); ++i)
        if (!std::isfinite(cxy[i])) return fail(DNNMG_EINVAL, "coarse_xy_host[%zu] is not finite", i);
    if (!shared) {
        if (!weights) return fail(DNNMG_EINVAL, "weights_host is NULL");
        if (nw != weight_count(*cfg))
            return fail(DNNMG_EINVAL, "n_weights = %zu, expected %zu", nw, weight_count(*cfg));
    } else if (shared->K != cfg->K || shared->H != cfg->H || shared->Hm != cfg->Hm || shared->prec != cfg->precision ||
               shared->netflags != (cfg->flags & kNetFlags)) {
        return fail(DNNMG_EINVAL, "shared weights have another K/H/Hm/precision/network form");
    }
    hipStream_t st = (hipStream_t)stream;
    dnnmg_ctx *c = new dnnmg_ctx();
    c->cfg = *cfg;
    c->s = sizes_of(*cfg);
    c->L = layout_of(*cfg);
    (void)hipGetDevice(&c->device);
    if (hipMalloc((void **)&c->ws, c->L.total) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return fail(DNNMG_ENOMEM, "hipMalloc of %zu workspace bytes failed", c->L.total);
    }
    auto bail = [&](int code) {
        (void)hipFree(c->ws);
        if (c->w) release_weights(c->w);
        delete c;
        return code;
    };
    if (shared) {
        ++shared->refs;
        c->w = shared;
    } else {
        rc = build_weights(*cfg, weights, st, &c->w);
        if (rc) { c->w = nullptr; return bail(rc); }
    }
    const Sizes &s = c->s;
    hipError_t e = hipMemcpyAsync(c->ws + c->L.cxy, cxy, sizeof(double) * 2 * s.Nc, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(c->h(), 0, sizeof(float) * (size_t)s.P * cfg->H, st);
    if (e == hipSuccess) e = hipMemsetAsync(c->uprev(), 0, sizeof(float) * 2 * s.Fu, st);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + c->L.bad, 0, sizeof(int), st);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + c->L.nonfinite, 0, sizeof(int), st);
    if (e == hipSuccess) e = hipMemsetAsync(c->first_flag(), 1, sizeof(int), st);
    if (e == hipSuccess)
        e = launch_geometry((const double *)(c->ws + c->L.cxy), cfg->nx, cfg->ny, c->geo(), c->geo64(), c->map64(),
                            c->feat(), c->geo12(), (int *)(c->ws + c->L.bad), st);
    int bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, c->ws + c->L.bad, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bail(fail(DNNMG_EDEVICE, "create: %s", hipGetErrorString(e)));
    if (bad) return bail(fail(DNNMG_EINVAL, "coarse mesh has an element that is not positively oriented"));
    *out = c;
    return DNNMG_OK;
}

int check_ctx(const dnnmg_ctx *c)
{
    if (!c) return fail(DNNMG_EINVAL, "ctx is NULL");
    return DNNMG_OK;
}

// ----------------------------------------------------- unstructured meshes
UArgs uargs(const dnnmg_ctx *c, const float *v, const float *p)
{
    const UMeshDev &m = *c->um;
    UArgs u{};
    u.K = c->cfg.K;
    u.P = m.ne;
    u.Fn = m.Fn;
    u.Nc = m.nc;
    u.nin = c->s.nin;
    u.xfmt = c->cfg.precision;
    u.inv_dt = (float)(1.0 / c->cfg.dt);
    u.nu = (float)c->cfg.nu;
    u.inv_dt64 = 1.0 / c->cfg.dt;
    u.v = v;
    u.p = p;
    u.corners = m.corners;
    u.pmap = m.pmap;
    u.rel = m.rel;
    u.dgeo = m.dgeo;
    u.cidx = m.cidx;
    u.W = m.W;
    u.M4 = m.M4;
    u.tab = c->tables();
    u.feat = m.feat;
    u.mask = m.mask;
    u.node_ptr = m.node_ptr;
    u.node_occ = m.node_occ;
    u.cnode_ptr = m.cnode_ptr;
    u.cnode_occ = m.cnode_occ;
    u.first_flag = c->first_flag();
    u.uprev = m.uprev;
    u.dloc = m.dloc;
    u.D = m.D;
    u.X = c->X();
    u.dpatch = c->dpatch();
    u.part = c->part();
    u.nonfinite = (c->cfg.flags & DNNMG_F_NANCHECK) ? (int *)(c->ws + c->L.nonfinite) : nullptr;
    return u;
}

// The network launch of an unstructured context: its patches as one row of
// ne elements.
FlowArgs unet_args(const dnnmg_ctx *c)
{
    FlowArgs f{};
    f.nx = c->um->ne;
    f.ny = 1;
    f.h = c->h();
    f.X = c->X();
    f.xfmt = c->cfg.precision;
    f.dpatch = c->dpatch();
    return f;
}

}  // namespace

// ------------------------------------------------------------------ arena
// Device memory for serving: one hipMalloc when the arena is made; contexts
// made in it take their workspace from it (first fit, 256-byte blocks) and
// give it back when destroyed, so admitting and retiring flows neither
// allocates, frees nor synchronises.  Coarse coordinates reach the device
// through a pinned staging ring (asynchronous copies); a ring slot is reused
// once the event recorded after its copy has completed.  The bookkeeping
// (BlockList, StageRing) is host code in arena.h.
struct dnnmg_arena {
    unsigned char *base = nullptr;
    BlockList blocks;
    int live = 0;                           // contexts holding a block
    unsigned char *stage = nullptr;         // pinned staging ring
    StageRing ring;
    std::deque<hipEvent_t> slot_events;     // one per live ring slot, oldest first
    std::vector<hipEvent_t> events;         // idle events
    int device = 0;
};

namespace {

// Release the ring slots whose copies have completed (oldest first); with
// wait, first block on the oldest one.
int arena_reclaim(dnnmg_arena *a, bool wait)
{
    while (!a->slot_events.empty()) {
        hipEvent_t ev = a->slot_events.front();
        hipError_t e = wait ? hipEventSynchronize(ev) : hipEventQuery(ev);
        if (e == hipErrorNotReady) return DNNMG_OK;
        if (e != hipSuccess) return fail(DNNMG_EDEVICE, "staging event: %s", hipGetErrorString(e));
        a->slot_events.pop_front();
        a->events.push_back(ev);
        a->ring.pop_oldest();
        wait = false;
    }
    return DNNMG_OK;
}

// A staging slot of `bytes` and an idle event for it, waiting for the oldest
// slots' copies only when the ring (or the event pool) is full.
int arena_stage(dnnmg_arena *a, size_t bytes, size_t *off)
{
    if (arena_round(bytes) > a->ring.bytes)
        return fail(DNNMG_EINVAL, "%zu coordinate bytes exceed the arena's staging ring", bytes);
    int rc = arena_reclaim(a, false);
    while (rc == DNNMG_OK && (a->events.empty() || !a->ring.place(bytes, off))) rc = arena_reclaim(a, true);
    return rc;
}

// The check the geometry kernel makes, on the host: det J of the bilinear
// map is positive at the four corners of every element.
bool mesh_positively_oriented(const double *cxy, int nx, int ny)
{
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const double *c00 = cxy + 2 * ((size_t)j * (nx + 1) + i), *c10 = c00 + 2;
            const double *c01 = c00 + 2 * (nx + 1), *c11 = c01 + 2;
            const double exx = c10[0] - c00[0], exy = c10[1] - c00[1];
            const double eyx = c01[0] - c00[0], eyy = c01[1] - c00[1];
            const double twx = c11[0] - c10[0] - c01[0] + c00[0], twy = c11[1] - c10[1] - c01[1] + c00[1];
            const double d0 = exx * eyy - exy * eyx, d1 = exx * twy - exy * twx, d2 = twx * eyy - twy * eyx;
            if (!(d0 > 0.0 && d0 + d1 > 0.0 && d0 + d2 > 0.0 && d0 + d1 + d2 > 0.0)) return false;
        }
    return true;
}

}  // namespace

// ================================================================ ABI
extern "C" size_t dnnmg_weight_count(const dnnmg_config *cfg)
{
    if (!cfg || cfg->K < 1 || cfg->K > 3 || cfg->H <= 0 || cfg->Hm < 0) return 0;
    return weight_count(*cfg);
}

extern "C" size_t dnnmg_workspace_bytes(const dnnmg_config *cfg)
{
    if (check_config(cfg) != DNNMG_OK) return 0;
    return layout_of(*cfg).total + weight_bytes_estimate(*cfg);
}

extern "C" int dnnmg_create(const dnnmg_config *cfg, const double *coarse_xy_host, const float *weights_host,
                            size_t n_weights, void *stream, dnnmg_ctx **out)
{
    return create_common(cfg, coarse_xy_host, weights_host, n_weights, nullptr, stream, out);
}

extern "C" int dnnmg_create_shared(const dnnmg_config *cfg, const double *coarse_xy_host, const dnnmg_ctx *model,
                                   void *stream, dnnmg_ctx **out)
{
    if (!model) return fail(DNNMG_EINVAL, "model is NULL");
    return create_common(cfg, coarse_xy_host, nullptr, 0, model->w, stream, out);
}

extern "C" int dnnmg_umesh_counts(const dnnmg_umesh *mesh, int K, int *n_edges, int *n_fine_nodes)
{
    if (!mesh || !n_edges || !n_fine_nodes || !mesh->xy || !mesh->elems)
        return fail(DNNMG_EINVAL, "mesh, its xy and elems, n_edges and n_fine_nodes must not be NULL");
    UMeshHost m;
    const std::string err = build_umesh(mesh->n_nodes, mesh->n_elems, mesh->xy, mesh->elems, mesh->n_dirichlet,
                                        mesh->dirichlet_edges, mesh->n_circles, mesh->circles, mesh->n_curved,
                                        mesh->curved_edges, K, m);
    if (!err.empty()) return fail(DNNMG_EINVAL, "mesh: %s", err.c_str());
    *n_edges = m.E;
    *n_fine_nodes = m.Fn;
    return DNNMG_OK;
}

extern "C" int dnnmg_create_umesh(const dnnmg_config *cfg, const dnnmg_umesh *mesh, const float *weights,
                                  size_t nw, void *stream, dnnmg_ctx **out)
{
    if (!out) return fail(DNNMG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg || !mesh || !mesh->xy || !mesh->elems) return fail(DNNMG_EINVAL, "cfg, mesh, its xy and elems must not be NULL");
    if ((mesh->n_dirichlet > 0 && !mesh->dirichlet_edges) || (mesh->n_circles > 0 && !mesh->circles) ||
        (mesh->n_curved > 0 && !mesh->curved_edges))
        return fail(DNNMG_EINVAL, "a mesh list with entries has a NULL pointer");
    dnnmg_config g = *cfg;
    g.nx = std::max(mesh->n_elems, 1);   // the patches as one row (sizes, network launch)
    g.ny = 1;
    g.dirichlet = 0;
    int rc = check_config(&g);
    if (rc) return rc;
    if (g.flags & ~(unsigned)(DNNMG_F_NANCHECK | DNNMG_F_UNFUSED | DNNMG_F_GRU_RESET_AFTER | DNNMG_F_PATCH_OUTPUTS))
        return fail(DNNMG_EUNSUPPORTED,
                    "unstructured meshes take DNNMG_F_NANCHECK, DNNMG_F_GRU_RESET_AFTER and DNNMG_F_PATCH_OUTPUTS only");
    if (g.precision == DNNMG_FP8_E4M3) return fail(DNNMG_EUNSUPPORTED, "unstructured meshes run FP32 or BF16 operands");
    if (!weights) return fail(DNNMG_EINVAL, "weights_host is NULL");
    if (nw != weight_count(g)) return fail(DNNMG_EINVAL, "n_weights = %zu, expected %zu", nw, weight_count(g));
    UMeshHost m;
    const std::string err = build_umesh(mesh->n_nodes, mesh->n_elems, mesh->xy, mesh->elems, mesh->n_dirichlet,
                                        mesh->dirichlet_edges, mesh->n_circles, mesh->circles, mesh->n_curved,
                                        mesh->curved_edges, g.K, m);
    if (!err.empty()) return fail(DNNMG_EINVAL, "mesh: %s", err.c_str());

    hipStream_t st = (hipStream_t)stream;
    dnnmg_ctx *c = new dnnmg_ctx();
    c->cfg = g;
    c->s = sizes_of(g);
    c->s.Fn = m.Fn;
    c->s.Nc = m.nc;
    c->L = layout_of(g, false);
    (void)hipGetDevice(&c->device);
    UMeshDev *d = new UMeshDev();
    d->nc = m.nc; d->ne = m.ne; d->E = m.E; d->Fn = m.Fn;
    c->um = d;
    // one device block for the mesh: offsets of the arrays, 256-byte aligned
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t r = off; off += align256(bytes); return r; };
    const size_t o_corn = take(sizeof(int) * m.corners.size()), o_pmap = take(sizeof(int) * m.pmap.size());
    const size_t o_nptr = take(sizeof(int) * m.node_ptr.size()), o_nocc = take(sizeof(int) * m.node_occ.size());
    const size_t o_cptr = take(sizeof(int) * m.cnode_ptr.size()), o_cocc = take(sizeof(int) * m.cnode_occ.size());
    const size_t o_rel = take(sizeof(float) * m.rel32.size()), o_feat = take(sizeof(float) * m.feat.size());
    const size_t o_W = take(sizeof(double) * m.W.size()), o_M4 = take(sizeof(double) * m.M4.size());
    const size_t o_dgeo = take(sizeof(double) * m.dgeo.size()), o_cidx = take(sizeof(int) * m.cidx.size());
    const size_t o_mask = take(m.mask.size()), o_up = take(sizeof(float) * 2 * (size_t)m.Fn);
    const size_t o_dloc = take(sizeof(float) * 2 * (size_t)m.ne * m.nf), o_D = take(sizeof(float) * 2 * (size_t)m.Fn);
    auto bail = [&](int code) {
        (void)hipFree(c->ws);
        (void)hipFree(d->dev);
        if (c->w) release_weights(c->w);
        delete d;
        delete c;
        return code;
    };
    if (hipMalloc((void **)&c->ws, c->L.total) != hipSuccess || hipMalloc((void **)&d->dev, off) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(DNNMG_ENOMEM, "hipMalloc of %zu + %zu bytes failed", c->L.total, off));
    }
    d->corners = (int *)(d->dev + o_corn); d->pmap = (int *)(d->dev + o_pmap);
    d->node_ptr = (int *)(d->dev + o_nptr); d->node_occ = (int *)(d->dev + o_nocc);
    d->cnode_ptr = (int *)(d->dev + o_cptr); d->cnode_occ = (int *)(d->dev + o_cocc);
    d->rel = (float *)(d->dev + o_rel); d->feat = (float *)(d->dev + o_feat);
    d->W = (double *)(d->dev + o_W); d->M4 = (double *)(d->dev + o_M4);
    d->dgeo = (double *)(d->dev + o_dgeo); d->cidx = (int *)(d->dev + o_cidx);
    d->mask = d->dev + o_mask; d->uprev = (float *)(d->dev + o_up);
    d->dloc = (float *)(d->dev + o_dloc); d->D = (float *)(d->dev + o_D);
    rc = build_weights(g, weights, st, &c->w);
    if (rc) { c->w = nullptr; return bail(rc); }
    hipError_t e = hipSuccess;
    auto up = [&](void *dst, const void *src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    };
    up(d->corners, m.corners.data(), sizeof(int) * m.corners.size());
    up(d->pmap, m.pmap.data(), sizeof(int) * m.pmap.size());
    up(d->node_ptr, m.node_ptr.data(), sizeof(int) * m.node_ptr.size());
    up(d->node_occ, m.node_occ.data(), sizeof(int) * m.node_occ.size());
    up(d->cnode_ptr, m.cnode_ptr.data(), sizeof(int) * m.cnode_ptr.size());
    up(d->cnode_occ, m.cnode_occ.data(), sizeof(int) * m.cnode_occ.size());
    up(d->rel, m.rel32.data(), sizeof(float) * m.rel32.size());
    up(d->feat, m.feat.data(), sizeof(float) * m.feat.size());
    up(d->W, m.W.data(), sizeof(double) * m.W.size());
    up(d->M4, m.M4.data(), sizeof(double) * m.M4.size());
    up(d->dgeo, m.dgeo.data(), sizeof(double) * m.dgeo.size());
    up(d->cidx, m.cidx.data(), sizeof(int) * m.cidx.size());
    up(d->mask, m.mask.data(), m.mask.size());
    if (e == hipSuccess) e = hipMemsetAsync(d->uprev, 0, sizeof(float) * 2 * (size_t)m.Fn, st);
    if (e == hipSuccess) e = hipMemsetAsync(c->h(), 0, sizeof(float) * (size_t)m.ne * g.H, st);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + c->L.nonfinite, 0, sizeof(int), st);
    if (e == hipSuccess) e = hipMemsetAsync(c->first_flag(), 1, sizeof(int), st);
    // the host vectors are the copies' sources: wait before they go
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bail(fail(DNNMG_EDEVICE, "create_umesh: %s", hipGetErrorString(e)));
    *out = c;
    return DNNMG_OK;
}

extern "C" int dnnmg_destroy(dnnmg_ctx *ctx)
{
    if (!ctx) return fail(DNNMG_EINVAL, "ctx is NULL");
    for (hipEvent_t e : ctx->prof.ev) (void)hipEventSynchronize(e);
    for (hipEvent_t e : ctx->prof.evg) (void)hipEventSynchronize(e);
    profile_release(ctx->prof);
    if (ctx->um) {
        (void)hipFree(ctx->um->dev);
        delete ctx->um;
    }
    if (ctx->arena) {
        ctx->arena->blocks.give((size_t)(ctx->ws - ctx->arena->base), ctx->L.total);
        ctx->arena->live--;
    } else {
        (void)hipFree(ctx->ws);
    }
    release_weights(ctx->w);
    delete ctx;
    return DNNMG_OK;
}

extern "C" size_t dnnmg_arena_block_bytes(const dnnmg_config *cfg)
{
    if (check_config(cfg) != DNNMG_OK) return 0;
    return align256(layout_of(*cfg).total);
}

extern "C" int dnnmg_arena_create(size_t bytes, size_t staging_bytes, dnnmg_arena **out)
{
    if (!out) return fail(DNNMG_EINVAL, "out is NULL");
    *out = nullptr;
    if (bytes < 256 || staging_bytes < 256) return fail(DNNMG_EINVAL, "arena and staging sizes must be >= 256 bytes");
    dnnmg_arena *a = new dnnmg_arena();
    a->blocks.init(bytes);
    a->ring.init(staging_bytes);
    (void)hipGetDevice(&a->device);
    bool ok = hipMalloc((void **)&a->base, a->blocks.bytes) == hipSuccess &&
              hipHostMalloc((void **)&a->stage, a->ring.bytes, hipHostMallocDefault) == hipSuccess;
    for (int i = 0; ok && i < 64; ++i) {
        hipEvent_t e = nullptr;
        ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
        if (ok) a->events.push_back(e);
    }
    if (!ok) {
        (void)hipGetLastError();
        if (a->base) (void)hipFree(a->base);
        if (a->stage) (void)hipHostFree(a->stage);
        for (hipEvent_t e : a->events) (void)hipEventDestroy(e);
        delete a;
        return fail(DNNMG_ENOMEM, "arena of %zu bytes (staging %zu) could not be allocated", bytes, staging_bytes);
    }
    *out = a;
    return DNNMG_OK;
}

extern "C" int dnnmg_arena_destroy(dnnmg_arena *a)
{
    if (!a) return fail(DNNMG_EINVAL, "arena is NULL");
    if (a->live > 0) return fail(DNNMG_ESTATE, "%d contexts still use the arena", a->live);
    while (!a->slot_events.empty()) {
        int rc = arena_reclaim(a, true);
        if (rc) return rc;
    }
    for (hipEvent_t e : a->events) (void)hipEventDestroy(e);
    (void)hipFree(a->base);
    (void)hipHostFree(a->stage);
    delete a;
    return DNNMG_OK;
}

extern "C" int dnnmg_arena_usage(const dnnmg_arena *a, size_t *used, size_t *largest_free)
{
    if (!a || !used || !largest_free) return fail(DNNMG_EINVAL, "arena, used and largest_free must not be NULL");
    *used = a->blocks.used;
    *largest_free = a->blocks.largest();
    return DNNMG_OK;
}

extern "C" int dnnmg_arena_upload(dnnmg_arena *a, void *dst_dev, const void *src_host, size_t bytes, void *stream)
{
    if (!a || !dst_dev || !src_host) return fail(DNNMG_EINVAL, "arena, dst and src must not be NULL");
    if (bytes == 0) return DNNMG_OK;
    size_t soff = 0;
    int rc = arena_stage(a, bytes, &soff);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    std::memcpy(a->stage + soff, src_host, bytes);
    HIP_OR_FAIL(hipMemcpyAsync(dst_dev, a->stage + soff, bytes, hipMemcpyHostToDevice, st));
    hipEvent_t ev = a->events.back();
    HIP_OR_FAIL(hipEventRecord(ev, st));
    a->events.pop_back();
    a->ring.push(soff, bytes);
    a->slot_events.push_back(ev);
    return DNNMG_OK;
}

extern "C" int dnnmg_create_in_arena(dnnmg_arena *a, const dnnmg_config *cfg, const double *cxy,
                                     const dnnmg_ctx *model, void *stream, dnnmg_ctx **out)
{
    if (!out) return fail(DNNMG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!a) return fail(DNNMG_EINVAL, "arena is NULL");
    if (!model) return fail(DNNMG_EINVAL, "model is NULL");
    int rc = check_config(cfg);
    if (rc) return rc;
    if (!cxy) return fail(DNNMG_EINVAL, "coarse_xy_host is NULL");
    const Weights *w = model->w;
    if (w->K != cfg->K || w->H != cfg->H || w->Hm != cfg->Hm || w->prec != cfg->precision ||
        w->netflags != (cfg->flags & kNetFlags))
        return fail(DNNMG_EINVAL, "shared weights have another K/H/Hm/precision/network form");
    const size_t ncxy = 2 * (size_t)(cfg->nx + 1) * (cfg->ny + 1);
    for (size_t i = 0; i < ncxy; ++i)
        if (!std::isfinite(cxy[i])) return fail(DNNMG_EINVAL, "coarse_xy_host[%zu] is not finite", i);
    if (!mesh_positively_oriented(cxy, cfg->nx, cfg->ny))
        return fail(DNNMG_EINVAL, "coarse mesh has an element that is not positively oriented");
    const Layout L = layout_of(*cfg);
    size_t off = 0, soff = 0;
    if (!a->blocks.take(L.total, &off))
        return fail(DNNMG_ENOMEM, "arena has no free block of %zu bytes (%zu of %zu in use)", align256(L.total),
                    a->blocks.used, a->blocks.bytes);
    rc = arena_stage(a, sizeof(double) * ncxy, &soff);
    if (rc) { a->blocks.give(off, L.total); return rc; }
    hipStream_t st = (hipStream_t)stream;
    dnnmg_ctx *c = new dnnmg_ctx();
    c->cfg = *cfg;
    c->s = sizes_of(*cfg);
    c->L = L;
    c->device = a->device;
    c->arena = a;
    c->ws = a->base + off;
    c->w = model->w;
    const Sizes &s = c->s;
    std::memcpy(a->stage + soff, cxy, sizeof(double) * ncxy);
    hipError_t e = hipMemcpyAsync(c->ws + L.cxy, a->stage + soff, sizeof(double) * ncxy, hipMemcpyHostToDevice, st);
    hipEvent_t ev = a->events.back();
    if (e == hipSuccess) e = hipEventRecord(ev, st);
    if (e == hipSuccess) {
        a->events.pop_back();
        a->ring.push(soff, sizeof(double) * ncxy);
        a->slot_events.push_back(ev);
    }
    if (e == hipSuccess) e = hipMemsetAsync(c->h(), 0, sizeof(float) * (size_t)s.P * cfg->H, st);
    if (e == hipSuccess) e = hipMemsetAsync(c->uprev(), 0, sizeof(float) * 2 * s.Fu, st);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.nonfinite, 0, sizeof(int), st);
    if (e == hipSuccess) e = hipMemsetAsync(c->first_flag(), 1, sizeof(int), st);
    if (e == hipSuccess)
        e = launch_geometry((const double *)(c->ws + L.cxy), cfg->nx, cfg->ny, c->geo(), c->geo64(), c->map64(),
                            c->feat(), c->geo12(), (int *)(c->ws + L.bad), st);
    if (e != hipSuccess) {
        // the enqueued work may still touch the block: wait for it before returning the block
        (void)hipStreamSynchronize(st);
        a->blocks.give(off, L.total);
        delete c;
        return fail(DNNMG_EDEVICE, "create in arena: %s", hipGetErrorString(e));
    }
    ++c->w->refs;
    a->live++;
    *out = c;
    return DNNMG_OK;
}

extern "C" long long dnnmg_step_count(const dnnmg_ctx *ctx) { return ctx ? ctx->steps : -1; }

static int enqueue_ustep(dnnmg_ctx *c, const UArgs &u, hipStream_t st)
{
    const dnnmg_config &g = c->cfg;
    Profile &pr = c->prof;
    hipEvent_t *ev = (pr.max_steps > 0 && pr.steps < pr.max_steps) ? &pr.ev[4 * pr.steps] : nullptr;
    if (ev) HIP_OR_FAIL(hipEventRecord(ev[0], st));
    HIP_OR_FAIL(launch_udefect(u, nullptr, st));     // contributions; the input rows sum them per node
    HIP_OR_FAIL(launch_uinput(u, st));
    if (ev) HIP_OR_FAIL(hipEventRecord(ev[1], st));
    HIP_OR_FAIL(launch_net(unet_args(c), nullptr, blocks_for(kKindNet, c->um->ne, 1, g.K), c->w->net, st));
    if (ev) HIP_OR_FAIL(hipEventRecord(ev[2], st));
    HIP_OR_FAIL(launch_uaverage(u, st));            // D now holds the averaged correction
    HIP_OR_FAIL(launch_urhs(u, c->um->D, st));
    if (ev) {
        HIP_OR_FAIL(hipEventRecord(ev[3], st));
        pr.steps++;
    }
    return DNNMG_OK;
}

static int enqueue_step(dnnmg_ctx *c, const FlowArgs &f, hipStream_t st)
{
    const dnnmg_config &g = c->cfg;
    Profile &pr = c->prof;
    hipEvent_t *ev = (pr.max_steps > 0 && pr.steps < pr.max_steps) ? &pr.ev[4 * pr.steps] : nullptr;
    if (ev) HIP_OR_FAIL(hipEventRecord(ev[0], st));
    FlowArgs fs = f;
    if (fused_step(c->w->net) && !(g.flags & (DNNMG_F_UNFUSED | DNNMG_F_CRANK_NICOLSON))) {
        // defect, network input, GRU, MLP and the averaging inside the tiles in
        // one launch (stage 1 then times nothing); the rhs completes the frame
        if (!c->frame()) return fail(DNNMG_EINVAL, "internal: one-launch step without a tile frame");
        fs.frame = c->frame();
        fs.keep_dpatch = (g.flags & DNNMG_F_PATCH_OUTPUTS) ? 1 : 0;
        HIP_OR_FAIL(launch_defect_net(fs, nullptr, blocks_for(kKindDefect, g.nx, g.ny, g.K), c->w->net, st));
        if (ev) HIP_OR_FAIL(hipEventRecord(ev[1], st));
    } else {
        HIP_OR_FAIL(launch_defect(f, nullptr, blocks_for(kKindDefect, g.nx, g.ny, g.K), g.K, f.xfmt, st));
        if (ev) HIP_OR_FAIL(hipEventRecord(ev[1], st));
        HIP_OR_FAIL(launch_net(f, nullptr, blocks_for(kKindNet, g.nx, g.ny, g.K), c->w->net, st));
    }
    if (ev) HIP_OR_FAIL(hipEventRecord(ev[2], st));
    HIP_OR_FAIL(launch_rhs(fs, nullptr, blocks_for(kKindRhs, g.nx, g.ny, g.K), g.K, c->tables(), 1, st));
    c->dpatch_kept = !fs.frame || fs.keep_dpatch;
    if (ev) {
        HIP_OR_FAIL(hipEventRecord(ev[3], st));
        pr.steps++;
    }
    return DNNMG_OK;
}

static void profile_release(Profile &pr)
{
    for (hipEvent_t e : pr.ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : pr.evg) (void)hipEventDestroy(e);
    pr.ev.clear();
    pr.evg.clear();
    pr.max_steps = pr.steps = pr.gathers = 0;
}

extern "C" int dnnmg_profile_enable(dnnmg_ctx *ctx, int max_steps)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (max_steps < 0 || max_steps > 100000) return fail(DNNMG_EINVAL, "max_steps must be in 0..100000");
    for (hipEvent_t e : ctx->prof.ev) HIP_OR_FAIL(hipEventSynchronize(e));
    profile_release(ctx->prof);
    if (max_steps == 0) return DNNMG_OK;
    Profile &pr = ctx->prof;
    pr.ev.resize(4 * (size_t)max_steps);
    pr.evg.resize(2 * (size_t)max_steps);
    for (auto *v : {&pr.ev, &pr.evg})
        for (hipEvent_t &e : *v)
            // no system-scope release at each record: a record then costs about
            // 2 us of stream time instead of 3.6 us, and the timings stay exact
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
                e = nullptr;
                (void)hipGetLastError();
                profile_release(pr);
                return fail(DNNMG_EDEVICE, "hipEventCreate failed");
            }
    pr.max_steps = max_steps;
    return DNNMG_OK;
}

extern "C" int dnnmg_profile_read(dnnmg_ctx *ctx, double *ms, int *count)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!ms || !count) return fail(DNNMG_EINVAL, "ms_per_stage and launches_per_stage must not be NULL");
    Profile &pr = ctx->prof;
    for (int k = 0; k < DNNMG_STAGES; ++k) { ms[k] = 0.0; count[k] = 0; }
    for (int s = 0; s < pr.steps; ++s)
        for (int k = 0; k < 3; ++k) {
            float t = 0.f;
            HIP_OR_FAIL(hipEventSynchronize(pr.ev[4 * s + k + 1]));
            HIP_OR_FAIL(hipEventElapsedTime(&t, pr.ev[4 * s + k], pr.ev[4 * s + k + 1]));
            ms[k] += t;
            count[k]++;
        }
    for (int s = 0; s < pr.gathers; ++s) {
        float t = 0.f;
        HIP_OR_FAIL(hipEventSynchronize(pr.evg[2 * s + 1]));
        HIP_OR_FAIL(hipEventElapsedTime(&t, pr.evg[2 * s], pr.evg[2 * s + 1]));
        ms[3] += t;
        count[3]++;
    }
    pr.steps = pr.gathers = 0;
    return DNNMG_OK;
}

extern "C" int dnnmg_step(dnnmg_ctx *ctx, const float *v, const float *p, float *d_fine, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!v) return fail(DNNMG_EINVAL, "v_coarse_dev is NULL");
    if (ctx->um) {
        UArgs u = uargs(ctx, v, p);
        u.dbar_out = d_fine;
        rc = enqueue_ustep(ctx, u, (hipStream_t)stream);
        if (rc) return rc;
        ctx->steps++;
        return DNNMG_OK;
    }
    FlowArgs f = flow_args(ctx, v, p);
    f.dbar_out = d_fine;
    rc = enqueue_step(ctx, f, (hipStream_t)stream);
    if (rc) return rc;
    ctx->steps++;
    return DNNMG_OK;
}

extern "C" int dnnmg_restrict_rhs(dnnmg_ctx *ctx, double *b, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!b) return fail(DNNMG_EINVAL, "b_coarse_dev is NULL");
    if (ctx->steps == 0) return fail(DNNMG_ESTATE, "no step has been taken yet");
    FlowArgs f = flow_args(ctx, nullptr, nullptr);
    f.bL = b;
    Profile &pr = ctx->prof;
    hipEvent_t *ev = (pr.max_steps > 0 && pr.gathers < pr.max_steps) ? &pr.evg[2 * pr.gathers] : nullptr;
    if (ev) HIP_OR_FAIL(hipEventRecord(ev[0], (hipStream_t)stream));
    if (ctx->um) {
        UArgs u = uargs(ctx, nullptr, nullptr);
        u.bL = b;
        HIP_OR_FAIL(launch_ugather(u, (hipStream_t)stream));
    } else {
        HIP_OR_FAIL(launch_gather(f, nullptr, blocks_for(kKindGather, ctx->cfg.nx, ctx->cfg.ny, ctx->cfg.K),
                                  (hipStream_t)stream));
    }
    if (ev) {
        HIP_OR_FAIL(hipEventRecord(ev[1], (hipStream_t)stream));
        pr.gathers++;
    }
    return DNNMG_OK;
}

extern "C" int dnnmg_prolong(dnnmg_ctx *ctx, const float *v, const float *p, float *pv, float *pp, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!v) return fail(DNNMG_EINVAL, "v_coarse_dev is NULL");
    if (ctx->um) {
        UArgs u = uargs(ctx, v, p);
        u.pv_out = pv;
        u.pp_out = pp;
        HIP_OR_FAIL(launch_uprolong(u, (hipStream_t)stream));
        return DNNMG_OK;
    }
    FlowArgs f = flow_args(ctx, v, p);
    HIP_OR_FAIL(launch_prolong(f, ctx->cfg.K, pv, pp, (hipStream_t)stream));
    return DNNMG_OK;
}

extern "C" int dnnmg_defect(dnnmg_ctx *ctx, const float *v, const float *p, float *D, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!v || !D) return fail(DNNMG_EINVAL, "v_coarse_dev and D_out_dev must not be NULL");
    if (ctx->um) {
        HIP_OR_FAIL(launch_udefect(uargs(ctx, v, p), D, (hipStream_t)stream));
        return DNNMG_OK;
    }
    FlowArgs f = flow_args(ctx, v, p);
    f.D = D;
    f.X = nullptr;   // the stage leaves the network input alone
    HIP_OR_FAIL(launch_defect(f, nullptr, blocks_for(kKindDefect, ctx->cfg.nx, ctx->cfg.ny, ctx->cfg.K), ctx->cfg.K,
                              f.xfmt, (hipStream_t)stream));
    return DNNMG_OK;
}

extern "C" int dnnmg_rhs_restrict(dnnmg_ctx *ctx, const float *v, const float *dbar, double *b, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!v || !dbar || !b) return fail(DNNMG_EINVAL, "v, dbar and b_out must not be NULL");
    if (ctx->um) {
        UArgs u = uargs(ctx, v, nullptr);
        u.part = (double *)(ctx->ws + ctx->L.part2);
        u.bL = b;
        HIP_OR_FAIL(launch_urhs(u, dbar, (hipStream_t)stream));
        HIP_OR_FAIL(launch_ugather(u, (hipStream_t)stream));
        return DNNMG_OK;
    }
    FlowArgs f = flow_args(ctx, v, nullptr);
    f.dbar_in = dbar;
    f.part = (double *)(ctx->ws + ctx->L.part2);   // keeps the step's own partial sums intact
    f.bL = b;
    const dnnmg_config &g = ctx->cfg;
    hipStream_t st = (hipStream_t)stream;
    HIP_OR_FAIL(launch_rhs(f, nullptr, blocks_for(kKindRhs, g.nx, g.ny, g.K), g.K, ctx->tables(), 0, st));
    HIP_OR_FAIL(launch_gather(f, nullptr, blocks_for(kKindGather, g.nx, g.ny, g.K), st));
    return DNNMG_OK;
}

// ------------------------------------------- allocation-free rhs + restriction
// dnnmg_rhs_restrict without a context: the kernels' scratch (the patches'
// map coefficients, the FP64 corner partial sums, the moment tables) lives in
// one file-scope device array instead of a hipMalloc'd workspace.
namespace {
constexpr size_t cround(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t kStaticTabA = 0;                                              // moment table A (K <= 3)
constexpr size_t kStaticTabM = kStaticTabA + cround(sizeof(double) * 4 * 9);  // moment table M
constexpr size_t kStaticGeo = kStaticTabM + cround(sizeof(double) * kMomentMSize);
constexpr size_t kStaticGeo64 = kStaticGeo + cround(sizeof(float) * 6 * DNNMG_NOALLOC_MAX_PATCHES);
constexpr size_t kStaticFeat = kStaticGeo64 + cround(sizeof(double) * 4 * DNNMG_NOALLOC_MAX_PATCHES);
constexpr size_t kStaticPart = kStaticFeat + cround(sizeof(float) * 4 * DNNMG_NOALLOC_MAX_PATCHES);
constexpr size_t kStaticBad = kStaticPart + cround(sizeof(double) * 8 * DNNMG_NOALLOC_MAX_PATCHES);
constexpr size_t kStaticBytes = kStaticBad + 256;
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
unsigned char *g_scratch_dev[kMaxDevices] = {};   // the array's device address, per device
}  // namespace

// (its name in host code is a host-side stand-in: host code uses only the
// addresses hipGetSymbolAddress returns)
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

// The array's address on the current device, looked up once per device.
static int static_scratch(unsigned char **out)
{
    int dev = 0;
    HIP_OR_FAIL(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DNNMG_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIP_OR_FAIL(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(DNNMG_EDEVICE, "hipGetSymbolAddress returned NULL");
        g_scratch_dev[dev] = (unsigned char *)p;
    }
    *out = g_scratch_dev[dev];
    return DNNMG_OK;
}

extern "C" size_t dnnmg_noalloc_scratch_bytes(void) { return kStaticBytes; }

extern "C" int dnnmg_rhs_restrict_noalloc(int nx, int ny, int K, double dt, const double *cxy, const float *v,
                                          const float *dbar, double *b, void *stream)
{
    if (!cxy || !v || !dbar || !b) return fail(DNNMG_EINVAL, "coarse_xy, v, dbar and b_out must not be NULL");
    if (nx < 1 || ny < 1) return fail(DNNMG_EINVAL, "nx, ny must be >= 1 (got %d, %d)", nx, ny);
    if (K < 1 || K > 3) return fail(DNNMG_EINVAL, "K must be 1, 2 or 3 (got %d)", K);
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DNNMG_EINVAL, "dt must be > 0");
    if ((long long)nx * ny > DNNMG_NOALLOC_MAX_PATCHES)
        return fail(DNNMG_EINVAL, "%d x %d = %lld patches exceed the allocation-free limit of %d", nx, ny,
                    (long long)nx * ny, DNNMG_NOALLOC_MAX_PATCHES);
    unsigned char *sc = nullptr;
    int rc = static_scratch(&sc);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    double *tabA = (double *)(sc + kStaticTabA), *tabM = (double *)(sc + kStaticTabM);
    FlowArgs f{};
    f.nx = nx;
    f.ny = ny;
    f.inv_dt = (float)(1.0 / dt);
    f.inv_dt64 = 1.0 / dt;
    f.v = v;
    f.geo = (const float *)(sc + kStaticGeo);
    f.geo64 = (const double *)(sc + kStaticGeo64);
    f.feat = (const float *)(sc + kStaticFeat);
    f.upitch = nx * (1 << K) + 1;
    f.dbar_in = dbar;
    f.part = (double *)(sc + kStaticPart);
    f.bL = b;
    // every scratch word the kernels read is written earlier in this call
    // (geometry, tables, partial sums), so nothing needs clearing
    HIP_OR_FAIL(launch_geometry(cxy, nx, ny, (float *)f.geo, (double *)f.geo64, nullptr, (float *)f.feat, nullptr,
                                (int *)(sc + kStaticBad), st));
    HIP_OR_FAIL(launch_moment_tables(K, tabA, tabM, st));
    HIP_OR_FAIL(launch_rhs(f, nullptr, blocks_for(kKindRhs, nx, ny, K), K, RhsTables{tabA, tabM}, 0, st));
    HIP_OR_FAIL(launch_gather(f, nullptr, blocks_for(kKindGather, nx, ny, K), st));
    return DNNMG_OK;
}

extern "C" int dnnmg_get_state(dnnmg_ctx *ctx, float *h, float *u, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (h) HIP_OR_FAIL(hipMemcpyAsync(h, ctx->h(), sizeof(float) * (size_t)ctx->s.P * ctx->cfg.H,
                                      hipMemcpyDeviceToDevice, st));
    if (ctx->um) {
        if (u) HIP_OR_FAIL(hipMemcpyAsync(u, ctx->um->uprev, sizeof(float) * 2 * (size_t)ctx->um->Fn,
                                          hipMemcpyDeviceToDevice, st));
        return DNNMG_OK;
    }
    // (the state's rows are padded to upitch nodes; the caller's are NX+1)
    const size_t row = sizeof(float) * 2 * (size_t)(ctx->cfg.nx * ctx->s.n + 1);
    if (u) HIP_OR_FAIL(hipMemcpy2DAsync(u, row, ctx->uprev(), sizeof(float) * 2 * (size_t)ctx->s.upitch, row,
                                        ctx->cfg.ny * ctx->s.n + 1, hipMemcpyDeviceToDevice, st));
    return DNNMG_OK;
}

extern "C" int dnnmg_set_state(dnnmg_ctx *ctx, const float *h, const float *u, long long steps, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (steps < 0) return fail(DNNMG_EINVAL, "steps must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    if (h) HIP_OR_FAIL(hipMemcpyAsync(ctx->h(), h, sizeof(float) * (size_t)ctx->s.P * ctx->cfg.H,
                                      hipMemcpyDeviceToDevice, st));
    if (ctx->um) {
        if (u) HIP_OR_FAIL(hipMemcpyAsync(ctx->um->uprev, u, sizeof(float) * 2 * (size_t)ctx->um->Fn,
                                          hipMemcpyDeviceToDevice, st));
    } else {
        const size_t row = sizeof(float) * 2 * (size_t)(ctx->cfg.nx * ctx->s.n + 1);
        if (u) HIP_OR_FAIL(hipMemcpy2DAsync(ctx->uprev(), sizeof(float) * 2 * (size_t)ctx->s.upitch, u, row, row,
                                            ctx->cfg.ny * ctx->s.n + 1, hipMemcpyDeviceToDevice, st));
    }
    HIP_OR_FAIL(hipMemsetAsync(ctx->first_flag(), steps == 0 ? 1 : 0, sizeof(int), st));
    ctx->steps = steps;
    return DNNMG_OK;
}

extern "C" int dnnmg_nonfinite(dnnmg_ctx *ctx, int clear, int *flags_out, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!flags_out) return fail(DNNMG_EINVAL, "flags_out is NULL");
    if (!(ctx->cfg.flags & DNNMG_F_NANCHECK)) return fail(DNNMG_ESTATE, "context created without DNNMG_F_NANCHECK");
    hipStream_t st = (hipStream_t)stream;
    int v = 0;
    HIP_OR_FAIL(hipMemcpyAsync(&v, ctx->ws + ctx->L.nonfinite, sizeof(int), hipMemcpyDeviceToHost, st));
    if (clear) HIP_OR_FAIL(hipMemsetAsync(ctx->ws + ctx->L.nonfinite, 0, sizeof(int), st));
    HIP_OR_FAIL(hipStreamSynchronize(st));
    *flags_out = v;
    return DNNMG_OK;
}

extern "C" int dnnmg_patch_output(dnnmg_ctx *ctx, float *d, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!d) return fail(DNNMG_EINVAL, "d_out_dev is NULL");
    if (ctx->steps == 0) return fail(DNNMG_ESTATE, "no step has been taken yet");
    if (!ctx->dpatch_kept)
        return fail(DNNMG_ESTATE, "the last step kept no per-patch outputs (one-launch step: create the context "
                                  "with DNNMG_F_PATCH_OUTPUTS)");
    HIP_OR_FAIL(hipMemcpyAsync(d, ctx->dpatch(), sizeof(float) * (size_t)ctx->s.P * ctx->s.nout,
                               hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return DNNMG_OK;
}

// ------------------------------------------------------------- batches
extern "C" int dnnmg_batch_create(int max_flows, dnnmg_batch **out)
{
    if (!out) return fail(DNNMG_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_flows < 1 || max_flows > kMaxBatch)
        return fail(DNNMG_EINVAL, "max_flows must be in 1..%d", kMaxBatch);
    dnnmg_batch *b = new dnnmg_batch();
    b->max_flows = max_flows;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) {
        (void)hipGetLastError();
        delete b;
        return fail(DNNMG_EDEVICE, "cannot query the device's compute units");
    }
    // eight blocks per CU: room for every batched kernel's resident
    // workgroups (up to six per CU for the rhs), the rest wait their turn
    b->cap = 8 * ncu;
    bool ok = hipMalloc((void **)&b->dev, sizeof(BatchTable)) == hipSuccess;
    for (int i = 0; ok && i < 2; ++i)
        ok = hipHostMalloc((void **)&b->host[i], sizeof(BatchTable), hipHostMallocDefault) == hipSuccess &&
             hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        dnnmg_batch_destroy(b);
        return fail(DNNMG_ENOMEM, "batch table allocation failed");
    }
    *out = b;
    return DNNMG_OK;
}

static bool same_net(const NetArgs &a, const NetArgs &b)
{
    return a.K == b.K && a.H == b.H && a.Hm == b.Hm && a.nin == b.nin && a.nout == b.nout && a.prec == b.prec &&
           a.kc1 == b.kc1 && a.B1 == b.B1 && a.B2 == b.B2 && a.B3 == b.B3 && a.B4 == b.B4;
}

static void batch_drop_graph(dnnmg_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_gather = -1;
}

extern "C" int dnnmg_batch_destroy(dnnmg_batch *b)
{
    if (!b) return fail(DNNMG_EINVAL, "batch is NULL");
    for (int i = 0; i < 2; ++i)
        if (b->ev[i]) { (void)hipEventSynchronize(b->ev[i]); (void)hipEventDestroy(b->ev[i]); }
    batch_drop_graph(b);
    if (b->dev) (void)hipFree(b->dev);
    for (int i = 0; i < 2; ++i)
        if (b->host[i]) (void)hipHostFree(b->host[i]);
    delete b;
    return DNNMG_OK;
}

extern "C" int dnnmg_batch_prepare(dnnmg_batch *b, dnnmg_ctx *const *ctxs, int nflows, const float *const *v,
                                   const float *const *p, float *const *d_out, double *const *b_out, void *stream)
{
    if (!b || !ctxs || !v) return fail(DNNMG_EINVAL, "batch, ctxs and v must not be NULL");
    if (nflows < 1 || nflows > b->max_flows) return fail(DNNMG_EINVAL, "nflows must be in 1..%d", b->max_flows);
    Weights *w = ctxs[0] ? ctxs[0]->w : nullptr;
    for (int i = 0; i < nflows; ++i) {
        if (!ctxs[i]) return fail(DNNMG_EINVAL, "ctxs[%d] is NULL", i);
        if (!v[i]) return fail(DNNMG_EINVAL, "v[%d] is NULL", i);
        if (b_out && !b_out[i]) return fail(DNNMG_EINVAL, "b_out[%d] is NULL", i);
        if (ctxs[i]->w != w) return fail(DNNMG_EINVAL, "ctxs[%d] does not share the weights of ctxs[0]", i);
        if (ctxs[i]->um) return fail(DNNMG_EINVAL, "ctxs[%d] is an unstructured-mesh context: it steps alone", i);
        if (ctxs[i]->cfg.flags & (DNNMG_F_CRANK_NICOLSON | DNNMG_F_PAPER_NET))
            return fail(DNNMG_EINVAL, "ctxs[%d] uses DNNMG_F_CRANK_NICOLSON or DNNMG_F_PAPER_NET: such flows step "
                                      "alone (dnnmg_step)", i);
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(DNNMG_EINVAL, "ctxs[%d] repeats ctxs[%d]", i, j);
    }
    hipStream_t st = (hipStream_t)stream;
    // the one-launch tiles average inside the tile and hand the rest over in
    // the tile frame when every flow has one (as in dnnmg_step)
    bool frame = fused_step(w->net);
    for (int i = 0; i < nflows && frame; ++i) frame = ctxs[i]->frame() != nullptr;
    const int slot = b->slot;
    if (b->used[slot]) HIP_OR_FAIL(hipEventSynchronize(b->ev[slot]));
    BatchTable *t = b->host[slot];
    t->nflows = nflows;
    for (int k = 0; k < kKinds; ++k) t->prefix[k][0] = 0;
    for (int i = 0; i < nflows; ++i) {
        const dnnmg_config &g = ctxs[i]->cfg;
        for (int k = 0; k < kKinds; ++k) t->prefix[k][i + 1] = t->prefix[k][i] + blocks_for(k, g.nx, g.ny, g.K);
        FlowArgs f = flow_args(ctxs[i], v[i], p ? p[i] : nullptr);
        f.dbar_out = d_out ? d_out[i] : nullptr;
        f.bL = b_out ? b_out[i] : nullptr;
        f.frame = frame ? ctxs[i]->frame() : nullptr;
        f.keep_dpatch = !frame || (g.flags & DNNMG_F_PATCH_OUTPUTS) ? 1 : 0;
        ctxs[i]->dpatch_kept = f.keep_dpatch != 0;
        t->flows[i] = f;
    }
    const size_t bytes = offsetof(BatchTable, flows) + sizeof(FlowArgs) * nflows;
    HIP_OR_FAIL(hipMemcpyAsync(b->dev, t, bytes, hipMemcpyHostToDevice, st));
    HIP_OR_FAIL(hipEventRecord(b->ev[slot], st));
    b->used[slot] = true;
    b->slot ^= 1;
    b->prepared = true;
    b->nflows = nflows;
    b->K = ctxs[0]->cfg.K;
    b->xfmt = ctxs[0]->cfg.precision;
    b->gather = b_out != nullptr;
    b->frame = frame ? 1 : 0;
    b->net = w->net;
    b->tab = ctxs[0]->tables();
    for (int k = 0; k < kKinds; ++k) b->totals[k] = t->prefix[k][nflows];
    for (int i = 0; i < nflows; ++i) ctxs[i]->steps++;
    return DNNMG_OK;
}

// Grids of the batched launches.  The kernels stride over the table's tiles,
// so any grid is correct; a graph uses the fixed cap so that one capture
// serves every membership, an eager launch trims the grid to the work.
static int batch_enqueue(dnnmg_batch *b, bool graph, hipStream_t st)
{
    FlowArgs dummy{};
    int grid[kKinds];
    for (int k = 0; k < kKinds; ++k) grid[k] = graph ? b->cap : std::min(b->totals[k], b->cap);
    // the one-launch tiles and the rhs of the tile frame take one tile per block
    auto tiles = [&](int k) { return graph ? b->tile_grid : b->totals[k]; };
    if (fused_step(b->net)) {
        HIP_OR_FAIL(launch_defect_net(dummy, b->dev, tiles(kKindDefect), b->net, st));
    } else {
        HIP_OR_FAIL(launch_defect(dummy, b->dev, grid[kKindDefect], b->K, b->xfmt, st));
        HIP_OR_FAIL(launch_net(dummy, b->dev, grid[kKindNet], b->net, st));
    }
    if (b->frame) HIP_OR_FAIL(launch_rhs(dummy, b->dev, tiles(kKindRhs), b->K, b->tab, 2, st));
    else HIP_OR_FAIL(launch_rhs(dummy, b->dev, b->K == 3 ? tiles(kKindRhs) : grid[kKindRhs], b->K, b->tab, 1, st));
    if (b->gather) HIP_OR_FAIL(launch_gather(dummy, b->dev, grid[kKindGather], st));
    return DNNMG_OK;
}

extern "C" int dnnmg_batch_launch(dnnmg_batch *b, int use_graph, void *stream)
{
    if (!b) return fail(DNNMG_EINVAL, "batch is NULL");
    if (!b->prepared) return fail(DNNMG_ESTATE, "dnnmg_batch_prepare has not been called");
    hipStream_t st = (hipStream_t)stream;
    if (!use_graph) return batch_enqueue(b, false, st);
    if (!st) return fail(DNNMG_EINVAL, "graph launches need a non-default stream");
    // (only the one-launch batches have one-tile-per-block launches)
    const int tiles = fused_step(b->net) ? std::max(b->totals[kKindDefect], b->totals[kKindRhs])
                                         : (b->K == 3 ? b->totals[kKindRhs] : 0);
    const bool same = b->exec && b->graph_K == b->K && b->graph_xfmt == b->xfmt &&
                      b->graph_gather == b->gather && b->graph_frame == b->frame && tiles <= b->tile_grid &&
                      same_net(b->graph_net, b->net) &&
                      b->graph_tab.A == b->tab.A && b->graph_tab.M == b->tab.M;
    if (!same) {
        batch_drop_graph(b);
        if (tiles > b->tile_grid) b->tile_grid = std::max(b->cap, 2 * tiles);
        HIP_OR_FAIL(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        int rc = batch_enqueue(b, true, st);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(st, &g);
        if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (e != hipSuccess) return fail(DNNMG_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        b->graph = g;
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) { batch_drop_graph(b); return fail(DNNMG_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e)); }
        b->graph_K = b->K;
        b->graph_xfmt = b->xfmt;
        b->graph_gather = b->gather;
        b->graph_frame = b->frame;
        b->graph_net = b->net;
        b->graph_tab = b->tab;
        b->captures++;
    }
    HIP_OR_FAIL(hipGraphLaunch(b->exec, st));
    return DNNMG_OK;
}

extern "C" int dnnmg_quantize_e4m3(const float *a_dev, int rows, int cols, unsigned char *q_dev, float *scale_dev,
                                   void *stream)
{
    if (!a_dev || !q_dev || !scale_dev) return fail(DNNMG_EINVAL, "a, q and scale must not be NULL");
    if (rows < 1 || cols < 1) return fail(DNNMG_EINVAL, "rows and cols must be >= 1 (got %d, %d)", rows, cols);
    HIP_OR_FAIL(launch_quantize(a_dev, rows, cols, q_dev, scale_dev, (hipStream_t)stream));
    return DNNMG_OK;
}

extern "C" int dnnmg_batch_captures(const dnnmg_batch *b)
{
    return b ? b->captures : -1;
}

extern "C" int dnnmg_step_batch(dnnmg_batch *b, dnnmg_ctx *const *ctxs, int nflows, const float *const *v,
                                const float *const *p, float *const *d_out, void *stream)
{
    int rc = dnnmg_batch_prepare(b, ctxs, nflows, v, p, d_out, nullptr, stream);
    if (rc) return rc;
    return dnnmg_batch_launch(b, 0, stream);
}
