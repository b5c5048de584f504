// Per-patch GRU (Eq. (gru), no biases) and MLP head on gfx950 matrix cores.
//
//   z  = sigma(W_z x + U_z h)          r = sigma(W_r x + U_r h)
//   h' = z h + (1 - z) tanh(W_h x + U_h (r h))
//   d  = M2 relu(M1 h')   (or M h')
//
// Patches are the rows of tall-skinny products.  A workgroup takes 64 patch
// rows; each of its four wave64s owns 16 of them and runs the whole chain on
// 16 x 16 MFMA tiles with FP32 accumulation:
//   phase 1: [x | h] against the stacked gate weights [W_g | U_g] (U_h part 0),
//   gates in registers, r*h to LDS (rows private to the wave),
//   phase 2: (r*h) against U_h, then the update of h (FP32 state),
//   MLP: h' -> LDS -> M1 -> relu -> LDS -> M2 -> per-patch output.
// Operands are FP32 (v_mfma_f32_16x16x4_f32) or BF16 with round-to-nearest-
// even (v_mfma_f32_16x16x32_bf16).  Weights are pre-packed at create time
// into per-lane fragments so that each lane reads 16 contiguous bytes.
//
// Fragment convention (both forms): in k-chunk kc, lane l = i + 16 q holds
// operand values at k = kc*KC + q*KQ + e, e < KQ (A: row i; B: column i).
// The 16 x 16 f32 result tile gives lane l rows 4 q + e (e < 4) of column i.
#include "device.h"
#include "fp8.h"
#include "internal.h"
#include "net_index.h"

namespace dnnmg {


template <int PREC> struct Op;

// FP32 operands: a 16-wide k-chunk is four 16x16x4 MFMAs; lane element e of
// the chunk feeds the e-th of them.
template <> struct Op<0> {
    typedef float T;
    typedef f4 Frag;
    static constexpr int KC = 16, KQ = 4;
    __device__ static inline f4 mma(f4 acc, Frag a, Frag b)
    {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc, 0, 0, 0);
        return acc;
    }
    __device__ static inline T cvt(float x) { return x; }
    // A fragment from FP32 global memory (4 contiguous values).
    __device__ static inline Frag load_f32(const float *p) { return *reinterpret_cast<const f4 *>(p); }
    // A fragment of the network input (stored FP32 in this form).
    __device__ static inline Frag load_x(const void *X, size_t off)
    {
        return *reinterpret_cast<const f4 *>(reinterpret_cast<const float *>(X) + off);
    }
    // The same through global address-space pointers.
    __device__ static inline Frag load_f32(gptr<float> p) { return *(gptr<f4>)p; }
    __device__ static inline Frag load_x(gptr<T> X, size_t off) { return *(gptr<f4>)(X + off); }
};

// BF16 operands: one 16x16x32 MFMA per 32-wide k-chunk.
template <> struct Op<1> {
    typedef __bf16 T;
    typedef bf8 Frag;
    static constexpr int KC = 32, KQ = 8;
    __device__ static inline f4 mma(f4 acc, Frag a, Frag b)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    __device__ static inline T cvt(float x) { return (__bf16)x; }
    __device__ static inline Frag load_f32(const float *p)
    {
        f4 u = *reinterpret_cast<const f4 *>(p), w = *reinterpret_cast<const f4 *>(p + 4);
        Frag r;
        r[0] = (__bf16)u.x; r[1] = (__bf16)u.y; r[2] = (__bf16)u.z; r[3] = (__bf16)u.w;
        r[4] = (__bf16)w.x; r[5] = (__bf16)w.y; r[6] = (__bf16)w.z; r[7] = (__bf16)w.w;
        return r;
    }
    // A fragment of the network input (stored BF16 in this form).
    __device__ static inline Frag load_x(const void *X, size_t off)
    {
        return *reinterpret_cast<const bf8 *>(reinterpret_cast<const __bf16 *>(X) + off);
    }
    // The same through global address-space pointers.
    __device__ static inline Frag load_f32(gptr<float> p)
    {
        f4 u = *(gptr<f4>)p, w = *(gptr<f4>)(p + 4);
        Frag r;
        r[0] = (__bf16)u.x; r[1] = (__bf16)u.y; r[2] = (__bf16)u.z; r[3] = (__bf16)u.w;
        r[4] = (__bf16)w.x; r[5] = (__bf16)w.y; r[6] = (__bf16)w.z; r[7] = (__bf16)w.w;
        return r;
    }
    __device__ static inline Frag load_x(gptr<T> X, size_t off) { return *(gptr<bf8>)(X + off); }
};


// One 64-patch tile.  Wave w takes row tiles 2 (w & 1) and 2 (w & 1) + 1 and
// half of the hidden (and MLP output) tiles, w >> 1, so that every weight
// fragment it reads feeds two row tiles and the workgroup reads each weight
// fragment twice.  HMC is the MLP hidden width rounded up to 64, 128 or 256
// (0 without the hidden layer): it sizes the LDS.
template <int PREC, int H, int HMC>
__device__ __forceinline__ void net_tile(const FlowArgs &f, int blk, NetArgs net)
{
    typedef Op<PREC> O;
    typedef typename O::T T;
    typedef typename O::Frag Frag;
    constexpr int KC = O::KC, KQ = O::KQ;
    constexpr int HT = H / 16, HW = HT / 2;    // hidden-unit tiles, per wave
    static_assert(HT % 2 == 0, "hidden tiles split over two wave pairs");
    constexpr int PAD = 16 / sizeof(T);        // 16-byte row padding
    constexpr int LDH = H + PAD;
    constexpr int LDM = HMC + PAD;

    // r*h (phase 2 operand) and the MLP hidden layer share one buffer: the
    // former is dead once phase 2 is done.  Rows are the tile's 64 patches.
    constexpr int LDB = LDH > LDM ? LDH : LDM;
    __shared__ __align__(16) T sBuf[kNetRows * LDB];
    __shared__ __align__(16) T sHp[kNetRows * LDH];
    T *sR = sBuf, *sAm = sBuf;

    const int P = f.nx * f.ny;
    const int nin = net.nin, nout = net.nout, Hm = net.Hm, kc1 = net.kc1;
    const bool reset_after = net.reset_after != 0;
    // (tile_thread(): in the batched tile loop the index math is redone per
    // tile instead of hoisted out of the loop and held in registers)
    const int tid = tile_thread();
    const int wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lq = lane >> 4;
    const int rg = wave & 1, hg = wave >> 1;
    // the flow's buffers through global address-space pointers: global, not
    // flat, memory instructions where the pointers come from the batch table
    typedef __attribute__((address_space(1))) float gfloat;
    const gptr<T> Xg = (gptr<T>)f.X;
    gfloat *const hG = (gfloat *)f.h;
    gfloat *const dG = (gfloat *)f.dpatch;
    const int r0 = 32 * rg;                         // first tile-local row of this wave
    const int rbase = blk * kNetRows + r0;          // first patch row of this wave

    const Frag *B1 = reinterpret_cast<const Frag *>(net.B1);
    const Frag *B2 = reinterpret_cast<const Frag *>(net.B2);
    const Frag *B3 = reinterpret_cast<const Frag *>(net.B3);
    const Frag *B4 = reinterpret_cast<const Frag *>(net.B4);

    // ---- phase 1: [x | h] x [W_g | U_g]^T for g = z, r, h
    f4 az[HW][2], ar[HW][2], ah[HW][2];
#pragma unroll
    for (int t = 0; t < HW; ++t)
#pragma unroll
        for (int q = 0; q < 2; ++q) az[t][q] = ar[t][q] = ah[t][q] = f4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < kc1; ++kc) {
        const int k0 = kc * KC + lq * KQ;
        Frag a[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int arow = rbase + 16 * q + li;      // row this lane supplies operand values for
            if (arow < P && k0 < nin) a[q] = O::load_x(Xg, (size_t)arow * nin + k0);
            else if (arow < P && k0 < nin + H) a[q] = O::load_f32((gptr<float>)(hG + (size_t)arow * H + (k0 - nin)));
            else {
#pragma unroll
                for (int e = 0; e < KQ; ++e) a[q][e] = O::cvt(0.f);
            }
        }
#pragma unroll
        for (int tw = 0; tw < HW; ++tw) {
            const int t = hg * HW + tw;
            const Frag wz = B1[((0 * HT + t) * kc1 + kc) * 64 + lane];
            const Frag wr = B1[((1 * HT + t) * kc1 + kc) * 64 + lane];
            const Frag wh = B1[((2 * HT + t) * kc1 + kc) * 64 + lane];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                az[tw][q] = O::mma(az[tw][q], a[q], wz);
                ar[tw][q] = O::mma(ar[tw][q], a[q], wr);
                ah[tw][q] = O::mma(ah[tw][q], a[q], wh);
            }
        }
    }

    // ---- gates; r*h to LDS.  Lane holds rows 16 q + 4 lq + e (of the
    //      wave's 32), column 16 t + li.
    float hold[HW][2][4];
#pragma unroll
    for (int tw = 0; tw < HW; ++tw)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int lr = r0 + 16 * q + 4 * lq + e, row = blk * kNetRows + lr, k = 16 * (hg * HW + tw) + li;
                const float h0 = row < P ? hG[(size_t)row * H + k] : 0.f;
                hold[tw][q][e] = h0;
                // (BF16 weights come pre-multiplied for 2^x, see sigmoid_l2)
                az[tw][q][e] = PREC == 1 ? sigmoid_l2(az[tw][q][e]) : sigmoid(az[tw][q][e]);
                const float r = PREC == 1 ? sigmoid_l2(ar[tw][q][e]) : sigmoid(ar[tw][q][e]);
                // reset after U_h: phase 2 takes h itself, r stays for the candidate
                ar[tw][q][e] = r;
                sR[lr * LDH + k] = O::cvt(reset_after ? h0 : r * h0);
            }
    __syncthreads();

    // ---- phase 2: (r*h) x U_h^T (or h x U_h^T, then times r); update h
    f4 au[HW][2];
#pragma unroll
    for (int tw = 0; tw < HW; ++tw)
#pragma unroll
        for (int q = 0; q < 2; ++q) au[tw][q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < H / KC; ++kc) {
        Frag a[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) a[q] = *reinterpret_cast<const Frag *>(&sR[(r0 + 16 * q + li) * LDH + kc * KC + lq * KQ]);
#pragma unroll
        for (int tw = 0; tw < HW; ++tw) {
            const Frag w = B2[((hg * HW + tw) * (H / KC) + kc) * 64 + lane];
#pragma unroll
            for (int q = 0; q < 2; ++q) au[tw][q] = O::mma(au[tw][q], a[q], w);
        }
    }
#pragma unroll
    for (int tw = 0; tw < HW; ++tw)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int lr = r0 + 16 * q + 4 * lq + e, row = blk * kNetRows + lr, k = 16 * (hg * HW + tw) + li;
                const float z = az[tw][q][e];
                const float u = reset_after ? ar[tw][q][e] * au[tw][q][e] : au[tw][q][e];
                const float hh = PREC == 1 ? tanh_l2(ah[tw][q][e] + u) : fast_tanh(ah[tw][q][e] + u);
                const float hn = hh + z * (hold[tw][q][e] - hh);   // z h + (1 - z) hh
                if (row < P) hG[(size_t)row * H + k] = hn;
                sHp[lr * LDH + k] = O::cvt(hn);
            }
    __syncthreads();

    // ---- MLP head; the wave pair hg takes every other output tile
    const int ot_n = (nout + 15) / 16;
    auto out_tile = [&](int ot, const T *src, int ld, int kcn, const Frag *Bw) {
        f4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
        for (int kc = 0; kc < kcn; ++kc) {
            const Frag w = Bw[(ot * kcn + kc) * 64 + lane];
#pragma unroll
            for (int q = 0; q < 2; ++q)
                acc[q] = O::mma(acc[q], *reinterpret_cast<const Frag *>(&src[(r0 + 16 * q + li) * ld + kc * KC + lq * KQ]), w);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = rbase + 16 * q + 4 * lq + e, o = 16 * ot + li;
                if (row < P && o < nout) dG[(size_t)row * nout + o] = acc[q][e];
            }
    };
    if constexpr (HMC > 0) {
        for (int mt = hg; mt < Hm / 16; mt += 2) {
            f4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
            for (int kc = 0; kc < H / KC; ++kc) {
                const Frag w = B3[(mt * (H / KC) + kc) * 64 + lane];
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    acc[q] = O::mma(acc[q], *reinterpret_cast<const Frag *>(&sHp[(r0 + 16 * q + li) * LDH + kc * KC + lq * KQ]), w);
            }
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    sAm[(r0 + 16 * q + 4 * lq + e) * LDM + 16 * mt + li] = O::cvt(fmaxf(acc[q][e], 0.f));
        }
        __syncthreads();
        for (int ot = hg; ot < ot_n; ot += 2) out_tile(ot, sAm, LDM, Hm / KC, B4);
    } else {
        for (int ot = hg; ot < ot_n; ot += 2) out_tile(ot, sHp, LDH, H / KC, B3);
    }
}

// MLP hidden width class of the generic kernel (LDS sizing).
static constexpr int hm_class(int Hm) { return Hm == 0 ? 0 : (Hm <= 64 ? 64 : (Hm <= 128 ? 128 : 256)); }

// Waves per SIMD of the generic kernel: two workgroups per CU where the LDS
// allows it.
template <int PREC, int H, int HMC>
constexpr int net_waves()
{
    constexpr int sz = PREC == 0 ? 4 : 2, pad = 16 / sz, ldh = H + pad, ldm = HMC + pad;
    return kNetRows * ((ldh > ldm ? ldh : ldm) + ldh) * sz <= 80 * 1024 ? 2 : 1;
}

// Single flow: one tile per block.  Batched: the blocks stride over the
// table's tiles of all flows, so the grid need not match the batch.
template <int PREC, int H, int HMC, bool BATCHED>
__global__ __launch_bounds__(kThreads, (net_waves<PREC, H, HMC>())) void k_net(FlowArgs single, const BatchTable *__restrict__ bt, NetArgs net)
{
    if (!BATCHED) {
        net_tile<PREC, H, HMC>(single, blockIdx.x, net);
        return;
    }
    const int total = bt->prefix[kKindNet][bt->nflows];
#pragma unroll 1
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        int blk = g;
        const FlowArgs &f = *batch_flow(bt, kKindNet, blk);
        net_tile<PREC, H, HMC>(f, blk, net);
        __syncthreads();   // LDS is reused by the next tile
    }
}


// ---------------------------------------------------------------- FP8 E4M3
// Every product takes E4M3 operands with one FP32 scale per row and
// accumulates in FP32: weights per output row (packed at create), the
// network input per patch (quantised by the defect kernel), and the state h,
// r*h, h' and the MLP hidden layer per patch, quantised here.  The input and
// the state of the gate products carry separate scales, so their k-chunks are
// accumulated separately: the input part is rescaled by s_x / s_h before the
// state part is added, and the sum by s_h s_w at the end.
typedef long f8x8;   // 8 E4M3 codes: one MFMA operand fragment

__device__ inline f8x8 mma_fp8_operand(const uint8_t *p) { return *reinterpret_cast<const f8x8 *>(p); }

__device__ inline f4 mma_fp8(f4 acc, f8x8 a, f8x8 b)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, acc, 0, 0, 0);
}

// Row maximum over the 16 lanes that share lq (the 16 columns of a tile).
__device__ inline float max16(float m)
{
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) m = fmaxf(m, __shfl_xor(m, o));
    return m;
}

template <int H>
__device__ __forceinline__ void net_tile_fp8(const FlowArgs &f, int blk, NetArgs net)
{
    constexpr int KC = 32, KQ = 8, HT = H / 16, HC = H / 32;
    constexpr int LDH = H + 16;                // bytes per staged row (16-byte padding)
    constexpr int LDM = 256 + 16;
    constexpr int MT_MAX = 256 / 16;           // MLP hidden tiles (Hm <= 256)
    __shared__ __align__(16) uint8_t sR[4][16 * LDH];
    __shared__ __align__(16) uint8_t sHp[4][16 * LDH];
    __shared__ __align__(16) uint8_t sAm[4][16 * LDM];

    const int P = f.nx * f.ny;
    const int nin = net.nin, nout = net.nout, Hm = net.Hm, kc1 = net.kc1;
    const int XS = xstride_fp8(nin), kcx = XS / KC;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 15, lq = lane >> 4;
    const int rbase = blk * kNetRows + wave * 16;   // first patch row of this wave
    const int arow = rbase + li;                    // row this lane supplies A values for
    const bool aok = arow < P;
    const uint8_t *X8 = reinterpret_cast<const uint8_t *>(f.X);
    const f8x8 *B1 = reinterpret_cast<const f8x8 *>(net.B1);
    const f8x8 *B2 = reinterpret_cast<const f8x8 *>(net.B2);
    const f8x8 *B3 = reinterpret_cast<const f8x8 *>(net.B3);
    const f8x8 *B4 = reinterpret_cast<const f8x8 *>(net.B4);

    // ---- the state row of this lane's A row: scale and codes
    float hv[HC][KQ];
    float mh = 0.0f;
#pragma unroll
    for (int kh = 0; kh < HC; ++kh)
#pragma unroll
        for (int e = 0; e < KQ; ++e) {
            hv[kh][e] = aok ? f.h[(size_t)arow * H + kh * KC + lq * KQ + e] : 0.0f;
            mh = fmaxf(mh, fabsf(hv[kh][e]));
        }
    mh = fmaxf(mh, __shfl_xor(mh, 16));
    mh = fmaxf(mh, __shfl_xor(mh, 32));
    mh = fmaxf(mh, kFp8MinMax);
    const float rh_li = 448.0f / mh, sh_li = mh / 448.0f;
    f8x8 qh[HC];
#pragma unroll
    for (int kh = 0; kh < HC; ++kh) {
        const uint32_t lo = pack4_e4m3(hv[kh][0] * rh_li, hv[kh][1] * rh_li, hv[kh][2] * rh_li, hv[kh][3] * rh_li);
        const uint32_t hi = pack4_e4m3(hv[kh][4] * rh_li, hv[kh][5] * rh_li, hv[kh][6] * rh_li, hv[kh][7] * rh_li);
        qh[kh] = (f8x8)(((unsigned long)hi << 32) | lo);
    }

    // ---- phase 1, input chunks: x . [W_z W_r W_h]
    f4 az[HT], ar[HT], ah[HT];
#pragma unroll
    for (int t = 0; t < HT; ++t) az[t] = ar[t] = ah[t] = f4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < kcx; ++kc) {
        const f8x8 a = aok ? mma_fp8_operand(X8 + (size_t)arow * XS + kc * KC + lq * KQ) : 0;
#pragma unroll
        for (int t = 0; t < HT; ++t) {
            az[t] = mma_fp8(az[t], a, B1[((0 * HT + t) * kc1 + kc) * 64 + lane]);
            ar[t] = mma_fp8(ar[t], a, B1[((1 * HT + t) * kc1 + kc) * 64 + lane]);
            ah[t] = mma_fp8(ah[t], a, B1[((2 * HT + t) * kc1 + kc) * 64 + lane]);
        }
    }
    // accumulator element e is patch row rbase + 4 lq + e
    float sx[4], sh[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = rbase + 4 * lq + e;
        sx[e] = row < P ? f.sx[row] : 1.0f;
        sh[e] = __shfl(sh_li, 4 * lq + e);
        const float ratio = sx[e] / sh[e];
#pragma unroll
        for (int t = 0; t < HT; ++t) { az[t][e] *= ratio; ar[t][e] *= ratio; }
    }
    // ---- phase 1, state chunks: h . [U_z U_r] (the candidate has no U block here)
#pragma unroll
    for (int kh = 0; kh < HC; ++kh)
#pragma unroll
        for (int t = 0; t < HT; ++t) {
            az[t] = mma_fp8(az[t], qh[kh], B1[((0 * HT + t) * kc1 + kcx + kh) * 64 + lane]);
            ar[t] = mma_fp8(ar[t], qh[kh], B1[((1 * HT + t) * kc1 + kcx + kh) * 64 + lane]);
        }

    // ---- gates; r*h.  Lane holds rows rbase + 4 lq + e, column 16 t + li.
    float hold[HT][4];
    float mr[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < HT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = rbase + 4 * lq + e, k = 16 * t + li;
            const float h0 = row < P ? f.h[(size_t)row * H + k] : 0.f;
            hold[t][e] = h0;
            az[t][e] = sigmoid(az[t][e] * sh[e] * net.s1[k]);
            const float rh = sigmoid(ar[t][e] * sh[e] * net.s1[H + k]) * h0;
            ar[t][e] = rh;
            mr[e] = fmaxf(mr[e], fabsf(rh));
            ah[t][e] *= sx[e] * net.s1[2 * H + k];
        }
    float srh[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float m = fmaxf(max16(mr[e]), kFp8MinMax);
        const float r = 448.0f / m;
        srh[e] = m / 448.0f;
#pragma unroll
        for (int t = 0; t < HT; ++t) sR[wave][(4 * lq + e) * LDH + 16 * t + li] = to_e4m3(ar[t][e] * r);
    }
    __syncthreads();

    // ---- phase 2: (r*h) . U_h^T; new state
    f4 au[HT];
#pragma unroll
    for (int t = 0; t < HT; ++t) au[t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < HC; ++kc) {
        const f8x8 a = mma_fp8_operand(&sR[wave][li * LDH + kc * KC + lq * KQ]);
#pragma unroll
        for (int t = 0; t < HT; ++t) au[t] = mma_fp8(au[t], a, B2[(t * HC + kc) * 64 + lane]);
    }
    float mp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < HT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = rbase + 4 * lq + e, k = 16 * t + li;
            const float z = az[t][e];
            const float hh = fast_tanh(ah[t][e] + au[t][e] * srh[e] * net.s2[k]);
            const float hn = hh + z * (hold[t][e] - hh);   // z h + (1 - z) hh
            if (row < P) f.h[(size_t)row * H + k] = hn;
            au[t][e] = hn;
            mp[e] = fmaxf(mp[e], fabsf(hn));
        }
    float shp[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float m = fmaxf(max16(mp[e]), kFp8MinMax);
        const float r = 448.0f / m;
        shp[e] = m / 448.0f;
#pragma unroll
        for (int t = 0; t < HT; ++t) sHp[wave][(4 * lq + e) * LDH + 16 * t + li] = to_e4m3(au[t][e] * r);
    }
    __syncthreads();

    // ---- MLP head
    const int ot_n = (nout + 15) / 16;
    const uint8_t *src = sHp[wave];
    int lds = LDH, kcs = HC;
    const f8x8 *Bo = B3;
    const float *so = net.s3;
    float sin_[4] = {shp[0], shp[1], shp[2], shp[3]};
    if (Hm > 0) {
        float am[MT_MAX][4];
        float ma[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mt = 0; mt < MT_MAX; ++mt) {
            if (mt < Hm / 16) {
                f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kc = 0; kc < HC; ++kc) {
                    const f8x8 a = mma_fp8_operand(&sHp[wave][li * LDH + kc * KC + lq * KQ]);
                    acc = mma_fp8(acc, a, B3[(mt * HC + kc) * 64 + lane]);
                }
                const float sw = net.s3[16 * mt + li];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    am[mt][e] = fmaxf(acc[e] * shp[e] * sw, 0.f);
                    ma[e] = fmaxf(ma[e], am[mt][e]);
                }
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float m = fmaxf(max16(ma[e]), kFp8MinMax);
            const float r = 448.0f / m;
            sin_[e] = m / 448.0f;
#pragma unroll
            for (int mt = 0; mt < MT_MAX; ++mt)
                if (mt < Hm / 16) sAm[wave][(4 * lq + e) * LDM + 16 * mt + li] = to_e4m3(am[mt][e] * r);
        }
        __syncthreads();
        src = sAm[wave];
        lds = LDM;
        kcs = Hm / KC;
        Bo = B4;
        so = net.s4;
    }
    for (int ot = 0; ot < ot_n; ++ot) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int kc = 0; kc < kcs; ++kc) {
            const f8x8 a = mma_fp8_operand(&src[li * lds + kc * KC + lq * KQ]);
            acc = mma_fp8(acc, a, Bo[(ot * kcs + kc) * 64 + lane]);
        }
        const int o = 16 * ot + li;
        if (o < nout) {
            const float sw = so[o];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = rbase + 4 * lq + e;
                if (row < P) f.dpatch[(size_t)row * nout + o] = acc[e] * sin_[e] * sw;
            }
        }
    }
}

// Stage entry point: the per-row activation quantiser of the FP8 form on its
// own, one workgroup per row.
__global__ __launch_bounds__(kThreads) void k_quantize(const float *a, int rows, int cols, uint8_t *q, float *s)
{
    __shared__ float sm[kThreads / 64];
    const int row = blockIdx.x;
    const float *ar = a + (size_t)row * cols;
    float m = 0.0f;
    for (int k = threadIdx.x; k < cols; k += kThreads) m = fmaxf(m, fabsf(ar[k]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    m = fmaxf(fmaxf(sm[0], sm[1]), fmaxf(sm[2], sm[3]));
    m = fmaxf(m, kFp8MinMax);
    const float r = 448.0f / m;
    if (threadIdx.x == 0) s[row] = m / 448.0f;
    for (int k = threadIdx.x; k < cols; k += kThreads) q[(size_t)row * cols + k] = to_e4m3(ar[k] * r);
}

hipError_t launch_quantize(const float *a, int rows, int cols, uint8_t *q, float *s, hipStream_t st)
{
    hipLaunchKernelGGL(k_quantize, dim3(rows), dim3(kThreads), 0, st, a, rows, cols, q, s);
    return hipGetLastError();
}

template <int H, bool BATCHED>
__global__ __launch_bounds__(kThreads) void k_net_fp8(FlowArgs single, const BatchTable *__restrict__ bt, NetArgs net)
{
    if (!BATCHED) {
        net_tile_fp8<H>(single, blockIdx.x, net);
        return;
    }
    const int total = bt->prefix[kKindNet][bt->nflows];
#pragma unroll 1
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        int blk = g;
        const FlowArgs &f = *batch_flow(bt, kKindNet, blk);
        net_tile_fp8<H>(f, blk, net);
        __syncthreads();   // LDS is reused by the next tile
    }
}

// Persistent BF16 kernel for H = 64 (and Hm 0 or 64).  Eight waves: wave w
// owns hidden tile w % 4 for row tiles 2 (w / 4) and 2 (w / 4) + 1 of each
// 64-patch tile, and keeps that hidden tile's weight fragments (three gates,
// U_h, M1 and M2 / M) in registers for the whole launch.  The workgroup loops
// over 64-patch row tiles staged through LDS, so each weight fragment is read
// from memory once per workgroup.
constexpr int kNetH64Threads = 512;

template <int K>
__global__ __launch_bounds__(kNetH64Threads, 2) void k_net_h64(FlowArgs single, const BatchTable *__restrict__ bt, NetArgs net,
                                                               int ntiles)
{
    typedef Op<1> O;
    constexpr int H = 64, KC = 32, KQ = 8, HT = 4, RTW = 2;
    constexpr int n = 1 << K, nf = (n + 1) * (n + 1), nin = 4 * nf + 4, nout = 2 * nf;
    if (bt) ntiles = bt->prefix[kKindNet][bt->nflows];   // batched: the table's row tiles
    constexpr int KC1 = (nin + H + KC - 1) / KC;
    constexpr int LDA = KC1 * KC + 8;          // +16 bytes per row
    constexpr int LDH = H + 8;
    constexpr int OT = (nout + 15) / 16;       // output tiles (<= 4 here)
    constexpr int PADK = KC1 * KC - nin - H;
    static_assert(OT <= 4, "one output tile per hidden-tile slot");

    __shared__ __align__(16) __bf16 sA[64 * LDA];
    constexpr int LDS32 = H + 4;              // FP32 state rows, padded against bank conflicts
    __shared__ __align__(16) float sH[64 * LDS32];
    __shared__ __align__(16) __bf16 sR[64 * LDH];
    __shared__ __align__(16) __bf16 sHp[64 * LDH];
    __shared__ __align__(16) __bf16 sAm[64 * LDH];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lq = lane >> 4;
    const int ht = wave & 3, rt0 = RTW * (wave >> 2);
    const int Hm = net.Hm;
    const bf8 *B1 = reinterpret_cast<const bf8 *>(net.B1);
    const bf8 *B2 = reinterpret_cast<const bf8 *>(net.B2);
    const bf8 *B3 = reinterpret_cast<const bf8 *>(net.B3);
    const bf8 *B4 = reinterpret_cast<const bf8 *>(net.B4);

    // gate and U_h fragments in registers; the MLP fragments in LDS
    __shared__ __align__(16) bf8 sW3[4 * (H / KC) * 64];
    __shared__ __align__(16) bf8 sW4[4 * (H / KC) * 64];
    bf8 w1[3][KC1], w2[H / KC];
#pragma unroll
    for (int g = 0; g < 3; ++g)
#pragma unroll
        for (int kc = 0; kc < KC1; ++kc) w1[g][kc] = B1[((g * HT + ht) * KC1 + kc) * 64 + lane];
#pragma unroll
    for (int kc = 0; kc < H / KC; ++kc) w2[kc] = B2[(ht * (H / KC) + kc) * 64 + lane];
    for (int t = tid; t < 4 * (H / KC) * 64; t += kNetH64Threads) {
        const int tile_m = t / ((H / KC) * 64);
        sW3[t] = (Hm > 0 || tile_m < OT) ? B3[t] : bf8{};
        sW4[t] = (Hm > 0 && tile_m < OT) ? B4[t] : bf8{};
    }

    // Tiles are contiguous in memory: the network input (BF16, 64 x nin) and
    // the state (FP32, 64 x H).  Each thread prefetches its 16-byte pieces of
    // the next two tiles into two register buffers while the current one is
    // computed, so two tiles' loads are in flight per workgroup.
    constexpr int XCH = 64 * nin / 8, HCH = 64 * H / 4;            // 16-byte pieces per tile
    constexpr int XPT = (XCH + kNetH64Threads - 1) / kNetH64Threads;
    constexpr int HPT = (HCH + kNetH64Threads - 1) / kNetH64Threads;
    bf8 xrA[XPT], xrB[XPT];
    f4 hrA[HPT], hrB[HPT];
    // A row tile's buffers.  The fields are read in two branches: a pointer
    // that may point at either the kernel argument or the batch table would
    // make them flat loads (and the lambdas below would reach the argument
    // through a generic pointer).
    typedef __attribute__((address_space(1))) float gfloat;
    struct Rows {
        gptr<bf8> X;
        gfloat *h, *dp;
        int nrows;
    };
    const void *const s_X = single.X;
    float *const s_h = single.h, *const s_dp = single.dpatch;
    const int s_P = single.nx * single.ny;
    auto rows_of = [&](int tile) -> Rows {
        int blk = tile;
        const void *X;
        float *h, *dp;
        int P;
        if (bt) {
            const FlowArgs &F = *batch_flow(bt, kKindNet, blk);
            X = F.X; h = F.h; dp = F.dpatch; P = F.nx * F.ny;
        } else {
            X = s_X; h = s_h; dp = s_dp; P = s_P;
        }
        const int row0 = blk * 64;
        Rows r;
        r.X = (gptr<bf8>)(reinterpret_cast<const __bf16 *>(X) + (size_t)row0 * nin);
        r.h = (gfloat *)(h + (size_t)row0 * H);
        r.dp = (gfloat *)(dp + (size_t)row0 * nout);
        r.nrows = min(64, P - row0);
        return r;
    };
    // (index math from tile_thread(): recomputed in each tile instead of
    // hoisted out of the tile loop and held in registers)
    typedef __attribute__((address_space(1))) const f4 gf4;
    auto load_tile = [&](int tile, bf8 (&xr)[XPT], f4 (&hr)[HPT]) {
        const Rows rw = rows_of(tile);
        const int t0 = tile_thread();
#pragma unroll
        for (int i = 0; i < XPT; ++i) {
            const int c = t0 + i * kNetH64Threads;
            xr[i] = tile_piece_in(c, nin / 8, rw.nrows) ? rw.X[c] : bf8{};
        }
#pragma unroll
        for (int i = 0; i < HPT; ++i) {
            const int c = t0 + i * kNetH64Threads;
            hr[i] = tile_piece_in(c, H / 4, rw.nrows) ? ((gf4 *)rw.h)[c] : f4{0.f, 0.f, 0.f, 0.f};
        }
    };
    // the k-padding columns of [x | h] stay zero for the whole launch
    if (PADK > 0)
        for (int t = tid; t < 64 * PADK; t += kNetH64Threads) sA[(t / PADK) * LDA + nin + H + t % PADK] = (__bf16)0.f;
    const int G = gridDim.x;
    if (blockIdx.x < ntiles) load_tile(blockIdx.x, xrA, hrA);
    if (blockIdx.x + G < ntiles) load_tile(blockIdx.x + G, xrB, hrB);

    // one 64-patch tile: stage the prefetched registers, refill them with
    // tile `next`, compute
    auto process = [&](int tile, bf8 (&xr)[XPT], f4 (&hr)[HPT], int next) {
        const Rows rw = rows_of(tile);
        const int nrows = rw.nrows;
        gfloat *const hg = rw.h;
        gfloat *const dp = rw.dp;

        __syncthreads();   // the previous tile's readers of LDS are done
        const int t1 = tile_thread();
#pragma unroll
        for (int i = 0; i < XPT; ++i) {
            const int c = t1 + i * kNetH64Threads;
            if (c < XCH) *reinterpret_cast<bf8 *>(&sA[(c / (nin / 8)) * LDA + 8 * (c % (nin / 8))]) = xr[i];
        }
#pragma unroll
        for (int i = 0; i < HPT; ++i) {
            const int c = t1 + i * kNetH64Threads;
            if (c < HCH) {
                const int r = c / (H / 4), k = 4 * (c % (H / 4));
                *reinterpret_cast<f4 *>(&sH[r * LDS32 + k]) = hr[i];
                bf4 hb;
                hb[0] = (__bf16)hr[i].x; hb[1] = (__bf16)hr[i].y; hb[2] = (__bf16)hr[i].z; hb[3] = (__bf16)hr[i].w;
                *reinterpret_cast<bf4 *>(&sA[r * LDA + nin + k]) = hb;
            }
        }
        if (next < ntiles) load_tile(next, xr, hr);
        __syncthreads();

        // The products are formed transposed (weights x activations^T), so the
        // 16 x 16 result tile gives lane (li, lq) patch row 16 rt + li and the
        // four consecutive hidden units 16 ht + 4 lq + e: gate inputs, r*h, h'
        // and the MLP activations move as 8- and 16-byte vectors.
        const int ucol = 16 * ht + 4 * lq;       // first of this lane's four units
        // ---- phase 1: the three gates of this wave's hidden tile
        f4 az[RTW], ar[RTW], ah[RTW];
#pragma unroll
        for (int q = 0; q < RTW; ++q) az[q] = ar[q] = ah[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < KC1; ++kc)
#pragma unroll
            for (int q = 0; q < RTW; ++q) {
                const bf8 a = *reinterpret_cast<const bf8 *>(&sA[(16 * (rt0 + q) + li) * LDA + kc * KC + lq * KQ]);
                az[q] = O::mma(az[q], w1[0][kc], a);
                ar[q] = O::mma(ar[q], w1[1][kc], a);
                ah[q] = O::mma(ah[q], w1[2][kc], a);
            }
        f4 hold[RTW];
#pragma unroll
        for (int q = 0; q < RTW; ++q) {
            const int r = 16 * (rt0 + q) + li;
            hold[q] = *reinterpret_cast<const f4 *>(&sH[r * LDS32 + ucol]);
            bf4 rh;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                az[q][e] = sigmoid_l2(az[q][e]);
                rh[e] = (__bf16)(sigmoid_l2(ar[q][e]) * hold[q][e]);
            }
            *reinterpret_cast<bf4 *>(&sR[r * LDH + ucol]) = rh;
        }
        __syncthreads();

        // ---- phase 2: U_h (r*h); new state
#pragma unroll
        for (int q = 0; q < RTW; ++q) {
            const int r = 16 * (rt0 + q) + li;
            f4 au = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < H / KC; ++kc) {
                const bf8 a = *reinterpret_cast<const bf8 *>(&sR[r * LDH + kc * KC + lq * KQ]);
                au = O::mma(au, w2[kc], a);
            }
            f4 hn;
            bf4 hb;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float z = az[q][e];
                // h' = z h + (1 - z) c = c + z (h - c), c the candidate state
                const float c = tanh_l2(ah[q][e] + au[e]);
                hn[e] = c + z * (hold[q][e] - c);
                hb[e] = (__bf16)hn[e];
            }
            if (r < nrows) *(__attribute__((address_space(1))) f4 *)(hg + r * H + ucol) = hn;
            *reinterpret_cast<bf4 *>(&sHp[r * LDH + ucol]) = hb;
        }
        __syncthreads();

        // ---- MLP head
        const __bf16 *src = sHp;
        if (Hm > 0) {
#pragma unroll
            for (int q = 0; q < RTW; ++q) {
                const int r = 16 * (rt0 + q) + li;
                f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kc = 0; kc < H / KC; ++kc) {
                    const bf8 a = *reinterpret_cast<const bf8 *>(&sHp[r * LDH + kc * KC + lq * KQ]);
                    acc = O::mma(acc, sW3[(ht * (H / KC) + kc) * 64 + lane], a);
                }
                bf4 m;
#pragma unroll
                for (int e = 0; e < 4; ++e) m[e] = (__bf16)fmaxf(acc[e], 0.f);
                *reinterpret_cast<bf4 *>(&sAm[r * LDH + ucol]) = m;
            }
            __syncthreads();
            src = sAm;
        }
        if (ht < OT) {
#pragma unroll
            for (int q = 0; q < RTW; ++q) {
                const int r = 16 * (rt0 + q) + li;
                f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kc = 0; kc < H / KC; ++kc) {
                    const bf8 a = *reinterpret_cast<const bf8 *>(&src[r * LDH + kc * KC + lq * KQ]);
                    acc = O::mma(acc, Hm > 0 ? sW4[(ht * (H / KC) + kc) * 64 + lane] : sW3[(ht * (H / KC) + kc) * 64 + lane], a);
                }
                // nout is even: the pairs (ucol, ucol+1), (ucol+2, ucol+3) are inside or outside together
                if (r < nrows) {
                    typedef float v2 __attribute__((ext_vector_type(2)));
                    typedef __attribute__((address_space(1))) v2 gv2;
                    gfloat *o = dp + r * nout + ucol;
                    if (ucol < nout) *(gv2 *)o = v2{acc[0], acc[1]};
                    if (ucol + 2 < nout) *(gv2 *)(o + 2) = v2{acc[2], acc[3]};
                }
            }
        }
    };
    for (int tile = blockIdx.x; tile < ntiles; tile += 2 * G) {
        process(tile, xrA, hrA, tile + 2 * G);
        if (tile + G < ntiles) process(tile + G, xrB, hrB, tile + 3 * G);
    }
}

// Persistent FP8 kernel (H = 64 or 128, Hm = 0 or H, K <= 3).  Eight waves:
// wave w owns hidden tile w % HT for 4 / (8 / HT) row tiles of each 64-patch
// tile and keeps that hidden tile's gate and U_h fragments in registers for
// the whole launch (90 VGPRs at K = 3, H = 128: the FP8 weights that BF16
// could not keep resident); the MLP fragments live in LDS.  Products are
// formed transposed (weights x activations^T) as in k_net_h64, so a lane
// holds one patch row and four consecutive units; the per-patch row maxima
// of the quantised activations are reduced over lanes and then over the
// waves of the row through LDS.
template <int K, int H, int HM>
__global__ __launch_bounds__(kNetH64Threads, 2) void k_net_q8p(FlowArgs single, const BatchTable *__restrict__ bt,
                                                               NetArgs net, int ntiles)
{
    constexpr int n = 1 << K, nf = (n + 1) * (n + 1), nin = 4 * nf + 4, nout = 2 * nf;
    constexpr int KC = 32, KQ = 8;
    constexpr int XS = xstride_fp8(nin), KCX = XS / KC, HC = H / KC, KC1 = KCX + HC;
    // wave w: hidden tile w % HT, row tiles RTW (w / HT) .. + RTW - 1 of a pass;
    // a 64-patch tile takes PASSES passes (2 at H = 128, to bound registers)
    constexpr int HT = H / 16, WPH = 8 / HT, RTW = 2, PASSES = 4 / (WPH * RTW);
    constexpr int OT = (nout + 15) / 16;
    constexpr int MC = HM / KC;
    constexpr int LDX = XS + 16, LDQ = H + 16, LDS32 = H + 4;
    constexpr int W3N = (HM > 0 ? HM / 16 : OT) * HC * 64, W4N = HM > 0 ? OT * MC * 64 : 1;
    static_assert(HM == 0 || HM == H, "MLP hidden tiles follow the hidden tiles");
    if (bt) ntiles = bt->prefix[kKindNet][bt->nflows];   // batched: the table's row tiles

    __shared__ __align__(16) uint8_t sX[64 * LDX];       // network input codes of the tile
    __shared__ __align__(16) float sH[64 * LDS32];       // FP32 state of the tile
    __shared__ __align__(16) uint8_t sQ[64 * LDQ];       // state codes, then r*h codes
    __shared__ __align__(16) uint8_t sHp[64 * LDQ];      // h' codes
    __shared__ __align__(16) uint8_t sAm[64 * LDQ];      // MLP hidden codes
    __shared__ __align__(16) f8x8 sW3[W3N];
    __shared__ __align__(16) f8x8 sW4[W4N];
    __shared__ float sMax[HT * 64];                     // per-wave partial row maxima
    __shared__ float sSx[64], sSh[64];                  // row scales of x and h

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lq = lane >> 4;
    const int ht = wave % HT, rt0 = RTW * (wave / HT);   // row-tile offset within a pass
    const int ucol = 16 * ht + 4 * lq;                  // first of this lane's four units
    const f8x8 *B1 = reinterpret_cast<const f8x8 *>(net.B1);
    const f8x8 *B2 = reinterpret_cast<const f8x8 *>(net.B2);
    const f8x8 *B3 = reinterpret_cast<const f8x8 *>(net.B3);
    const f8x8 *B4 = reinterpret_cast<const f8x8 *>(net.B4);

    f8x8 wz[KC1], wr[KC1], wh[KCX], w2[HC];
#pragma unroll
    for (int kc = 0; kc < KC1; ++kc) {
        wz[kc] = B1[((0 * HT + ht) * KC1 + kc) * 64 + lane];
        wr[kc] = B1[((1 * HT + ht) * KC1 + kc) * 64 + lane];
    }
#pragma unroll
    for (int kc = 0; kc < KCX; ++kc) wh[kc] = B1[((2 * HT + ht) * KC1 + kc) * 64 + lane];
#pragma unroll
    for (int kc = 0; kc < HC; ++kc) w2[kc] = B2[(ht * HC + kc) * 64 + lane];
    for (int t = tid; t < W3N; t += kNetH64Threads) sW3[t] = B3[t];
    for (int t = tid; t < W4N; t += kNetH64Threads) sW4[t] = HM > 0 ? B4[t] : 0;
    // per-unit weight scales: read where they are used (global, cached)
    const gptr<float> S1 = pinned<float>(net.s1), S2 = pinned<float>(net.s2);

    // A row tile's buffers.  The fields are read in two branches: a pointer
    // that may point at either the kernel argument or the batch table would
    // make them flat loads (and the lambdas below would reach the argument
    // through a generic pointer).
    typedef __attribute__((address_space(1))) float gfloat;
    struct Rows {
        gptr<uint8_t> X;
        gptr<float> sx;
        gfloat *h, *dp;
        int nrows;
    };
    const void *const s_X = single.X;
    const float *const s_sx = single.sx;
    float *const s_h = single.h, *const s_dp = single.dpatch;
    const int s_P = single.nx * single.ny;
    auto rows_of = [&](int tile) -> Rows {
        int blk = tile;
        const void *X;
        const float *sxp;
        float *h, *dp;
        int P;
        if (bt) {
            const FlowArgs &F = *batch_flow(bt, kKindNet, blk);
            X = F.X; sxp = F.sx; h = F.h; dp = F.dpatch; P = F.nx * F.ny;
        } else {
            X = s_X; sxp = s_sx; h = s_h; dp = s_dp; P = s_P;
        }
        const int row0 = blk * 64;
        Rows r;
        r.X = (gptr<uint8_t>)(reinterpret_cast<const uint8_t *>(X) + (size_t)row0 * XS);
        r.sx = (gptr<float>)(sxp + row0);
        r.h = (gfloat *)(h + (size_t)row0 * H);
        r.dp = (gfloat *)(dp + (size_t)row0 * nout);
        r.nrows = min(64, P - row0);
        return r;
    };

    // next-tile prefetch into registers: network input codes, FP32 state, x
    // scales (index math from tile_thread(): recomputed in each tile instead
    // of hoisted out of the tile loop and held in registers)
    constexpr int XCH = 64 * XS / 16, HCH = 64 * H / 4;
    constexpr int XPT = (XCH + kNetH64Threads - 1) / kNetH64Threads;
    constexpr int HPT = (HCH + kNetH64Threads - 1) / kNetH64Threads;
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(1))) const u4 gu4;
    typedef __attribute__((address_space(1))) const f4 gf4;
    u4 xr[XPT];
    f4 hr[HPT];
    float sxr = 1.0f;
    auto load_tile = [&](int tile) {
        const Rows rw = rows_of(tile);
        const int t0 = tile_thread();
#pragma unroll
        for (int i = 0; i < XPT; ++i) {
            const int c = t0 + i * kNetH64Threads;
            xr[i] = tile_piece_in(c, XS / 16, rw.nrows) ? ((gu4 *)rw.X)[c] : u4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int i = 0; i < HPT; ++i) {
            const int c = t0 + i * kNetH64Threads;
            hr[i] = tile_piece_in(c, H / 4, rw.nrows) ? ((gf4 *)rw.h)[c] : f4{0.f, 0.f, 0.f, 0.f};
        }
        sxr = t0 < rw.nrows ? rw.sx[t0] : 1.0f;
    };
    if (blockIdx.x < ntiles) load_tile(blockIdx.x);

    // row maximum of |v| over the 16 units a wave holds for its row, then over
    // the HT waves of the row (the caller brackets this with barriers)
    auto wave_max = [&](float m, int row) {
        m = fmaxf(m, __shfl_xor(m, 16));
        m = fmaxf(m, __shfl_xor(m, 32));
        if (lq == 0) sMax[ht * 64 + row] = m;
    };
    auto row_max = [&](int row) {
        float m = kFp8MinMax;
#pragma unroll
        for (int t = 0; t < HT; ++t) m = fmaxf(m, sMax[t * 64 + row]);
        return m;
    };

    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const Rows rw = rows_of(tile);
        const int nrows = rw.nrows;
        gfloat *const hg = rw.h;
        gfloat *const dp = rw.dp;

        __syncthreads();   // the previous tile's readers of LDS are done
        const int t1 = tile_thread();
#pragma unroll
        for (int i = 0; i < XPT; ++i) {
            const int c = t1 + i * kNetH64Threads;
            if (c < XCH) *reinterpret_cast<u4 *>(&sX[(c / (XS / 16)) * LDX + 16 * (c % (XS / 16))]) = xr[i];
        }
        // the state: FP32 rows and their codes; the H / 4 consecutive threads
        // that hold one row's pieces reduce its maximum by shuffles
        static_assert(HCH % kNetH64Threads == 0 && (H / 4) <= 64, "whole rows per pass");
#pragma unroll
        for (int i = 0; i < HPT; ++i) {
            const int c = t1 + i * kNetH64Threads;
            const int row = c / (H / 4), k = 4 * (c % (H / 4));
            *reinterpret_cast<f4 *>(&sH[row * LDS32 + k]) = hr[i];
            float m = fmaxf(fmaxf(fabsf(hr[i].x), fabsf(hr[i].y)), fmaxf(fabsf(hr[i].z), fabsf(hr[i].w)));
#pragma unroll
            for (int o = 1; o < H / 4; o <<= 1) m = fmaxf(m, __shfl_xor(m, o));
            m = fmaxf(m, kFp8MinMax);
            const float r = 448.0f / m;
            if (k == 0) sSh[row] = m / 448.0f;
            *reinterpret_cast<uint32_t *>(&sQ[row * LDQ + k]) =
                pack4_e4m3(hr[i].x * r, hr[i].y * r, hr[i].z * r, hr[i].w * r);
        }
        if (t1 < 64) sSx[t1] = sxr;
        if (tile + (int)gridDim.x < ntiles) load_tile(tile + gridDim.x);
        __syncthreads();

        for (int pass = 0; pass < PASSES; ++pass) {
            const int rtb = pass * WPH * RTW + rt0;      // first row tile of this wave in the pass
            // ---- phase 1: the three gates of this wave's hidden tile
            f4 az[RTW], ar[RTW], ah[RTW];
            float sx[RTW], sh[RTW];
#pragma unroll
            for (int q = 0; q < RTW; ++q) {
                const int row = 16 * (rtb + q) + li;
                az[q] = ar[q] = ah[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kc = 0; kc < KCX; ++kc) {
                    const f8x8 a = mma_fp8_operand(&sX[row * LDX + kc * KC + lq * KQ]);
                    az[q] = mma_fp8(az[q], wz[kc], a);
                    ar[q] = mma_fp8(ar[q], wr[kc], a);
                    ah[q] = mma_fp8(ah[q], wh[kc], a);
                }
                sx[q] = sSx[row];
                sh[q] = sSh[row];
                const float ratio = sx[q] / sh[q];
                az[q] *= ratio;
                ar[q] *= ratio;
#pragma unroll
                for (int kh = 0; kh < HC; ++kh) {
                    const f8x8 a = mma_fp8_operand(&sQ[row * LDQ + kh * KC + lq * KQ]);
                    az[q] = mma_fp8(az[q], wz[KCX + kh], a);
                    ar[q] = mma_fp8(ar[q], wr[KCX + kh], a);
                }
            }
            f4 hold[RTW];
#pragma unroll
            for (int q = 0; q < RTW; ++q) {
                const int row = 16 * (rtb + q) + li;
                hold[q] = *reinterpret_cast<const f4 *>(&sH[row * LDS32 + ucol]);
                float m = 0.0f;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    az[q][e] = sigmoid(az[q][e] * sh[q] * S1[ucol + e]);
                    ar[q][e] = sigmoid(ar[q][e] * sh[q] * S1[H + ucol + e]) * hold[q][e];   // r*h
                    ah[q][e] *= sx[q] * S1[2 * H + ucol + e];
                    m = fmaxf(m, fabsf(ar[q][e]));
                }
                wave_max(m, row);
            }
            __syncthreads();
            float srh[RTW];
#pragma unroll
            for (int q = 0; q < RTW; ++q) {
                const int row = 16 * (rtb + q) + li;
                const float m = row_max(row), r = 448.0f / m;
                srh[q] = m / 448.0f;
                *reinterpret_cast<uint32_t *>(&sQ[row * LDQ + ucol]) =
                    pack4_e4m3(ar[q][0] * r, ar[q][1] * r, ar[q][2] * r, ar[q][3] * r);
            }
            __syncthreads();

            // ---- phase 2: U_h (r*h); new state
#pragma unroll
            for (int q = 0; q < RTW; ++q) {
                const int row = 16 * (rtb + q) + li;
                f4 au = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kc = 0; kc < HC; ++kc) au = mma_fp8(au, w2[kc], mma_fp8_operand(&sQ[row * LDQ + kc * KC + lq * KQ]));
                float m = 0.0f;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float z = az[q][e];
                    const float c = fast_tanh(ah[q][e] + au[e] * srh[q] * S2[ucol + e]);
                    const float hn = c + z * (hold[q][e] - c);   // z h + (1 - z) c
                    az[q][e] = hn;
                    m = fmaxf(m, fabsf(hn));
                }
                if (row < nrows) *(__attribute__((address_space(1))) f4 *)(hg + row * H + ucol) = az[q];
                wave_max(m, row);
            }
            __syncthreads();
            float shp[RTW];
#pragma unroll
            for (int q = 0; q < RTW; ++q) {
                const int row = 16 * (rtb + q) + li;
                const float m = row_max(row), r = 448.0f / m;
                shp[q] = m / 448.0f;
                *reinterpret_cast<uint32_t *>(&sHp[row * LDQ + ucol]) =
                    pack4_e4m3(az[q][0] * r, az[q][1] * r, az[q][2] * r, az[q][3] * r);
            }
            __syncthreads();

            // ---- MLP head
            const uint8_t *src = sHp;
            const f8x8 *Wo = sW3;
            const float *so = net.s3;
            constexpr int CO = HM > 0 ? MC : HC;             // k-chunks of the output layer
            float sin_[RTW];
#pragma unroll
            for (int q = 0; q < RTW; ++q) sin_[q] = shp[q];
            if constexpr (HM > 0) {
                float s3u[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) s3u[e] = net.s3[ucol + e];
#pragma unroll
                for (int q = 0; q < RTW; ++q) {
                    const int row = 16 * (rtb + q) + li;
                    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kc = 0; kc < HC; ++kc)
                        acc = mma_fp8(acc, sW3[(ht * HC + kc) * 64 + lane], mma_fp8_operand(&sHp[row * LDQ + kc * KC + lq * KQ]));
                    float m = 0.0f;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        ar[q][e] = fmaxf(acc[e] * shp[q] * s3u[e], 0.f);
                        m = fmaxf(m, ar[q][e]);
                    }
                    wave_max(m, row);
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < RTW; ++q) {
                    const int row = 16 * (rtb + q) + li;
                    const float m = row_max(row), r = 448.0f / m;
                    sin_[q] = m / 448.0f;
                    *reinterpret_cast<uint32_t *>(&sAm[row * LDQ + ucol]) =
                        pack4_e4m3(ar[q][0] * r, ar[q][1] * r, ar[q][2] * r, ar[q][3] * r);
                }
                __syncthreads();
                src = sAm;
                Wo = sW4;
                so = net.s4;
            }
            for (int ot = ht; ot < OT; ot += HT) {
                const int oc = 16 * ot + 4 * lq;
                float so4[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) so4[e] = oc + e < nout ? so[oc + e] : 0.0f;
#pragma unroll
                for (int q = 0; q < RTW; ++q) {
                    const int row = 16 * (rtb + q) + li;
                    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kc = 0; kc < CO; ++kc)
                        acc = mma_fp8(acc, Wo[(ot * CO + kc) * 64 + lane], mma_fp8_operand(&src[row * LDQ + kc * KC + lq * KQ]));
                    // nout is even: the pairs (oc, oc+1), (oc+2, oc+3) are inside or outside together
                    if (row < nrows) {
                        typedef float v2 __attribute__((ext_vector_type(2)));
                        typedef __attribute__((address_space(1))) v2 gv2;
                        gfloat *o = dp + row * nout + oc;
                        if (oc < nout) *(gv2 *)o = v2{acc[0] * sin_[q] * so4[0], acc[1] * sin_[q] * so4[1]};
                        if (oc + 2 < nout) *(gv2 *)(o + 2) = v2{acc[2] * sin_[q] * so4[2], acc[3] * sin_[q] * so4[3]};
                    }
                }
            }
        }
    }
}

// Persistent BF16 kernel on 128-patch tiles for the shapes k_net_h64 does not
// cover (H = 128, or K = 3), Hm = 0 or H.  Eight waves; wave w owns hidden
// tile w % HT for the 8 / (8 / HT) row tiles of its row group, so each weight
// fragment streamed from L2 (the weights, 368 KB at K = 3, H = 128, fit
// neither in registers nor in LDS) feeds 8 (H = 128) or 4 (H = 64) row tiles
// per gate.  LDS holds three regions: the tile's input rows (pitch nin, which
// keeps the fragment reads free of bank conflicts), the gate rows' state part
// [h | 0] (later r * h, then the MLP hidden layer) and h'.  The next tile's
// input rows are copied from global memory straight into their region as
// soon as the gate products are done with it, and its FP32 state into
// registers once the update has read the current one, while the current tile
// runs its state update, MLP and output products; the weights of those
// products are requested first, so the waits for them never wait for the
// copy.  A 128-patch tile is a pair of
// the launch's 64-patch row tiles, each of which may belong to another flow
// of a batch.
constexpr int kWideRows = 128;
constexpr int kCPolNT = 2;   // cache-policy operand of a global load: non-temporal

// Workgroup barrier for LDS data only: this wave's LDS accesses complete,
// then s_barrier.  Unlike __syncthreads() it does not wait for the wave's
// outstanding global loads, so a copy into LDS (global_load_lds) of another
// region can stay in flight across it.  (The memory clobber keeps the
// compiler from moving memory accesses across it.)
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <int K, int H, int HM>
__global__ __launch_bounds__(kNetH64Threads, 1) void k_net_b16w(FlowArgs single, const BatchTable *__restrict__ bt,
                                                                NetArgs net, int ntiles64)
{
    typedef Op<1> O;
    constexpr int n = 1 << K, nf = (n + 1) * (n + 1), nin = 4 * nf + 4, nout = 2 * nf;
    constexpr int KC = 32, KQ = 8, KC1 = (nin + H + KC - 1) / KC, HC = H / KC;
    constexpr int HT = H / 16, WPH = 8 / HT, RTW = (kWideRows / 16) / WPH;
    constexpr int OT = (nout + 15) / 16;
    constexpr int LDG = KC1 * KC - nin, LDH = H + 8;
    constexpr int XP = nin / 8;                       // 16-byte pieces per input row
    constexpr int XBYTES = kWideRows * nin * 2;
    constexpr int GBYTES = kWideRows * (LDG > LDH ? LDG : LDH) * 2;
    constexpr int HBYTES = kWideRows * LDH * 2;
    constexpr int KX = nin / KC;                      // k-chunks of input alone; chunk KX may straddle
    static_assert(HM == 0 || HM == H, "MLP hidden tiles follow the hidden tiles");
    static_assert(nin % 8 == 0 && LDG >= H && (LDG - H) % 8 == 0, "rows in 16-byte pieces");
    static_assert(kNetH64Threads == 512 && (H == 64 || H == 128), "eight waves over 4 or 8 hidden tiles");
    static_assert(XBYTES + GBYTES + HBYTES <= 160 * 1024, "LDS of one CU");
    if (bt) ntiles64 = bt->prefix[kKindNet][bt->nflows];
    const int ntiles = (ntiles64 + 1) / 2;

    // (three arrays, not one: the compiler then knows that reads of sG and
    // sHp cannot see the copy into sX and need not wait for it)
    __shared__ __align__(16) __bf16 sX[XBYTES / 2];     // input rows
    __shared__ __align__(16) __bf16 sG[GBYTES / 2];     // [h | 0], then r * h, then MLP hidden
    __shared__ __align__(16) __bf16 sHp[HBYTES / 2];    // h'

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lq = lane >> 4;
    const int ht = wave % HT, rt0 = RTW * (wave / HT);
    const int ucol = 16 * ht + 4 * lq;

    // the two 64-row halves of a tile: input, state and output rows, row count
    // (global address-space pointers: global, not flat, loads and stores;
    // the single flow's fields copied out, since the lambdas below would
    // otherwise reach the argument through a generic pointer)
    typedef __attribute__((address_space(1))) float gfloat;
    typedef __attribute__((address_space(1))) void gvoid;
    typedef __attribute__((address_space(3))) void lvoid;
    const void *const sXg = single.X;
    float *const sh = single.h, *const sdp = single.dpatch;
    const int sP = single.nx * single.ny;
    struct Half {
        gptr<__bf16> X;
        gfloat *h, *dp;
        int nrows;
    };
    auto half_of = [&](int t64) -> Half {
        Half r{nullptr, nullptr, nullptr, 0};
        if (t64 >= ntiles64) return r;
        int blk = t64;
        // (fields read in two branches: a pointer that may point at either the
        // kernel argument or the batch table would make them flat loads)
        const void *X;
        float *h, *dp;
        int P;
        if (bt) {
            const FlowArgs &F = *batch_flow(bt, kKindNet, blk);
            X = F.X; h = F.h; dp = F.dpatch; P = F.nx * F.ny;
        } else {
            X = sXg; h = sh; dp = sdp; P = sP;
        }
        const int row0 = blk * 64;
        r.X = (gptr<__bf16>)(reinterpret_cast<const __bf16 *>(X) + (size_t)row0 * nin);
        r.h = (gfloat *)(h + (size_t)row0 * H);
        r.dp = (gfloat *)(dp + (size_t)row0 * nout);
        r.nrows = min(64, P - row0);
        return r;
    };

    // a tile's input rows, copied into sX without passing through registers:
    // one wave load moves 64 consecutive 16-byte pieces (a half's rows are
    // consecutive in global memory and in sX).  The loads are unconditional,
    // so that the waits for later loads can count past them; wide_x_piece
    // keeps every read inside the half's rows (rows past a flow's end read
    // its last row at the same column, an empty half reads the other half's
    // rows; those rows' results are never stored).  (Lane index from
    // tile_thread(): the index math is recomputed in each tile instead of
    // hoisted out of the tile loop into registers.)
    auto fill_x = [&](const Half &a, const Half &b) {
        const int l = tile_thread() & 63;
#pragma unroll
        for (int i = 0; i < (2 * XP + 7) / 8; ++i) {
            const WidePiece w = wide_x_piece(i, wave, l, XP, a.nrows, b.nrows);
            const Half &hh = w.half ? b : a;
            // (non-temporal: the rows are read once, and the weights that
            // every tile reads stay in L2 instead)
            __builtin_amdgcn_global_load_lds((gvoid *)(hh.X + w.src), (lvoid *)(sX + w.dst), 16, 0, kCPolNT);
        }
    };
    // a tile's FP32 state in the lane layout of the update (rows 16 q + li
    // of the wave's row tiles, units ucol .. ucol + 3); unconditional loads
    // as above (wide_h_row: rows past the flow's end read its last row)
    f4 hold[RTW];
    auto load_hold = [&](const Half &a, const Half &b) {
        const int l = tile_thread() & 15;
#pragma unroll
        for (int q = 0; q < RTW; ++q) {
            int half;
            const int row = wide_h_row(16 * (rt0 + q) + l, a.nrows, b.nrows, half);
            const Half &hh = half ? b : a;
            hold[q] = *(const __attribute__((address_space(1))) f4 *)(hh.h + row * H + ucol);
        }
    };
    if ((int)blockIdx.x < ntiles) {
        const Half a = half_of(2 * blockIdx.x), b = half_of(2 * blockIdx.x + 1);
        fill_x(a, b);
        load_hold(a, b);
    }

    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const Half ha = half_of(2 * tile), hb = half_of(2 * tile + 1);
        const bool more = tile + (int)gridDim.x < ntiles;
        const gptr<bf8> B1 = pinned<bf8>(net.B1);
        const gptr<bf8> B2 = pinned<bf8>(net.B2);
        const gptr<bf8> B3 = pinned<bf8>(net.B3);
        const gptr<bf8> B4 = pinned<bf8>(net.B4);

        __syncthreads();   // the previous tile's readers of sG and sHp are done
        // the state's BF16 copy and the zeros after it (the last k-chunk
        // reads them)
#pragma unroll
        for (int q = 0; q < RTW; ++q) {
            const int r = 16 * (rt0 + q) + li;
            bf4 hb4;
            hb4[0] = (__bf16)hold[q].x; hb4[1] = (__bf16)hold[q].y; hb4[2] = (__bf16)hold[q].z; hb4[3] = (__bf16)hold[q].w;
            *reinterpret_cast<bf4 *>(&sG[r * LDG + ucol]) = hb4;
        }
        if (LDG > H)
            for (int t = tile_thread(); t < kWideRows * ((LDG - H) / 8); t += kNetH64Threads)
                *reinterpret_cast<uint4 *>(&sG[(t / ((LDG - H) / 8)) * LDG + H + 8 * (t % ((LDG - H) / 8))]) = make_uint4(0u, 0u, 0u, 0u);
        __builtin_amdgcn_s_waitcnt(0);   // this wave's pieces of the input rows have landed in LDS
        __syncthreads();

        // ---- gates: weight fragments streamed chunk by chunk
        f4 az[RTW], ar[RTW], ah[RTW];
#pragma unroll
        for (int q = 0; q < RTW; ++q) az[q] = ar[q] = ah[q] = f4{0.f, 0.f, 0.f, 0.f};
        // (each chunk requests the fragments of the chunk two ahead before its
        // products, so the products never wait for the chunk's own)
        bf8 wz = B1[((0 * HT + ht) * KC1 + 0) * 64 + lane];
        bf8 wr = B1[((1 * HT + ht) * KC1 + 0) * 64 + lane];
        bf8 wh = B1[((2 * HT + ht) * KC1 + 0) * 64 + lane];
        bf8 vz = B1[((0 * HT + ht) * KC1 + 1) * 64 + lane];
        bf8 vr = B1[((1 * HT + ht) * KC1 + 1) * 64 + lane];
        bf8 vh = B1[((2 * HT + ht) * KC1 + 1) * 64 + lane];
        auto chunk = [&](int kc, const __bf16 *base, int pitch, int lrow) {
            const int kn = min(kc + 2, KC1 - 1);
            const bf8 nz = B1[((0 * HT + ht) * KC1 + kn) * 64 + lane];
            const bf8 nr = B1[((1 * HT + ht) * KC1 + kn) * 64 + lane];
            const bf8 nh = B1[((2 * HT + ht) * KC1 + kn) * 64 + lane];
#pragma unroll
            for (int q = 0; q < RTW; ++q) {
                const bf8 a = *reinterpret_cast<const bf8 *>(&base[(16 * (rt0 + q) + lrow) * pitch]);
                az[q] = O::mma(az[q], wz, a);
                ar[q] = O::mma(ar[q], wr, a);
                ah[q] = O::mma(ah[q], wh, a);
            }
            wz = vz;
            wr = vr;
            wh = vh;
            vz = nz;
            vr = nr;
            vh = nh;
        };
#pragma unroll 1
        for (int kc = 0; kc < KX; ++kc) chunk(kc, sX + kc * KC + lq * KQ, nin, li);
        {
            // chunk KX: a lane's 8 columns lie in the input or in the state
            // part (lane indices from tile_thread(): the row addresses are
            // recomputed in each tile, not held in registers across tiles)
            const int tt = tile_thread() & 63;
            const int k0 = KX * KC + (tt >> 4) * KQ;
            const bool inx = k0 < nin;
            chunk(KX, inx ? sX + k0 : sG + (k0 - nin), inx ? nin : LDG, tt & 15);
        }
#pragma unroll 1
        for (int kc = KX + 1; kc < KC1; ++kc) chunk(kc, sG + (kc * KC + lq * KQ - nin), LDG, li);
        __syncthreads();   // every wave is done with sX and sG

        // the weights of U_h, of the MLP hidden layer and of this wave's
        // output tiles (ht, ht + HT, ...), requested before the copy below so
        // that the waits for them do not wait for the copy
        bf8 w2[HC], w3[HC];
#pragma unroll
        for (int kc = 0; kc < HC; ++kc) w2[kc] = B2[(ht * HC + kc) * 64 + lane];
        if constexpr (HM > 0) {
#pragma unroll
            for (int kc = 0; kc < HC; ++kc) w3[kc] = B3[(ht * HC + kc) * 64 + lane];
        }
        const gptr<bf8> Wo = HM > 0 ? B4 : B3;
        constexpr int NOT = (OT + HT - 1) / HT;
        bf8 wo[NOT][HC];
#pragma unroll
        for (int j = 0; j < NOT; ++j) {
            const int ot = min(ht + j * HT, OT - 1);
#pragma unroll
            for (int kc = 0; kc < HC; ++kc) wo[j][kc] = Wo[(ot * HC + kc) * 64 + lane];
        }
#pragma unroll
        for (int q = 0; q < RTW; ++q) {
            const int r = 16 * (rt0 + q) + li;
            bf4 rh;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                az[q][e] = sigmoid_l2(az[q][e]);
                rh[e] = (__bf16)(sigmoid_l2(ar[q][e]) * hold[q][e]);
            }
            *reinterpret_cast<bf4 *>(&sG[r * LDH + ucol]) = rh;
        }
        // the next tile's input rows, copied into sX (free from here on) while
        // this tile runs its state update, MLP and output products.  The
        // weights above land first: while a copy into LDS is outstanding, a
        // wait for any load waits for the copy too.  The barriers until the
        // tile's end are lds_barrier(), which do not wait for the copy.  (The
        // last tile of the block copies itself again: no branch.)
        __builtin_amdgcn_s_waitcnt(0);
        const int nt = more ? tile + (int)gridDim.x : tile;
        const Half na = half_of(2 * nt), nb = half_of(2 * nt + 1);
        fill_x(na, nb);
        lds_barrier();

        // ---- U_h (r * h); new state
#pragma unroll
        for (int q = 0; q < RTW; ++q) {
            const int r = 16 * (rt0 + q) + li;
            f4 au = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < HC; ++kc)
                au = O::mma(au, w2[kc], *reinterpret_cast<const bf8 *>(&sG[r * LDH + kc * KC + lq * KQ]));
            f4 hn;
            bf4 hb4;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float z = az[q][e];
                // h' = z h + (1 - z) c = c + z (h - c), c the candidate state
                const float c = tanh_l2(ah[q][e] + au[e]);
                hn[e] = c + z * (hold[q][e] - c);
                hb4[e] = (__bf16)hn[e];
            }
            const Half &hh = r < 64 ? ha : hb;
            if ((r & 63) < hh.nrows) *(__attribute__((address_space(1))) f4 *)(hh.h + (r & 63) * H + ucol) = hn;
            *reinterpret_cast<bf4 *>(&sHp[r * LDH + ucol]) = hb4;
        }
        // the next tile's state (this tile's is no longer read)
        load_hold(na, nb);
        lds_barrier();

        // ---- MLP head
        const __bf16 *src = sHp;
        if constexpr (HM > 0) {
#pragma unroll
            for (int q = 0; q < RTW; ++q) {
                const int r = 16 * (rt0 + q) + li;
                f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kc = 0; kc < HC; ++kc)
                    acc = O::mma(acc, w3[kc], *reinterpret_cast<const bf8 *>(&sHp[r * LDH + kc * KC + lq * KQ]));
                bf4 m;
#pragma unroll
                for (int e = 0; e < 4; ++e) m[e] = (__bf16)fmaxf(acc[e], 0.f);
                *reinterpret_cast<bf4 *>(&sG[r * LDH + ucol]) = m;
            }
            lds_barrier();
            src = sG;
        }
        const int lo = tile_thread() & 15;   // (row addresses recomputed in each tile)
#pragma unroll
        for (int j = 0; j < NOT; ++j) {
            const int ot = ht + j * HT;
            if (ot >= OT) break;
            const int oc = 16 * ot + 4 * lq;
#pragma unroll
            for (int q = 0; q < RTW; ++q) {
                const int r = 16 * (rt0 + q) + li;
                f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kc = 0; kc < HC; ++kc)
                    acc = O::mma(acc, wo[j][kc], *reinterpret_cast<const bf8 *>(&src[r * LDH + kc * KC + lq * KQ]));
                // nout is even: the pairs (oc, oc+1), (oc+2, oc+3) are inside or outside together
                const int ro = 16 * (rt0 + q) + lo;
                const Half &hh = ro < 64 ? ha : hb;
                if ((ro & 63) < hh.nrows) {
                    gfloat *o = hh.dp + (ro & 63) * nout + oc;
                    typedef float v2 __attribute__((ext_vector_type(2)));
                    typedef __attribute__((address_space(1))) v2 gv2;
                    if (oc < nout) *(gv2 *)o = v2{acc[0], acc[1]};
                    if (oc + 2 < nout) *(gv2 *)(o + 2) = v2{acc[2], acc[3]};
                }
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);   // the last tile's repeated copy into LDS has landed
}

static int g_num_cus = 0;

// The persistent kernels take rows of the standard width 4 nf + 4 and the
// GRU as printed; other forms run the generic kernels.
static bool standard_rows(const NetArgs &net)
{
    const int n = 1 << net.K;
    return net.nin == 4 * (n + 1) * (n + 1) + 4 && !net.reset_after;
}
static bool use_h64(int prec, int K, int H, int Hm) { return prec == 1 && H == 64 && K <= 2 && (Hm == 0 || Hm == 64); }
static bool use_h64(const NetArgs &net) { return standard_rows(net) && use_h64(net.prec, net.K, net.H, net.Hm); }
static bool use_q8p(const NetArgs &net)
{
    return standard_rows(net) && net.prec == 2 && (net.H == 64 || net.H == 128) && (net.Hm == 0 || net.Hm == net.H);
}
static bool use_b16w(const NetArgs &net)
{
    return standard_rows(net) && net.prec == 1 && !use_h64(net) && (net.H == 64 || net.H == 128) &&
           (net.Hm == 0 || net.Hm == net.H);
}
static bool persistent(const NetArgs &net) { return use_h64(net) || use_q8p(net) || use_b16w(net); }


int net_blocks(const NetArgs &net, int row_tiles)
{
    if (persistent(net)) {
        if (g_num_cus == 0) {
            int dev = 0;
            (void)hipGetDevice(&dev);
            if (hipDeviceGetAttribute(&g_num_cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
                g_num_cus = 256;
        }
        return row_tiles < g_num_cus ? row_tiles : g_num_cus;
    }
    return row_tiles;
}

template <int PREC, int H, int HMC>
static void launch_net_m(const FlowArgs &f, const BatchTable *bt, int nblocks, const NetArgs &net, hipStream_t s)
{
    if (bt) hipLaunchKernelGGL((k_net<PREC, H, HMC, true>), dim3(nblocks), dim3(kThreads), 0, s, f, bt, net);
    else hipLaunchKernelGGL((k_net<PREC, H, HMC, false>), dim3(nblocks), dim3(kThreads), 0, s, f, bt, net);
}

template <int PREC, int H>
static hipError_t launch_net_t(const FlowArgs &f, const BatchTable *bt, int nblocks, const NetArgs &net,
                               hipStream_t s)
{
    switch (hm_class(net.Hm)) {
    case 0: launch_net_m<PREC, H, 0>(f, bt, nblocks, net, s); break;
    case 64: launch_net_m<PREC, H, 64>(f, bt, nblocks, net, s); break;
    case 128: launch_net_m<PREC, H, 128>(f, bt, nblocks, net, s); break;
    default: launch_net_m<PREC, H, 256>(f, bt, nblocks, net, s);
    }
    return hipGetLastError();
}

hipError_t launch_net(const FlowArgs &f, const BatchTable *bt, int ntiles, const NetArgs &net, hipStream_t s)
{
    const int nblocks = net_blocks(net, ntiles);
    if (use_h64(net)) {
        if (net.K == 1) hipLaunchKernelGGL(k_net_h64<1>, dim3(nblocks), dim3(kNetH64Threads), 0, s, f, bt, net, ntiles);
        else hipLaunchKernelGGL(k_net_h64<2>, dim3(nblocks), dim3(kNetH64Threads), 0, s, f, bt, net, ntiles);
        return hipGetLastError();
    }
    if (use_b16w(net)) {
        // 128-patch tiles: half as many blocks are enough
        dim3 g(net_blocks(net, (ntiles + 1) / 2)), b(kNetH64Threads);
#define DNNMG_B16W(KK, HH, MM) hipLaunchKernelGGL((k_net_b16w<KK, HH, MM>), g, b, 0, s, f, bt, net, ntiles)
#define DNNMG_B16W_H(KK)                                                                             \
        if (net.H == 64) { if (net.Hm == 64) DNNMG_B16W(KK, 64, 64); else DNNMG_B16W(KK, 64, 0); }    \
        else { if (net.Hm == 128) DNNMG_B16W(KK, 128, 128); else DNNMG_B16W(KK, 128, 0); }
        switch (net.K) {
        case 1: DNNMG_B16W_H(1) break;
        case 2: DNNMG_B16W_H(2) break;
        case 3: DNNMG_B16W_H(3) break;
        default: return hipErrorInvalidValue;
        }
#undef DNNMG_B16W_H
#undef DNNMG_B16W
        return hipGetLastError();
    }
    if (use_q8p(net)) {
        dim3 g(nblocks), b(kNetH64Threads);
#define DNNMG_Q8P(KK, HH, MM) hipLaunchKernelGGL((k_net_q8p<KK, HH, MM>), g, b, 0, s, f, bt, net, ntiles)
#define DNNMG_Q8P_H(KK)                                                                            \
        if (net.H == 64) { if (net.Hm == 64) DNNMG_Q8P(KK, 64, 64); else DNNMG_Q8P(KK, 64, 0); }    \
        else { if (net.Hm == 128) DNNMG_Q8P(KK, 128, 128); else DNNMG_Q8P(KK, 128, 0); }
        switch (net.K) {
        case 1: DNNMG_Q8P_H(1) break;
        case 2: DNNMG_Q8P_H(2) break;
        case 3: DNNMG_Q8P_H(3) break;
        default: return hipErrorInvalidValue;
        }
#undef DNNMG_Q8P_H
#undef DNNMG_Q8P
        return hipGetLastError();
    }
    if (net.prec == 2) {
        dim3 g(nblocks), b(kThreads);
#define DNNMG_FP8_CASE(HH)                                                                  \
        if (net.H == HH) {                                                                  \
            if (bt) hipLaunchKernelGGL((k_net_fp8<HH, true>), g, b, 0, s, f, bt, net);      \
            else hipLaunchKernelGGL((k_net_fp8<HH, false>), g, b, 0, s, f, bt, net);        \
            return hipGetLastError();                                                       \
        }
        DNNMG_FP8_CASE(32)
        DNNMG_FP8_CASE(64)
        DNNMG_FP8_CASE(128)
#undef DNNMG_FP8_CASE
        return hipErrorInvalidValue;
    }
    if (net.prec == 0) {
        if (net.H == 32) return launch_net_t<0, 32>(f, bt, nblocks, net, s);
        if (net.H == 64) return launch_net_t<0, 64>(f, bt, nblocks, net, s);
        if (net.H == 96) return launch_net_t<0, 96>(f, bt, nblocks, net, s);
        if (net.H == 128) return launch_net_t<0, 128>(f, bt, nblocks, net, s);
    } else if (net.prec == 1) {
        if (net.H == 32) return launch_net_t<1, 32>(f, bt, nblocks, net, s);
        if (net.H == 64) return launch_net_t<1, 64>(f, bt, nblocks, net, s);
        if (net.H == 96) return launch_net_t<1, 96>(f, bt, nblocks, net, s);
        if (net.H == 128) return launch_net_t<1, 128>(f, bt, nblocks, net, s);
    }
    return hipErrorInvalidValue;
}


}  // namespace dnnmg
