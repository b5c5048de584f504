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
#include "internal.h"

namespace dnnmg {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

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
};

__device__ inline float sigmoid(float t) { return 1.0f / (1.0f + expf(-t)); }

template <int PREC, int H>
__global__ __launch_bounds__(kThreads) void k_net(FlowArgs single, const BatchTable *bt, NetArgs net)
{
    typedef Op<PREC> O;
    typedef typename O::T T;
    typedef typename O::Frag Frag;
    constexpr int KC = O::KC, KQ = O::KQ;
    constexpr int HT = H / 16;                 // hidden-unit tiles
    constexpr int PAD = 16 / sizeof(T);        // 16-byte row padding
    constexpr int LDH = H + PAD;
    constexpr int LDM = 256 + PAD;             // MLP hidden width <= 256

    // r*h (phase 2 operand) and the MLP hidden layer share one buffer: the
    // former is dead once phase 2 is done.
    constexpr int LDB = LDH > LDM ? LDH : LDM;
    __shared__ __align__(16) T sBuf[4][16 * LDB];
    __shared__ __align__(16) T sHp[4][16 * LDH];
    T *sR = sBuf[0], *sAm = sBuf[0];

    int blk = blockIdx.x;
    const FlowArgs f = bt ? *batch_flow(bt, kKindNet, blk) : single;
    const int P = f.nx * f.ny;
    const int nin = net.nin, nout = net.nout, Hm = net.Hm, kc1 = net.kc1;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 15, lq = lane >> 4;
    const int rbase = blk * kNetRows + wave * 16;   // first patch row of this wave
    const int arow = rbase + li;                    // row this lane supplies A values for
    const bool aok = arow < P;

    const Frag *B1 = reinterpret_cast<const Frag *>(net.B1);
    const Frag *B2 = reinterpret_cast<const Frag *>(net.B2);
    const Frag *B3 = reinterpret_cast<const Frag *>(net.B3);
    const Frag *B4 = reinterpret_cast<const Frag *>(net.B4);

    // ---- phase 1: [x | h] x [W_g | U_g]^T for g = z, r, h
    f4 az[HT], ar[HT], ah[HT];
#pragma unroll
    for (int t = 0; t < HT; ++t) az[t] = ar[t] = ah[t] = f4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < kc1; ++kc) {
        const int k0 = kc * KC + lq * KQ;
        Frag a;
        if (aok && k0 < nin) a = O::load_f32(f.X + (size_t)arow * nin + k0);
        else if (aok && k0 < nin + H) a = O::load_f32(f.h + (size_t)arow * H + (k0 - nin));
        else {
#pragma unroll
            for (int e = 0; e < KQ; ++e) a[e] = O::cvt(0.f);
        }
#pragma unroll
        for (int t = 0; t < HT; ++t) {
            az[t] = O::mma(az[t], a, B1[((0 * HT + t) * kc1 + kc) * 64 + lane]);
            ar[t] = O::mma(ar[t], a, B1[((1 * HT + t) * kc1 + kc) * 64 + lane]);
            ah[t] = O::mma(ah[t], a, B1[((2 * HT + t) * kc1 + kc) * 64 + lane]);
        }
    }

    // ---- gates; r*h to LDS.  Lane holds rows rbase + 4 lq + e, column 16 t + li.
    float hold[HT][4];
#pragma unroll
    for (int t = 0; t < HT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = rbase + 4 * lq + e, k = 16 * t + li;
            const float h0 = row < P ? f.h[(size_t)row * H + k] : 0.f;
            hold[t][e] = h0;
            az[t][e] = sigmoid(az[t][e]);
            const float r = sigmoid(ar[t][e]);
            sR[wave * 16 * LDB + (4 * lq + e) * LDH + k] = O::cvt(r * h0);
        }
    __syncthreads();

    // ---- phase 2: (r*h) x U_h^T; update h
    f4 au[HT];
#pragma unroll
    for (int t = 0; t < HT; ++t) au[t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < H / KC; ++kc) {
        Frag a = *reinterpret_cast<const Frag *>(&sR[wave * 16 * LDB + li * LDH + kc * KC + lq * KQ]);
#pragma unroll
        for (int t = 0; t < HT; ++t) au[t] = O::mma(au[t], a, B2[(t * (H / KC) + kc) * 64 + lane]);
    }
#pragma unroll
    for (int t = 0; t < HT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = rbase + 4 * lq + e, k = 16 * t + li;
            const float z = az[t][e];
            const float hh = tanhf(ah[t][e] + au[t][e]);
            const float hn = z * hold[t][e] + (1.0f - z) * hh;
            if (row < P) f.h[(size_t)row * H + k] = hn;
            sHp[wave][(4 * lq + e) * LDH + k] = O::cvt(hn);
        }
    __syncthreads();

    // ---- MLP head
    const int ot_n = (nout + 15) / 16;
    if (Hm > 0) {
        for (int mt = 0; mt < Hm / 16; ++mt) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < H / KC; ++kc) {
                Frag a = *reinterpret_cast<const Frag *>(&sHp[wave][li * LDH + kc * KC + lq * KQ]);
                acc = O::mma(acc, a, B3[(mt * (H / KC) + kc) * 64 + lane]);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) sAm[wave * 16 * LDB + (4 * lq + e) * LDM + 16 * mt + li] = O::cvt(fmaxf(acc[e], 0.f));
        }
        __syncthreads();
        const int kcm = Hm / KC;
        for (int ot = 0; ot < ot_n; ++ot) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
            for (int kc = 0; kc < kcm; ++kc) {
                Frag a = *reinterpret_cast<const Frag *>(&sAm[wave * 16 * LDB + li * LDM + kc * KC + lq * KQ]);
                acc = O::mma(acc, a, B4[(ot * kcm + kc) * 64 + lane]);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = rbase + 4 * lq + e, o = 16 * ot + li;
                if (row < P && o < nout) f.dpatch[(size_t)row * nout + o] = acc[e];
            }
        }
    } else {
        for (int ot = 0; ot < ot_n; ++ot) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < H / KC; ++kc) {
                Frag a = *reinterpret_cast<const Frag *>(&sHp[wave][li * LDH + kc * KC + lq * KQ]);
                acc = O::mma(acc, a, B3[(ot * (H / KC) + kc) * 64 + lane]);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = rbase + 4 * lq + e, o = 16 * ot + li;
                if (row < P && o < nout) f.dpatch[(size_t)row * nout + o] = acc[e];
            }
        }
    }
}

template <int PREC, int H>
static hipError_t launch_net_t(const FlowArgs &f, const BatchTable *bt, int nblocks, const NetArgs &net,
                               hipStream_t s)
{
    hipLaunchKernelGGL((k_net<PREC, H>), dim3(nblocks), dim3(kThreads), 0, s, f, bt, net);
    return hipGetLastError();
}

hipError_t launch_net(const FlowArgs &f, const BatchTable *bt, int nblocks, const NetArgs &net, hipStream_t s)
{
    if (net.prec == 0) {
        if (net.H == 32) return launch_net_t<0, 32>(f, bt, nblocks, net, s);
        if (net.H == 64) return launch_net_t<0, 64>(f, bt, nblocks, net, s);
        if (net.H == 128) return launch_net_t<0, 128>(f, bt, nblocks, net, s);
    } else if (net.prec == 1) {
        if (net.H == 32) return launch_net_t<1, 32>(f, bt, nblocks, net, s);
        if (net.H == 64) return launch_net_t<1, 64>(f, bt, nblocks, net, s);
        if (net.H == 128) return launch_net_t<1, 128>(f, bt, nblocks, net, s);
    }
    return hipErrorInvalidValue;
}

hipError_t net_set_attributes(int, int) { return hipSuccess; }
size_t net_lds_bytes(const NetArgs &) { return 0; }

}  // namespace dnnmg
