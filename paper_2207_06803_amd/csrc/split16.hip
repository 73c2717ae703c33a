// Complex64 FFT whose DFT_16 stages run on the matrix cores (gfx950
// v_mfma_f32_16x16x32_{f16,bf16}) with split low-precision operands.
//
// A radix-16 stage applies DFT_16 (x) I_{N/16}: as (A (x) I_n) vec(X) =
// vec(A X), it is the dense product of the 16 x 16 DFT matrix W with a
// 16 x (N/16) matrix whose columns are the butterflies.  In real form, for
// a group of 16 butterflies (columns), with V = Vr + i Vi the twiddled inputs:
//     Yr = Wr Vr - Wi Vi,   Yi = Wi Vr + Wr Vi
// each a 16 x 32 by 32 x 16 product over the stacked real and imaginary
// parts: one MFMA.  Operands are split as
// X = X_hi + 2^-s X_lo (X_lo stored scaled by 2^s so it stays normal), and
//     Y ~ W_hi V_hi + 2^-s (W_hi V_lo + W_lo V_hi)
// accumulated in FP32 (the split-operand refinement of Markidis et al. 2018
// and Ootomo & Yokota 2022).  Modes: fp16 hi+lo (s = 11), bf16 hi+lo
// (s = 8), bf16 hi+mid+lo (three terms, s = 8 per level) and plain fp16.
//
// Data path per transform (one workgroup): the first radix-16 stage reads
// its inputs from HBM (each 16 lanes 128 contiguous bytes), the stages
// exchange through interleaved complex LDS, and the last stage -- radix 16,
// or a final radix-2/4/8 stage on the VALU -- writes HBM in natural order.  Each stage multiplies its outputs by
// the twiddle factors of the next stage (same table layout as the Stockham
// plans), so MFMA inputs need no complex multiply.  The contraction index
// pairs each input's real and imaginary parts (k = 2 r + c), so a lane's
// eight B values are four whole complex inputs: one 8-byte LDS read per
// complex element and stage, split once into hi and lo parts, and one 8-byte
// write of each complex output.
//
// MFMA lane layouts (16x16x32, 64 lanes, l = lane):
//   A[m][k]: m = l % 16, k = 8 (l / 16) + i   (8 values per lane)
//   B[k][n]: k = 8 (l / 16) + i, n = l % 16
//   C[m][n]: m = 4 (l / 16) + i, n = l % 16   (4 floats per lane)
#include "codelets.h"
#include "plan.h"
#include "split16.h"

namespace fftc {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int MODE> struct SplitTraits;
template <> struct SplitTraits<FFTC_C64_SPLIT_F16> {
    using V = f16x8; using E = _Float16;
    static constexpr int TERMS = 2; static constexpr float SCALE = 2048.f;
};
template <> struct SplitTraits<FFTC_C64_SPLIT_BF16> {
    using V = bf16x8; using E = __bf16;
    static constexpr int TERMS = 2; static constexpr float SCALE = 256.f;
};
template <> struct SplitTraits<FFTC_C64_SPLIT3_BF16> {
    using V = bf16x8; using E = __bf16;
    static constexpr int TERMS = 3; static constexpr float SCALE = 256.f;
};
template <> struct SplitTraits<FFTC_C64_F16> {
    using V = f16x8; using E = _Float16;
    static constexpr int TERMS = 1; static constexpr float SCALE = 1.f;
};

__device__ __forceinline__ f32x4 mma(f16x8 a, f16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Split x into TERMS low-precision parts: x ~ p0 + p1 / S + p2 / S^2.
template <int MODE>
__device__ __forceinline__ void split(float x, typename SplitTraits<MODE>::E* p) {
    using T = SplitTraits<MODE>;
    using E = typename T::E;
    float r = x;
#pragma unroll
    for (int t = 0; t < T::TERMS; ++t) {
        p[t] = (E)r;
        r = (r - (float)p[t]) * T::SCALE;
    }
}

// cos / sin (2 pi t / 16), t = 0..15.  Selects rather than an indexed
// array: a runtime-indexed local table is placed in memory, and its loads
// then stood in front of the transform's own HBM loads in every workgroup.
__device__ __forceinline__ float cos16(int q) {  // cos of q sixteenths of a turn, q = 0..4
    const float c1 = 0.9238795325112867f, s1 = 0.3826834323650898f, h = 0.7071067811865476f;
    return q == 0 ? 1.f : q == 1 ? c1 : q == 2 ? h : q == 3 ? s1 : 0.f;
}
__device__ __forceinline__ void w16(int t, float* c, float* s) {
    const int q = t & 3, o = (t >> 2) & 3;  // t = 4 o + q
    // angle = o pi/2 + q pi/8
    float cc = cos16(q), ss = cos16(4 - q);
    float rc, rs;
    switch (o) {
        case 0: rc = cc; rs = ss; break;
        case 1: rc = -ss; rs = cc; break;
        case 2: rc = -cc; rs = -ss; break;
        default: rc = ss; rs = -cc; break;
    }
    *c = rc;
    *s = rs;
}

// radix list: NS16 stages of 16, then RT in {1 (none), 2, 4, 8}
template <int N> constexpr int split_stages16() {
    int s = 0, m = N;
    while (m % 16 == 0) { m /= 16; ++s; }
    return s;
}
template <int N> constexpr int split_tail() {
    int m = N;
    while (m % 16 == 0) m /= 16;
    return m;
}
// Waves per transform: one per group of 16 butterflies for N = 256 and 512,
// two for N = 1024 and 2048 (two and four groups each), four for 4096, then
// one per 1024 elements.  Measured at batch 8192, N = 1024: two waves of two
// groups took 32.2 us (fp16 split) and 39.2 us (bf16 three-term) against
// 33.7 and 45.2 us with four waves of one group, and one wave of four groups
// was slower still; N = 2048: 60.7 / 69.8 us against 61.9 / 72.9 us; N =
// 4096: two waves were slower (125.9 / 211.6 us against 115.8 / 172.6 us).
__host__ __device__ constexpr int split_waves_for(int64_t n) {
    return (n == 1024 || n == 2048) ? 2 : n <= 4096 ? (n / 256 < 4 ? (n / 256 < 1 ? 1 : (int)(n / 256)) : 4) : (int)(n / 1024);
}
template <int N> constexpr int split_waves() { return split_waves_for(N); }

__device__ __forceinline__ int spad(int i) { return i + (i >> 4); }

// The twiddle element p needs as an input of the stage with radix R2 after
// NS2 (table segment at TW2): w_{NS2 R2}^{r k} (1 when r = 0 or NS2 = 1).
template <int N, int R2, int NS2, int TW2>
__device__ __forceinline__ float2 next_twiddle(int p, const float2* __restrict__ tw) {
    if constexpr (NS2 > 1) {
        constexpr int NR2 = N / R2;
        const int r = p / NR2, j = p - r * NR2, k = j % NS2;
        // r = 0 reads the table's first entry and discards it (no branch)
        const float2 w = tw[TW2 + (r > 0 ? (r - 1) * NS2 + k : 0)];
        return r > 0 ? w : make_float2(1.f, 0.f);
    }
    return make_float2(1.f, 0.f);
}

// The same factor applied in place, read only where r > 0.
template <int N, int R2, int NS2, int TW2>
__device__ __forceinline__ void apply_next_twiddle(int p, float& re, float& im, const float2* __restrict__ tw) {
    if constexpr (NS2 > 1) {
        constexpr int NR2 = N / R2;
        const int r = p / NR2, j = p - r * NR2, k = j % NS2;
        if (r > 0) {
            const float2 w = tw[TW2 + (r - 1) * NS2 + k];
            const float a = re, b = im;
            re = a * w.x - b * w.y;
            im = a * w.y + b * w.x;
        }
    }
}

// One radix-16 MFMA stage (NS = product of earlier radices).  R2/NS2/TW2
// describe the next stage (R2 = 0: none).  The contraction index k runs over
// (input r, real or imaginary part) as k = 2 r + c, so the lane holding
// B[k][n], k = 8 (l / 16) + i, takes inputs r = 4 (l / 16) .. + 3 of
// butterfly n whole: four complex values read from the interleaved LDS.
template <int N, int W> constexpr int split_gpw() { return (N / 256 + W - 1) / W; }

template <int N, int MODE, int NS, int R2, int NS2, int TW2, int W, bool INV, bool FIRST, bool LASTG>
__device__ __forceinline__ void mfma_stage(float2* x, float2* gout, const float2* __restrict__ tw,
                                           const typename SplitTraits<MODE>::V (&a1)[3],
                                           const typename SplitTraits<MODE>::V (&a2)[3],
                                           const float2 (&raw)[split_gpw<N, W>()][4]) {
    using T = SplitTraits<MODE>;
    using V = typename T::V;
    using E = typename T::E;
    constexpr int NB = N / 16;        // butterflies
    constexpr int G = NB / 16;        // groups of 16 butterflies
    constexpr int GPW = (G + W - 1) / W;
    constexpr bool EVENG = G % W == 0;  // every wave has GPW groups
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const int n = lane & 15, g4 = lane >> 4;
    V b[GPW][3];
#pragma unroll
    for (int gi = 0; gi < GPW; ++gi) {
        const int grp = wave + gi * W;
        if (EVENG || grp < G) {
            const int j = grp * 16 + n;
            E parts[8][3];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // the first stage's inputs were loaded from HBM at the start
                const float2 v = FIRST ? raw[gi][i] : x[spad(j + (4 * g4 + i) * NB)];
                split<MODE>(v.x, parts[2 * i]);
                split<MODE>(v.y, parts[2 * i + 1]);
            }
#pragma unroll
            for (int t = 0; t < T::TERMS; ++t)
#pragma unroll
                for (int i = 0; i < 8; ++i) b[gi][t][i] = parts[i][t];
        }
    }
    // the next stage's twiddles for this lane's outputs, loaded before the
    // products so their latency overlaps the matrix-core work (workgroups of
    // up to 4 waves: with 16 waves the registers they take cost more)
    constexpr bool PREFETCH = R2 > 0 && W <= 4;
    float2 wn[PREFETCH ? GPW : 1][4];
    if constexpr (PREFETCH) {
#pragma unroll
        for (int gi = 0; gi < GPW; ++gi) {
            const int grp = wave + gi * W;
            const int j = grp * 16 + n;
            const int kk = j % NS, q = j / NS;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                wn[gi][c] = (EVENG || grp < G) ? next_twiddle<N, R2, NS2, TW2>(q * NS * 16 + (4 * g4 + c) * NS + kk, tw)
                                    : make_float2(1.f, 0.f);
        }
    }
    if constexpr (!FIRST) __syncthreads();  // every read of the LDS before it is overwritten
    const float inv1 = 1.f / T::SCALE, inv2 = inv1 * inv1;
#pragma unroll
    for (int gi = 0; gi < GPW; ++gi) {
        const int grp = wave + gi * W;
        if (EVENG || grp < G) {
            const f32x4 z = {0.f, 0.f, 0.f, 0.f};
            f32x4 yr0 = mma(a1[0], b[gi][0], z), yi0 = mma(a2[0], b[gi][0], z);
            f32x4 yr1 = z, yi1 = z, yr2 = z, yi2 = z;
            if constexpr (T::TERMS >= 2) {
                yr1 = mma(a1[0], b[gi][1], mma(a1[1], b[gi][0], z));
                yi1 = mma(a2[0], b[gi][1], mma(a2[1], b[gi][0], z));
            }
            if constexpr (T::TERMS >= 3) {
                yr2 = mma(a1[0], b[gi][2], mma(a1[1], b[gi][1], mma(a1[2], b[gi][0], z)));
                yi2 = mma(a2[0], b[gi][2], mma(a2[1], b[gi][1], mma(a2[2], b[gi][0], z)));
            }
            const int j = grp * 16 + n;
            const int kk = j % NS, q = j / NS;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int m = 4 * g4 + c;
                float vr = yr0[c], vi = yi0[c];
                if constexpr (T::TERMS >= 2) { vr += inv1 * yr1[c]; vi += inv1 * yi1[c]; }
                if constexpr (T::TERMS >= 3) { vr += inv2 * yr2[c]; vi += inv2 * yi2[c]; }
                const int p = q * NS * 16 + m * NS + kk;
                if constexpr (PREFETCH) {
                    const float2 w = wn[gi][c];
                    const float a = vr, bb = vi;
                    vr = a * w.x - bb * w.y;
                    vi = a * w.y + bb * w.x;
                } else if constexpr (R2 > 0) {
                    apply_next_twiddle<N, R2, NS2, TW2>(p, vr, vi, tw);
                }
                // the last stage writes HBM in natural order (p = m N/16 + j)
                if constexpr (LASTG)
                    st_out<INV>(gout + p, make_float2(vr, vi));
                else
                    x[spad(p)] = make_float2(vr, vi);
            }
        }
    }
    if constexpr (!LASTG) __syncthreads();
}

// Final radix-RT stage on the VALU (its input twiddles already applied),
// writing HBM in natural order.
template <int N, int RT, int NS, int NT, bool INV>
__device__ __forceinline__ void tail_stage(float2* x, float2* gout) {
    constexpr int NR = N / RT;
    constexpr int NB = (NR + NT - 1) / NT;
    float2 v[NB][RT];
    const int t = (int)threadIdx.x;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = t + i * NT;
        if (j < NR) {
#pragma unroll
            for (int r = 0; r < RT; ++r) v[i][r] = x[spad(j + r * NR)];
            Codelet<RT, float2>::run(v[i]);
        }
    }
    static_assert(NS * RT == N, "the tail is the last stage");
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = t + i * NT;
        if (j < NR) {
#pragma unroll
            for (int r = 0; r < RT; ++r) st_out<INV>(gout + j + r * NS, v[i][r]);
        }
    }
}

template <int N, int MODE, int S, int NS, int TWOFF, int W, bool INV>
__device__ __forceinline__ void run_mfma_stages(float2* x, float2* gout,
                                                const float2* __restrict__ tw,
                                                const typename SplitTraits<MODE>::V (&a1)[3],
                                                const typename SplitTraits<MODE>::V (&a2)[3],
                                                const float2 (&raw)[split_gpw<N, W>()][4]) {
    constexpr int S16 = split_stages16<N>();
    constexpr int RT = split_tail<N>();
    if constexpr (S < S16) {
        constexpr int TW2 = TWOFF + 15 * NS;  // next stage's twiddle segment
        constexpr int R2 = (S + 1 < S16) ? 16 : (RT > 1 ? RT : 0);
        mfma_stage<N, MODE, NS, R2, NS * 16, TW2, W, INV, S == 0, R2 == 0>(x, gout, tw, a1, a2, raw);
        run_mfma_stages<N, MODE, S + 1, NS * 16, TW2, W, INV>(x, gout, tw, a1, a2, raw);
    } else if constexpr (RT > 1) {
        tail_stage<N, RT, NS, 64 * W, INV>(x, gout);
    }
}

// Four-wave transforms (N = 1024 .. 4096) of the two-term modes are compiled
// for four resident workgroups per CU, the most their LDS allows (N = 4096,
// split fp16: 137 VGPRs + 16 AGPRs and three workgroups without the bound,
// 116 VGPRs with it: 155 -> 135 us at batch 8192; the three-term mode spills
// under it).
template <int MODE> constexpr bool split_bound4() { return MODE != FFTC_C64_SPLIT3_BF16; }
template <int N, int MODE, bool INV>
__global__ void __launch_bounds__(64 * split_waves<N>(), (split_waves<N>() == 4 && split_bound4<MODE>()) ? 4 : 1)
split_fft(const float2* in, float2* out, const float2* __restrict__ tw, int64_t batch) {
    using T = SplitTraits<MODE>;
    using V = typename T::V;
    using E = typename T::E;
    constexpr int W = split_waves<N>();
    constexpr int NT = 64 * W;
    constexpr int L = lds_len(N);
    __shared__ float2 xs[L];
    const int64_t b = blockIdx.x;
    const float2* x = in + b * N;
    float2* y = out + b * N;
    const int t = (int)threadIdx.x;
    // the first stage's inputs, loaded before anything else so the HBM
    // latency overlaps the operand setup below (16 lanes: 128 contiguous
    // bytes; a wave past the last group loads group 0 and discards it)
    constexpr int GPW = split_gpw<N, W>();
    float2 raw[GPW][4];
    {
        const int lane = t & 63, wave = t >> 6, n = lane & 15, g4 = lane >> 4;
#pragma unroll
        for (int gi = 0; gi < GPW; ++gi) {
            const int grp = wave + gi * W;
            const int j = (grp < N / 256 ? grp : 0) * 16 + n;
#pragma unroll
            for (int i = 0; i < 4; ++i) raw[gi][i] = ld_in<INV>(x + j + (4 * g4 + i) * (N / 16));
        }
    }
    // operands A1 = [Wr | -Wi], A2 = [Wi | Wr] for this lane, split, with the
    // contraction index k = 2 r + c (c = 0: real parts, 1: imaginary parts)
    V a1[3], a2[3];
    {
        const int lane = t & 63, m = lane & 15, g4 = lane >> 4;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = 8 * g4 + i, col = k >> 1;
            float c, s;
            w16((m * col) & 15, &c, &s);
            // W[m][col] = cos - i sin
            const float wr = c, wi = -s;
            const float v1 = (k & 1) ? -wi : wr;
            const float v2 = (k & 1) ? wr : wi;
            E p1[3], p2[3];
            split<MODE>(v1, p1);
            split<MODE>(v2, p2);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                a1[q][i] = q < T::TERMS ? p1[q] : (E)0.f;
                a2[q][i] = q < T::TERMS ? p2[q] : (E)0.f;
            }
        }
    }
    // the first stage reads HBM and the last writes it
    run_mfma_stages<N, MODE, 0, 1, 0, W, INV>(xs, y, tw, a1, a2, raw);
}

// ---------------------------------------------------------------------------

template <int N, int MODE>
static const void* split_fn(bool inv) {
    return inv ? reinterpret_cast<const void*>(&split_fft<N, MODE, true>)
               : reinterpret_cast<const void*>(&split_fft<N, MODE, false>);
}

template <int MODE>
static const void* split_fn_mode(int64_t n, bool inv) {
    switch (n) {
        case 256: return split_fn<256, MODE>(inv);
        case 512: return split_fn<512, MODE>(inv);
        case 1024: return split_fn<1024, MODE>(inv);
        case 2048: return split_fn<2048, MODE>(inv);
        case 4096: return split_fn<4096, MODE>(inv);
        case 8192: return split_fn<8192, MODE>(inv);
        case 16384: return split_fn<16384, MODE>(inv);
        default: return nullptr;
    }
}

bool split_supported(int64_t n) {
    return n == 256 || n == 512 || n == 1024 || n == 2048 || n == 4096 || n == 8192 || n == 16384;
}

std::vector<int> split_radices(int64_t n) {
    std::vector<int> rs;
    int64_t m = n;
    while (m % 16 == 0) {
        rs.push_back(16);
        m /= 16;
    }
    if (m > 1) rs.push_back((int)m);
    return rs;
}

int split_threads(int64_t n) { return 64 * split_waves_for(n); }

fftc_status launch_split(const fftc_plan_s* p, const void* in, void* out, int64_t batch, hipStream_t s) {
    const bool inv = p->direction == FFTC_INVERSE;
    const void* fn = nullptr;
    switch (p->dtype) {
        case FFTC_C64_SPLIT_F16: fn = split_fn_mode<FFTC_C64_SPLIT_F16>(p->n, inv); break;
        case FFTC_C64_SPLIT_BF16: fn = split_fn_mode<FFTC_C64_SPLIT_BF16>(p->n, inv); break;
        case FFTC_C64_SPLIT3_BF16: fn = split_fn_mode<FFTC_C64_SPLIT3_BF16>(p->n, inv); break;
        case FFTC_C64_F16: fn = split_fn_mode<FFTC_C64_F16>(p->n, inv); break;
        default: break;
    }
    if (!fn) return fail(FFTC_ERR_INTERNAL, "no split-precision kernel for this plan");
    const float2* tin = static_cast<const float2*>(in);
    float2* tout = static_cast<float2*>(out);
    const float2* tw = static_cast<const float2*>(p->tw);
    void* args[] = {(void*)&tin, (void*)&tout, (void*)&tw, (void*)&batch};
    hipError_t e = hipLaunchKernel(fn, dim3((unsigned)batch), dim3(split_threads(p->n)), args, 0, s);
    if (e != hipSuccess) return fail_hip(e, "hipLaunchKernel(split_fft)");
    return FFTC_OK;
}

}  // namespace fftc
