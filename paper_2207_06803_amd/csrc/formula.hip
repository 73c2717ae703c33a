// Execution of lowered formulas (passes I_p (x) E (x) I_q, see formula.h).
//
// Vectors that fit in LDS twice (two buffers) run as ONE kernel: a workgroup
// loads T whole vectors from HBM, runs every pass LDS to LDS (in place for
// DFT codelets and diagonals, ping-pong for Stockham stages, direct sums and
// permutations), and stores once -- the same one-read-one-write traffic as
// the Stockham kernels.  Longer vectors run one kernel per pass over HBM,
// alternating between the output and a scratch buffer.
//
// Index arithmetic: a pass on a tile of whole vectors is the same pass with
// p scaled by the number of vectors, so every unit index u decomposes with
// divisions by q, by the size of E and by one inner size.  These divide by
// runtime constants with the multiply-high method of Granlund and
// Montgomery (PLDI 1994): for d >= 1, l = ceil(log2 d),
// m = floor(2^32 (2^l - d) / d) + 1, and u div d = (mulhi(u, m) + u) >> l,
// exact for u < 2^31 (the sum cannot overflow 32 bits).
#include <array>

#include "codelets.h"
#include "cplx.h"
#include "formula.h"

namespace fftc {

struct FDiv {
    uint32_t m, l;
};

static FDiv make_fdiv(uint32_t d) {
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    const uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1;
    return {(uint32_t)m, l};
}

__device__ __forceinline__ uint32_t fdiv(uint32_t u, FDiv f) { return (__umulhi(u, f.m) + u) >> f.l; }

// Device descriptor of one pass.
struct FPass {
    int32_t kind, r;
    uint32_t n;      // size of E
    uint32_t q;      // I_q to the right of E
    uint32_t inner;  // STAGE: ns;  PERM: M = n / K;  DIAG: (unused)
    uint32_t k;      // PERM: K;  STAGE: n / r
    int32_t twoff;
    uint32_t units;  // work units per vector
    FDiv dq, dn, di; // divide by q, by n (STAGE: n / r), by inner
};

template <typename C> __device__ __forceinline__ C cj(C v, bool on) { return on ? cconj(v) : v; }

// LDS buffers are padded by one element every 16 (index i at i + i / 16),
// which spreads the stride-16 and stride-8 accesses of radix-16 / radix-8
// stages over the banks; HBM buffers are not (PAD = 0).
template <int PAD> __device__ __forceinline__ uint32_t ix(uint32_t i) { return PAD ? i + (i >> PAD) : i; }
__host__ __device__ constexpr uint32_t padded_len(uint32_t n) { return n + (n >> 4); }

// I_p (x) DFT_R (x) I_q: unit u = (group w, offset qi), elements w R q + qi + t q
template <int R, int PAD, typename C>
__device__ __forceinline__ void unit_dft(const FPass& ps, const C* src, C* dst, uint32_t u, bool ci, bool co) {
    const uint32_t w = fdiv(u, ps.dq), qi = u - w * ps.q;
    const uint32_t base = w * (uint32_t)R * ps.q + qi;
    C v[R];
#pragma unroll
    for (int t = 0; t < R; ++t) v[t] = cj(src[ix<PAD>(base + t * ps.q)], ci);
    Codelet<R, C>::run(v);
#pragma unroll
    for (int t = 0; t < R; ++t) dst[ix<PAD>(base + t * ps.q)] = cj(v[t], co);
}

// One Stockham stage of I_p (x) DFT_n (x) I_q, radix R after ns:
//   v_t = x[j + t n/R] w_{ns R}^{t (j mod ns)},  v = DFT_R v,
//   y[(j div ns) ns R + t ns + (j mod ns)] = v_t   (positions scaled by q)
template <int R, int PAD, typename C>
__device__ __forceinline__ void unit_stage(const FPass& ps, const C* src, C* dst, const C* __restrict__ tw, uint32_t u,
                                           bool ci, bool co) {
    const uint32_t w = fdiv(u, ps.dq), qi = u - w * ps.q;
    const uint32_t g = fdiv(w, ps.dn), j = w - g * ps.k;  // k = n / R
    const uint32_t jd = fdiv(j, ps.di), kk = j - jd * ps.inner;
    const uint32_t gb = g * ps.n * ps.q + qi;
    C v[R];
#pragma unroll
    for (int t = 0; t < R; ++t) v[t] = cj(src[ix<PAD>(gb + (j + t * ps.k) * ps.q)], ci);
    if (ps.inner > 1) {
        const C* twr = tw + ps.twoff + kk;
#pragma unroll
        for (int t = 1; t < R; ++t) v[t] = cmul(v[t], twr[(t - 1) * ps.inner]);
    }
    Codelet<R, C>::run(v);
    const uint32_t ob = gb + (jd * ps.inner * R + kk) * ps.q;
#pragma unroll
    for (int t = 0; t < R; ++t) dst[ix<PAD>(ob + t * ps.inner * ps.q)] = cj(v[t], co);
}

// Output u = (g, k, qi) of I_p (x) DFT_n (x) I_q summed directly.
template <int PAD, typename C>
__device__ __forceinline__ void unit_direct(const FPass& ps, const C* src, C* dst, const C* __restrict__ tw, uint32_t u,
                                            bool ci, bool co) {
    const uint32_t w = fdiv(u, ps.dq), qi = u - w * ps.q;
    const uint32_t g = fdiv(w, ps.dn), kk = w - g * ps.n;
    const uint32_t xb = g * ps.n * ps.q + qi;
    const C* wt = tw + ps.twoff;
    C acc;
    acc.x = 0;
    acc.y = 0;
    uint32_t e = 0;
    for (uint32_t j = 0; j < ps.n; ++j) {
        const C xv = cj(src[ix<PAD>(xb + j * ps.q)], ci), wv = wt[e];
        acc = mk(acc.x + xv.x * wv.x - xv.y * wv.y, acc.y + xv.x * wv.y + xv.y * wv.x);
        e += kk;
        if (e >= ps.n) e -= ps.n;
    }
    dst[ix<PAD>(u)] = cj(acc, co);
}

// I_p (x) D^n_M (x) I_q: element u times w_n^{i j}, (i M + j) = (u div q) mod n
template <int PAD, typename C>
__device__ __forceinline__ void unit_diag(const FPass& ps, const C* src, C* dst, const C* __restrict__ tw, uint32_t u,
                                          bool ci, bool co) {
    const uint32_t w = fdiv(u, ps.dq);
    const uint32_t t = w - fdiv(w, ps.dn) * ps.n;
    dst[ix<PAD>(u)] = cj(cmul(cj(src[ix<PAD>(u)], ci), tw[ps.twoff + t]), co);
}

// I_p (x) Pi^n_K (x) I_q: output (g, i M + j, qi) <- input (g, j K + i, qi)
template <int PAD, typename C>
__device__ __forceinline__ void unit_perm(const FPass& ps, const C* src, C* dst, uint32_t u, bool ci, bool co) {
    const uint32_t w = fdiv(u, ps.dq), qi = u - w * ps.q;
    const uint32_t g = fdiv(w, ps.dn), o = w - g * ps.n;
    const uint32_t i = fdiv(o, ps.di), j = o - i * ps.inner;
    dst[ix<PAD>(u)] = cj(src[ix<PAD>((g * ps.n + j * ps.k + i) * ps.q + qi)], ci ^ co);
}

#define FFTC_RADIX_CASES(X) X(2) X(3) X(4) X(5) X(7) X(8) X(16)

// Units [u0, U) with stride `step` of one pass; src == dst allowed for DFT and DIAG.
template <int PAD, typename C>
__device__ __forceinline__ void run_pass(const FPass& ps, const C* src, C* dst, const C* __restrict__ tw, uint32_t U,
                                         uint32_t u0, uint32_t step, bool ci, bool co) {
    switch (ps.kind) {
        case FP_DFT:
            switch (ps.r) {
#define FFTC_CASE(R) \
    case R:          \
        for (uint32_t u = u0; u < U; u += step) unit_dft<R, PAD>(ps, src, dst, u, ci, co); \
        break;
                FFTC_RADIX_CASES(FFTC_CASE)
#undef FFTC_CASE
            }
            break;
        case FP_STAGE:
            switch (ps.r) {
#define FFTC_CASE(R) \
    case R:          \
        for (uint32_t u = u0; u < U; u += step) unit_stage<R, PAD>(ps, src, dst, tw, u, ci, co); \
        break;
                FFTC_RADIX_CASES(FFTC_CASE)
#undef FFTC_CASE
            }
            break;
        case FP_DIRECT:
            for (uint32_t u = u0; u < U; u += step) unit_direct<PAD>(ps, src, dst, tw, u, ci, co);
            break;
        case FP_DIAG:
            for (uint32_t u = u0; u < U; u += step) unit_diag<PAD>(ps, src, dst, tw, u, ci, co);
            break;
        case FP_PERM:
            for (uint32_t u = u0; u < U; u += step) unit_perm<PAD>(ps, src, dst, u, ci, co);
            break;
        default:
            for (uint32_t u = u0; u < U; u += step) dst[ix<PAD>(u)] = cj(src[ix<PAD>(u)], ci ^ co);
            break;
    }
}

__host__ __device__ constexpr bool pass_in_place(int kind) { return kind == FP_DFT || kind == FP_DIAG; }

// One LDS run: passes that all act within sub-vectors of length L.  The
// vector (per batch row) is viewed as [o < P0][l < L][i < Q0] and a run whose
// passes have P0 | p and Q0 | q acts on each sub-vector (o, ., i) as the
// passes with p / P0 and q / Q0.  A workgroup takes T consecutive outer
// indices g = row P0 + o (g < G) and Cc consecutive inner indices i (Cc | Q0)
// and keeps them in LDS as [t][l][c], on which the passes are
// I_{T p/P0} (x) E (x) I_{(q/Q0) Cc} -- so the pass code is unchanged and
// rows of Cc contiguous elements are read and written.  The tile is read
// whole before any write, so a run may write over its own input.
struct RunGeom {
    uint32_t L, Q0, Cc, T, nib;  // nib = Q0 / Cc
    int64_t G;
    FDiv d_lc, d_c, d_nib;       // divide by L Cc, by Cc, by nib
};

template <typename C>
__global__ void __launch_bounds__(512)
formula_lds(const C* in, C* out, const FPass* __restrict__ passes, int npass, const C* __restrict__ tw,
            RunGeom g, int ci, int co) {
    extern __shared__ unsigned char formula_smem[];
    const uint32_t tile = g.T * g.L * g.Cc;
    C* a = reinterpret_cast<C*>(formula_smem);
    C* b = a + padded_len(tile);
    const uint32_t blk = blockIdx.x;
    const uint32_t gb = fdiv(blk, g.d_nib), ib = blk - gb * g.nib;
    const int64_t g0 = (int64_t)gb * g.T;
    const uint32_t nv = (uint32_t)min<int64_t>(g.T, g.G - g0);
    const uint32_t valid = nv * g.L * g.Cc;
    const uint32_t i0 = ib * g.Cc;
    const uint32_t tid = threadIdx.x, nth = blockDim.x;
    const uint32_t rowlen = g.L * g.Q0;  // elements per outer index
    C zero;
    zero.x = 0;
    zero.y = 0;
    // tile element e = (t, l, c) lives at (g0 + t) L Q0 + l Q0 + i0 + c
    const bool contiguous = g.Q0 == 1;  // whole vectors: the tile is one contiguous range
    auto addr = [&](uint32_t e) {
        if (contiguous) return (uint32_t)g0 * rowlen + e;
        const uint32_t t = fdiv(e, g.d_lc), rem = e - t * g.L * g.Cc;
        const uint32_t l = fdiv(rem, g.d_c), c = rem - l * g.Cc;
        return (uint32_t)g0 * rowlen + t * rowlen + l * g.Q0 + i0 + c;
    };
    // loads in batches of kLoadBatch per thread, issued before any is used,
    // so each batch waits for HBM once
    constexpr int kLoadBatch = 8;
    for (uint32_t base = 0; base < tile; base += kLoadBatch * nth) {
        C r[kLoadBatch];
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k) {
            const uint32_t e = base + k * nth + tid;
            r[k] = e < valid ? in[addr(e)] : zero;
        }
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k) {
            const uint32_t e = base + k * nth + tid;
            if (e < tile) a[ix<4>(e)] = cj(r[k], ci != 0);
        }
    }
    __syncthreads();
    C* cur = a;
    C* oth = b;
    for (int k = 0; k < npass; ++k) {
        const FPass ps = passes[k];
        const uint32_t U = ps.units * g.T;
        if (pass_in_place(ps.kind)) {
            run_pass<4>(ps, cur, cur, tw, U, tid, nth, false, false);
        } else {
            run_pass<4>(ps, cur, oth, tw, U, tid, nth, false, false);
            C* t = cur;
            cur = oth;
            oth = t;
        }
        __syncthreads();
    }
    for (uint32_t e = tid; e < valid; e += nth) out[addr(e)] = cj(cur[ix<4>(e)], co != 0);
}

// One pass over every vector in HBM.
template <typename C>
__global__ void __launch_bounds__(256)
formula_pass(const C* src, C* dst, FPass ps, const C* __restrict__ tw, uint32_t U, int ci, int co) {
    run_pass<0>(ps, src, dst, tw, U, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, ci != 0, co != 0);
}

// A launch of the execution: an LDS run of passes [first, first + count) of
// the device list (localised to its sub-vectors), or one HBM pass.
struct FStep {
    bool lds;
    int first, count;  // device descriptors
    RunGeom geom;      // LDS run
    int threads;
    size_t lds_bytes;
};

struct FormulaExec {
    int dtype = FFTC_C64;
    int64_t dim = 0, batch = 0;
    std::vector<FPass> host;  // device descriptors, runs back to back
    std::vector<FStep> steps;
    FPass* dev = nullptr;
    void* tw = nullptr;
    void* scratch = nullptr;
};

static size_t csize(int dtype) { return dtype == FFTC_C128 ? 16 : 8; }

// largest L with two padded buffers in one workgroup's LDS
int64_t formula_lds_max_dim(int dtype) {
    const int64_t per = kLdsMaxPerGroup / (2 * (int64_t)csize(dtype));
    int64_t L = per * 16 / 17;
    while (padded_len((uint32_t)(L + 1)) <= per) ++L;
    return L;
}

// Device descriptor of a pass acting on vectors of length `len` as
// I_p (x) E (x) I_q.
static FPass to_dev(const FormulaPass& s, int64_t len, int64_t p, int64_t q) {
    FPass d{};
    d.kind = s.kind;
    d.r = s.r;
    d.n = (uint32_t)s.n;
    d.q = (uint32_t)q;
    (void)p;
    d.twoff = (int32_t)std::max<int64_t>(s.twoff, 0);
    uint32_t dn = (uint32_t)s.n, di = 1;
    switch (s.kind) {
        case FP_DFT: d.units = (uint32_t)(len / s.r); break;
        case FP_STAGE:
            d.inner = (uint32_t)s.ns;
            d.k = (uint32_t)(s.n / s.r);
            dn = d.k;
            di = d.inner;
            d.units = (uint32_t)(len / s.r);
            break;
        case FP_PERM:
            d.k = (uint32_t)s.a;
            d.inner = (uint32_t)(s.n / s.a);
            di = d.inner;
            d.units = (uint32_t)len;
            break;
        default:
            d.units = (uint32_t)len;
            break;
    }
    d.dq = make_fdiv(d.q);
    d.dn = make_fdiv(dn);
    d.di = make_fdiv(di);
    return d;
}

static int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Geometry of an LDS run with outer / inner factors P0, Q0 over `batch` vectors.
static RunGeom make_geom(int64_t dim, int64_t batch, int64_t P0, int64_t Q0, size_t cs, int* threads, size_t* lds) {
    RunGeom g{};
    g.L = (uint32_t)(dim / (P0 * Q0));
    g.Q0 = (uint32_t)Q0;
    // columns per tile: the largest divisor of Q0 up to 16 (rows of up to
    // 128 B of complex64) that still fits two buffers in LDS
    uint32_t cc = 1;
    for (uint32_t c = 16; c >= 1; --c)
        if (Q0 % c == 0 && 2 * (size_t)padded_len(g.L * c) * cs <= (size_t)kLdsMaxPerGroup) {
            cc = c;
            break;
        }
    g.Cc = cc;
    g.nib = (uint32_t)(Q0 / cc);
    g.G = batch * P0;
    // tiles of about 8 KiB per buffer (or one sub-vector) and about 8
    // elements per thread: measured best over 8-32 KiB and 4-16 elements
    const int64_t sub = (int64_t)g.L * cc;
    int64_t T = std::max<int64_t>(1, 8192 / (sub * (int64_t)cs));
    T = std::min<int64_t>(T, g.G);
    g.T = (uint32_t)T;
    g.d_lc = make_fdiv((uint32_t)sub);
    g.d_c = make_fdiv(cc);
    g.d_nib = make_fdiv(g.nib);
    *lds = 2 * (size_t)padded_len((uint32_t)(T * sub)) * cs;
    const int64_t th = (T * sub / 8 + 63) / 64 * 64;
    *threads = (int)std::min<int64_t>(512, std::max<int64_t>(64, th));
    return g;
}

void formula_destroy(FormulaExec* fx) {
    if (!fx) return;
    if (fx->dev) hipFree(fx->dev);
    if (fx->tw) hipFree(fx->tw);
    if (fx->scratch) hipFree(fx->scratch);
    delete fx;
}

fftc_status formula_prepare(const FormulaProgram& prog, int dtype, int64_t batch, int flags, FormulaExec** out,
                            size_t* table_bytes, size_t* scratch_bytes, int* kernels) {
    *out = nullptr;
    if (prog.dim * batch >= (int64_t(1) << 31))
        return fail(FFTC_ERR_INVALID_ARG, "formula plans take batch * dim < 2^31 elements");
    FormulaExec* fx = new (std::nothrow) FormulaExec();
    if (!fx) return fail(FFTC_ERR_OUT_OF_MEMORY, "host allocation failed");
    fx->dtype = dtype;
    fx->dim = prog.dim;
    fx->batch = batch;
    const size_t cs = csize(dtype);
    const int64_t D = prog.dim, cap = formula_lds_max_dim(dtype);
    const bool per_pass = (flags & FFTC_FORMULA_HBM_PASSES) != 0;
    // Greedy runs: extend while the sub-vector length D / (gcd p, gcd q) fits LDS.
    const auto& ps = prog.passes;
    size_t k = 0;
    while (k < ps.size()) {
        int64_t P0 = ps[k].p, Q0 = ps[k].q;
        size_t e = k + 1;
        const bool fits = !per_pass && D / (P0 * Q0) <= cap;
        if (fits) {
            while (e < ps.size()) {
                const int64_t p2 = gcd64(P0, ps[e].p), q2 = gcd64(Q0, ps[e].q);
                if (D / (p2 * q2) > cap) break;
                P0 = p2;
                Q0 = q2;
                ++e;
            }
            FStep st{};
            st.lds = true;
            st.first = (int)fx->host.size();
            st.count = (int)(e - k);
            st.geom = make_geom(D, batch, P0, Q0, cs, &st.threads, &st.lds_bytes);
            const int64_t L = st.geom.L, Cc = st.geom.Cc;
            for (size_t j = k; j < e; ++j)
                fx->host.push_back(to_dev(ps[j], L * Cc, ps[j].p / P0, ps[j].q / Q0 * Cc));
            fx->steps.push_back(st);
        } else {
            FStep st{};
            st.lds = false;
            st.first = (int)fx->host.size();
            st.count = 1;
            fx->host.push_back(to_dev(ps[k], D, ps[k].p, ps[k].q));
            fx->steps.push_back(st);
        }
        k = e;
    }
    *kernels = (int)fx->steps.size();
    // (scratch: every execution but a single LDS run may need a second buffer)
    hipError_t e = hipSuccess;
    fftc_status st = dev_malloc((void**)&fx->dev, sizeof(FPass) * fx->host.size(), "hipMalloc(formula passes)");
    if (st == FFTC_OK) {
        e = hipMemcpy(fx->dev, fx->host.data(), sizeof(FPass) * fx->host.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) st = fail_hip(e, "formula pass list");
    }
    *table_bytes = (size_t)std::max<int64_t>(prog.table_entries, 1) * cs;
    if (st == FFTC_OK) st = dev_malloc(&fx->tw, *table_bytes, "hipMalloc(formula tables)");
    if (st == FFTC_OK) st = make_twiddles(fx->tw, dtype, prog.tables, nullptr);
    *scratch_bytes = 0;
    const bool one_lds = fx->steps.size() == 1 && fx->steps[0].lds;
    if (st == FFTC_OK && !one_lds) {
        *scratch_bytes = (size_t)batch * (size_t)prog.dim * cs;
        st = dev_malloc(&fx->scratch, *scratch_bytes, "hipMalloc(formula scratch)");
    }
    if (st == FFTC_OK) {
        // per kernel, not per plan: allow the largest tile any plan uses
        const void* kf = dtype == FFTC_C128 ? (const void*)&formula_lds<double2> : (const void*)&formula_lds<float2>;
        e = hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMaxPerGroup);
        if (e != hipSuccess) st = fail_hip(e, "hipFuncSetAttribute(formula)");
    }
    if (st != FFTC_OK) {
        formula_destroy(fx);
        return st;
    }
    *out = fx;
    return FFTC_OK;
}

// Buffers of a multi-kernel execution: which buffer every step writes.
// Steps that are not in place (Stockham stages, direct sums, permutations
// as HBM passes) need a destination other than their source; the input is
// written only when it is also the output; the last step must write the
// output.  Backward feasibility over the buffers, then a forward choice that
// prefers staying in place; the caller adds a final copy when nothing fits.
enum { BUF_IN = 0, BUF_OUT = 1, BUF_SCR = 2 };

static bool assign_buffers(const std::vector<bool>& inplace, bool same, std::vector<int>* dst) {
    const size_t k = inplace.size();
    auto legal = [&](size_t i, int from, int to) { return inplace[i] || to != from; };
    // ok[i][b]: with the data in buffer b before step i, the steps can end in BUF_OUT
    std::vector<std::array<bool, 3>> ok(k + 1);
    ok[k] = {false, true, false};
    for (size_t i = k; i-- > 0;)
        for (int b = 0; b < 3; ++b)
            ok[i][b] = (legal(i, b, BUF_OUT) && ok[i + 1][BUF_OUT]) || (legal(i, b, BUF_SCR) && ok[i + 1][BUF_SCR]);
    int cur = same ? BUF_OUT : BUF_IN;  // in place: the input is the output buffer
    if (!ok[0][cur]) return false;
    dst->assign(k, BUF_OUT);
    for (size_t i = 0; i < k; ++i) {
        int pick = -1;
        if (cur != BUF_IN && inplace[i] && ok[i + 1][cur]) pick = cur;
        for (int d = BUF_OUT; d <= BUF_SCR && pick < 0; ++d)
            if (legal(i, cur, d) && ok[i + 1][d]) pick = d;
        if (pick < 0) return false;
        (*dst)[i] = pick;
        cur = pick;
    }
    return true;
}

template <typename C>
static void launch_step(const FormulaExec* fx, const FStep& st, const FPass* hostpass, const void* src, void* dst,
                        int64_t batch, int ci, int co, hipStream_t s) {
    if (st.lds) {
        RunGeom g = st.geom;
        g.G = g.G / fx->batch * batch;  // G = batch P0
        g.T = (uint32_t)std::min<int64_t>(g.T, g.G);
        const int64_t tiles = (g.G + g.T - 1) / g.T * g.nib;
        const size_t lds = 2 * (size_t)padded_len(g.T * g.L * g.Cc) * sizeof(C);
        hipLaunchKernelGGL(formula_lds<C>, dim3((unsigned)tiles), dim3(st.threads), lds, s, (const C*)src, (C*)dst,
                           fx->dev + st.first, st.count, (const C*)fx->tw, g, ci, co);
    } else {
        const uint32_t U = (uint32_t)(hostpass->units * batch);
        const int64_t blocks = std::min<int64_t>((U + 255) / 256, 65536);
        hipLaunchKernelGGL(formula_pass<C>, dim3((unsigned)blocks), dim3(256), 0, s, (const C*)src, (C*)dst,
                           *hostpass, (const C*)fx->tw, U, ci, co);
    }
}

fftc_status formula_launch(FormulaExec* fx, const void* in, void* out, int64_t batch, bool inverse, hipStream_t s) {
    std::vector<FStep> steps = fx->steps;
    std::vector<FPass> extra;  // a final copy, if the buffers need one
    std::vector<bool> inplace;
    for (const auto& st : steps) inplace.push_back(st.lds || pass_in_place(fx->host[st.first].kind));
    const bool same = in == out;
    std::vector<int> dsts;
    if (!assign_buffers(inplace, same, &dsts)) {
        FormulaPass cp;
        cp.kind = FP_COPY;
        cp.n = fx->dim;
        extra.push_back(to_dev(cp, fx->dim, 1, 1));
        FStep st{};
        st.lds = false;
        st.first = -1;
        st.count = 1;
        steps.push_back(st);
        inplace.push_back(false);
        if (!assign_buffers(inplace, same, &dsts)) return fail(FFTC_ERR_INTERNAL, "formula buffer assignment");
    }
    const void* bufs[3] = {in, out, fx->scratch};
    const void* cur = in;
    for (size_t i = 0; i < steps.size(); ++i) {
        const FStep& st = steps[i];
        void* dst = const_cast<void*>(bufs[dsts[i]]);
        const FPass* hp = st.first >= 0 ? &fx->host[st.first] : &extra[0];
        const int ci = (i == 0 && inverse) ? 1 : 0, co = (i + 1 == steps.size() && inverse) ? 1 : 0;
        if (fx->dtype == FFTC_C128)
            launch_step<double2>(fx, st, hp, cur, dst, batch, ci, co, s);
        else
            launch_step<float2>(fx, st, hp, cur, dst, batch, ci, co, s);
        FFTC_HIP_TRY(hipGetLastError());
        cur = dst;
    }
    return FFTC_OK;
}

}  // namespace fftc
