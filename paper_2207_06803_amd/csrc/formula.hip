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

// I_p (x) DFT_R (x) I_q: unit u = (group w, offset qi), elements w R q + qi + t q
template <int R, typename C>
__device__ __forceinline__ void unit_dft(const FPass& ps, const C* src, C* dst, uint32_t u, bool ci, bool co) {
    const uint32_t w = fdiv(u, ps.dq), qi = u - w * ps.q;
    const uint32_t base = w * (uint32_t)R * ps.q + qi;
    C v[R];
#pragma unroll
    for (int t = 0; t < R; ++t) v[t] = cj(src[base + t * ps.q], ci);
    Codelet<R, C>::run(v);
#pragma unroll
    for (int t = 0; t < R; ++t) dst[base + t * ps.q] = cj(v[t], co);
}

// One Stockham stage of I_p (x) DFT_n (x) I_q, radix R after ns:
//   v_t = x[j + t n/R] w_{ns R}^{t (j mod ns)},  v = DFT_R v,
//   y[(j div ns) ns R + t ns + (j mod ns)] = v_t   (positions scaled by q)
template <int R, typename C>
__device__ __forceinline__ void unit_stage(const FPass& ps, const C* src, C* dst, const C* __restrict__ tw, uint32_t u,
                                           bool ci, bool co) {
    const uint32_t w = fdiv(u, ps.dq), qi = u - w * ps.q;
    const uint32_t g = fdiv(w, ps.dn), j = w - g * ps.k;  // k = n / R
    const uint32_t jd = fdiv(j, ps.di), kk = j - jd * ps.inner;
    const uint32_t gb = g * ps.n * ps.q + qi;
    C v[R];
#pragma unroll
    for (int t = 0; t < R; ++t) v[t] = cj(src[gb + (j + t * ps.k) * ps.q], ci);
    if (ps.inner > 1) {
        const C* twr = tw + ps.twoff + kk;
#pragma unroll
        for (int t = 1; t < R; ++t) v[t] = cmul(v[t], twr[(t - 1) * ps.inner]);
    }
    Codelet<R, C>::run(v);
    const uint32_t ob = gb + (jd * ps.inner * R + kk) * ps.q;
#pragma unroll
    for (int t = 0; t < R; ++t) dst[ob + t * ps.inner * ps.q] = cj(v[t], co);
}

// Output u = (g, k, qi) of I_p (x) DFT_n (x) I_q summed directly.
template <typename C>
__device__ __forceinline__ void unit_direct(const FPass& ps, const C* src, C* dst, const C* __restrict__ tw, uint32_t u,
                                            bool ci, bool co) {
    const uint32_t w = fdiv(u, ps.dq), qi = u - w * ps.q;
    const uint32_t g = fdiv(w, ps.dn), kk = w - g * ps.n;
    const C* x = src + g * ps.n * ps.q + qi;
    const C* wt = tw + ps.twoff;
    C acc;
    acc.x = 0;
    acc.y = 0;
    uint32_t e = 0;
    for (uint32_t j = 0; j < ps.n; ++j) {
        const C xv = cj(x[j * ps.q], ci), wv = wt[e];
        acc = mk(acc.x + xv.x * wv.x - xv.y * wv.y, acc.y + xv.x * wv.y + xv.y * wv.x);
        e += kk;
        if (e >= ps.n) e -= ps.n;
    }
    dst[u] = cj(acc, co);
}

// I_p (x) D^n_M (x) I_q: element u times w_n^{i j}, (i M + j) = (u div q) mod n
template <typename C>
__device__ __forceinline__ void unit_diag(const FPass& ps, const C* src, C* dst, const C* __restrict__ tw, uint32_t u,
                                          bool ci, bool co) {
    const uint32_t w = fdiv(u, ps.dq);
    const uint32_t t = w - fdiv(w, ps.dn) * ps.n;
    dst[u] = cj(cmul(cj(src[u], ci), tw[ps.twoff + t]), co);
}

// I_p (x) Pi^n_K (x) I_q: output (g, i M + j, qi) <- input (g, j K + i, qi)
template <typename C>
__device__ __forceinline__ void unit_perm(const FPass& ps, const C* src, C* dst, uint32_t u, bool ci, bool co) {
    const uint32_t w = fdiv(u, ps.dq), qi = u - w * ps.q;
    const uint32_t g = fdiv(w, ps.dn), o = w - g * ps.n;
    const uint32_t i = fdiv(o, ps.di), j = o - i * ps.inner;
    dst[u] = cj(src[(g * ps.n + j * ps.k + i) * ps.q + qi], ci ^ co);
}

#define FFTC_RADIX_CASES(X) X(2) X(3) X(4) X(5) X(7) X(8) X(16)

// Units [u0, U) with stride `step` of one pass; src == dst allowed for DFT and DIAG.
template <typename C>
__device__ __forceinline__ void run_pass(const FPass& ps, const C* src, C* dst, const C* __restrict__ tw, uint32_t U,
                                         uint32_t u0, uint32_t step, bool ci, bool co) {
    switch (ps.kind) {
        case FP_DFT:
            switch (ps.r) {
#define FFTC_CASE(R) \
    case R:          \
        for (uint32_t u = u0; u < U; u += step) unit_dft<R>(ps, src, dst, u, ci, co); \
        break;
                FFTC_RADIX_CASES(FFTC_CASE)
#undef FFTC_CASE
            }
            break;
        case FP_STAGE:
            switch (ps.r) {
#define FFTC_CASE(R) \
    case R:          \
        for (uint32_t u = u0; u < U; u += step) unit_stage<R>(ps, src, dst, tw, u, ci, co); \
        break;
                FFTC_RADIX_CASES(FFTC_CASE)
#undef FFTC_CASE
            }
            break;
        case FP_DIRECT:
            for (uint32_t u = u0; u < U; u += step) unit_direct(ps, src, dst, tw, u, ci, co);
            break;
        case FP_DIAG:
            for (uint32_t u = u0; u < U; u += step) unit_diag(ps, src, dst, tw, u, ci, co);
            break;
        case FP_PERM:
            for (uint32_t u = u0; u < U; u += step) unit_perm(ps, src, dst, u, ci, co);
            break;
        default:
            for (uint32_t u = u0; u < U; u += step) dst[u] = cj(src[u], ci ^ co);
            break;
    }
}

__host__ __device__ constexpr bool pass_in_place(int kind) { return kind == FP_DFT || kind == FP_DIAG; }

// One workgroup: T whole vectors through every pass in LDS.
template <typename C>
__global__ void __launch_bounds__(512)
formula_lds(const C* in, C* out, const FPass* __restrict__ passes, int npass, const C* __restrict__ tw,
            uint32_t dim, uint32_t T, int64_t nvec, int inv) {
    extern __shared__ unsigned char formula_smem[];
    C* a = reinterpret_cast<C*>(formula_smem);
    C* b = a + (size_t)T * dim;
    const int64_t v0 = (int64_t)blockIdx.x * T;
    const uint32_t nv = (uint32_t)min<int64_t>(T, nvec - v0);
    const uint32_t tot = T * dim, valid = nv * dim;
    const uint32_t tid = threadIdx.x, nth = blockDim.x;
    const C* src = in + v0 * dim;
    C zero;
    zero.x = 0;
    zero.y = 0;
    for (uint32_t i = tid; i < tot; i += nth) a[i] = i < valid ? cj(src[i], inv != 0) : zero;
    __syncthreads();
    C* cur = a;
    C* oth = b;
    for (int k = 0; k < npass; ++k) {
        const FPass ps = passes[k];
        const uint32_t U = ps.units * T;
        if (pass_in_place(ps.kind)) {
            run_pass(ps, cur, cur, tw, U, tid, nth, false, false);
        } else {
            run_pass(ps, cur, oth, tw, U, tid, nth, false, false);
            C* t = cur;
            cur = oth;
            oth = t;
        }
        __syncthreads();
    }
    C* dst = out + v0 * dim;
    for (uint32_t i = tid; i < valid; i += nth) dst[i] = cj(cur[i], inv != 0);
}

// One pass over every vector in HBM.
template <typename C>
__global__ void __launch_bounds__(256)
formula_pass(const C* src, C* dst, FPass ps, const C* __restrict__ tw, uint32_t U, int ci, int co) {
    run_pass(ps, src, dst, tw, U, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, ci != 0, co != 0);
}

struct FormulaExec {
    int dtype = FFTC_C64;
    int64_t dim = 0, batch = 0;
    bool lds = false;
    uint32_t T = 1;
    int threads = 256;
    size_t lds_bytes = 0;
    std::vector<FPass> host;
    FPass* dev = nullptr;
    void* tw = nullptr;
    void* scratch = nullptr;
};

static size_t csize(int dtype) { return dtype == FFTC_C128 ? 16 : 8; }

int64_t formula_lds_max_dim(int dtype) { return kLdsMaxPerGroup / (2 * (int64_t)csize(dtype)); }

static FPass to_dev(const FormulaPass& s, int64_t dim) {
    FPass d{};
    d.kind = s.kind;
    d.r = s.r;
    d.n = (uint32_t)s.n;
    d.q = (uint32_t)s.q;
    d.twoff = (int32_t)std::max<int64_t>(s.twoff, 0);
    uint32_t dn = (uint32_t)s.n, di = 1;
    switch (s.kind) {
        case FP_DFT: d.units = (uint32_t)(dim / s.r); break;
        case FP_STAGE:
            d.inner = (uint32_t)s.ns;
            d.k = (uint32_t)(s.n / s.r);
            dn = d.k;
            di = d.inner;
            d.units = (uint32_t)(dim / s.r);
            break;
        case FP_PERM:
            d.k = (uint32_t)s.a;
            d.inner = (uint32_t)(s.n / s.a);
            di = d.inner;
            d.units = (uint32_t)dim;
            break;
        default:
            d.units = (uint32_t)dim;
            break;
    }
    d.dq = make_fdiv(d.q);
    d.dn = make_fdiv(dn);
    d.di = make_fdiv(di);
    return d;
}

void formula_destroy(FormulaExec* fx) {
    if (!fx) return;
    if (fx->dev) hipFree(fx->dev);
    if (fx->tw) hipFree(fx->tw);
    if (fx->scratch) hipFree(fx->scratch);
    delete fx;
}

fftc_status formula_prepare(const FormulaProgram& prog, int dtype, int64_t batch, int flags, FormulaExec** out,
                            size_t* table_bytes, size_t* scratch_bytes) {
    *out = nullptr;
    if (prog.dim * batch >= (int64_t(1) << 31))
        return fail(FFTC_ERR_INVALID_ARG, "formula plans take batch * dim < 2^31 elements");
    FormulaExec* fx = new (std::nothrow) FormulaExec();
    if (!fx) return fail(FFTC_ERR_OUT_OF_MEMORY, "host allocation failed");
    fx->dtype = dtype;
    fx->dim = prog.dim;
    fx->batch = batch;
    const size_t cs = csize(dtype);
    fx->lds = !(flags & FFTC_FORMULA_HBM_PASSES) && prog.dim <= formula_lds_max_dim(dtype);
    if (fx->lds) {
        // about 32 KiB per buffer: two workgroups of two buffers fit a CU
        int64_t T = std::max<int64_t>(1, 32768 / (prog.dim * (int64_t)cs));
        T = std::min<int64_t>(T, batch);
        fx->T = (uint32_t)T;
        fx->lds_bytes = 2 * (size_t)T * (size_t)prog.dim * cs;
        fx->threads = (size_t)T * prog.dim > 4096 ? 512 : 256;
    }
    for (const auto& s : prog.passes) fx->host.push_back(to_dev(s, prog.dim));
    fftc_status st = FFTC_OK;
    hipError_t e = hipMalloc(&fx->dev, sizeof(FPass) * fx->host.size());
    if (e == hipSuccess)
        e = hipMemcpy(fx->dev, fx->host.data(), sizeof(FPass) * fx->host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) st = fail_hip(e, "formula pass list");
    *table_bytes = (size_t)std::max<int64_t>(prog.table_entries, 1) * cs;
    if (st == FFTC_OK) {
        e = hipMalloc(&fx->tw, *table_bytes);
        if (e != hipSuccess) st = fail_hip(e, "hipMalloc(formula tables)");
    }
    if (st == FFTC_OK) st = make_twiddles(fx->tw, dtype, prog.tables, nullptr);
    *scratch_bytes = 0;
    if (st == FFTC_OK && !fx->lds) {
        *scratch_bytes = (size_t)batch * (size_t)prog.dim * cs;
        e = hipMalloc(&fx->scratch, *scratch_bytes);
        if (e != hipSuccess) st = fail_hip(e, "hipMalloc(formula scratch)");
    }
    if (st == FFTC_OK && fx->lds) {
        const void* k = dtype == FFTC_C128 ? (const void*)&formula_lds<double2> : (const void*)&formula_lds<float2>;
        // per kernel, not per plan: allow the largest tile any plan uses
        e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMaxPerGroup);
        if (e != hipSuccess) st = fail_hip(e, "hipFuncSetAttribute(formula)");
    }
    if (st != FFTC_OK) {
        formula_destroy(fx);
        return st;
    }
    *out = fx;
    return FFTC_OK;
}

// Buffers of the HBM path: which buffer every pass writes.  Out-of-place
// passes need a destination other than their source; the input is written
// only when it is also the output; the last pass must write the output.
// Backward feasibility over the buffers, then a forward choice that prefers
// staying in place; the caller adds a final copy when nothing fits.
enum { BUF_IN = 0, BUF_OUT = 1, BUF_SCR = 2 };

static bool assign_buffers(const std::vector<int>& kinds, bool same, std::vector<int>* dst) {
    const size_t k = kinds.size();
    auto legal = [&](size_t i, int from, int to) { return pass_in_place(kinds[i]) || to != from; };
    // ok[i][b]: with the data in buffer b before pass i, the passes can end in BUF_OUT
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
        if (cur != BUF_IN && pass_in_place(kinds[i]) && ok[i + 1][cur]) pick = cur;
        for (int d = BUF_OUT; d <= BUF_SCR && pick < 0; ++d)
            if (legal(i, cur, d) && ok[i + 1][d]) pick = d;
        if (pick < 0) return false;
        (*dst)[i] = pick;
        cur = pick;
    }
    return true;
}

fftc_status formula_launch(FormulaExec* fx, const void* in, void* out, int64_t batch, bool inverse, hipStream_t s) {
    const size_t cs = csize(fx->dtype);
    if (fx->lds) {
        const uint32_t T = (uint32_t)std::min<int64_t>(fx->T, batch);
        const int64_t groups = (batch + T - 1) / T;
        const size_t lds = 2 * (size_t)T * (size_t)fx->dim * cs;
        if (groups > 0x7fffffff) return fail(FFTC_ERR_INVALID_ARG, "batch too large");
        if (fx->dtype == FFTC_C128)
            hipLaunchKernelGGL(formula_lds<double2>, dim3((unsigned)groups), dim3(fx->threads), lds, s,
                               (const double2*)in, (double2*)out, fx->dev, (int)fx->host.size(),
                               (const double2*)fx->tw, (uint32_t)fx->dim, T, batch, inverse ? 1 : 0);
        else
            hipLaunchKernelGGL(formula_lds<float2>, dim3((unsigned)groups), dim3(fx->threads), lds, s,
                               (const float2*)in, (float2*)out, fx->dev, (int)fx->host.size(),
                               (const float2*)fx->tw, (uint32_t)fx->dim, T, batch, inverse ? 1 : 0);
        FFTC_HIP_TRY(hipGetLastError());
        return FFTC_OK;
    }
    std::vector<FPass> passes = fx->host;
    std::vector<int> kinds;
    for (const auto& p : passes) kinds.push_back(p.kind);
    const bool same = in == out;
    std::vector<int> dsts;
    if (!assign_buffers(kinds, same, &dsts)) {
        FormulaPass cp;
        cp.kind = FP_COPY;
        cp.n = fx->dim;
        passes.push_back(to_dev(cp, fx->dim));
        kinds.push_back(FP_COPY);
        if (!assign_buffers(kinds, same, &dsts)) return fail(FFTC_ERR_INTERNAL, "formula buffer assignment");
    }
    const void* bufs[3] = {in, out, fx->scratch};
    const void* cur = in;
    for (size_t i = 0; i < passes.size(); ++i) {
        void* dst = const_cast<void*>(bufs[dsts[i]]);
        const uint32_t U = (uint32_t)(passes[i].units * batch);
        const int ci = (i == 0 && inverse) ? 1 : 0, co = (i + 1 == passes.size() && inverse) ? 1 : 0;
        const int64_t blocks = std::min<int64_t>((U + 255) / 256, 65536);
        if (fx->dtype == FFTC_C128)
            hipLaunchKernelGGL(formula_pass<double2>, dim3((unsigned)blocks), dim3(256), 0, s, (const double2*)cur,
                               (double2*)dst, passes[i], (const double2*)fx->tw, U, ci, co);
        else
            hipLaunchKernelGGL(formula_pass<float2>, dim3((unsigned)blocks), dim3(256), 0, s, (const float2*)cur,
                               (float2*)dst, passes[i], (const float2*)fx->tw, U, ci, co);
        FFTC_HIP_TRY(hipGetLastError());
        cur = dst;
    }
    return FFTC_OK;
}

}  // namespace fftc
