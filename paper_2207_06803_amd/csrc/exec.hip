// Kernel launches for single-kernel and two-pass plans.
#include <algorithm>
#include <type_traits>

#include "plan.h"

namespace fftc {

extern "C" __shared__ __align__(16) unsigned char fftc_dyn_lds[];

// ---------------------------------------------------------------------------
// Runtime-length single kernel: one workgroup owns d.t transforms.
// ---------------------------------------------------------------------------
// Up to 256 threads per workgroup: stage bodies inlined.  Larger groups
// (lengths above 4096) call the bodies to stay within 128 registers.
template <typename Real, bool INV, int MAXT>
__global__ void __launch_bounds__(MAXT)
stockham_generic(const cplx<Real>* in, cplx<Real>* out, const cplx<Real>* __restrict__ tw,
                 int64_t batch, GenDesc d) {
    using C = cplx<Real>;
    C* lds = reinterpret_cast<C*>(fftc_dyn_lds);
    const int tr = (int)threadIdx.x / d.tpt;
    const int t = (int)threadIdx.x - tr * d.tpt;
    const int64_t b = (int64_t)blockIdx.x * d.t + tr;
    const bool valid = b < batch;
    const int64_t off = (valid ? b : 0) * (int64_t)d.n;
    if (d.nst == 0) {  // N = 1: DFT_1 is the identity
        if (valid && t == 0) out[off] = in[off];
        return;
    }
    gen_transform<INV, (MAXT > 256)>(in + off, out + off, lds + tr * lds_len(d.n), tw, d, t, valid);
}

// ---------------------------------------------------------------------------
// Two-pass plan for N = M K (Eq. 2):
//   pass 1: for each column i < K, DFT_M of x[j K + i] (j < M), i.e.
//           (I_K (x) DFT_M) Pi^N_K, then the twiddle D^N_M: element (i, p)
//           is scaled by w_N^{i p} and written to row i: z[i M + p].
//   pass 2: for each p < M, DFT_K of z[i M + p] (i < K), written to
//           y[q M + p] (q < K): (DFT_K (x) I_M).
// A workgroup owns `tc` adjacent columns so every global access touches
// tc * sizeof(complex) contiguous bytes; the column tile is staged in LDS.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int udiv(int a, uint32_t mul, int d) {
    return d == 1 ? a : (int)__umulhi((uint32_t)a, mul);
}

template <typename Real, bool INV, int PASS>
__global__ void __launch_bounds__(1024)
four_step_pass(const cplx<Real>* src, cplx<Real>* dst, const cplx<Real>* __restrict__ tw,
               const cplx<Real>* __restrict__ twn, GenDesc d, int64_t n, int ncols, int tc,
               uint32_t len_mul) {
    using C = cplx<Real>;
    C* lds = reinterpret_cast<C*>(fftc_dyn_lds);
    const int len = d.n;             // transform length of this pass
    const int ldl = tile_pitch(len);
    const int col0 = (int)blockIdx.x * tc;
    const int cols = min(tc, ncols - col0);
    const int64_t base = (int64_t)blockIdx.y * n;
    const int nthr = (int)blockDim.x;
    const int tot = tc * len;
    // stride between successive elements of one column in src: pass 1 reads
    // x[j K + i] (stride K = ncols), pass 2 reads z[i M + p] (stride M = ncols)
    for (int l = (int)threadIdx.x; l < tot; l += nthr) {
        const int c = l % tc, j = l / tc;
        C v = mk((Real)0, (Real)0);
        if (c < cols) {
            v = src[base + (int64_t)j * ncols + col0 + c];
            if (PASS == 1 && INV) v = cconj(v);
        }
        lds[c * ldl + lds_pad(j)] = v;
    }
    __syncthreads();
    const int tr = (int)threadIdx.x / d.tpt;
    const int t = (int)threadIdx.x - tr * d.tpt;
    gen_transform<false, true>((const C*)nullptr, (C*)nullptr, lds + tr * ldl, tw, d, t, true, false, false);
    if (PASS == 1) {
        // row-major store z[(col0 + c) M + p] * w_N^{(col0 + c) p}; (col0+c) p < N.
        // When a thread's p is the same at every step, the factor is
        // w_N^{col0 p} (once) times twc[c M + p] = w_N^{c p}.
        const C* twc = twn + kTwSplit + (int)((n + kTwSplit - 1) / kTwSplit);
        const bool fixed_p = nthr % len == 0;
        C a = mk((Real)1, (Real)0);
        if (fixed_p) {
            const int e = col0 * ((int)threadIdx.x % len);
            a = cmul(twn[e % kTwSplit], twn[kTwSplit + e / kTwSplit]);
        }
        for (int l = (int)threadIdx.x; l < tot; l += nthr) {
            const int c = udiv(l, len_mul, len);
            const int p = l - c * len;
            if (c < cols) {
                const int i = col0 + c;
                C w;
                if (fixed_p) {
                    w = cmul(a, twc[c * len + p]);
                } else {
                    const int e = i * p;  // < N <= 2^20
                    w = cmul(twn[e % kTwSplit], twn[kTwSplit + e / kTwSplit]);
                }
                dst[base + (int64_t)i * len + p] = cmul(lds[c * ldl + lds_pad(p)], w);
            }
        }
    } else {
        // y[q M + col0 + c]
        for (int l = (int)threadIdx.x; l < tot; l += nthr) {
            const int c = l % tc, q = l / tc;
            if (c < cols) {
                C v = lds[c * ldl + lds_pad(q)];
                dst[base + (int64_t)q * ncols + col0 + c] = INV ? cconj(v) : v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
void fill_gen_desc(int64_t n, const std::vector<int>& rs, int tpt, int t, int64_t twbase, GenDesc* d) {
    *d = GenDesc{};
    d->n = (int)n;
    d->nst = (int)rs.size();
    d->tpt = tpt;
    d->t = t;
    int64_t ns = 1, off = twbase;
    for (size_t q = 0; q < rs.size(); ++q) {
        StageRt& s = d->st[q];
        s.r = rs[q];
        s.ns = (int)ns;
        s.twoff = (int)off;
        s.ns_mul = ns > 1 ? (uint32_t)(((uint64_t(1) << 32) + ns - 1) / ns) : 0u;
        off += (rs[q] - 1) * ns;
        ns *= rs[q];
    }
}

static uint32_t mul_for(int d) { return d > 1 ? (uint32_t)(((uint64_t(1) << 32) + d - 1) / d) : 0u; }

template <typename Real>
static fftc_status launch_single_t(const fftc_plan_s* p, const void* in, void* out, int64_t batch,
                                   hipStream_t s) {
    using C = cplx<Real>;
    const C* tin = static_cast<const C*>(in);
    C* tout = static_cast<C*>(out);
    const C* tw = static_cast<const C*>(p->tw);
    const bool inv = p->direction == FFTC_INVERSE;
    if (!grid_fits((batch + p->t - 1) / std::max(p->t, 1)))
        return fail(FFTC_ERR_INVALID_ARG, "batch too large for one launch");
    if (p->spec) {
        const int64_t groups = (batch + p->spec->t - 1) / p->spec->t;
        void* args[] = {(void*)&tin, (void*)&tout, (void*)&tw, (void*)&batch};
        hipError_t e = hipLaunchKernel(inv ? p->spec->inv : p->spec->fwd, dim3((unsigned)groups),
                                       dim3(p->spec->tpt * p->spec->t), args, 0, s);
        if (e != hipSuccess) return fail_hip(e, "hipLaunchKernel(stockham_spec)");
    } else {
        const int64_t groups = (batch + p->t - 1) / p->t;
        const int threads = p->tpt * p->t;
        dim3 g((unsigned)groups), b(threads);
        if (threads <= 256) {
            if (inv)
                hipLaunchKernelGGL((stockham_generic<Real, true, 256>), g, b, p->lds_bytes, s, tin, tout, tw, batch, p->gdesc);
            else
                hipLaunchKernelGGL((stockham_generic<Real, false, 256>), g, b, p->lds_bytes, s, tin, tout, tw, batch, p->gdesc);
        } else {
            if (inv)
                hipLaunchKernelGGL((stockham_generic<Real, true, 1024>), g, b, p->lds_bytes, s, tin, tout, tw, batch, p->gdesc);
            else
                hipLaunchKernelGGL((stockham_generic<Real, false, 1024>), g, b, p->lds_bytes, s, tin, tout, tw, batch, p->gdesc);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail_hip(e, "launch(stockham_generic)");
    }
    return FFTC_OK;
}

fftc_status launch_reqs(const SpecEntry* e, bool inv, const ReqList& list, int64_t groups, const void* tw,
                        hipStream_t s) {
    if (!grid_fits(groups)) return fail(FFTC_ERR_INVALID_ARG, "requests too large for one launch");
    ReqList l = list;
    const void* t = tw;
    void* args[] = {(void*)&l, (void*)&t};
    hipError_t err = hipLaunchKernel(inv ? e->inv : e->fwd, dim3((unsigned)groups), dim3(e->tpt * e->t), args, 0, s);
    if (err != hipSuccess) return fail_hip(err, "hipLaunchKernel(stockham_spec_reqs)");
    return FFTC_OK;
}

fftc_status launch_order(const fftc_plan_s* p, const void* in, void* out, int64_t batch, hipStream_t s) {
    const OrderEntry* o = p->order;
    const int64_t groups = (batch + o->t - 1) / o->t;
    if (!grid_fits(groups)) return fail(FFTC_ERR_INVALID_ARG, "batch too large for one launch");
    const void* tw = p->tw;
    void* args[] = {(void*)&in, (void*)&out, (void*)&tw, (void*)&batch};
    hipError_t e = hipLaunchKernel(p->direction == FFTC_INVERSE ? o->inv : o->fwd, dim3((unsigned)groups),
                                   dim3(o->tpt * o->t), args, 0, s);
    if (e != hipSuccess) return fail_hip(e, "hipLaunchKernel(order_kernel)");
    return FFTC_OK;
}

// Layout plans: the compiled kernel with GAcc accessors.  Interleaved sides
// count in reals (element step 2 stride, transform step 2 dist, im = re + 1).
template <typename Real>
static GAcc<Real> make_acc(const fftc_layout& l, const void* re, const void* im) {
    GAcc<Real> a;
    a.re = static_cast<Real*>(const_cast<void*>(re));
    if (l.planar) {
        a.im = static_cast<Real*>(const_cast<void*>(im));
        a.es = l.stride;
        a.ts = l.dist;
    } else {
        a.im = a.re + 1;
        a.es = 2 * l.stride;
        a.ts = 2 * l.dist;
    }
    return a;
}

// Both sides interleaved: strides in complex elements.
template <typename Real>
static GAccI<Real> make_acc_i(const fftc_layout& l, const void* p) {
    GAccI<Real> a;
    a.p = static_cast<cplx<Real>*>(const_cast<void*>(p));
    a.es = l.stride;
    a.ts = l.dist;
    return a;
}

template <typename Real, class ACC>
static fftc_status launch_layout_cols(const fftc_plan_s* p, const ACC& a, const ACC& b, int64_t batch,
                                      hipStream_t s) {
    constexpr bool IL = std::is_same<ACC, GAccI<Real>>::value;
    const bool inv = p->direction == FFTC_INVERSE;
    const cplx<Real>* tw = static_cast<const cplx<Real>*>(p->tw);
    const cplx<Real>* tw1 = tw + p->tw1_off;
    const cplx<Real>* tw2 = tw + p->tw2_off;
    const cplx<Real>* twn = tw + p->twn_off;
    cplx<Real>* scr = static_cast<cplx<Real>*>(p->scratch);
    const FourStepEntry* f1 = p->col1;
    const FourStepEntry* f2 = p->col2;
    int k = (int)p->k, m = (int)p->m;
    const int64_t g1 = (batch + f1->tc - 1) / f1->tc, g2 = (batch + f2->tc - 1) / f2->tc;
    if (!grid_fits(g1) || !grid_fits(g2)) return fail(FFTC_ERR_INVALID_ARG, "batch too large for one launch");
    ACC aa = a, bb = b;
    const void* fn1 = IL ? f1->fn_il[0][inv ? 1 : 0] : f1->fn[0][inv ? 1 : 0];
    const void* fn2 = IL ? f2->fn_il[1][inv ? 1 : 0] : f2->fn[1][inv ? 1 : 0];
    if (!fn1 || !fn2) return fail(FFTC_ERR_INTERNAL, "column-layout pass kernel missing");
    void* args1[] = {(void*)&aa, (void*)&bb, (void*)&scr, (void*)&tw1, (void*)&twn, (void*)&batch, (void*)&k};
    hipError_t e = hipLaunchKernel(fn1, dim3((unsigned)g1, (unsigned)k), dim3(f1->tpt * f1->tc), args1, 0, s);
    if (e != hipSuccess) return fail_hip(e, "hipLaunchKernel(col_two_pass 1)");
    void* args2[] = {(void*)&aa, (void*)&bb, (void*)&scr, (void*)&tw2, (void*)&twn, (void*)&batch, (void*)&m};
    e = hipLaunchKernel(fn2, dim3((unsigned)g2, (unsigned)m), dim3(f2->tpt * f2->tc), args2, 0, s);
    if (e != hipSuccess) return fail_hip(e, "hipLaunchKernel(col_two_pass 2)");
    return FFTC_OK;
}

fftc_status launch_layout(const fftc_plan_s* p, const void* in_re, const void* in_im, void* out_re, void* out_im,
                          int64_t batch, hipStream_t s) {
    const bool inv = p->direction == FFTC_INVERSE;
    // both sides interleaved: the kernels with one vector access per element
    const bool il = !p->lin.planar && !p->lout.planar;
    if (p->col1) {
        if (p->dtype == FFTC_C128)
            return il ? launch_layout_cols<double>(p, make_acc_i<double>(p->lin, in_re),
                                                   make_acc_i<double>(p->lout, out_re), batch, s)
                      : launch_layout_cols<double>(p, make_acc<double>(p->lin, in_re, in_im),
                                                   make_acc<double>(p->lout, out_re, out_im), batch, s);
        return il ? launch_layout_cols<float>(p, make_acc_i<float>(p->lin, in_re), make_acc_i<float>(p->lout, out_re),
                                              batch, s)
                  : launch_layout_cols<float>(p, make_acc<float>(p->lin, in_re, in_im),
                                              make_acc<float>(p->lout, out_re, out_im), batch, s);
    }
    // column-like sides (dist < stride) go through the tile kernel
    int in_cols = p->lin.dist < p->lin.stride ? 1 : 0, out_cols = p->lout.dist < p->lout.stride ? 1 : 0;
    const bool tile = (in_cols || out_cols) && p->spec->tile_fwd;
    const int per = tile ? p->spec->tile_tc : p->spec->t;
    const int threads = tile ? p->spec->tile_tpt * p->spec->tile_tc : p->spec->tpt * p->spec->t;
    const int64_t groups = (batch + per - 1) / per;
    if (!grid_fits(groups)) return fail(FFTC_ERR_INVALID_ARG, "batch too large for one launch");
    const void* fn = tile ? (il ? (inv ? p->spec->tile_il_inv : p->spec->tile_il_fwd)
                                : (inv ? p->spec->tile_inv : p->spec->tile_fwd))
                          : (il ? (inv ? p->spec->il_inv : p->spec->il_fwd) : (inv ? p->spec->inv : p->spec->fwd));
    if (!fn) return fail(FFTC_ERR_INTERNAL, "layout kernel missing");
    hipError_t e;
    // one side planar, the other interleaved (row layouts): the interleaved
    // side takes its own accessor
    const bool mixed_pi = !tile && p->lin.planar && !p->lout.planar && p->spec->pi_fwd;
    const bool mixed_ip = !tile && !p->lin.planar && p->lout.planar && p->spec->ip_fwd;
    if (mixed_pi || mixed_ip) {
        const void* fm = mixed_pi ? (inv ? p->spec->pi_inv : p->spec->pi_fwd) : (inv ? p->spec->ip_inv : p->spec->ip_fwd);
        if (p->dtype == FFTC_C128) {
            const double2* tw = static_cast<const double2*>(p->tw);
            GAcc<double> ga = make_acc<double>(mixed_pi ? p->lin : p->lout, mixed_pi ? in_re : out_re,
                                               mixed_pi ? in_im : out_im);
            GAccI<double> gi = make_acc_i<double>(mixed_pi ? p->lout : p->lin, mixed_pi ? out_re : in_re);
            void* args_pi[] = {(void*)&ga, (void*)&gi, (void*)&tw, (void*)&batch};
            void* args_ip[] = {(void*)&gi, (void*)&ga, (void*)&tw, (void*)&batch};
            e = hipLaunchKernel(fm, dim3((unsigned)groups), dim3(threads), mixed_pi ? args_pi : args_ip, 0, s);
        } else {
            const float2* tw = static_cast<const float2*>(p->tw);
            GAcc<float> ga = make_acc<float>(mixed_pi ? p->lin : p->lout, mixed_pi ? in_re : out_re,
                                             mixed_pi ? in_im : out_im);
            GAccI<float> gi = make_acc_i<float>(mixed_pi ? p->lout : p->lin, mixed_pi ? out_re : in_re);
            void* args_pi[] = {(void*)&ga, (void*)&gi, (void*)&tw, (void*)&batch};
            void* args_ip[] = {(void*)&gi, (void*)&ga, (void*)&tw, (void*)&batch};
            e = hipLaunchKernel(fm, dim3((unsigned)groups), dim3(threads), mixed_pi ? args_pi : args_ip, 0, s);
        }
        if (e != hipSuccess) return fail_hip(e, "hipLaunchKernel(stockham_spec_layout)");
        return FFTC_OK;
    }
    // the tile kernel takes the two order flags as well
    if (p->dtype == FFTC_C128) {
        const double2* tw = static_cast<const double2*>(p->tw);
        if (il) {
            GAccI<double> a = make_acc_i<double>(p->lin, in_re), b = make_acc_i<double>(p->lout, out_re);
            void* args[] = {(void*)&a, (void*)&b, (void*)&tw, (void*)&batch, (void*)&in_cols, (void*)&out_cols};
            void* args4[] = {(void*)&a, (void*)&b, (void*)&tw, (void*)&batch};
            e = hipLaunchKernel(fn, dim3((unsigned)groups), dim3(threads), tile ? args : args4, 0, s);
        } else {
            GAcc<double> a = make_acc<double>(p->lin, in_re, in_im), b = make_acc<double>(p->lout, out_re, out_im);
            void* args[] = {(void*)&a, (void*)&b, (void*)&tw, (void*)&batch, (void*)&in_cols, (void*)&out_cols};
            void* args4[] = {(void*)&a, (void*)&b, (void*)&tw, (void*)&batch};
            e = hipLaunchKernel(fn, dim3((unsigned)groups), dim3(threads), tile ? args : args4, 0, s);
        }
    } else {
        const float2* tw = static_cast<const float2*>(p->tw);
        if (il) {
            GAccI<float> a = make_acc_i<float>(p->lin, in_re), b = make_acc_i<float>(p->lout, out_re);
            void* args[] = {(void*)&a, (void*)&b, (void*)&tw, (void*)&batch, (void*)&in_cols, (void*)&out_cols};
            void* args4[] = {(void*)&a, (void*)&b, (void*)&tw, (void*)&batch};
            e = hipLaunchKernel(fn, dim3((unsigned)groups), dim3(threads), tile ? args : args4, 0, s);
        } else {
            GAcc<float> a = make_acc<float>(p->lin, in_re, in_im), b = make_acc<float>(p->lout, out_re, out_im);
            void* args[] = {(void*)&a, (void*)&b, (void*)&tw, (void*)&batch, (void*)&in_cols, (void*)&out_cols};
            void* args4[] = {(void*)&a, (void*)&b, (void*)&tw, (void*)&batch};
            e = hipLaunchKernel(fn, dim3((unsigned)groups), dim3(threads), tile ? args : args4, 0, s);
        }
    }
    if (e != hipSuccess) return fail_hip(e, "hipLaunchKernel(stockham_spec_layout)");
    return FFTC_OK;
}

fftc_status launch_single(const fftc_plan_s* p, const void* in, void* out, int64_t batch, hipStream_t s) {
    return p->dtype == FFTC_C128 ? launch_single_t<double>(p, in, out, batch, s)
                                 : launch_single_t<float>(p, in, out, batch, s);
}

// Columns per workgroup in a two-pass plan: 128 contiguous bytes per access.
int two_pass_cols(int dtype) { return dtype == FFTC_C128 ? 8 : 16; }

template <typename Real, bool INV>
static fftc_status launch_two_pass_chunk(const fftc_plan_s* p, const cplx<Real>* tin, cplx<Real>* mid,
                                         cplx<Real>* tout, const cplx<Real>* tw, const cplx<Real>* twn,
                                         int tc, size_t csz, int64_t nb, hipStream_t s);

template <typename Real, bool INV>
static fftc_status launch_two_pass_t(const fftc_plan_s* p, const void* in, void* out, int64_t batch,
                                     hipStream_t s) {
    using C = cplx<Real>;
    const C* tin = static_cast<const C*>(in);
    C* tout = static_cast<C*>(out);
    const C* tw = static_cast<const C*>(p->tw);
    const C* twn = tw + p->twn_off;
    // the intermediate goes through `out` unless the call is in place
    C* mid = (in == out) ? static_cast<C*>(p->scratch) : tout;
    const int tc = two_pass_cols(p->dtype);
    const size_t csz = sizeof(C);
    // grid.y carries the transform index; split very large batches
    constexpr int64_t kMaxY = 65535;
    for (int64_t b0 = 0; b0 < batch; b0 += kMaxY) {
        const int64_t nb = std::min<int64_t>(kMaxY, batch - b0);
        const int64_t o = b0 * p->n;
        fftc_status st = launch_two_pass_chunk<Real, INV>(p, tin + o, mid + o, tout + o, tw, twn, tc, csz, nb, s);
        if (st != FFTC_OK) return st;
    }
    return FFTC_OK;
}

template <typename Real, bool INV>
static fftc_status launch_two_pass_chunk(const fftc_plan_s* p, const cplx<Real>* tin, cplx<Real>* mid,
                                         cplx<Real>* tout, const cplx<Real>* tw, const cplx<Real>* twn,
                                         int tc, size_t csz, int64_t nb, hipStream_t s) {
    using C = cplx<Real>;
    if (p->fs1) {  // compiled column kernels
        const FourStepEntry* f = p->fs1;
        const C* tw1 = tw + p->tw1_off;
        int64_t n = p->n;
        int ncols = (int)p->k;
        void* args[] = {(void*)&tin, (void*)&mid, (void*)&tw1, (void*)&twn, (void*)&n, (void*)&ncols};
        hipError_t e = hipLaunchKernel(f->fn[0][INV ? 1 : 0], dim3((unsigned)((p->k + f->tc - 1) / f->tc), (unsigned)nb),
                                       dim3(f->tpt * f->tc), args, 0, s);
        if (e != hipSuccess) return fail_hip(e, "hipLaunchKernel(fourstep pass 1)");
    } else {
        const GenDesc& d = p->pass1;
        dim3 grid((unsigned)((p->k + tc - 1) / tc), (unsigned)nb);
        const size_t lds = (size_t)tc * tile_pitch(d.n) * csz;
        hipLaunchKernelGGL((four_step_pass<Real, INV, 1>), grid, dim3(d.tpt * tc), lds, s, tin, mid, tw,
                           twn, d, p->n, (int)p->k, tc, mul_for(d.n));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail_hip(e, "launch(four_step_pass 1)");
    }
    if (p->fs2) {
        const FourStepEntry* f = p->fs2;
        const C* tw2 = tw + p->tw2_off;
        const C* cmid = mid;
        int64_t n = p->n;
        int ncols = (int)p->m;
        void* args[] = {(void*)&cmid, (void*)&tout, (void*)&tw2, (void*)&twn, (void*)&n, (void*)&ncols};
        hipError_t e = hipLaunchKernel(f->fn[1][INV ? 1 : 0], dim3((unsigned)((p->m + f->tc - 1) / f->tc), (unsigned)nb),
                                       dim3(f->tpt * f->tc), args, 0, s);
        if (e != hipSuccess) return fail_hip(e, "hipLaunchKernel(fourstep pass 2)");
    } else {
        const GenDesc& d = p->pass2;
        dim3 grid((unsigned)((p->m + tc - 1) / tc), (unsigned)nb);
        const size_t lds = (size_t)tc * tile_pitch(d.n) * csz;
        hipLaunchKernelGGL((four_step_pass<Real, INV, 2>), grid, dim3(d.tpt * tc), lds, s,
                           (const C*)mid, tout, tw, twn, d, p->n, (int)p->m, tc, mul_for(d.n));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail_hip(e, "launch(four_step_pass 2)");
    }
    return FFTC_OK;
}

fftc_status launch_two_pass(const fftc_plan_s* p, const void* in, void* out, int64_t batch, hipStream_t s) {
    const bool inv = p->direction == FFTC_INVERSE;
    if (in == out && !p->scratch) return fail(FFTC_ERR_INVALID_ARG, "this two-pass plan has no scratch for in-place use");
    if (p->dtype == FFTC_C128)
        return inv ? launch_two_pass_t<double, true>(p, in, out, batch, s)
                   : launch_two_pass_t<double, false>(p, in, out, batch, s);
    return inv ? launch_two_pass_t<float, true>(p, in, out, batch, s)
               : launch_two_pass_t<float, false>(p, in, out, batch, s);
}

// Allow the dynamic-LDS kernels to use up to the gfx950 per-group maximum.
fftc_status enable_large_lds() {
    static bool done = false;
    if (done) return FFTC_OK;
    const void* ks[] = {
        (const void*)&stockham_generic<float, false, 256>, (const void*)&stockham_generic<float, true, 256>,
        (const void*)&stockham_generic<double, false, 256>, (const void*)&stockham_generic<double, true, 256>,
        (const void*)&stockham_generic<float, false, 1024>, (const void*)&stockham_generic<float, true, 1024>,
        (const void*)&stockham_generic<double, false, 1024>, (const void*)&stockham_generic<double, true, 1024>,
        (const void*)&four_step_pass<float, false, 1>, (const void*)&four_step_pass<float, false, 2>,
        (const void*)&four_step_pass<float, true, 1>, (const void*)&four_step_pass<float, true, 2>,
        (const void*)&four_step_pass<double, false, 1>, (const void*)&four_step_pass<double, false, 2>,
        (const void*)&four_step_pass<double, true, 1>, (const void*)&four_step_pass<double, true, 2>,
    };
    for (const void* k : ks) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMaxPerGroup);
        if (e != hipSuccess) return fail_hip(e, "hipFuncSetAttribute(MaxDynamicSharedMemorySize)");
    }
    done = true;
    return FFTC_OK;
}

// ---------------------------------------------------------------------------
// Bandwidth reference: a plain device copy in the transforms' access form
// (one 16-byte nontemporal load and store per thread).
// ---------------------------------------------------------------------------
typedef float copy_vec __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) copy16(const copy_vec* __restrict__ in, copy_vec* __restrict__ out,
                                              int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(in + i), out + i);
}

fftc_status launch_copy16(const void* in, void* out, int64_t nvec, hipStream_t s) {
    const int64_t blocks = (nvec + 255) / 256;
    if (!grid_fits(blocks)) return fail(FFTC_ERR_TOO_LARGE, "copy needs more workgroups than one launch holds");
    hipLaunchKernelGGL(copy16, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const copy_vec*>(in),
                       static_cast<copy_vec*>(out), nvec);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? FFTC_OK : fail_hip(e, "launch(copy16)");
}

}  // namespace fftc
