// rq_lmm_adj.h -- pathwise Greeks of the LIBOR caplet book by a
// hand-written adjoint (reverse-mode) sweep, one path per lane.
//
// Forward pass (same scheme as rq_lmm.hip, state X_n = log2(L_n / L_n(0))):
//   step k:  w = sqrt(delta) z_k;  for n = k..n_fwd-1 in ascending order:
//     g_n = G(X_n) = 1 / (1 + kappa_n 2^{-X_n}),  kappa_n = 1 / (delta L_n(0))
//     w  += g_n delta a_n                       (w is now w_n)
//     X_n += log2(e) (c_n + a_n . w_n)
//   and the lane stores the step's final w (d numbers).
// Payoffs (FP64): L_n(T_n) = L_n(0) 2^{X_n}; P_n = delta (L_n - K_n)^+ / num_{n+1},
//   num_{n+1} = num_0 prod_{j<=n} (1 + delta L_j(T_j)); book = sum_n P_n.
//
// Reverse sweep.  The payoff adjoint is
//   dbook/dL_n(T_n) = delta [L_n > K_n] / num_{n+1} - delta / (1 + delta L_n) * sum_{j>=n} P_j
// and Xbar_n = dbook/dL_n(T_n) * L_n(T_n) ln 2.  Steps then run backwards,
// k = n_fwd-1..0.  Step k restarts from its stored final w and visits its
// forwards in descending order.  With w_n known, the pre-step state and the
// drift factor are explicit (nothing is solved, no normal is drawn again):
//   P = log2(e) a_n . w_n,   X_n -= P + log2(e) c_n,   g_n = G(X_n)
// and the adjoint of the forward-step is
//   Wbar += Xbar_n log2(e) a_n            (adjoint of w_n: a suffix sum over n)
//   h     = g_n delta a_n . Wbar
//   vega_n += Xbar_n log2(e) (b_n . w_n - delta sigma_n |b_n|^2) + h / sigma_n
//   Xbar_n += h ln2 (1 - g_n)             (delta a_n . Wbar G'(X_n), G' = ln2 G (1 - G))
//   w    -= g_n delta a_n                 (back to w_{n-1})
// with a_n = sigma_n b_n.  The lane accumulates sigma_n vega_n,
//   sigma_n vega_n += Xbar_n (P + 2 log2(e) c_n) + h,   (c_n = -delta |a_n|^2 / 2)
// so that the one dot product P serves the state and the vega, and h both
// the vega and Xbar with constant factors; the sums are divided by sigma_n
// once, in FP64, at the end (a zero sigma_n is carried as 2^-60).
// After step 0, Xbar_n is the adjoint of log2 L_n(0), so
//   dbook/dL_n(0) = Xbar_n / (L_n(0) ln 2);  dbook/dL_0(0) = -delta book / num_0.
// The reconstructed states differ from the forward pass's by rounding only
// (one rounding of the increment per step, as in the forward pass).
//
// Per path: n_fwd+1 prices (caplets, book) and 2 n_fwd + 1 Greeks (deltas,
// spot delta, vegas).  A task is one wave of 64 paths.  A single call runs
// the forward halves of a chunk of tasks in one kernel (storing w and the
// final states per task) and their payoffs and reverse sweeps in a second;
// the batch does the same per window of its work items (and runs whole
// tasks without Greeks for its prices).  State and adjoint state live in
// registers, the vega accumulators in LDS ([forward][lane], conflict-free;
// before the sweep the same rows hold the payoff adjoint; in the FP32
// reverse half at capacity 80 the two top forwards' accumulators are
// registers, to leave LDS room for the drift constants).  Outputs are wave
// sums (transpose butterfly), one partial row per path block: deterministic.
#pragma once

#include <type_traits>

#include "rq_device.h"

namespace rq {

// r = the first K entries of a table row (scalar loads: the row address is
// uniform)
template <typename T, int K> __device__ __forceinline__ void load_row(T (&r)[K], cptr<T> q)
{
#pragma unroll
    for (int e = 0; e < K; ++e) r[e] = q[e];
}

// "no loads to issue" for the forward-step bodies below (their scheduling is
// then left alone)
struct NoPre {
    __device__ void operator()() const {}
};

// p, made to depend on the scalar value dep: loads through the result issue
// only once dep (the current row's first entry used) has arrived, so the wait
// for the current row does not also wait for the next one
template <typename T> __device__ __forceinline__ cptr<T> after(cptr<T> p, T dep)
{
    uint64_t u = (uint64_t)p;
    asm volatile("" : "+s"(u) : "s"(dep));
    return (cptr<T>)u;
}

template <typename T> __device__ __forceinline__ T adj_exp2(T x);
template <> __device__ __forceinline__ float adj_exp2<float>(float x) { return __builtin_amdgcn_exp2f(x); }
template <> __device__ __forceinline__ double adj_exp2<double>(double x) { return exp2_f64(x); }
template <typename T> __device__ __forceinline__ T adj_rcp(T x);
template <> __device__ __forceinline__ float adj_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
// 1/x for the drift factor's denominator 1 + kappa 2^-X >= 1: the Newton
// reciprocal, or 0 beyond 2^1000 (as a division would give for an
// overflowing denominator)
template <> __device__ __forceinline__ double adj_rcp<double>(double x)
{
    return x < 0x1p1000 ? recip64(x) : 0.0;
}

// One task: the 64 paths of block `blk` of replication m (task = m n_blk + blk
// indexes the partial rows).  GREEKS = false runs the forward pass and the
// payoffs only (the batch kernel's pricing form).  MC draws the path's
// uniforms from Philox instead of the Halton replication (a separate
// instantiation, so the Halton form carries no pseudo-random code).  wt is the lane's entry of
// the task's stored-w rows ([k][f][64]); vbar the block's LDS rows.
// PART selects the whole task (kTaskWhole: forward, payoffs, reverse) or one
// of its two halves for the two-kernel form: kTaskFwd runs the forward pass
// and stores the final states at xs ([n][lane], n < NFC); kTaskRev loads them
// and runs the payoffs and the reverse sweep.  The halves do exactly the
// arithmetic of the whole task.  c6s is the block's LDS table of the NFC
// drift constants log2(e) c_n, filled by the task; the forward pass always
// uses it, the FP32 reverse sweep too (FP64 passes none to its reverse half).
// The vega rows of forwards n >= NFC - VR are held in registers, the others
// in vbar (NFC - VR rows).
constexpr int kTaskWhole = 0, kTaskFwd = 1, kTaskRev = 2;

// LDS of one 64-lane wave at two waves per SIMD: the CU's 160 KB over 8
constexpr int kLdsPerWave2 = 160 * 1024 / 8;
// Vega rows an FP32 reverse half holds in registers so that its NFC vega
// rows and its NFC drift constants fit kLdsPerWave2 (two at NFC = 80; the
// registers are there, as the sweep's state takes about 190 of 256)
template <int NFC, typename T>
constexpr int rev_reg_rows()
{
    constexpr int over = (NFC * kWave + NFC) * (int)sizeof(T) - kLdsPerWave2;
    return sizeof(T) == 4 && over > 0 ? (over + kWave * (int)sizeof(T) - 1) / (kWave * (int)sizeof(T)) : 0;
}

template <int NFC, int D, typename T, bool GREEKS, bool MC, int PART = kTaskWhole, int VR = 0, int XL = 0>
__device__ __forceinline__ void lmm_task(const LmmArgs &a, int m, int blk, int64_t task, T *__restrict__ wt,
                                         T (*__restrict__ vbar)[kWave], T *__restrict__ xs = nullptr,
                                         T *__restrict__ c6s = nullptr, T (*__restrict__ xl)[kWave] = nullptr)
{
    static_assert(NFC % 16 == 0 && NFC % kGrp == 0, "capacity must be a multiple of 16");
    static_assert(VR >= 0 && VR < kGrp, "at most kGrp - 1 vega rows in registers");
    static_assert(XL == 0 || (PART == kTaskFwd && XL % kGrp == 0 && XL < NFC), "LDS states: forward halves only");
    constexpr bool kF32 = sizeof(T) == 4;
    constexpr T kLn2 = T(0.69314718055994530942);
    const int lane = threadIdx.x;
    // per task: keeps the forward count, the tables and all that derives
    // from them out of scalar registers between tasks
    const cptr<double> fwd = opaque_u(as_const<double>(a.fwd));
    const cptr<T> tab = opaque_u(as_const<T>(a.adj));
    const int nf = opaque_u(a.n_fwd);
    const double delta = a.delta;
    const T sqd = (T)a.sqrt_delta;

    auto G = [&](T x, T c) -> T { return adj_rcp<T>(ffma(c, adj_exp2<T>(-x), T(1))); };

    const int64_t i = (int64_t)blk * kWave + lane;
    const bool active = i < a.g.N;
    const int seg = (int)(((int64_t)blk * kWave) >> a.g.log2S);   // blocks never straddle segments
    const uint32_t t = (uint32_t)(i - ((int64_t)seg << a.g.log2S));
    const StartEnt *__restrict__ st = a.g.starts + ((size_t)m * a.g.n_seg + seg) * a.g.s;

    T X[NFC], Xb[NFC];
    // state of forward n: X[n], or in the forward half the LDS row xl[n]
    // for the XL lowest forwards (forward n moves in steps 0..n only, so these
    // take few of the forward-steps; their registers go to a fifth wave per
    // SIMD).  n is a compile-time constant at every use.
    auto xget = [&](int n) -> T { return n < XL ? xl[n][lane] : X[n]; };
    auto xset = [&](int n, T v) {
        if (n < XL) xl[n][lane] = v;
        else X[n] = v;
    };
    // vega row n: vbar[n][lane], or a register for n >= kLdsRows (n is a
    // compile-time constant at every use, in unrolled loops)
    constexpr int kLdsRows = NFC - VR;
    T vr[VR > 0 ? VR : 1] = {};
    auto vget = [&](int n) -> T { return n >= kLdsRows ? vr[n - kLdsRows] : vbar[n][lane]; };
    auto vset = [&](int n, T v) {
        if (n >= kLdsRows) vr[n - kLdsRows] = v;
        else vbar[n][lane] = v;
    };
#pragma unroll
    // (the stored w and final states are written once and read once, far
    // beyond the caches: non-temporal stores and loads, -0.4% per step)
    for (int n = 0; n < NFC; ++n) xset(n, PART == kTaskRev ? __builtin_nontemporal_load(xs + n * kWave) : T(0));
    if constexpr (PART != kTaskRev) {
        // the drift constants log2(e) c_n, broadcast from LDS (c6s, NFC
        // entries): a forward-step's first FMA then takes one scalar operand
        // (the loading) and one vector operand (the constant), and no
        // constant is moved to a vector register
        for (int n = lane; n < NFC; n += kWave) c6s[n] = tab[n * kAdjRow + 6];
        __syncthreads();
    }

    // ---- forward pass ----
    McPath mc;
#pragma unroll 1
    for (int k = 0; k < (PART == kTaskRev ? 0 : nf); ++k) {
        T w[D];
        // the step's base and start entries, all requested before the first
        // is used: one scalar-load wait per step instead of one per dimension
        PointCtx cs[D];
        StartEnt ses[D];
        if constexpr (!MC) {
#pragma unroll
            for (int f = 0; f < D; ++f) {
                cs[f] = load_base_uniform(a.g.base, k * D + f);
                ses[f] = load_uniform<StartEnt>(st + k * D + f);
            }
        }
#pragma unroll
        for (int f = 0; f < D; ++f) {
            const int j = k * D + f;
            double x;
            if constexpr (MC) {
                x = mc.point(a.g.seed, (uint64_t)(a.g.m_offset + m), (uint64_t)i, j);
            } else {
                x = a.g.perm_on ? radinv_x<true, !kF32>(cs[f], ses[f], t, a.g.perm + (size_t)m * a.g.perm_stride)
                                : radinv_x<false, !kF32>(cs[f], ses[f], t, a.g.perm);
            }
            w[f] = sqd * inv_normal(x, T(0));
        }
        // one forward-step of forward n (alive in this step); c6 is its drift
        // constant log2(e) c_n, read from LDS
        auto body = [&](int n, T c6) __attribute__((always_inline)) {
            const cptr<T> q = tab + n * kAdjRow;
            const T xn = xget(n);
            const T g = G(xn, q[7]);
#pragma unroll
            for (int f = 0; f < D; ++f) w[f] = ffma(g, q[3 + f], w[f]);
            // the (small) increment log2(e) (c_n + a_n . w) is formed first and
            // added to the O(1) state once
            T e = ffma(q[0], w[0], c6);
#pragma unroll
            for (int f = 1; f < D; ++f) e = ffma(q[f], w[f], e);
            xset(n, xn + e);
        };
        const unsigned alive = (unsigned)(nf - k);
        const lds_ptr<T> c6k = lds_base(c6s);
        if constexpr (kF32) {
            // groups of kGrp forwards: in the one holding forward k (n0 < k <
            // n0 + kGrp) each live forward runs behind its own uniform branch,
            // first; the wholly alive groups (k <= n0 < n_fwd) run after it
            // (two passes over the groups keep the two forms out of one branch)
#pragma unroll
            for (int gq = 0; gq < NFC / kGrp; ++gq) {
                const int n0 = gq * kGrp;
                if ((unsigned)(k - n0 - 1) < (unsigned)(kGrp - 1)) {
                    const Quad<T> c4 = lds_quad(c6k, n0);
#pragma unroll
                    for (int u = 0; u < kGrp; ++u)   // its live forwards only, one uniform branch each
                        if ((unsigned)(n0 + u - k) < alive) body(n0 + u, c4.v[u]);
                }
            }
#pragma unroll
            for (int gq = 0; gq < NFC / kGrp; ++gq) {
                const int n0 = gq * kGrp;
                if ((unsigned)(n0 - k) < alive) {
                    const Quad<T> c4 = lds_quad(c6k, n0);
#pragma unroll
                    for (int u = 0; u < kGrp; ++u) body(n0 + u, c4.v[u]);
                }
            }
        } else {
#pragma unroll
            for (int n = 0; n < NFC; ++n)
                if ((unsigned)(n - k) < alive) body(n, c6k[n]);
        }
        if constexpr (GREEKS) {
#pragma unroll
            for (int f = 0; f < D; ++f) __builtin_nontemporal_store(w[f], wt + (size_t)(k * D + f) * kWave);
        }
    }

    if constexpr (PART == kTaskFwd) {
#pragma unroll
        for (int n = 0; n < NFC; ++n) __builtin_nontemporal_store(xget(n), xs + n * kWave);
        return;
    }

    // ---- payoffs and their adjoint (FP64) ----
    // (In FP32, 2^X is formed in FP32, one more rounding of the size the FP32
    // state already carries; the fixing value, numeraire and payoffs are FP64.)
    // With Greeks, pass 1 forms the book and pass 2 (16 forwards at a time)
    // the payoffs again, their wave sums, and the adjoint of the fixing
    // values, parked in the (not yet used) vega rows of LDS so that the
    // state registers are not doubled while the FP64 payoff work needs
    // registers.  Without Greeks only pass 2 runs.
    const double act = active ? 1.0 : 0.0;
    double *pp = (a.per_path && active) ? a.per_path + ((size_t)m * (size_t)a.g.N + (size_t)i) * a.n_out
                                        : nullptr;
    double *out = a.partial + (size_t)task * a.n_out;
    double *gout = GREEKS ? a.partial_g + (size_t)task * a.n_g : nullptr;
    double book = 0.0;
    // Rows beyond n_fwd are zero (L_n(0) = 0: no numeraire factor, no
    // payoff, no adjoint), so the loops need no per-forward guard; the
    // caplet flag multiplies the payoff.  Each pass re-reads the table
    // through a fresh pointer so that no row value stays live in scalar
    // registers from one pass to the next.
    if constexpr (GREEKS) {
        // the book over a common denominator: B = num_{n+1} sum_{j<=n} P_j
        // grows as B <- B (1 + delta L_n) + delta (L_n - K_n)^+, and
        // book = B / num at the end (one division instead of one per forward)
        const cptr<double> f1 = opaque_u(fwd);
        double num = a.num0, B = 0.0;
#pragma unroll
        for (int c = 0; c < NFC / 16; ++c) {
            if (c * 16 < nf) {
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int n = c * 16 + q;
                    const double Lf = f1[n * kFwdRow + 7] * (double)adj_exp2<T>(X[n]);
                    const double onep = 1.0 + delta * Lf;
                    num *= onep;
                    const double ex = __builtin_fmax(Lf - f1[n * kFwdRow + 8], 0.0);   // (L_n - K_n)^+
                    B = __builtin_fma(B, onep, f1[n * kFwdRow + 9] * (delta * ex));
                }
            }
        }
        book = B / num;
    }
    if constexpr (GREEKS) {   // pass 2 forms 2^X again: keep pass 1's values from living on in registers
#pragma unroll
        for (int n = 0; n < NFC; ++n) asm volatile("" : "+v"(X[n]));
    }
    {
        const cptr<double> f2 = opaque_u(fwd);
        double num = a.num0;
        double before = 0.0;   // sum_{j<n} P_j
#pragma unroll
        for (int c = 0; c < NFC / 16; ++c) {
            if (c * 16 < nf) {
                double V[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int n = c * 16 + q;
                    const double Lf = f2[n * kFwdRow + 7] * (double)adj_exp2<T>(X[n]);
                    const double onep = 1.0 + delta * Lf;
                    const double num_prev = num;
                    num *= onep;
                    const double rn = delta * recip64(num);
                    const double ex = Lf - f2[n * kFwdRow + 8];
                    const double flag = f2[n * kFwdRow + 9];
                    const double Pn = ex > 0.0 ? flag * (ex * rn) : 0.0;
                    if constexpr (GREEKS) {
                        // delta / (1 + delta L_n) = rn num_{n-1}: no second division
                        double dL = -(rn * num_prev) * (book - before);
                        if (ex > 0.0) dL += flag * rn;
                        vset(n, (T)(dL * Lf * 0.69314718055994530942));
                        before += Pn;
                    } else {
                        book += Pn;
                    }
                    V[q] = Pn * act;
                }
                if (pp) {   // (an active lane: V = Pn) beyond n_fwd: 0 into the book slot, rewritten below
#pragma unroll
                    for (int q = 0; q < 16; ++q) pp[c * 16 + q < nf ? c * 16 + q : nf] = V[q];
                }
                const double sv = wave_sum16(V, lane);
                const int o = c * 16 + (lane >> 2);
                if ((lane & 3) == 0 && o < nf) out[o] = sv;
            }
        }
    }
    if (pp) pp[nf] = book;
    {
        const double b = wave_sum(book * act);
        const double sp = GREEKS ? wave_sum(-delta * book / a.num0 * act) : 0.0;
        if (lane == 0) {
            out[nf] = b;
            if (GREEKS) gout[nf] = sp;
        }
    }
    if constexpr (!GREEKS) return;

    // ---- reverse sweep ----
#pragma unroll
    for (int n = 0; n < NFC; ++n) {   // rows beyond n_fwd hold 0
        Xb[n] = vget(n);
        vset(n, T(0));
    }
    if constexpr (kF32 && PART == kTaskRev) {   // the drift constants, as the forward half has them
        for (int n = lane; n < NFC; n += kWave) c6s[n] = tab[n * kAdjRow + 6];
        __syncthreads();
    }
    // The state rebuild and adjoint of one forward-step come in two parts, so
    // that two independent forward-steps can share a wait:
    //  * incr() forms the increment e = log2(e) (c_n + a_n . w_n) as the
    //    forward pass forms it (c6 = log2(e) c_n: in FP32 a vector operand
    //    read from LDS, so that the first FMA takes it beside the row's scalar
    //    loading);
    //  * rest() takes forward n from there with a chain's state (w = w_n on
    //    entry, w_{n-1} on exit; Wbar) and returns the new sigma-scaled vega
    //    entry vb + term.  on = 0 (masked form) leaves everything unchanged.
    struct Chain {
        T w[D], Wb[D];
    };
    auto incr = [&](const Chain &c, const auto &q, T c6) __attribute__((always_inline)) -> T {
        T e = ffma(q[0], c.w[0], c6);
#pragma unroll
        for (int f = 1; f < D; ++f) e = ffma(q[f], c.w[f], e);
        return e;
    };
    auto rest = [&](Chain &c, int n, const auto &q, T vb, T e, T on, auto masked) __attribute__((always_inline)) -> T {
        constexpr bool MASKED = decltype(masked)::value;
        const T y = MASKED ? ffma(-e, on, X[n]) : X[n] - e;
        X[n] = y;
        const T g = G(y, q[7]);
        const T ge = MASKED ? g * on : g;
        const T xb = MASKED ? Xb[n] * on : Xb[n];
#pragma unroll
        for (int f = 0; f < D; ++f) c.Wb[f] = ffma(xb, q[f], c.Wb[f]);
        T da = q[3] * c.Wb[0];                      // delta a_n . Wbar
#pragma unroll
        for (int f = 1; f < D; ++f) da = ffma(q[3 + f], c.Wb[f], da);
        const T h = ge * da;
        const T vnew = vb + ffma(xb, e + q[6], h);   // P + 2 log2(e) c_n = e + log2(e) c_n
        Xb[n] = ffma(kLn2, ffma(-g, h, h), Xb[n]);
#pragma unroll
        for (int f = 0; f < D; ++f) c.w[f] = ffma(-ge, q[3 + f], c.w[f]);
        return vnew;
    };
    // Final w of the next two steps to run, loaded a step (or pair) ahead.
    T wp0[D] = {}, wp1[D] = {};
    auto load_w = [&](T(&dst)[D], int k) {
        if (k >= 0) {
#pragma unroll
            for (int f = 0; f < D; ++f) dst[f] = __builtin_nontemporal_load(wt + (size_t)(k * D + f) * kWave);
        }
    };
    auto take = [&](Chain &c, const T(&src)[D]) {
#pragma unroll
        for (int f = 0; f < D; ++f) {
            c.w[f] = src[f];
            c.Wb[f] = T(0);
        }
    };
    load_w(wp0, nf - 1);
    load_w(wp1, nf - 2);
    const NoPre none;

    // One step k alone (the first step when n_fwd is odd; the rest run in
    // pairs below).  In FP32 the wholly alive groups come first (unmasked), the group
    // holding forward k last, as in the forward pass but in reverse order;
    // the live groups' rows, vega entries and drift constants are
    // software-pipelined (rr, vo and co hold the next forward's), and pre()
    // runs right after the row's first use, once the wave has waited for it:
    // it issues the next forward's loads and stores the previous forward-step's
    // vega entry, so that the one wait per forward-step finds them long done.
    auto one_step = [&](Chain &c, int k) __attribute__((always_inline)) {
        T pend = T(0);   // the previous unmasked forward-step's new vega entry, not yet stored
        const int nfk = opaque_u(nf);   // tests on it stay inside the step loop
        auto body = [&](int n, const auto &q, T vb, T c6, T on, auto masked, auto pre) __attribute__((always_inline)) {
            constexpr bool MASKED = decltype(masked)::value;
            const T e = incr(c, q, c6);
            if constexpr (!std::is_same<decltype(pre), NoPre>::value) {
                __builtin_amdgcn_sched_barrier(0);
                pre();
                __builtin_amdgcn_sched_barrier(0);
            }
            const T vnew = rest(c, n, q, vb, e, on, masked);
            if constexpr (MASKED || std::is_same<decltype(pre), NoPre>::value)
                vset(n, vnew);
            else
                pend = vnew;   // written by the next forward-step, after its wait
        };
        const unsigned alive = (unsigned)(nf - k);
        if constexpr (kF32) {
            const lds_ptr<T> c6k = lds_base(c6s);
            T rr[kAdjRow] = {};
            T vo = T(0), co = T(0);
#pragma unroll
            for (int gq = NFC / kGrp - 1; gq >= 0; --gq) {
                const int n0 = gq * kGrp;
                if ((unsigned)(n0 - k) < alive) {                           // k <= n0 < n_fwd
                    if (n0 + kGrp >= nfk) {                                 // highest live group
                        load_row(rr, tab + (n0 + kGrp - 1) * kAdjRow);
                        vo = vget(n0 + kGrp - 1);
                        co = c6k[n0 + kGrp - 1];
                    }
#pragma unroll
                    for (int u = kGrp - 1; u >= 0; --u) {
                        const int n = n0 + u;
                        T q[kAdjRow];
#pragma unroll
                        for (int e = 0; e < kAdjRow; ++e) q[e] = rr[e];
                        const T vb = vo, c6 = co;
                        body(n, q, vb, c6, T(1), std::false_type{}, [&] {
                            const cptr<T> t2 = after(tab, q[0]);
                            __builtin_amdgcn_sched_barrier(0);
                            if (n > 0) {
                                load_row(rr, t2 + (n - 1) * kAdjRow);
                                vo = vget(n - 1);
                                co = c6k[n - 1];
                            }
                            // the previous forward-step (n + 1) ran unless this is
                            // the highest live group's first
                            if (n + 1 < NFC && (u < kGrp - 1 || n0 + kGrp < nfk)) vset(n + 1, pend);
                        });
                    }
                }
            }
            {   // the last unmasked forward-step's entry: forward n = k rounded up to
                // kGrp, below NFC and so (VR < kGrp) an LDS row
                const int nl = (k + kGrp - 1) & ~(kGrp - 1);
                if (nl < nf) vbar[nl][lane] = pend;
            }
#pragma unroll
            for (int gq = NFC / kGrp - 1; gq >= 0; --gq) {
                const int n0 = gq * kGrp;
                if ((unsigned)(k - n0 - 1) < (unsigned)(kGrp - 1)) {        // n0 < k < n0 + kGrp
                    // the group's rows, all requested before the first is used
                    // (one scalar-load wait for the group, not one per forward).
                    // Forward n0 < k is dead and skipped; forward n0 + kGrp - 1 >= k
                    // is live, or beyond the model, where its zero row makes the
                    // forward-step a no-op, so it runs unmasked.  One uniform
                    // branch skips the ones between when k = n0 + kGrp - 1; inside
                    // it forward n0 + kGrp - 2 is live (or beyond the model) and
                    // runs unmasked, the rest are masked (a branch per forward
                    // costs SGPRs the loop needs).
                    T qg[kGrp][kAdjRow];
#pragma unroll
                    for (int u = 1; u < kGrp; ++u) load_row(qg[u], tab + (n0 + u) * kAdjRow);
                    const Quad<T> c4 = lds_quad(c6k, n0);
                    body(n0 + kGrp - 1, qg[kGrp - 1], vget(n0 + kGrp - 1), c4.v[kGrp - 1], T(1), std::false_type{},
                         none);
                    if (k <= n0 + kGrp - 2) {
                        body(n0 + kGrp - 2, qg[kGrp - 2], vget(n0 + kGrp - 2), c4.v[kGrp - 2], T(1),
                             std::false_type{}, none);
#pragma unroll
                        for (int u = kGrp - 3; u >= 1; --u)
                            body(n0 + u, qg[u], vget(n0 + u), c4.v[u],
                                 __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(
                                     (unsigned)(n0 + u - k) < alive ? 0x3f800000u : 0u)),
                                 std::true_type{}, none);
                    }
                }
            }
        } else {
#pragma unroll
            for (int n = NFC - 1; n >= 0; --n)
                if ((unsigned)(n - k) < alive) {
                    const cptr<T> q = tab + n * kAdjRow;
                    body(n, q, vget(n), q[6], T(1), std::false_type{}, none);
                }
        }
    };

    {
        static_assert(kGrp == 4, "the paired sweep's boundary group is written for groups of four");
        int k = nf - 1;
        if (nf & 1) {
            Chain c;
            take(c, wp0);
#pragma unroll
            for (int f = 0; f < D; ++f) wp0[f] = wp1[f];
            load_w(wp1, k - 2);
            one_step(c, k);
            --k;
        }
        // Then two steps at a time: the leading chain runs step kp, the
        // trailing chain step kp - 1 one forward behind it.  Each slot of the
        // wholly alive groups holds the leading chain's forward-step n and the
        // trailing chain's n + 1, independent work that shares one wait; the
        // trailing chain takes forward n + 1's row and drift constant from the
        // slot before and the leading chain's new vega entry from a register,
        // so only the trailing chain writes vega rows (after the next wait).
        // Both precisions: FP64, at one wave per SIMD, has the more latency
        // to hide (its whole step with Greeks took 13% less time than with
        // one step at a time; the FP32 reverse half 5% less).
#pragma unroll 1
        for (int kp = k; kp >= 1; kp -= 2) {
            Chain cL, cT;
            take(cL, wp0);
            take(cT, wp1);
            load_w(wp0, kp - 2);
            load_w(wp1, kp - 3);
            const int nfk = opaque_u(nf);
            const unsigned aliveL = (unsigned)(nf - kp);
            // drift constants: FP32 from the LDS table (a vector operand),
            // FP64 from the row's entry 6
            lds_ptr<T> c6k{};
            if constexpr (kF32) c6k = lds_base(c6s);
            T rr[kAdjRow] = {}, qT[kAdjRow] = {};
            T vo = T(0), co = T(0), c6T = T(0), vbT = T(0), pendT = T(0);
#pragma unroll
            for (int gq = NFC / kGrp - 1; gq >= 0; --gq) {
                const int n0 = gq * kGrp;
                if ((unsigned)(n0 - kp) < aliveL) {                         // kp <= n0 < n_fwd
                    const bool top = n0 + kGrp >= nfk;                      // highest live group
                    if (top) {
                        load_row(rr, tab + (n0 + kGrp - 1) * kAdjRow);
                        vo = vget(n0 + kGrp - 1);
                        if constexpr (kF32) co = c6k[n0 + kGrp - 1];
                    }
#pragma unroll
                    for (int u = kGrp - 1; u >= 0; --u) {
                        const int n = n0 + u;
                        T q[kAdjRow];
#pragma unroll
                        for (int e = 0; e < kAdjRow; ++e) q[e] = rr[e];
                        const T vbL = vo, c6L = kF32 ? co : q[6];
                        // the trailing chain at n + 1: none in the first slot
                        const bool hasT = n + 1 < NFC && !(top && u == kGrp - 1);
                        const T eL = incr(cL, q, c6L);
                        T eT = T(0);
                        if (hasT) eT = incr(cT, qT, c6T);
                        __builtin_amdgcn_sched_barrier(0);
                        {
                            const cptr<T> t2 = after(tab, q[0]);
                            __builtin_amdgcn_sched_barrier(0);
                            if (n > 0) {
                                load_row(rr, t2 + (n - 1) * kAdjRow);
                                vo = vget(n - 1);
                                if constexpr (kF32) co = c6k[n - 1];
                            }
                            // the trailing chain's entry of forward n + 2, from the
                            // slot before the previous one (none in the first two)
                            if (n + 2 < NFC && !(top && u >= kGrp - 2)) vset(n + 2, pendT);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                        const T vnL = rest(cL, n, q, vbL, eL, T(1), std::false_type{});
                        if (hasT) pendT = rest(cT, n + 1, qT, vbT, eT, T(1), std::false_type{});
#pragma unroll
                        for (int e = 0; e < kAdjRow; ++e) qT[e] = q[e];
                        c6T = c6L;
                        vbT = vnL;
                    }
                    if (n0 - kGrp < kp) {
                        // the lowest such group: the trailing chain's forward n0
                        vset(n0 + 1, pendT);
                        const T eT = incr(cT, qT, c6T);
                        vset(n0, rest(cT, n0, qT, vbT, eT, T(1), std::false_type{}));
                    }
                }
            }
            // The group holding forward kp (n0 < kp <= n0 + 4, r = kp - n0):
            // forward n0 + 3 is the leading chain's if r <= 3 (masked) and the
            // trailing chain's always; n0 + 2 the leading chain's if r <= 2 and
            // the trailing chain's if r <= 3; n0 + 1 likewise with r <= 1 and
            // r <= 2; n0 the trailing chain's if r = 1.  Uniform branches skip
            // the levels no chain needs; each level runs the leading chain's
            // forward-step (masked), then the trailing chain's (unmasked; a
            // forward beyond the model has a zero row and is a no-op).
#pragma unroll
            for (int gq = NFC / kGrp - 1; gq >= 0; --gq) {
                const int n0 = gq * kGrp;
                if ((unsigned)(kp - n0 - 1) < (unsigned)kGrp) {
                    const int r = kp - n0;
                    T qg[kGrp][kAdjRow];
#pragma unroll
                    for (int u = 1; u < kGrp; ++u) load_row(qg[u], tab + (n0 + u) * kAdjRow);
                    Quad<T> c4{};
                    if constexpr (kF32) c4 = lds_quad(c6k, n0);
                    auto c6g = [&](int u) __attribute__((always_inline)) -> T {
                        if constexpr (kF32) return c4.v[u];
                        else return qg[u][6];
                    };
                    auto level = [&](int u) __attribute__((always_inline)) {
                        const int n = n0 + u;
                        T on;
                        if constexpr (kF32)
                            on = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(n >= kp ? 0x3f800000u : 0u));
                        else
                            on = n >= kp ? 1.0 : 0.0;
                        vset(n, rest(cL, n, qg[u], vget(n), incr(cL, qg[u], c6g(u)), on, std::true_type{}));
                        vset(n, rest(cT, n, qg[u], vget(n), incr(cT, qg[u], c6g(u)), T(1), std::false_type{}));
                    };
                    level(3);
                    if (r <= 3) {
                        level(2);
                        if (r <= 2) {
                            level(1);
                            if (r <= 1) {
                                load_row(qg[0], tab + n0 * kAdjRow);
                                vset(n0, rest(cT, n0, qg[0], vget(n0), incr(cT, qg[0], c6g(0)), T(1),
                                              std::false_type{}));
                            }
                        }
                    }
                }
            }
        }
    }

    // ---- Greeks [2 nf + 1]: deltas, spot delta (above), vegas ----
    // dbook/dL_n(0) = Xbar_n / (L_n(0) ln 2): row entry 10 is 1/(L_n(0) ln 2)
    // and entry 11 the vega rows' 1/sigma~_n, both 0 beyond n_fwd, where Xbar
    // and the vega rows are 0 as well
    const cptr<double> f3 = opaque_u(fwd);
#pragma unroll
    for (int c = 0; c < NFC / 16; ++c) {
        if (c * 16 < nf) {
            const int o = c * 16 + (lane >> 2);
            const bool wr = (lane & 3) == 0 && o < nf;
            double V[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int n = c * 16 + q;
                V[q] = (double)Xb[n] * f3[n * kFwdRow + 10] * act;
            }
            double s = wave_sum16(V, lane);
            if (wr) gout[o] = s;
#pragma unroll
            for (int q = 0; q < 16; ++q)   // sigma_n vega_n / sigma_n
                V[q] = (double)vget(c * 16 + q) * f3[(c * 16 + q) * kFwdRow + 11] * act;
            s = wave_sum16(V, lane);
            if (wr) gout[nf + 1 + o] = s;
        }
    }
}

// Single-call adjoint, two kernels per chunk of tasks (task = m n_blk + blk,
// one 64-path wave per block, one block per task):
//  * lmm_adj_fwd_kernel runs the forward passes.  Its state is the 80
//    forwards (the 16 lowest in LDS at capacity 80) and w only, so it runs
//    at five waves per SIMD in FP32 (the point generation and the
//    forward-steps hide each other's latencies); it stores w per step and
//    the final states, 82 KB per task in FP32.
//  * lmm_adj_rev_kernel loads the final states and runs the payoffs and the
//    reverse sweep with the vega rows in LDS, at two waves per SIMD (X and
//    Xbar in registers).
// Forward states held in LDS by the FP32 forward half: the 16 lowest
// forwards' at capacity 80 (a fifth wave per SIMD), none below
template <int NFC, typename T>
constexpr int fwd_lds_states()
{
    return sizeof(T) == 4 && NFC == 80 ? 16 : 0;
}

template <int NFC, int D, typename T, bool MC>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(fwd_lds_states<NFC, T>() ? 5 : sizeof(T) == 4 ? 4 : 2)))
void lmm_adj_fwd_kernel(LmmArgs a)
{
    constexpr int XL = fwd_lds_states<NFC, T>();
    __shared__ T vbar[NFC][kWave];   // not touched by the forward half
    __shared__ __align__(32) T c6s[NFC];
    __shared__ T xl[XL > 0 ? XL : 1][kWave];
    const int64_t local = blockIdx.x;
    const int64_t task = a.task0 + local;
    const int m = (int)(task / a.n_blk);
    const int blk = (int)(task - (int64_t)m * a.n_blk);
    T *wt = (T *)a.wtop + local * ((int64_t)a.n_fwd * D * kWave) + threadIdx.x;
    T *xs = (T *)a.xs + local * ((int64_t)NFC * kWave) + threadIdx.x;
    lmm_task<NFC, D, T, true, MC, kTaskFwd, 0, XL>(a, m, blk, task, wt, vbar, xs, c6s, xl);
}

// FP32: the compiler is asked for two waves per SIMD (at most 256 registers;
// the sweep takes about 195, without spills); FP64: one.
template <int NFC, int D, typename T, bool MC>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 2 : 1)))
void lmm_adj_rev_kernel(LmmArgs a)
{
    constexpr int VR = rev_reg_rows<NFC, T>();
    __shared__ T vbar[NFC - VR][kWave];
    const int64_t local = blockIdx.x;
    const int64_t task = a.task0 + local;
    const int m = (int)(task / a.n_blk);
    const int blk = (int)(task - (int64_t)m * a.n_blk);
    T *wt = (T *)a.wtop + local * ((int64_t)a.n_fwd * D * kWave) + threadIdx.x;
    T *xs = (T *)a.xs + local * ((int64_t)NFC * kWave) + threadIdx.x;
    if constexpr (sizeof(T) == 4) {
        __shared__ __align__(32) T c6s[NFC];
        lmm_task<NFC, D, T, true, MC, kTaskRev, VR>(a, m, blk, task, wt, vbar, xs, c6s);
    } else {   // FP64: the vega rows take the LDS of one wave per SIMD
        lmm_task<NFC, D, T, true, MC, kTaskRev>(a, m, blk, task, wt, vbar, xs);
    }
}

// One half (part kTaskFwd or kTaskRev) over tasks [a.task0, a.task0 +
// a.chunk).  The host launches the forward half, then the reverse half of
// the same tasks on the same stream, so the stored values are complete.
template <int NFC, int D, typename T, bool MC>
static hipError_t launch_adj_t(const LmmArgs &a, int part, hipStream_t st)
{
    if (part == kTaskFwd)
        hipLaunchKernelGGL((lmm_adj_fwd_kernel<NFC, D, T, MC>), dim3((unsigned)a.chunk), dim3(kWave), 0, st, a);
    else
        hipLaunchKernelGGL((lmm_adj_rev_kernel<NFC, D, T, MC>), dim3((unsigned)a.chunk), dim3(kWave), 0, st, a);
    return hipGetLastError();
}

template <int D, typename T, bool MC>
static hipError_t launch_adj_d(const LmmArgs &a, int part, hipStream_t st)
{
    if (a.n_fwd <= 16) return launch_adj_t<16, D, T, MC>(a, part, st);
    if (a.n_fwd <= 32) return launch_adj_t<32, D, T, MC>(a, part, st);
    if (a.n_fwd <= 48) return launch_adj_t<48, D, T, MC>(a, part, st);
    if (a.n_fwd <= 64) return launch_adj_t<64, D, T, MC>(a, part, st);
    return launch_adj_t<80, D, T, MC>(a, part, st);
}

// Adjoint launch for one precision and point generator (instantiated in
// rq_lmm_adj{32,64}{,mc}.hip, so that the four compile in parallel).
template <typename T, bool MC>
static hipError_t launch_adj_prec(const LmmArgs &a, int n_factors, int part, hipStream_t st)
{
    switch (n_factors) {
    case 1: return launch_adj_d<1, T, MC>(a, part, st);
    case 2: return launch_adj_d<2, T, MC>(a, part, st);
    case 3: return launch_adj_d<3, T, MC>(a, part, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lmm_adjoint_f32(const LmmArgs &a, int n_factors, int part, hipStream_t st);
hipError_t launch_lmm_adjoint_f64(const LmmArgs &a, int n_factors, int part, hipStream_t st);
hipError_t launch_lmm_adjoint_f32mc(const LmmArgs &a, int n_factors, int part, hipStream_t st);
hipError_t launch_lmm_adjoint_f64mc(const LmmArgs &a, int n_factors, int part, hipStream_t st);

}  // namespace rq
