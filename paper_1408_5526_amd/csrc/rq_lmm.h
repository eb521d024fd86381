// rq_lmm.h -- LIBOR market model caplet pricing, one path per lane.
//
// Model (caplet section): forwards L_1..L_n, spot measure, constant vol
// vectors a_n.  Step k (from T_k to T_{k+1}, k = 0..n-1) updates the alive
// forwards n = k+1..n_fwd in ascending order with the log-Euler form of the
// discretised SDE, drift from pre-step values:
//   g_n = delta L_n / (1 + delta L_n),  v += g_n a_n,  mu_n = a_n . v,
//   L_n <- L_n exp(mu_n delta - delta |a_n|^2 / 2 + sqrt(delta) a_n . z_k).
// The kernel carries w = delta v + sqrt(delta) z_k instead of v, so that
//   w += g_n (delta a_n),   exponent = a_n . w + c_n,   c_n = -delta|a_n|^2/2
// (the same quantities regrouped: 2d fused multiply-adds per forward-step).
// The caplet on L_n fixes at T_n and pays delta (L_n - K)^+ at T_{n+1},
// discounted by the spot numeraire prod_{j<=n} (1 + delta L_j(T_j)) (FP64).
// A forward is not touched after it fixes, so all payoffs are formed after
// the time loop from the final state.
//
// FP32 form: the lane keeps X_n = log2(L_n / L_n(0)).  With the constant
// kappa_n = 1 / (delta L_n(0)) the drift factor is
//   g_n = delta L_n / (1 + delta L_n) = 1 / (1 + kappa_n 2^{-X_n})
// (one v_exp_f32, one fused multiply-add, one v_rcp_f32), and the step is
//   X_n += log2(e) (a_n . w + c_n),
// the (small) increment being formed before it is added, so the O(1) state
// rounds once per step at its own scale (~3e-8) and the exponential's error
// is not carried from step to step.  Fixing values are formed in FP64,
// L_n(T_n) = L_n(0) 2^{X_n}.
//
// GPU mapping: a lane owns one path; the forward vector lives in registers.
// The inner loop over forwards is unrolled to a compile-time capacity NFC so
// that every state element is a fixed register; forwards that are dead
// (n < k) or beyond the model (n >= n_fwd) are skipped by one wave-uniform
// branch each.  Per-forward constants are wave-uniform (scalar loads).
// Points are produced in registers from the replication's start table (no
// point set is materialised).  Payoffs are summed over the wave 16 outputs
// at a time with a transpose butterfly, the four waves of a block in a fixed
// order, and the block writes one partial per output: the whole reduction is
// deterministic.
#pragma once

#include "rq_device.h"

namespace rq {


// GEN: 0 random-start Halton, 1 the same with permuted digits, 2 Philox
// pseudo-random points (the comparison baseline).  EULER: the plain Euler
// step of the paper's discretised SDE instead of the log-Euler step,
//   L_n <- L_n + mu_n L_n delta + L_n sqrt(delta) a_n . z_k = L_n (1 + a_n . w).
// Occupancy hints: FP32 forms at five waves per SIMD at capacity 80 (the
// 24 lowest forwards' states then live in LDS: forward n moves in steps
// 0..n only, so they take few of the forward-steps, and their registers go
// to the fifth wave; a few values are still spilled, and the kernel is 7%
// (Halton) and 4% (Philox) faster than at four waves); below capacity 80 the
// FP32 Halton forms at four; FP64 Halton forms at two (256 registers: the 80
// FP64 forwards take 160 of them, and the second wave hides the latency of
// the long dependent FP64 chains of the drift factor, the exponential and
// the digits); Philox forms otherwise at the compiler's choice.
template <int NFC, typename T, int GEN>
constexpr int price_lds_states()
{
    return sizeof(T) == 4 && NFC == 80 ? 24 : 0;
}

template <int NFC, int D, typename T, int GEN, bool EULER = false>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(price_lds_states<NFC, T, GEN>() ? 5 : GEN == 2 ? 1 : (sizeof(T) == 4 ? 4 : 2))))
void lmm_kernel(LmmArgs a)
{
    static_assert(NFC % 16 == 0, "capacity must be a multiple of 16");
    constexpr bool kF32 = sizeof(T) == 4;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int m = blockIdx.x / a.n_blk;
    const int blk = blockIdx.x - m * a.n_blk;
    const int64_t i = (int64_t)blk * kBlock + tid;
    const bool active = i < a.g.N;
    const int seg = (int)(((int64_t)blk * kBlock) >> a.g.log2S);
    const uint32_t t = (uint32_t)(i - ((int64_t)seg << a.g.log2S));
    const StartEnt *__restrict__ st = a.g.starts + ((size_t)m * a.g.n_seg + seg) * a.g.s;
    const cptr<double> fwd = as_const<double>(a.fwd);   // read-only tables: scalar loads
    const cptr<float> fwd32 = as_const<float>(a.fwd32);
    const int nf = a.n_fwd;

    __shared__ double red[kBlock / kWave][NFC];
    __shared__ double tot[NFC];
    // the drift constants (log2(e) c_n in FP32, c_n in FP64), broadcast from
    // LDS: a forward-step's first FMA then takes one scalar operand (the
    // loading) and one vector operand (the constant), and no constant is
    // moved to a vector register
    __shared__ __align__(32) T c6s[NFC];
    for (int n = tid; n < NFC; n += kBlock) c6s[n] = kF32 ? (T)fwd32[n * kRow32 + 6] : (T)fwd[n * kFwdRow + 6];
    __syncthreads();

    auto r64 = [&](int n, int c) -> double { return fwd[n * kFwdRow + c]; };

    // state: FP32 X_n = log2(L_n / L_n(0)); FP64 L_n.  Forward n's state is
    // X[n], or the thread's entry of the LDS row xl[n] for the XL lowest
    // forwards (n is a compile-time constant at every use).
    constexpr int XL = price_lds_states<NFC, T, GEN>();
    __shared__ T xl[XL > 0 ? XL : 1][kBlock];
    T X[NFC];
    auto xget = [&](int n) -> T { return n < XL ? xl[n][tid] : X[n]; };
    auto xset = [&](int n, T v) {
        if (n < XL) xl[n][tid] = v;
        else X[n] = v;
    };
#pragma unroll
    for (int n = 0; n < NFC; ++n) xset(n, kF32 ? T(0) : T(r64(n, 7)));   // rows beyond n_fwd are 0

    const T sqd = (T)a.sqrt_delta;
    const double delta = a.delta;

    McPath mc;
#pragma unroll 1
    for (int k = 0; k < nf; ++k) {
        T w[D];
        // the step's base and start entries, all requested before the first
        // is used: one scalar-load wait per step instead of one per dimension
        PointCtx cs[D];
        StartEnt ses[D];
        if constexpr (GEN != 2) {
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
            if constexpr (GEN == 2) {
                x = mc.point(a.g.seed, (uint64_t)(a.g.m_offset + m), (uint64_t)i, j);
            } else {
                x = radinv_x<GEN == 1, sizeof(T) == 8>(cs[f], ses[f], t, a.g.perm + (size_t)m * a.g.perm_stride);
            }
            w[f] = sqd * inv_normal(x, T(0));
        }
        // One forward-step of forward n (alive in this step); c6 is its drift
        // constant from LDS.
        auto body = [&](int n, T c6) __attribute__((always_inline)) {
            if constexpr (kF32) {
                const cptr<float> q = fwd32 + n * kRow32;
                const float xn = xget(n);
                const float g = __builtin_amdgcn_rcpf(ffma(q[7], fexp2(-xn), 1.0f));
#pragma unroll
                for (int f = 0; f < D; ++f) w[f] = ffma(g, q[3 + f], w[f]);
                // form the (small) step increment first, then add it to the
                // O(1) state once: one rounding at the state's scale per step
                if constexpr (EULER) {
                    // plain Euler: L <- L (1 + a_n . w), i.e. X += log2(1 + a_n . w);
                    // the argument is kept positive (an Euler step that would
                    // make L negative is outside what the log form holds)
                    float e = q[0] * w[0];
#pragma unroll
                    for (int f = 1; f < D; ++f) e = ffma(q[f], w[f], e);
                    const float r = fmaxf(ffma(e, 0.693147180559945309f, 1.0f), 0x1p-100f);
                    xset(n, xn + __builtin_amdgcn_logf(r));
                } else {
                    float e = ffma(q[0], w[0], (float)c6);
#pragma unroll
                    for (int f = 1; f < D; ++f) e = ffma(q[f], w[f], e);
                    xset(n, xn + e);
                }
            } else {
                // drift factor delta L / (1 + delta L) with the Newton
                // reciprocal (within an ulp or two of the quotient)
                const double dl = delta * X[n];
                const double g = dl * recip64(1.0 + dl);
#pragma unroll
                for (int f = 0; f < D; ++f) w[f] = ffma(g, r64(n, 3 + f), w[f]);
                if constexpr (EULER) {   // plain Euler: L <- L + L (a_n . w)
                    double e = r64(n, 0) * w[0];
#pragma unroll
                    for (int f = 1; f < D; ++f) e = ffma(r64(n, f), w[f], e);
                    X[n] = ffma(X[n], e, X[n]);
                } else {
                    double e = (double)c6;
#pragma unroll
                    for (int f = 0; f < D; ++f) e = ffma(r64(n, f), w[f], e);
                    X[n] = X[n] * exp(e);
                }
            }
        };
        const unsigned alive = (unsigned)(nf - k);
        const lds_ptr<T> c6k = lds_base(&c6s[0]);
        if constexpr (!kF32) {
            // FP64: one uniform branch per forward (its exp and division are
            // too costly to spend on dead forwards)
#pragma unroll
            for (int n = 0; n < NFC; ++n)
                if ((unsigned)(n - k) < alive) body(n, c6k[n]);
            continue;
        }
        // FP32: in the group holding forward k (n0 < k < n0 + kGrp) each live
        // forward runs behind its own uniform branch, first; the wholly alive
        // groups (k <= n0 < n_fwd) run after it as branch-free blocks (two
        // passes keep the two forms out of one branch)
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
    }

    // payoffs (FP64), 16 forwards at a time
    double num = a.num0;
    double book = 0.0;
    double *pp = (a.per_path && active) ? a.per_path + ((size_t)m * (size_t)a.g.N + (size_t)i) * a.n_out
                                        : nullptr;
#pragma unroll
    for (int c = 0; c < NFC / 16; ++c) {
        if (c * 16 < nf) {
            double P[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                // rows beyond n_fwd are 0 (no numeraire factor, no payoff);
                // the caplet flag multiplies the payoff
                const int n = c * 16 + q;
                // FP32: 2^X in FP32 (one more rounding, of the size the FP32
                // state already carries), the fixing value and payoff in FP64
                const double Lf = kF32 ? r64(n, 7) * (double)fexp2((float)xget(n)) : (double)X[n];
                const double onep = 1.0 + delta * Lf;
                const double ex = Lf - r64(n, 8);
                num *= onep;
                double pay = ex > 0.0 ? r64(n, 9) * (delta * ex * recip64(num)) : 0.0;
                pay = active ? pay : 0.0;
                book += pay;
                if (pp) pp[n < nf ? n : nf] = pay;   // beyond n_fwd: 0 into the book slot, rewritten below
                P[q] = pay;
            }
            const double s = wave_sum16(P, lane);
            if ((lane & 3) == 0) red[wave][c * 16 + (lane >> 2)] = s;
        }
    }
    if (pp) pp[nf] = book;
    __syncthreads();
    double *out = a.partial + ((size_t)m * a.n_blk + blk) * a.n_out;
    for (int o = tid; o < nf; o += kBlock) {
        double s = red[0][o];
        s += red[1][o];
        s += red[2][o];
        s += red[3][o];
        tot[o] = s;
        out[o] = s;
    }
    __syncthreads();
    if (tid == 0) {   // the book: sum of the block's caplet totals, in order
        double s = 0.0;
        for (int o = 0; o < nf; ++o) s += tot[o];
        out[nf] = s;
    }
}

template <int NFC, int D, typename T, int GEN, bool EULER>
static hipError_t launch_t(const LmmArgs &a, hipStream_t st)
{
    const int64_t blocks = (int64_t)a.n_blk * a.g.M;
    hipLaunchKernelGGL((lmm_kernel<NFC, D, T, GEN, EULER>), dim3((unsigned)blocks), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

template <int D, typename T, int GEN, bool EULER>
static hipError_t launch_d(const LmmArgs &a, hipStream_t st)
{
    if (a.n_fwd <= 16) return launch_t<16, D, T, GEN, EULER>(a, st);
    if (a.n_fwd <= 32) return launch_t<32, D, T, GEN, EULER>(a, st);
    if (a.n_fwd <= 48) return launch_t<48, D, T, GEN, EULER>(a, st);
    if (a.n_fwd <= 64) return launch_t<64, D, T, GEN, EULER>(a, st);
    return launch_t<80, D, T, GEN, EULER>(a, st);
}

// Pricing launch for one point generator (instantiated in rq_lmm.hip for
// the Halton forms and in rq_lmm_mc.hip for the pseudo-random one, so that
// they compile in parallel).
template <int GEN, bool EULER = false>
static hipError_t launch_lmm_gen_t(const LmmArgs &a, int n_factors, int fp32, hipStream_t st)
{
    switch (n_factors * 2 + (fp32 ? 1 : 0)) {
    case 2: return launch_d<1, double, GEN, EULER>(a, st);
    case 3: return launch_d<1, float, GEN, EULER>(a, st);
    case 4: return launch_d<2, double, GEN, EULER>(a, st);
    case 5: return launch_d<2, float, GEN, EULER>(a, st);
    case 6: return launch_d<3, double, GEN, EULER>(a, st);
    case 7: return launch_d<3, float, GEN, EULER>(a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lmm_mc(const LmmArgs &a, int n_factors, int fp32, hipStream_t st);
hipError_t launch_lmm_euler(const LmmArgs &a, int n_factors, int fp32, hipStream_t st);

}  // namespace rq
