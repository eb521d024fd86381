// rq_lmm_adj.h -- pathwise Greeks of the LIBOR caplet book by a
// hand-written adjoint (reverse-mode) sweep, one path per lane.
//
// Forward pass (same scheme as rq_lmm.hip, state X_n = log2(L_n / L_n(0))):
//   step k:  w = sqrt(delta) z_k;  for n = k..n_fwd-1:
//     g_n = G(X_n) = 1 / (1 + 2^{-(X_n + l_n)}),  l_n = log2(delta L_n(0))
//     w  += g_n delta a_n
//     X_n += log2(e) (c_n + a_n . w)
// Payoffs (FP64): L_n(T_n) = L_n(0) 2^{X_n}; P_n = delta (L_n - K_n)^+ / num_{n+1},
//   num_{n+1} = num_0 prod_{j<=n} (1 + delta L_j(T_j)); book = sum_n P_n.
//
// Reverse sweep.  The payoff adjoint is
//   dbook/dL_n(T_n) = delta [L_n > K_n] / num_{n+1} - delta / (1 + delta L_n) * sum_{j>=n} P_j
// and Xbar_n = dbook/dL_n(T_n) * L_n(T_n) ln 2.  Steps then run backwards.  The
// pre-step state of step k is not stored: it is recovered from the post-step
// state.  With C = X_post - log2(e) c_n - log2(e) a_n . w_{n-1} and
// q_n = log2(e) delta |a_n|^2 >= 0, the pre-state solves
//   y + q_n G(y) = C,
// whose left side is strictly increasing.  Newton from y0 = C - q_n G(X_post)
// converges quadratically (FP32: one step, FP64: two).  Ascending n rebuilds
// the states and w; descending n then applies the adjoint of each
// forward-step:
//   Wbar += Xbar_n log2(e) a_n           (adjoint of w_n, a suffix sum over n)
//   gbar  = delta a_n . Wbar
//   vega_n += Xbar_n log2(e) (b_n . w_n - delta sigma_n |b_n|^2) + g_n delta b_n . Wbar
//   Xbar_n += gbar G'(X_n),  G' = ln2 G (1 - G)
//   w    -= g_n delta a_n                (back to w_{n-1})
// After step 0, Xbar_n is the adjoint of log2 L_n(0), so
//   dbook/dL_n(0) = Xbar_n / (L_n(0) ln 2);  dbook/dL_0(0) = -delta book / num_0.
//
// Per path: n_fwd+1 prices (caplets, book) and 2 n_fwd + 1 Greeks (deltas,
// spot delta, vegas), reduced like the pricing kernel (wave transpose
// butterfly, fixed block order).  State and adjoint state live in registers;
// the vega accumulators live in LDS ([forward][lane], conflict-free).
#pragma once

#include "rq_device.h"

namespace rq {

constexpr int kAdjBlock = 128;   // two waves; LDS holds the vega accumulators

template <typename T> __device__ __forceinline__ T adj_exp2(T x);
template <> __device__ __forceinline__ float adj_exp2<float>(float x) { return __builtin_amdgcn_exp2f(x); }
template <> __device__ __forceinline__ double adj_exp2<double>(double x) { return exp2(x); }
template <typename T> __device__ __forceinline__ T adj_rcp(T x);
template <> __device__ __forceinline__ float adj_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double adj_rcp<double>(double x) { return 1.0 / x; }

template <int NFC, int D, typename T>
__global__ __launch_bounds__(kAdjBlock) void lmm_adjoint_kernel(LmmArgs a)
{
    static_assert(NFC % 16 == 0, "capacity must be a multiple of 16");
    constexpr bool kF32 = sizeof(T) == 4;
    constexpr T kLn2 = T(0.69314718055994530942);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int m = blockIdx.x / a.n_blk;
    const int blk = blockIdx.x - m * a.n_blk;
    const int64_t i = (int64_t)blk * kAdjBlock + tid;
    const bool active = i < a.g.N;
    const int seg = (int)(((int64_t)blk * kAdjBlock) >> a.g.log2S);
    const uint32_t t = (uint32_t)(i - ((int64_t)seg << a.g.log2S));
    const StartEnt *__restrict__ st = a.g.starts + ((size_t)m * a.g.n_seg + seg) * a.g.s;
    const double *__restrict__ fwd = a.fwd;
    const T *__restrict__ adj = (const T *)a.adj;
    const int nf = a.n_fwd;
    const double delta = a.delta;
    const T sqd = (T)a.sqrt_delta;

    __shared__ T vbar[NFC][kAdjBlock];
    __shared__ double red[kAdjBlock / kWave][3 * NFC];
    __shared__ double red2[kAdjBlock / kWave][2];

    auto r64 = [&](int n, int c) -> double { return fwd[n * kFwdRow + c]; };
    auto ra = [&](int n, int c) -> T { return adj[n * kAdjRow + c]; };
    auto G = [&](int n, T y) -> T { return adj_rcp<T>(T(1) + adj_exp2<T>(-(y + ra(n, 7)))); };
    auto normals = [&](int k, T (&w)[D]) {
#pragma unroll
        for (int f = 0; f < D; ++f) {
            const int j = k * D + f;
            const PointCtx c = load_base(a.g.base, j);
            const double x = a.g.perm_on ? radinv_x<true, !kF32>(c, st + j, t, a.g.perm)
                                         : radinv_x<false, !kF32>(c, st + j, t, a.g.perm);
            w[f] = sqd * inv_normal(x, T(0));
        }
    };

    T X[NFC], Xb[NFC];
#pragma unroll
    for (int n = 0; n < NFC; ++n) {
        X[n] = T(0);
        Xb[n] = T(0);
        vbar[n][tid] = T(0);
    }

    // ---- forward pass ----
#pragma unroll 1
    for (int k = 0; k < nf; ++k) {
        T w[D];
        normals(k, w);
        const unsigned alive = (unsigned)(nf - k);
#pragma unroll
        for (int n = 0; n < NFC; ++n) {
            if ((unsigned)(n - k) < alive) {
                const T g = G(n, X[n]);
#pragma unroll
                for (int f = 0; f < D; ++f) w[f] = ffma(g, ra(n, 3 + f), w[f]);
                T e = ra(n, 0) * w[0];
#pragma unroll
                for (int f = 1; f < D; ++f) e = ffma(ra(n, f), w[f], e);
                X[n] += e + ra(n, 6);
            }
        }
    }

    // ---- payoffs and their adjoint (FP64) ----
    // pass 1: the book; pass 2 (16 forwards at a time): payoffs again, their
    // wave sums, and the adjoint of the fixing values
    const double act = active ? 1.0 : 0.0;
    double *pp = (a.per_path && active) ? a.per_path + ((size_t)m * (size_t)a.g.N + (size_t)i) * a.n_out
                                        : nullptr;
    double book = 0.0;
    {
        double num = a.num0;
#pragma unroll
        for (int n = 0; n < NFC; ++n) {
            if (n < nf) {
                const double Lf = r64(n, 7) * exp2((double)X[n]);
                num *= 1.0 + delta * Lf;
                const double ex = Lf - r64(n, 8);
                if (r64(n, 9) != 0.0 && ex > 0.0) book += delta * ex / num;
            }
        }
    }
    {
        double num = a.num0;
        double before = 0.0;   // sum_{j<n} P_j
#pragma unroll
        for (int c = 0; c < NFC / 16; ++c) {
            if (c * 16 < nf) {
                double V[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int n = c * 16 + q;
                    double Pn = 0.0;
                    if (n < nf) {
                        const double Lf = r64(n, 7) * exp2((double)X[n]);
                        const double onep = 1.0 + delta * Lf;
                        num *= onep;
                        const double ex = Lf - r64(n, 8);
                        const bool itm = r64(n, 9) != 0.0 && ex > 0.0;
                        if (itm) Pn = delta * ex / num;
                        double dL = -delta / onep * (book - before);
                        if (itm) dL += delta / num;
                        Xb[n] = (T)(dL * Lf * 0.69314718055994530942);
                        before += Pn;
                        if (pp) pp[n] = Pn;
                    }
                    V[q] = Pn * act;
                }
                const double sv = wave_sum16(V, lane);
                if ((lane & 3) == 0) red[wave][c * 16 + (lane >> 2)] = sv;
            }
        }
    }
    if (pp) pp[nf] = book;

    // ---- reverse sweep ----
#pragma unroll 1
    for (int k = nf - 1; k >= 0; --k) {
        T w[D];
        normals(k, w);
        const unsigned alive = (unsigned)(nf - k);
        // ascending: rebuild the pre-step states and w
#pragma unroll
        for (int n = 0; n < NFC; ++n) {
            if ((unsigned)(n - k) < alive) {
                T C = X[n] - ra(n, 6);
#pragma unroll
                for (int f = 0; f < D; ++f) C = ffma(-ra(n, f), w[f], C);
                const T q = ra(n, 8);
                T y = C - q * G(n, X[n]);
#pragma unroll
                for (int it = 0; it < (kF32 ? 1 : 2); ++it) {
                    const T gy = G(n, y);
                    const T h = y + q * gy - C;
                    const T dh = T(1) + q * kLn2 * gy * (T(1) - gy);
                    y -= h * adj_rcp<T>(dh);
                }
                X[n] = y;
                const T g = G(n, y);
#pragma unroll
                for (int f = 0; f < D; ++f) w[f] = ffma(g, ra(n, 3 + f), w[f]);
            }
        }
        // descending: adjoint of each forward-step
        T Wb[D];
#pragma unroll
        for (int f = 0; f < D; ++f) Wb[f] = T(0);
#pragma unroll
        for (int nn = 0; nn < NFC; ++nn) {
            const int n = NFC - 1 - nn;
            if ((unsigned)(n - k) < alive) {
                const T g = G(n, X[n]);
                const T xb = Xb[n];
                T bw = T(0), dbw = T(0), gb = T(0);
#pragma unroll
                for (int f = 0; f < D; ++f) {
                    Wb[f] = ffma(xb, ra(n, f), Wb[f]);
                    bw = ffma(ra(n, 9 + f), w[f], bw);
                }
#pragma unroll
                for (int f = 0; f < D; ++f) {
                    dbw = ffma(ra(n, 12 + f), Wb[f], dbw);
                    gb = ffma(ra(n, 3 + f), Wb[f], gb);
                }
                vbar[n][tid] += ffma(xb, bw - ra(n, 15), g * dbw);
                Xb[n] = ffma(gb * kLn2 * g, T(1) - g, xb);
#pragma unroll
                for (int f = 0; f < D; ++f) w[f] = ffma(-g, ra(n, 3 + f), w[f]);
            }
        }
    }

    // ---- Greeks [2 nf + 1]: deltas, spot delta, vegas ----
#pragma unroll
    for (int c = 0; c < NFC / 16; ++c) {
        if (c * 16 < nf) {
            double V[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int n = c * 16 + q;
                V[q] = n < nf ? (double)Xb[n] / (r64(n, 7) * 0.69314718055994530942) * act : 0.0;
            }
            double s = wave_sum16(V, lane);
            if ((lane & 3) == 0) red[wave][NFC + c * 16 + (lane >> 2)] = s;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int n = c * 16 + q;
                V[q] = n < nf ? (double)vbar[n][tid] * act : 0.0;
            }
            s = wave_sum16(V, lane);
            if ((lane & 3) == 0) red[wave][2 * NFC + c * 16 + (lane >> 2)] = s;
        }
    }
    {
        const double b = wave_sum(book * act);
        const double sp = wave_sum(-delta * book / a.num0 * act);
        if (lane == 0) {
            red2[wave][0] = b;
            red2[wave][1] = sp;
        }
    }
    __syncthreads();
    double *out = a.partial + ((size_t)m * a.n_blk + blk) * a.n_out;
    double *gout = a.partial_g + ((size_t)m * a.n_blk + blk) * a.n_g;
    for (int o = tid; o < nf; o += kAdjBlock) {
        out[o] = red[0][o] + red[1][o];
        gout[o] = red[0][NFC + o] + red[1][NFC + o];
        gout[nf + 1 + o] = red[0][2 * NFC + o] + red[1][2 * NFC + o];
    }
    if (tid == 0) {
        out[nf] = red2[0][0] + red2[1][0];
        gout[nf] = red2[0][1] + red2[1][1];
    }
}

template <int NFC, int D, typename T>
static hipError_t launch_adj_t(const LmmArgs &a, hipStream_t st)
{
    const int64_t blocks = (int64_t)a.n_blk * a.g.M;
    hipLaunchKernelGGL((lmm_adjoint_kernel<NFC, D, T>), dim3((unsigned)blocks), dim3(kAdjBlock), 0, st, a);
    return hipGetLastError();
}

template <int D, typename T>
static hipError_t launch_adj_d(const LmmArgs &a, hipStream_t st)
{
    if (a.n_fwd <= 16) return launch_adj_t<16, D, T>(a, st);
    if (a.n_fwd <= 32) return launch_adj_t<32, D, T>(a, st);
    if (a.n_fwd <= 48) return launch_adj_t<48, D, T>(a, st);
    if (a.n_fwd <= 64) return launch_adj_t<64, D, T>(a, st);
    return launch_adj_t<80, D, T>(a, st);
}

// Adjoint launch for one precision (instantiated in rq_lmm_adj32.hip and
// rq_lmm_adj64.hip, so the two compile in parallel).
template <typename T>
static hipError_t launch_adj_prec(const LmmArgs &a, int n_factors, hipStream_t st)
{
    switch (n_factors) {
    case 1: return launch_adj_d<1, T>(a, st);
    case 2: return launch_adj_d<2, T>(a, st);
    case 3: return launch_adj_d<3, T>(a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lmm_adjoint_f32(const LmmArgs &a, int n_factors, hipStream_t st);
hipError_t launch_lmm_adjoint_f64(const LmmArgs &a, int n_factors, hipStream_t st);

}  // namespace rq
