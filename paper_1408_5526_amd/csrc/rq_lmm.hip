// rq_lmm.hip -- LIBOR market model caplet pricing, one path per lane.
//
// Model (caplet section): forwards L_1..L_n, spot measure, constant vol
// vectors a_n.  Step k (from T_k to T_{k+1}, k = 0..n-1) updates the alive
// forwards n = k+1..n_fwd in ascending order with the log-Euler form of the
// discretised SDE, drift from pre-step values:
//   g_n = delta L_n / (1 + delta L_n),  v += g_n a_n,  mu_n = a_n . v,
//   L_n <- L_n exp(mu_n delta - delta |a_n|^2 / 2 + sqrt(delta) a_n . z_k).
// After step k the caplet on L_{k+1} fixes and pays
//   delta (L_{k+1} - K)^+ / (num * (1 + delta L_{k+1})),
// num being the spot numeraire prod_{j<=k} (1 + delta L_j(T_j)) (FP64).
//
// GPU mapping: a lane owns one path; the forward vector lives in registers.
// The inner loop over forwards is unrolled to a compile-time capacity NFC so
// that every L[n] is a fixed register; forwards that are dead (n <= k) or
// beyond the model (n > n_fwd) are skipped by wave-uniform branches.  The
// per-forward constants are wave-uniform and come through scalar loads.
// Points are produced in registers from the replication's start table
// (no point set is materialised).  Each step's caplet is summed over the
// wave with a butterfly (fixed order), the four waves of a block are added
// in a fixed order, and the block writes one partial per output: the
// whole reduction is deterministic.
#include "rq_device.h"

namespace rq {

template <typename T> struct FwdRow;
template <> struct FwdRow<double> { using type = double; };
template <> struct FwdRow<float> { using type = float; };

template <int NFC, int D, typename T, bool PERM>
__global__ __launch_bounds__(kBlock) void lmm_kernel(LmmArgs a, const float *__restrict__ fwd32)
{
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
    const double *__restrict__ fwd = a.fwd;
    const int nf = a.n_fwd;

    __shared__ double red[kBlock / kWave][NFC + 1];

    // row of forward n: [a_0, a_1, a_2, c_n, K_n, L_n(0), has_caplet, -]
    auto rowv = [&](int n, int c) -> T {
        if constexpr (sizeof(T) == 8) return fwd[n * kFwdRow + c];
        else return fwd32[n * kFwdRow + c];
    };

    T L[NFC];
#pragma unroll
    for (int n = 0; n < NFC; ++n) L[n] = n < nf ? rowv(n, 5) : T(0);

    const T delta = (T)a.delta;
    const T sqd = (T)a.sqrt_delta;
    double num = a.num0;
    double book = 0.0;
    double *pp = (a.per_path && active) ? a.per_path + ((size_t)m * (size_t)a.g.N + (size_t)i) * a.n_out
                                        : nullptr;

#pragma unroll 1
    for (int k = 0; k < nf; ++k) {
        T z[D];
#pragma unroll
        for (int f = 0; f < D; ++f) {
            const int j = k * D + f;
            const PointCtx c = load_base(a.g.base, j);
            const double x = radinv_x<PERM>(c, st + j, t, a.g.perm);
            z[f] = inv_normal(x, T(0));
        }
        T v[D];
#pragma unroll
        for (int f = 0; f < D; ++f) v[f] = T(0);
        T Lfix = T(0);
#pragma unroll
        for (int n = 0; n < NFC; ++n) {
            if (n >= k && n < nf) {
                T an[D];
#pragma unroll
                for (int f = 0; f < D; ++f) an[f] = rowv(n, f);
                const T cn = rowv(n, 3);
                const T Ln = L[n];
                const T dl = delta * Ln;
                const T g = fdiv(dl, T(1) + dl);
                T mu = T(0), az = T(0);
#pragma unroll
                for (int f = 0; f < D; ++f) v[f] = __builtin_fma(g, an[f], v[f]);
#pragma unroll
                for (int f = 0; f < D; ++f) {
                    mu = __builtin_fma(an[f], v[f], mu);
                    az = __builtin_fma(an[f], z[f], az);
                }
                const T arg = __builtin_fma(mu, delta, __builtin_fma(sqd, az, cn));
                const T Lnew = Ln * fexp(arg);
                L[n] = Lnew;
                if (n == k) Lfix = Lnew;
            }
        }
        // caplet on forward k+1 fixes now (FP64 payoff and numeraire)
        const double *row = fwd + k * kFwdRow;
        const double Lf = (double)Lfix;
        const double onep = 1.0 + a.delta * Lf;
        double pay = 0.0;
        if (row[6] != 0.0) {
            const double ex = Lf - row[4];
            pay = ex > 0.0 ? a.delta * ex / (num * onep) : 0.0;
        }
        num *= onep;
        pay = active ? pay : 0.0;
        book += pay;
        if (pp) pp[k] = pay;
        const double w = wave_sum(pay);
        if (lane == 0) red[wave][k] = w;
    }
    if (pp) pp[nf] = book;
    const double wb = wave_sum(book);
    if (lane == 0) red[wave][nf] = wb;
    __syncthreads();
    double *out = a.partial + ((size_t)m * a.n_blk + blk) * a.n_out;
    for (int o = tid; o < a.n_out; o += kBlock) {
        double s = red[0][o];
        s += red[1][o];
        s += red[2][o];
        s += red[3][o];
        out[o] = s;
    }
}

template <int NFC, int D, typename T>
static hipError_t launch_t(const LmmArgs &a, const float *fwd32, hipStream_t st)
{
    const int64_t blocks = (int64_t)a.n_blk * a.g.M;
    if (a.g.perm_on)
        hipLaunchKernelGGL((lmm_kernel<NFC, D, T, true>), dim3((unsigned)blocks), dim3(kBlock), 0, st, a, fwd32);
    else
        hipLaunchKernelGGL((lmm_kernel<NFC, D, T, false>), dim3((unsigned)blocks), dim3(kBlock), 0, st, a, fwd32);
    return hipGetLastError();
}

template <int D, typename T>
static hipError_t launch_d(const LmmArgs &a, const float *fwd32, hipStream_t st)
{
    if (a.n_fwd <= 16) return launch_t<16, D, T>(a, fwd32, st);
    if (a.n_fwd <= 32) return launch_t<32, D, T>(a, fwd32, st);
    if (a.n_fwd <= 48) return launch_t<48, D, T>(a, fwd32, st);
    if (a.n_fwd <= 64) return launch_t<64, D, T>(a, fwd32, st);
    return launch_t<80, D, T>(a, fwd32, st);
}

hipError_t launch_lmm(const LmmArgs &a, int n_factors, int fp32, hipStream_t st)
{
    // the FP32 table follows the FP64 one in the workspace
    const float *fwd32 = reinterpret_cast<const float *>(a.fwd + (size_t)a.n_fwd * kFwdRow);
    switch (n_factors * 2 + (fp32 ? 1 : 0)) {
    case 2: return launch_d<1, double>(a, fwd32, st);
    case 3: return launch_d<1, float>(a, fwd32, st);
    case 4: return launch_d<2, double>(a, fwd32, st);
    case 5: return launch_d<2, float>(a, fwd32, st);
    case 6: return launch_d<3, double>(a, fwd32, st);
    case 7: return launch_d<3, float>(a, fwd32, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace rq
