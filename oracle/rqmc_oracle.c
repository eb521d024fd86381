/*
 * rqmc_oracle.c -- plain, slow FP64 CPU oracle for the RQMC pricing path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the GPU library: every piece
 * below is written out again from the paper's definitions (or, for the
 * generic pieces, from their own publications) so that the two
 * implementations can be checked against each other.
 *
 * What it computes (paper: Xu & Okten, "High Performance Financial
 * Simulation Using Randomized Quasi-Monte Carlo Methods"):
 *   - Random-start (optionally permuted) Halton points: the van der Corput
 *     radical inverse of eqs. (1)-(3), started at a random index per
 *     (replication, dimension) as in Algorithm 3, step 1.  Two independent
 *     generators: the direct definition, and the recursive digit/partial-sum
 *     update of Algorithm 2 carried out in exact integers.
 *   - The inverse normal CDF (Wichura's AS241, PPND16, FP64).
 *   - LIBOR market model paths under the spot measure (SDE "dL_n" and its
 *     Euler discretisation, taken in log form), caplet payoffs discounted
 *     by the spot numeraire (caplet section).
 *   - Caflisch MBS paths (MBS section): u_k, m_k, r_k, c_k, i_k, w_k.
 *   - The pseudo-random comparison (the paper's Philox baseline): the same
 *     paths driven by Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11)
 *     uniforms instead of Halton points.
 *   - Per-replication estimates theta_N^m, grand average RQ_{M,N}, sample
 *     standard deviation and standard error (Introduction).
 *
 * Everything is FP64 and scalar; OpenMP runs one replication per thread,
 * the paper's "parallel" paradigm (Introduction, Fig. 1(a)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ERANGE 2

#define ORC_START_ZERO 1
#define ORC_PERM_RANDOM 2
#define ORC_MC_PHILOX 8
#define ORC_LMM_EULER 16
#define ORC_PERM_PER_REP 32

/* ------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014).  The generator's state advances by the odd
 * constant gamma = 0x9e3779b97f4a7c15 and every output is mix64(state).
 * Output number k (0-based) of the stream seeded with `seed` is therefore
 * mix64(seed + (k+1)*gamma), which gives random access by counter. */
static uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix64(uint64_t seed, uint64_t k)
{
    return orc_mix64(seed + (k + 1ULL) * 0x9e3779b97f4a7c15ULL);
}

/* ------------------------------------------------------------------ */
/* Halton bases: the j-th prime (j = 0 -> 2), by trial division. */
int orc_nth_prime(int j)
{
    int count = -1;
    for (int c = 2;; ++c) {
        int is_p = 1;
        for (int q = 2; q * q <= c; ++q)
            if (c % q == 0) { is_p = 0; break; }
        if (is_p && ++count == j) return c;
    }
}

/* Number of base-p digits carried: D = max{D : p^D <= 2^53}; P = p^D.
 * The random start of Algorithm 3 is read as an index n uniform on [0, P):
 * omega truncated to D base-p digits is exactly a van der Corput term. */
int orc_digits(uint64_t p, uint64_t *P_out)
{
    const uint64_t lim = 1ULL << 53;
    uint64_t P = 1;
    int D = 0;
    while (P <= lim / p) { P *= p; ++D; }
    if (P_out) *P_out = P;
    return D;
}

/* Uniform integer in [0, range) from the counter stream, by rejection:
 * accept u < 2^64 - (2^64 mod range).  ctr0 is the counter of attempt 0;
 * attempt a uses ctr0 + a (a < 64). */
static int orc_uniform_below(uint64_t seed, uint64_t ctr0, uint64_t range, uint64_t *out)
{
    uint64_t rem = (0ULL - range) % range; /* == 2^64 mod range */
    for (uint64_t a = 0; a < 64; ++a) {
        uint64_t u = orc_splitmix64(seed, ctr0 + a);
        if (rem == 0 || u < 0ULL - rem) { *out = u % range; return ORC_OK; }
    }
    return ORC_ERANGE; /* probability < 2^-640; reported, never silent */
}

/* Random start of replication m_global in dimension j (Algorithm 3,
 * step 1): counter layout ((m_global*4096 + j)*64 + attempt). */
int orc_start(uint64_t seed, uint64_t m_global, int j, uint64_t P, int flags, uint64_t *n_out)
{
    if (flags & ORC_START_ZERO) { *n_out = 0; return ORC_OK; }
    return orc_uniform_below(seed, (m_global * 4096ULL + (uint64_t)j) * 64ULL, P, n_out);
}

/* Random digit permutation of base j (eq. (3), "picked at random"):
 * Fisher-Yates from the identity, step t = p-1 .. 1 swaps sigma[t] with
 * sigma[r], r uniform on [0, t], counter 2^60 + (j*65536 + t)*64 + attempt
 * (t < p <= 38873 < 65536).  One permutation per (seed, base), shared by all
 * replications. */
int orc_perm(uint64_t seed, int j, int p, int *sigma)
{
    for (int t = 0; t < p; ++t) sigma[t] = t;
    for (int t = p - 1; t >= 1; --t) {
        uint64_t r;
        uint64_t ctr = (1ULL << 60) + ((uint64_t)j * 65536ULL + (uint64_t)t) * 64ULL;
        if (orc_uniform_below(seed, ctr, (uint64_t)(t + 1), &r)) return ORC_ERANGE;
        int tmp = sigma[t]; sigma[t] = sigma[(int)r]; sigma[(int)r] = tmp;
    }
    return ORC_OK;
}

/* The other reading of "random permutations": replication m_global draws
 * its own permutation of every base -- the same Fisher-Yates, on the stream
 * whose seed is output 2^62 + m_global of the seed's stream. */
uint64_t orc_perm_rep_seed(uint64_t seed, uint64_t m_global)
{
    return orc_splitmix64(seed, (1ULL << 62) + m_global);
}

int orc_perm_rep(uint64_t seed, uint64_t m_global, int j, int p, int *sigma)
{
    return orc_perm(orc_perm_rep_seed(seed, m_global), j, p, sigma);
}

/* ------------------------------------------------------------------ */
/* Radical inverse by definition, eqs. (1)-(3):  idx = sum_t a_t p^t,
 * phi(idx) = sum_{t<=k} sigma(a_t) p^{-(t+1)} with k the top nonzero digit
 * (digits above k are absent from the sum).  Scaled by P = p^D this is the
 * exact integer R = sum_{t<=k} sigma(a_t) p^{D-1-t} < P <= 2^53. */
uint64_t orc_radinv_R(uint64_t p, int D, const int *sigma, uint64_t idx)
{
    int a[64];
    int top = -1;
    uint64_t v = idx;
    for (int t = 0; t < D; ++t) {
        a[t] = (int)(v % p);
        v /= p;
        if (a[t] != 0) top = t;
    }
    uint64_t R = 0;
    for (int t = 0; t <= top; ++t) {
        uint64_t w = 1;
        for (int e = 0; e < D - 1 - t; ++e) w *= p;
        uint64_t dig = sigma ? (uint64_t)sigma[a[t]] : (uint64_t)a[t];
        R += dig * w;
    }
    return R;
}

/* The point is the FP64 value of the exact rational R/P: one IEEE
 * division of two exactly representable integers (round to nearest). */
double orc_point_from_R(uint64_t R, uint64_t P)
{
    return (double)R / (double)P;
}

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11).  A counter (c0, c1, c2, c3) and a key (k0, k1)
 * of 64-bit words; one round replaces the counter by
 *   (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
 * where hi/lo are the halves of the 128-bit product, and then adds the
 * Weyl constants to the key; ten rounds.  Multipliers and Weyl constants
 * are those of the publication for the 4x64 member of the family. */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        const unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        const unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        const uint64_t n0 = (uint64_t)(p1 >> 64) ^ c1 ^ k0;
        const uint64_t n1 = (uint64_t)p1;
        const uint64_t n2 = (uint64_t)(p0 >> 64) ^ c3 ^ k1;
        const uint64_t n3 = (uint64_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Pseudo-random coordinate j of point i of replication m_global:
 * word (j mod 4) of Philox4x64-10 at counter (j / 4, i, 0, 0) under key
 * (seed, m_global), mapped to ((x >> 11) + 1/2) 2^-53, which lies in (0, 1)
 * and is exact in FP64. */
double orc_mc_point(uint64_t seed, uint64_t m_global, uint64_t i, int j)
{
    const uint64_t ctr[4] = {(uint64_t)j >> 2, i, 0, 0};
    const uint64_t key[2] = {seed, m_global};
    uint64_t w[4];
    orc_philox4x64(ctr, key, w);
    return ((double)(w[j & 3] >> 11) + 0.5) * 0x1p-53;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2 (recursive random-start permuted van der Corput) in exact
 * integers.  The paper keeps digits a_0..a_k of n and partial sums
 * S_j = sum_{i>=j} sigma(a_i)/p^{i+1}; here W_j = S_j * P is kept as an
 * exact integer so no rounding enters.  Going from n to n+1: find the
 * lowest digit m with a_m + 1 < p, raise it, zero the digits below it and
 * rebuild W_m..W_0 from W_{m+1}.  Indices wrap modulo P = p^D. */
typedef struct {
    uint64_t p;
    int D;
    const int *sigma;
    int a[64];
    uint64_t W[65];   /* W[D] = 0 */
    uint64_t pw[64];  /* pw[t] = p^{D-1-t} */
    int top;          /* highest nonzero digit, -1 when n = 0 */
} orc_alg2;

static uint64_t orc_sig(const orc_alg2 *g, int a) { return g->sigma ? (uint64_t)g->sigma[a] : (uint64_t)a; }

void orc_alg2_init(orc_alg2 *g, uint64_t p, int D, const int *sigma, uint64_t n)
{
    g->p = p; g->D = D; g->sigma = sigma;
    uint64_t w = 1;
    for (int t = D - 1; t >= 0; --t) { g->pw[t] = w; w *= p; }
    g->top = -1;
    uint64_t v = n;
    for (int t = 0; t < D; ++t) {
        g->a[t] = (int)(v % p); v /= p;
        if (g->a[t]) g->top = t;
    }
    g->W[D] = 0;
    for (int t = D - 1; t >= 0; --t)
        g->W[t] = (t > g->top) ? 0 : g->W[t + 1] + orc_sig(g, g->a[t]) * g->pw[t];
}

uint64_t orc_alg2_R(const orc_alg2 *g) { return g->W[0]; }

void orc_alg2_next(orc_alg2 *g)
{
    int m = 0;
    while (m < g->D && (uint64_t)g->a[m] + 1 >= g->p) ++m;
    if (m == g->D) { /* n + 1 == P wraps to index 0 */
        for (int t = 0; t < g->D; ++t) { g->a[t] = 0; g->W[t] = 0; }
        g->top = -1;
        return;
    }
    g->a[m] += 1;
    if (m > g->top) g->top = m;
    g->W[m] = g->W[m + 1] + orc_sig(g, g->a[m]) * g->pw[m];
    for (int i = m - 1; i >= 0; --i) {
        g->a[i] = 0;
        g->W[i] = g->W[i + 1] + orc_sig(g, 0) * g->pw[i];
    }
}

/* ------------------------------------------------------------------ */
/* Inverse standard normal CDF: Wichura, "Algorithm AS 241: The percentage
 * points of the normal distribution", Applied Statistics 37 (1988),
 * PPND16 (about 1e-16 relative).  The input is folded as
 * r = min(u, 1-u), clamped to >= 2^-64 so that the endpoint u = 0 (index
 * 0 at the start) maps to a finite value. */
double orc_ppnd16(double u)
{
    double q = u - 0.5;
    if (fabs(q) <= 0.425) {
        double r = 0.180625 - q * q;
        double num = (((((((2.5090809287301226727e3 * r + 3.3430575583588128105e4) * r
                       + 6.7265770927008700853e4) * r + 4.5921953931549871457e4) * r
                       + 1.3731693765509461125e4) * r + 1.9715909503065514427e3) * r
                       + 1.3314166789178437745e2) * r + 3.3871328727963666080e0);
        double den = (((((((5.2264952788528545610e3 * r + 2.8729085735721942674e4) * r
                       + 3.9307895800092710610e4) * r + 2.1213794301586595867e4) * r
                       + 5.3941960214247511077e3) * r + 6.8718700749205790830e2) * r
                       + 4.2313330701600911252e1) * r + 1.0);
        return q * num / den;
    }
    double r = q < 0 ? u : 1.0 - u;
    if (r < 0x1p-64) r = 0x1p-64;
    r = sqrt(-log(r));
    double z;
    if (r <= 5.0) {
        r -= 1.6;
        double num = (((((((7.74545014278341407640e-4 * r + 2.27238449892691845833e-2) * r
                       + 2.41780725177450611770e-1) * r + 1.27045825245236838258e0) * r
                       + 3.64784832476320460504e0) * r + 5.76949722146069140550e0) * r
                       + 4.63033784615654529590e0) * r + 1.42343711074968357734e0);
        double den = (((((((1.05075007164441684324e-9 * r + 5.47593808499534494600e-4) * r
                       + 1.51986665636164571966e-2) * r + 1.48103976427480074590e-1) * r
                       + 6.89767334985100004550e-1) * r + 1.67638483018380384940e0) * r
                       + 2.05319162663775882187e0) * r + 1.0);
        z = num / den;
    } else {
        r -= 5.0;
        double num = (((((((2.01033439929228813265e-7 * r + 2.71155556874348757815e-5) * r
                       + 1.24266094738807843860e-3) * r + 2.65321895265761230930e-2) * r
                       + 2.96560571828504891230e-1) * r + 1.78482653991729133580e0) * r
                       + 5.46378491116411436990e0) * r + 6.65790464350110377720e0);
        double den = (((((((2.04426310338993978564e-15 * r + 1.42151175831644588870e-7) * r
                       + 1.84631831751005468180e-5) * r + 7.86869131145613259100e-4) * r
                       + 1.48753612908506148525e-2) * r + 1.36929880922735805310e-1) * r
                       + 5.99832206555887937690e-1) * r + 1.0);
        z = num / den;
    }
    return q < 0 ? -z : z;
}

/* ------------------------------------------------------------------ */
/* LIBOR market model, spot measure (caplet section, SDE "dL_n").
 * Constant vols: forward n has vol vector a_n = sigma_n * b_n in R^d.
 * One period [T_k, T_{k+1}] (k = 0..n_fwd-1) is split in n_sub equal steps
 * of h = delta/n_sub (n_sub = 1 is the paper's grid t_i = T_i).  Inside
 * period k the drift sums over j = eta(t) .. n with eta = k+1, i.e. the
 * forwards still alive, using pre-step values.  The Euler step is taken on
 * log L (log-Euler):
 *   L_n <- L_n exp( (mu_n - |a_n|^2/2) h + sqrt(h) a_n . Z ),
 *   mu_n = sum_{j=k+1..n} delta L_j a_n.a_j / (1 + delta L_j).
 * After period k forward k+1 has fixed; the caplet on it pays
 * delta (L - K)^+ at T_{k+2}, discounted by the spot numeraire
 * prod_{j=0..k+1} (1 + delta L_j(T_j)).
 * Inputs:  L0[n_fwd+1], sigma[n_fwd+1] (sigma[0] unused), b[n_fwd*d],
 *          strike[n_fwd] (NaN = no caplet), z[n_fwd*n_sub*d] standard
 *          normals, time-major (period, sub-step, factor).
 * Outputs: pay[n_fwd + 1]: pay[n-1] = discounted caplet on L_n,
 *          pay[n_fwd] = book (sum of caplets).
 * euler != 0 selects the plain Euler update of the paper's eq. for
 * hat L_n(t_{i+1}) instead of the log form. */
void orc_lmm_path(int n_fwd, int d, double delta, const double *L0, const double *sigma,
                  const double *b, const double *strike, int n_sub, int euler,
                  const double *z, double *pay)
{
    double L[1024];
    double v[16];
    double h = delta / n_sub;
    double sqh = sqrt(h);
    for (int n = 1; n <= n_fwd; ++n) L[n] = L0[n];
    double num = 1.0 + delta * L0[0];
    double book = 0.0;
    for (int k = 0; k < n_fwd; ++k) {
        for (int sub = 0; sub < n_sub; ++sub) {
            const double *Z = z + ((size_t)k * n_sub + sub) * d;
            for (int f = 0; f < d; ++f) v[f] = 0.0;
            for (int n = k + 1; n <= n_fwd; ++n) {
                const double *bn = b + (size_t)(n - 1) * d;
                double g = delta * L[n] / (1.0 + delta * L[n]);
                double mu = 0.0, an2 = 0.0, az = 0.0;
                for (int f = 0; f < d; ++f) {
                    double anf = sigma[n] * bn[f];
                    v[f] += g * anf;
                }
                for (int f = 0; f < d; ++f) {
                    double anf = sigma[n] * bn[f];
                    mu += anf * v[f];
                    an2 += anf * anf;
                    az += anf * Z[f];
                }
                if (euler)
                    L[n] = L[n] + mu * L[n] * h + L[n] * sqh * az;
                else
                    L[n] = L[n] * exp((mu - 0.5 * an2) * h + sqh * az);
            }
        }
        int n = k + 1;
        double p = 0.0;
        if (!isnan(strike[n - 1])) {
            double ex = L[n] - strike[n - 1];
            if (ex < 0.0) ex = 0.0;
            p = delta * ex / (num * (1.0 + delta * L[n]));
        }
        pay[n - 1] = p;
        book += p;
        num *= 1.0 + delta * L[n];
    }
    pay[n_fwd] = book;
}

/* ------------------------------------------------------------------ */
/* Caflisch MBS model (MBS section).  Level monthly payment c on unit
 * principal, c = i0 / (1 - (1+i0)^{-K}); c_k = sum_{j=0}^{K-k} (1+i0)^{-j}
 * (remaining annuity / c); K0 = exp(-sigma^2/2).  For k = 1..K with
 * xi_k = sigma z_k:
 *   u_k = prod_{j<k} (1+i_j)^{-1},  i_k = K0 e^{xi_k} i_{k-1},
 *   w_k = K1 + K2 atan(K3 i_k + K4),  r_k = prod_{j=1}^{k-1} (1 - w_j),
 *   m_k = c r_k ((1 - w_k) + w_k c_k),  PV = sum_k u_k m_k.
 * orc_mbs_annuity fills ck[1..K] straight from the defining sum. */
void orc_mbs_annuity(int months, double i0, double *ck)
{
    ck[0] = 0.0;
    for (int k = 1; k <= months; ++k) {
        double a = 0.0;
        for (int j = 0; j <= months - k; ++j) a += pow(1.0 + i0, -(double)j);
        ck[k] = a;
    }
}

double orc_mbs_path(int months, double i0, double sig, double K1, double K2, double K3,
                    double K4, const double *ck, const double *z)
{
    double c = i0 / (1.0 - pow(1.0 + i0, -(double)months));
    double K0 = exp(-0.5 * sig * sig);
    double i = i0, u = 1.0, r = 1.0, pv = 0.0;
    for (int k = 1; k <= months; ++k) {
        u = u / (1.0 + i);
        i = K0 * exp(sig * z[k - 1]) * i;
        double w = K1 + K2 * atan(K3 * i + K4);
        pv += u * c * r * ((1.0 - w) + w * ck[k]);
        r = r * (1.0 - w);
    }
    return pv;
}

/* ------------------------------------------------------------------ */
/* Neumaier's compensated summation (improved Kahan). */
typedef struct { double s, c; } orc_acc;
static void orc_acc_add(orc_acc *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double orc_acc_val(const orc_acc *a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* Per-dimension generator state for one replication. */
typedef struct {
    uint64_t p, P;
    int D;
    int *sigma;       /* NULL = identity */
} orc_base;

static int orc_bases(int s, uint64_t seed, int flags, orc_base *bs)
{
    for (int j = 0; j < s; ++j) {
        bs[j].p = (uint64_t)orc_nth_prime(j);
        bs[j].D = orc_digits(bs[j].p, &bs[j].P);
        bs[j].sigma = NULL;
        if (flags & (ORC_PERM_RANDOM | ORC_PERM_PER_REP)) {
            bs[j].sigma = (int *)malloc(sizeof(int) * bs[j].p);
            if (!(flags & ORC_PERM_PER_REP) && orc_perm(seed, j, (int)bs[j].p, bs[j].sigma)) return ORC_ERANGE;
        }
    }
    return ORC_OK;
}

/* Per-replication permutations: a private copy of the bases for
 * replication m_global (freed by orc_bases_free). */
static int orc_bases_rep(int s, uint64_t seed, uint64_t m_global, const orc_base *shared, orc_base *bs)
{
    for (int j = 0; j < s; ++j) {
        bs[j] = shared[j];
        bs[j].sigma = (int *)malloc(sizeof(int) * bs[j].p);
        if (orc_perm_rep(seed, m_global, j, (int)bs[j].p, bs[j].sigma)) return ORC_ERANGE;
    }
    return ORC_OK;
}

static void orc_bases_free(int s, orc_base *bs)
{
    for (int j = 0; j < s; ++j) free(bs[j].sigma);
}

static int orc_check_N(int s, int64_t N, const orc_base *bs)
{
    for (int j = 0; j < s; ++j)
        if ((uint64_t)N > bs[j].P) return ORC_ERANGE;
    return ORC_OK;
}

/* Points x[M][N][s] (or exact integers R when out_R != NULL) of the
 * random-start Halton replications m_offset .. m_offset+M-1:
 * x_{i,j}^m = phi_{p_j}((n_j^m + i) mod P_j), i = 0..N-1.  gen = 0 uses
 * the direct definition, gen = 1 the Algorithm-2 recursion. */
int orc_sequence(int s, int64_t N, int M, uint64_t seed, int flags, int64_t m_offset, int gen,
                 double *out_x, uint64_t *out_R)
{
    if (s < 1 || N < 1 || M < 1 || s > 4096) return ORC_EINVAL;
    if (flags & ORC_MC_PHILOX) {
        if ((flags & (ORC_START_ZERO | ORC_PERM_RANDOM | ORC_PERM_PER_REP)) || out_R) return ORC_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
        for (int m = 0; m < M; ++m)
            for (int64_t i = 0; i < N; ++i)
                for (int j = 0; j < s; ++j)
                    out_x[((size_t)m * (size_t)N + (size_t)i) * (size_t)s + (size_t)j] =
                        orc_mc_point(seed, (uint64_t)(m_offset + m), (uint64_t)i, j);
        return ORC_OK;
    }
    orc_base *bs = (orc_base *)calloc((size_t)s, sizeof(orc_base));
    int st = orc_bases(s, seed, flags, bs);
    if (!st) st = orc_check_N(s, N, bs);
    if (st) { orc_bases_free(s, bs); free(bs); return st; }
    int err = 0;
    const int rep = (flags & ORC_PERM_PER_REP) != 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int m = 0; m < M; ++m) {
        orc_alg2 g;
        orc_base *bm = bs;
        if (rep) {
            bm = (orc_base *)calloc((size_t)s, sizeof(orc_base));
            if (orc_bases_rep(s, seed, (uint64_t)(m_offset + m), bs, bm)) err |= 1;
        }
        for (int j = 0; j < s; ++j) {
            uint64_t n;
            if (orc_start(seed, (uint64_t)(m_offset + m), j, bm[j].P, flags, &n)) { err |= 1; continue; }
            if (gen) orc_alg2_init(&g, bm[j].p, bm[j].D, bm[j].sigma, n);
            for (int64_t i = 0; i < N; ++i) {
                uint64_t R;
                if (gen) { R = orc_alg2_R(&g); orc_alg2_next(&g); }
                else R = orc_radinv_R(bm[j].p, bm[j].D, bm[j].sigma, (n + (uint64_t)i) % bm[j].P);
                size_t o = ((size_t)m * (size_t)N + (size_t)i) * (size_t)s + (size_t)j;
                if (out_R) out_R[o] = R;
                if (out_x) out_x[o] = orc_point_from_R(R, bm[j].P);
            }
        }
        if (rep) { orc_bases_free(s, bm); free(bm); }
    }
    orc_bases_free(s, bs);
    free(bs);
    return err ? ORC_ERANGE : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Shared driver for the two pricers: replication m walks i = 0..N-1 with
 * one Algorithm-2 generator per dimension (the paper's fastest CPU Halton
 * method), maps every coordinate through PPND16 and hands the normals of
 * one path to `path`.  theta[m][o] = (1/N) sum_i f_o(q_i^m) with
 * compensated summation.  per_path[m][i][o] is written when non-NULL. */
typedef void (*orc_path_fn)(const void *ctx, const double *z, double *f);

static int orc_price(int s, int n_out, orc_path_fn path, const void *ctx, int64_t N, int M,
                     uint64_t seed, int64_t m_offset, int flags, double *theta, double *per_path)
{
    if (s < 1 || N < 1 || M < 1 || s > 4096 || n_out < 1) return ORC_EINVAL;
    const int mc = (flags & ORC_MC_PHILOX) != 0;
    if (mc && (flags & (ORC_START_ZERO | ORC_PERM_RANDOM | ORC_PERM_PER_REP))) return ORC_EINVAL;
    orc_base *bs = (orc_base *)calloc((size_t)s, sizeof(orc_base));
    int st = mc ? ORC_OK : orc_bases(s, seed, flags, bs);
    if (!st && !mc) st = orc_check_N(s, N, bs);
    if (st) { orc_bases_free(s, bs); free(bs); return st; }
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int m = 0; m < M; ++m) {
        orc_alg2 *g = (orc_alg2 *)malloc(sizeof(orc_alg2) * (size_t)s);
        double *z = (double *)malloc(sizeof(double) * (size_t)s);
        double *f = (double *)malloc(sizeof(double) * (size_t)n_out);
        orc_acc *acc = (orc_acc *)calloc((size_t)n_out, sizeof(orc_acc));
        orc_base *bm = bs;
        if (!mc && (flags & ORC_PERM_PER_REP)) {
            bm = (orc_base *)calloc((size_t)s, sizeof(orc_base));
            if (orc_bases_rep(s, seed, (uint64_t)(m_offset + m), bs, bm)) err |= 1;
        }
        for (int j = 0; j < s && !mc; ++j) {
            uint64_t n;
            if (orc_start(seed, (uint64_t)(m_offset + m), j, bm[j].P, flags, &n)) err |= 1;
            orc_alg2_init(&g[j], bm[j].p, bm[j].D, bm[j].sigma, n);
        }
        for (int64_t i = 0; i < N; ++i) {
            for (int j = 0; j < s; ++j) {
                double x;
                if (mc) {
                    x = orc_mc_point(seed, (uint64_t)(m_offset + m), (uint64_t)i, j);
                } else {
                    x = orc_point_from_R(orc_alg2_R(&g[j]), bm[j].P);
                    orc_alg2_next(&g[j]);
                }
                z[j] = orc_ppnd16(x);
            }
            path(ctx, z, f);
            for (int o = 0; o < n_out; ++o) orc_acc_add(&acc[o], f[o]);
            if (per_path)
                memcpy(per_path + ((size_t)m * (size_t)N + (size_t)i) * (size_t)n_out, f,
                       sizeof(double) * (size_t)n_out);
        }
        for (int o = 0; o < n_out; ++o) theta[(size_t)m * n_out + o] = orc_acc_val(&acc[o]) / (double)N;
        free(g); free(z); free(f); free(acc);
        if (bm != bs) { orc_bases_free(s, bm); free(bm); }
    }
    orc_bases_free(s, bs);
    free(bs);
    return err ? ORC_ERANGE : ORC_OK;
}

typedef struct {
    int n_fwd, d;
    double delta;
    const double *L0, *sigma, *b, *strike;
    int euler;
} orc_lmm_ctx;

static void orc_lmm_fn(const void *c, const double *z, double *f)
{
    const orc_lmm_ctx *m = (const orc_lmm_ctx *)c;
    orc_lmm_path(m->n_fwd, m->d, m->delta, m->L0, m->sigma, m->b, m->strike, 1, m->euler, z, f);
}

int orc_price_caplets(int n_fwd, int d, double delta, const double *L0, const double *sigma,
                      const double *b, const double *strike, int64_t N, int M, uint64_t seed,
                      int64_t m_offset, int flags, double *theta, double *per_path)
{
    if (n_fwd < 1 || n_fwd > 1000 || d < 1 || d > 16 || !(delta > 0)) return ORC_EINVAL;
    orc_lmm_ctx c = {n_fwd, d, delta, L0, sigma, b, strike, (flags & ORC_LMM_EULER) ? 1 : 0};
    return orc_price(n_fwd * d, n_fwd + 1, orc_lmm_fn, &c, N, M, seed, m_offset, flags & ~ORC_LMM_EULER, theta,
                     per_path);
}

typedef struct {
    int months;
    double i0, sig, K1, K2, K3, K4;
    const double *ck;
} orc_mbs_ctx;

static void orc_mbs_fn(const void *c, const double *z, double *f)
{
    const orc_mbs_ctx *m = (const orc_mbs_ctx *)c;
    f[0] = orc_mbs_path(m->months, m->i0, m->sig, m->K1, m->K2, m->K3, m->K4, m->ck, z);
}

int orc_price_mbs(int months, double i0, double sig, double K1, double K2, double K3, double K4,
                  int64_t N, int M, uint64_t seed, int64_t m_offset, int flags, double *theta,
                  double *per_path)
{
    if (months < 1 || months > 4096) return ORC_EINVAL;
    double *ck = (double *)malloc(sizeof(double) * (size_t)(months + 1));
    orc_mbs_annuity(months, i0, ck);
    orc_mbs_ctx c = {months, i0, sig, K1, K2, K3, K4, ck};
    int st = orc_price(months, 1, orc_mbs_fn, &c, N, M, seed, m_offset, flags, theta, per_path);
    free(ck);
    return st;
}

/* Grand average, sample standard deviation (denominator M-1) and standard
 * error of the M replication estimates of each output (Introduction:
 * RQ_{M,N} and the spread of theta_N^1..theta_N^M). */
void orc_finalize(const double *theta, int M, int n_out, double *mean, double *sd, double *se)
{
    for (int o = 0; o < n_out; ++o) {
        orc_acc a = {0, 0};
        for (int m = 0; m < M; ++m) orc_acc_add(&a, theta[(size_t)m * n_out + o]);
        double mu = orc_acc_val(&a) / M;
        orc_acc q = {0, 0};
        for (int m = 0; m < M; ++m) {
            double dlt = theta[(size_t)m * n_out + o] - mu;
            orc_acc_add(&q, dlt * dlt);
        }
        mean[o] = mu;
        sd[o] = M > 1 ? sqrt(orc_acc_val(&q) / (M - 1)) : NAN;
        se[o] = M > 1 ? sd[o] / sqrt((double)M) : NAN;
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following calls (timing on one core or on all). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Batched helpers for the test-suite (same arithmetic as above). */
void orc_ppnd16_vec(int64_t n, const double *u, double *z)
{
    for (int64_t i = 0; i < n; ++i) z[i] = orc_ppnd16(u[i]);
}

void orc_lmm_paths(int64_t n_paths, int n_fwd, int d, double delta, const double *L0,
                   const double *sigma, const double *b, const double *strike, int n_sub,
                   int euler, const double *z, double *pay)
{
    size_t nz = (size_t)n_fwd * (size_t)n_sub * (size_t)d;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_paths; ++i)
        orc_lmm_path(n_fwd, d, delta, L0, sigma, b, strike, n_sub, euler, z + (size_t)i * nz,
                     pay + (size_t)i * (size_t)(n_fwd + 1));
}

void orc_mbs_paths(int64_t n_paths, int months, double i0, double sig, double K1, double K2,
                   double K3, double K4, const double *z, double *pv)
{
    double *ck = (double *)malloc(sizeof(double) * (size_t)(months + 1));
    orc_mbs_annuity(months, i0, ck);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_paths; ++i)
        pv[i] = orc_mbs_path(months, i0, sig, K1, K2, K3, K4, ck, z + (size_t)i * (size_t)months);
    free(ck);
}

/* Algorithm-2 run of `count` terms from index n (test hook). */
void orc_alg2_run(uint64_t p, const int *sigma, uint64_t n, int64_t count, uint64_t *out_R)
{
    orc_alg2 g;
    int D = orc_digits(p, NULL);
    orc_alg2_init(&g, p, D, sigma, n);
    for (int64_t i = 0; i < count; ++i) { out_R[i] = orc_alg2_R(&g); orc_alg2_next(&g); }
}
