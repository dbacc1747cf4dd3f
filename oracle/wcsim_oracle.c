/*
 * wcsim_oracle.c -- plain FP64 CPU oracle of the LArTPC signal-simulation hot
 * path (arXiv:2304.01841, Sec. 2: Rasterization, Scatter-Add, Convolution).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the HIP path is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load it.  It shares no code,
 * header, table or constant generator with the GPU library.
 *
 * Everything is double precision and written in the order the definitions
 * state it.  Build with -ffp-contract=off so that no multiply-add is fused:
 * the patch-window bounds are integers decided by floating point and must be
 * reproducible operation by operation.
 *
 * Paper coverage (Sec. 2 lists the three steps; the details below are the
 * readings recorded in the design notes, because the paper defers them to the
 * earlier Kokkos study):
 *   - drift + diffusion                        (Sec. 2, step 1, rasterization)
 *   - patch window, erf-difference weights     (Sec. 2, step 1)
 *   - statistical fluctuation from a counter-
 *     based Philox4x32-10 stream               (Sec. 4.1: random123 / Salmon et al. 2011)
 *   - scatter-add of patches into the grid     (Sec. 2, step 2)
 *   - linear 2-D convolution with a response   (Sec. 2, step 3), direct sum
 *     (the FFT route of the oracle lives in oracle.py and calls a library FFT)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11 (the random123 generator the paper uses on CPU,   */
/* Sec. 4.1).  Each round multiplies counter words 0 and 2 by the two round   */
/* multipliers, swaps the halves of the 64-bit products into place, and mixes */
/* the high halves with the other two counter words and the round key.  The   */
/* key is advanced by the two Weyl constants between rounds.                 */
/* ------------------------------------------------------------------------ */
#define PHILOX_MUL_A 0xD2511F53u /* multiplier applied to counter word 0 */
#define PHILOX_MUL_B 0xCD9E8D57u /* multiplier applied to counter word 2 */
#define PHILOX_WEYL_A 0x9E3779B9u /* key word 0 increment (golden ratio)  */
#define PHILOX_WEYL_B 0xBB67AE85u /* key word 1 increment (sqrt(3) - 1)   */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_WEYL_A;
            k1 += PHILOX_WEYL_B;
        }
        uint64_t prod_a = (uint64_t)PHILOX_MUL_A * (uint64_t)x0;
        uint64_t prod_b = (uint64_t)PHILOX_MUL_B * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(prod_b >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)prod_b;
        uint32_t y2 = (uint32_t)(prod_a >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)prod_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void oracle_philox_batch(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i)
        oracle_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

/* ------------------------------------------------------------------------ */
/* Problem description, passed as flat arrays so that ctypes needs no        */
/* structure layout.                                                          */
/*   phys[6]  = { drift speed v (mm/us) on the response plane, D_L (mm^2/us), */
/*                D_T (mm^2/us), nsigma, electron lifetime tau (us; 0: no     */
/*                absorption), drift acceleration a (mm/us^2; 0: constant     */
/*                speed) }                                                    */
/*   geom[7]  = { wire pitch (mm), tick (us), t0 (us), plane_x (mm),          */
/*                dir_y, dir_z (unit pitch direction), pitch_origin (mm) }    */
/*   dims[4]  = { plane_id, nwires, nimpact, nticks }                         */
/* Depos are rows of five doubles { x, y, z, t, q }.                          */
/* ------------------------------------------------------------------------ */
enum { ORACLE_OK = 0, ORACLE_INVALID = 1, ORACLE_EMPTY = 2 };

typedef struct {
    double T;                     /* drift time to the response plane (us)  */
    double mu_p, s_p, mu_t, s_t;  /* bin coordinates and widths (bin units)  */
    int64_t lo_p, lo_t;           /* first bin of the window, per axis       */
    int64_t n_p, n_t;             /* window lengths                           */
} oracle_window;

/* Drift, diffusion and window of one depo.  Returns ORACLE_INVALID for a
 * malformed depo (non-finite field, negative charge, behind the response
 * plane, or unable to reach it) and ORACLE_EMPTY for a depo whose window
 * misses the grid. */
static int depo_window(const double *d, const double *phys, const double *geom,
                       const int32_t *dims, oracle_window *w)
{
    const double x = d[0], y = d[1], z = d[2], t = d[3], q = d[4];
    const double v = phys[0], DL = phys[1], DT = phys[2], nsig = phys[3], a = phys[5];
    const double pitch = geom[0], tick = geom[1], t0 = geom[2], plane_x = geom[3];
    const double dir_y = geom[4], dir_z = geom[5], pitch_origin = geom[6];
    const int64_t nimpact = dims[2];
    const int64_t Np = (int64_t)dims[1] * nimpact, Nt = dims[3];

    if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !isfinite(t) || !isfinite(q))
        return ORACLE_INVALID;
    if (q < 0.0 || x < plane_x)
        return ORACLE_INVALID;

    /* Drift from the deposition point to the response plane.  The drift
     * speed changes linearly with drift time at the rate a and equals v on
     * the response plane (an extension beyond the paper, whose drift speed
     * is constant): over the remaining distance l to the plane the speed is
     * sqrt(v^2 - 2 a l), so a depo at distance L starts at
     * v_s = sqrt(v^2 - 2 a L) and arrives after T = 2 L / (v + v_s), the
     * distance over the mean of the start and end speeds.  A depo with
     * v^2 - 2 a L < 0 never reaches the plane and is invalid.  With a = 0,
     * v_s = v and T = L / v exactly.  The Gaussian widths grow as
     * sqrt(2 D T), the longitudinal one converted to time by the speed on
     * the plane. */
    double L = x - plane_x;
    double disc = v * v - 2.0 * a * L;
    if (disc < 0.0)
        return ORACLE_INVALID;
    double v_s = sqrt(disc);
    double T = (2.0 * L) / (v + v_s);
    double t_arr = t + T;
    w->T = T;
    double sigma_p = sqrt(2.0 * DT * T);
    double sigma_t = sqrt(2.0 * DL * T) / v;

    /* Continuous bin coordinates: pitch bin i covers [i, i+1), tick j covers
     * [j, j+1). */
    double dp = pitch / (double)nimpact;
    double proj = y * dir_y + z * dir_z;
    w->mu_p = (proj - pitch_origin) / dp;
    w->s_p = sigma_p / dp;
    w->mu_t = (t_arr - t0) / tick;
    w->s_t = sigma_t / tick;

    /* Inclusive window floor(mu - n s) .. floor(mu + n s) per axis. */
    double lo_p = floor(w->mu_p - nsig * w->s_p);
    double hi_p = floor(w->mu_p + nsig * w->s_p);
    double lo_t = floor(w->mu_t - nsig * w->s_t);
    double hi_t = floor(w->mu_t + nsig * w->s_t);

    if (hi_p < 0.0 || lo_p >= (double)Np || hi_t < 0.0 || lo_t >= (double)Nt)
        return ORACLE_EMPTY;
    w->lo_p = (int64_t)lo_p;
    w->lo_t = (int64_t)lo_t;
    w->n_p = (int64_t)hi_p - w->lo_p + 1;
    w->n_t = (int64_t)hi_t - w->lo_t + 1;
    return ORACLE_OK;
}

/* Normalised bin weights along one axis: the Gaussian integrated over each
 * bin of the window (difference of erf at the bin edges), divided by the sum
 * over the window.  A zero width puts all weight in the single bin. */
static void axis_weights(int64_t lo, int64_t n, double mu, double s, double *W)
{
    if (s == 0.0) {
        for (int64_t i = 0; i < n; ++i)
            W[i] = 0.0;
        W[0] = 1.0;
        return;
    }
    double sum = 0.0;
    double e_lo = erf(((double)lo - mu) / (M_SQRT2 * s));
    for (int64_t i = 0; i < n; ++i) {
        double e_hi = erf(((double)(lo + i + 1) - mu) / (M_SQRT2 * s));
        W[i] = 0.5 * (e_hi - e_lo);
        sum += W[i];
        e_lo = e_hi;
    }
    for (int64_t i = 0; i < n; ++i)
        W[i] = W[i] / sum;
}

static int64_t floor_div4(int64_t J)
{
    return (J >= 0) ? J / 4 : -((-J + 3) / 4);
}

/* Standard normal deviate for absolute bin (I, J) of depo d in event e.
 * One Philox call serves four consecutive ticks 4k..4k+3: ticks with
 * J mod 4 in {0,1} use output words (0,1), ticks with J mod 4 in {2,3} use
 * words (2,3); each word pair feeds one Box-Muller transform whose cosine
 * branch goes to the even tick and sine branch to the odd tick.  A word r is
 * mapped to the uniform ((r >> 9) + 1/2) 2^-23, which lies in (0, 1) and is
 * exact in binary32 and binary64 alike. */
double oracle_normal(int64_t I, int64_t J, int64_t d, uint64_t event_id, uint64_t seed,
                     int32_t plane_id)
{
    int64_t quad = floor_div4(J);
    int64_t m = J - 4 * quad;
    uint32_t ctr[4] = {(uint32_t)quad, (uint32_t)I, (uint32_t)d, (uint32_t)event_id};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ (uint32_t)plane_id};
    uint32_t r[4];
    oracle_philox4x32_10(ctr, key, r);
    uint32_t a = (m < 2) ? r[0] : r[2];
    uint32_t b = (m < 2) ? r[1] : r[3];
    double ua = ((double)(a >> 9) + 0.5) * 0x1p-23;
    double ub = ((double)(b >> 9) + 0.5) * 0x1p-23;
    double rho = sqrt(-2.0 * log(ua));
    double theta = 2.0 * M_PI * ub;
    return (m % 2 == 0) ? rho * cos(theta) : rho * sin(theta);
}

/* Electrons of a depo that survive the drift (an extension beyond the paper,
 * which starts from the drifted charge): with electron lifetime tau > 0 each
 * electron survives the drift time T with probability p = exp(-T / tau).
 * Without fluctuation the depo keeps its mean, q p; with fluctuation the
 * count is the normal approximation of Binomial(q, p), clamped at zero.
 * Absorption happens during the drift, before any readout plane is reached,
 * so the draw belongs to the depo alone: its deviate comes from
 * Philox4x32-10 under the lifetime key (seed low word XOR 0x6c696665, seed
 * high word) -- no plane enters it, so every plane of an event sees the same
 * surviving charge -- at counter (0, 0, depo index in the event, event id low
 * word), through the cosine branch of the Box-Muller transform of output
 * words 0 and 1. */
#define LIFETIME_KEY_XOR 0x6c696665u

double oracle_surviving_charge(double q, double T, double tau, int32_t fluctuate, int64_t d,
                               uint64_t event_id, uint64_t seed)
{
    if (!(tau > 0.0))
        return q;
    double p = exp(-T / tau);
    if (!fluctuate)
        return q * p;
    uint32_t ctr[4] = {0u, 0u, (uint32_t)d, (uint32_t)event_id};
    uint32_t key[2] = {(uint32_t)seed ^ LIFETIME_KEY_XOR, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    oracle_philox4x32_10(ctr, key, r);
    double ua = ((double)(r[0] >> 9) + 0.5) * 0x1p-23;
    double ub = ((double)(r[1] >> 9) + 0.5) * 0x1p-23;
    double z = sqrt(-2.0 * log(ua)) * cos(2.0 * M_PI * ub);
    double F = q * p + z * sqrt(q * p * (1.0 - p));
    return (F < 0.0) ? 0.0 : F;
}

/* Window of one depo, exposed for the tests.  out_d[5] = {mu_p, s_p, mu_t,
 * s_t, T}, out_i[4] = {lo_p, lo_t, n_p, n_t}.  Returns the status code. */
int oracle_depo_window(const double *depo, const double *phys, const double *geom,
                       const int32_t *dims, double *out_d, int64_t *out_i)
{
    oracle_window w;
    memset(&w, 0, sizeof w);
    int st = depo_window(depo, phys, geom, dims, &w);
    out_d[0] = w.mu_p; out_d[1] = w.s_p; out_d[2] = w.mu_t; out_d[3] = w.s_t; out_d[4] = w.T;
    out_i[0] = w.lo_p; out_i[1] = w.lo_t; out_i[2] = w.n_p; out_i[3] = w.n_t;
    return st;
}

/* Weights of one axis, exposed for the tests. */
void oracle_axis_weights(int64_t lo, int64_t n, double mu, double s, double *W)
{
    axis_weights(lo, n, mu, s, W);
}

/* Rasterization (Sec. 2 step 1): one patch per depo.
 *   meta[5 d + 0..4] = { lo_p, lo_t, n_p, n_t, offset } with offset the
 *   exclusive prefix sum of n_p n_t (invalid or empty depos get n_p = n_t = 0).
 *   values[offset + i n_t + j] = charge in absolute bin (lo_p + i, lo_t + j).
 *   status[d] = 0 ok, 1 invalid, 2 empty.
 * q is the charge that survives the drift (oracle_surviving_charge; the
 * depo's own charge when the lifetime is 0).
 * Without fluctuation a patch is q W_p[i] W_t[j].  With fluctuation each bin
 * takes the normal approximation of a binomial draw of the q electrons with
 * probability p = W_p W_t, clamped at zero, and the patch is rescaled so that
 * its total (over the whole window, in the grid or not) equals q again.
 * The normal deviates are keyed by each depo's index in its event (reading
 * A7): d itself, or ids[d] when ids is given (a subset of an event's depos).
 * Returns the number of values, or -(needed) when cap is too small. */
int64_t oracle_rasterize(const double *depos, int64_t n, const double *phys, int32_t fluctuate,
                         uint64_t seed, const double *geom, const int32_t *dims, uint64_t event_id,
                         const int64_t *ids, int64_t *meta, double *values, int64_t cap,
                         int32_t *status)
{
    int64_t total = 0;
    for (int64_t d = 0; d < n; ++d) {
        oracle_window w;
        int st = depo_window(depos + 5 * d, phys, geom, dims, &w);
        if (status)
            status[d] = st;
        int64_t cnt = (st == ORACLE_OK) ? w.n_p * w.n_t : 0;
        meta[5 * d + 0] = (st == ORACLE_OK) ? w.lo_p : 0;
        meta[5 * d + 1] = (st == ORACLE_OK) ? w.lo_t : 0;
        meta[5 * d + 2] = (st == ORACLE_OK) ? w.n_p : 0;
        meta[5 * d + 3] = (st == ORACLE_OK) ? w.n_t : 0;
        meta[5 * d + 4] = total;
        total += cnt;
    }
    if (total > cap)
        return -total;

    const int32_t plane_id = dims[0];
    for (int64_t d = 0; d < n; ++d) {
        int64_t n_p = meta[5 * d + 2], n_t = meta[5 * d + 3];
        if (n_p == 0)
            continue;
        oracle_window w;
        depo_window(depos + 5 * d, phys, geom, dims, &w);
        const double q = oracle_surviving_charge(depos[5 * d + 4], w.T, phys[4], fluctuate,
                                                 ids ? ids[d] : d, event_id, seed);
        double *Wp = (double *)malloc(sizeof(double) * (size_t)n_p);
        double *Wt = (double *)malloc(sizeof(double) * (size_t)n_t);
        axis_weights(w.lo_p, n_p, w.mu_p, w.s_p, Wp);
        axis_weights(w.lo_t, n_t, w.mu_t, w.s_t, Wt);
        double *P = values + meta[5 * d + 4];
        if (!fluctuate) {
            for (int64_t i = 0; i < n_p; ++i)
                for (int64_t j = 0; j < n_t; ++j)
                    P[i * n_t + j] = q * Wp[i] * Wt[j];
        } else {
            double S = 0.0;
            for (int64_t i = 0; i < n_p; ++i) {
                for (int64_t j = 0; j < n_t; ++j) {
                    double p = Wp[i] * Wt[j];
                    double z = oracle_normal(w.lo_p + i, w.lo_t + j, ids ? ids[d] : d, event_id,
                                             seed, plane_id);
                    double F = q * p + z * sqrt(q * p * (1.0 - p));
                    if (F < 0.0)
                        F = 0.0;
                    P[i * n_t + j] = F;
                    S += F;
                }
            }
            for (int64_t i = 0; i < n_p; ++i)
                for (int64_t j = 0; j < n_t; ++j)
                    P[i * n_t + j] = (S > 0.0) ? P[i * n_t + j] * q / S : q * Wp[i] * Wt[j];
        }
        free(Wp);
        free(Wt);
    }
    return total;
}

/* Scatter-Add (Sec. 2 step 2): sum every patch into the [Np][Nt] grid;
 * bins outside the grid are dropped. */
void oracle_scatter(const int64_t *meta, const double *values, int64_t n, int64_t Np, int64_t Nt,
                    double *G)
{
    for (int64_t d = 0; d < n; ++d) {
        int64_t lo_p = meta[5 * d + 0], lo_t = meta[5 * d + 1];
        int64_t n_p = meta[5 * d + 2], n_t = meta[5 * d + 3];
        const double *P = values + meta[5 * d + 4];
        for (int64_t i = 0; i < n_p; ++i) {
            int64_t I = lo_p + i;
            if (I < 0 || I >= Np)
                continue;
            for (int64_t j = 0; j < n_t; ++j) {
                int64_t J = lo_t + j;
                if (J < 0 || J >= Nt)
                    continue;
                G[I * Nt + J] += P[i * n_t + j];
            }
        }
    }
}

/* Convolution (Sec. 2 step 3) written as its defining sum:
 *   O[p][t] = sum_{r < Rp} sum_{s < Rt} R[r][s] G[p + r0 - r][t - s],
 * with G = 0 outside the grid.  The response's pitch origin r0 aligns response
 * row r0 with the output row; time is causal.  Evaluated at the listed
 * (p, t) points only; pts[2 k] = p, pts[2 k + 1] = t. */
void oracle_convolve_points(const double *G, int64_t Np, int64_t Nt, const double *R, int64_t Rp,
                            int64_t Rt, int64_t r0, const int64_t *pts, int64_t npts, double *out)
{
    for (int64_t k = 0; k < npts; ++k) {
        int64_t p = pts[2 * k], t = pts[2 * k + 1];
        double acc = 0.0;
        for (int64_t r = 0; r < Rp; ++r) {
            int64_t pp = p + r0 - r;
            if (pp < 0 || pp >= Np)
                continue;
            for (int64_t s = 0; s < Rt; ++s) {
                int64_t tt = t - s;
                if (tt < 0 || tt >= Nt)
                    continue;
                acc += R[r * Rt + s] * G[pp * Nt + tt];
            }
        }
        out[k] = acc;
    }
}

/* The whole [Np][Nt] output by the defining sum (tiny grids only). */
void oracle_convolve_direct(const double *G, int64_t Np, int64_t Nt, const double *R, int64_t Rp,
                            int64_t Rt, int64_t r0, double *O)
{
    for (int64_t p = 0; p < Np; ++p) {
        for (int64_t t = 0; t < Nt; ++t) {
            int64_t pt[2] = {p, t};
            oracle_convolve_points(G, Np, Nt, R, Rp, Rt, r0, pt, 1, O + p * Nt + t);
        }
    }
}
