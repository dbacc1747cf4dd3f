/* Driver for the sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host): runs every oracle entry point over
 * ordinary, edge and malformed inputs; any out-of-bounds access, leak or
 * undefined operation aborts the run. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_philox_batch(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out);
double oracle_normal(int64_t I, int64_t J, int64_t d, uint64_t event_id, uint64_t seed,
                     int32_t plane_id);
double oracle_surviving_charge(double q, double T, double tau, int32_t fluctuate, int64_t d,
                               uint64_t event_id, uint64_t seed);
int oracle_depo_window(const double *depo, const double *phys, const double *geom,
                       const int32_t *dims, double *out_d, int64_t *out_i);
void oracle_axis_weights(int64_t lo, int64_t n, double mu, double s, double *W);
int64_t oracle_rasterize(const double *depos, int64_t n, const double *phys, int32_t fluctuate,
                         uint64_t seed, const double *geom, const int32_t *dims, uint64_t event_id,
                         const int64_t *ids, int64_t *meta, double *values, int64_t cap,
                         int32_t *status);
void oracle_scatter(const int64_t *meta, const double *values, int64_t n, int64_t Np, int64_t Nt,
                    double *G);
void oracle_convolve_points(const double *G, int64_t Np, int64_t Nt, const double *R, int64_t Rp,
                            int64_t Rt, int64_t r0, const int64_t *pts, int64_t npts, double *out);
void oracle_convolve_direct(const double *G, int64_t Np, int64_t Nt, const double *R, int64_t Rp,
                            int64_t Rt, int64_t r0, double *O);

static double urand(uint64_t *s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) * 0x1p-53;
}

int main(void)
{
    uint64_t st = 12345;
    /* Philox over a few counters and keys */
    uint32_t ctr[40], key[20], out[40];
    for (int i = 0; i < 40; ++i)
        ctr[i] = (uint32_t)(urand(&st) * 4294967295.0);
    for (int i = 0; i < 20; ++i)
        key[i] = (uint32_t)(urand(&st) * 4294967295.0);
    oracle_philox_batch(10, ctr, key, out);
    double acc = 0.0;
    for (int j = -9; j < 9; ++j)
        acc += oracle_normal(j, -j, 3, 7, 0x2304018410ull, 2);
    acc += oracle_surviving_charge(5000.0, 700.0, 1500.0, 1, 4, 9, 77);
    acc += oracle_surviving_charge(5000.0, 700.0, 0.0, 1, 4, 9, 77);
    /* a small plane, depos inside, on the edges, outside, malformed */
    const double phys[6] = {1.6, 4e-4, 8.8e-4, 3.0, 1500.0, 1e-4};
    const double geom[7] = {5.0, 0.5, 0.0, 0.0, 0.0, 1.0, 0.0};
    const int32_t dims[4] = {1, 12, 10, 300};
    enum { N = 64 };
    double depos[N * 5];
    for (int d = 0; d < N; ++d) {
        depos[5 * d + 0] = 1.6 * 2500.0 * urand(&st);
        depos[5 * d + 1] = 0.0;
        depos[5 * d + 2] = -10.0 + 80.0 * urand(&st);
        depos[5 * d + 3] = -depos[5 * d + 0] / 1.6 + 160.0 * urand(&st);
        depos[5 * d + 4] = 5000.0 * urand(&st);
    }
    depos[5 * 0 + 4] = NAN;                   /* invalid */
    depos[5 * 1 + 4] = -1.0;                  /* invalid */
    depos[5 * 2 + 0] = -3.0;                  /* behind the plane */
    depos[5 * 3 + 0] = 0.0;                   /* zero drift: single bin */
    depos[5 * 4 + 2] = 1e6;                   /* far outside the grid */
    depos[5 * 5 + 0] = 1e5;                   /* beyond the reach of the speed change */
    double od[5];
    int64_t oi[4];
    for (int d = 0; d < N; ++d)
        acc += oracle_depo_window(depos + 5 * d, phys, geom, dims, od, oi);
    double W[40];
    oracle_axis_weights(-3, 40, 15.2, 3.1, W);
    oracle_axis_weights(7, 1, 7.5, 0.0, W);
    int64_t meta[N * 5];
    int32_t status[N];
    int64_t cap = 8;
    double *values = malloc(sizeof(double) * (size_t)cap);
    for (int fl = 0; fl < 2; ++fl) {
        int64_t got = oracle_rasterize(depos, N, phys, fl, 99, geom, dims, 5, NULL, meta, values,
                                       cap, status);
        if (got < 0) { /* too small: grow to the size asked for, as the caller does */
            cap = -got;
            free(values);
            values = malloc(sizeof(double) * (size_t)cap);
            got = oracle_rasterize(depos, N, phys, fl, 99, geom, dims, 5, NULL, meta, values, cap,
                                   status);
        }
        if (got < 0)
            return 1;
        const int64_t Np = 120, Nt = 300;
        double *G = calloc((size_t)(Np * Nt), sizeof(double));
        oracle_scatter(meta, values, N, Np, Nt, G);
        double R[7 * 5];
        for (int i = 0; i < 35; ++i)
            R[i] = urand(&st) - 0.5;
        int64_t pts[6] = {0, 0, 119, 299, 60, 150};
        double o[3];
        oracle_convolve_points(G, Np, Nt, R, 7, 5, 3, pts, 3, o);
        double *O = malloc(sizeof(double) * (size_t)(Np * Nt));
        oracle_convolve_direct(G, Np, Nt, R, 7, 5, 3, O);
        for (int64_t i = 0; i < Np * Nt; ++i)
            acc += O[i] * 1e-9;
        free(O);
        free(G);
    }
    int64_t ids[N];
    for (int d = 0; d < N; ++d)
        ids[d] = 1000 + d;
    oracle_rasterize(depos, N, phys, 1, 99, geom, dims, 5, ids, meta, values, cap, status);
    free(values);
    printf("sanitized oracle run ok %g\n", acc);
    return 0;
}
