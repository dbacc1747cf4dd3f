// Rasterization and Scatter-Add on gfx950 (arXiv:2304.01841, Sec. 2 steps 1-2).
//
// Per depo (FP64): drift to the response plane, Gaussian widths sqrt(2 D T),
// continuous bin coordinates and the inclusive window floor(mu -/+ n s) on each
// axis.  Bin weights are differences of erf at the bin edges normalised over
// the window (FP64); the patch is the outer product of the two weight vectors
// times the charge (FP32).  With fluctuation, every bin draws a normal deviate
// from a Philox4x32-10 stream keyed by (event, depo, absolute bin) and takes
// the normal approximation of a binomial draw, clamped at zero, and the patch
// is rescaled to the depo charge.
//
// Scatter-Add (Sec. 2 step 2) runs two ways:
//  * fused (simulate path): depos are binned by the grid tile holding their
//    window origin (count -> exclusive scan -> fill, the scan of Sec. 4.3);
//    a tile's list is cut into work items of a few dozen depos, and one
//    wavefront per work item rasterizes them, one patch at a time, into its
//    own LDS copy of the tile plus a halo, then adds the non-zero LDS cells to
//    the grid with float atomics, so the grid sees one atomic per touched cell
//    per work item instead of one per patch bin;
//  * unfused (patch-set API): patches are written to a flat buffer at the
//    scanned offsets and a second kernel adds them to the grid atomically.
#include <math.h>

#include <limits.h>

#include <atomic>

#include "wcsim_internal.h"

namespace wcs {
namespace {

constexpr double kSqrt2 = 1.41421356237309504880;  // sqrt(2), correctly rounded

// Philox4x32-10 round constants (Salmon et al., SC'11).
constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

// a ^ b ^ c in one gfx950 three-input bitwise instruction (truth table 0x96:
// the result bit is set when an odd number of input bits are)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t a = (uint64_t)kPhiloxM0 * c.x;
        const uint64_t b = (uint64_t)kPhiloxM1 * c.z;
        c = make_uint4(xor3((uint32_t)(b >> 32), c.y, k0), (uint32_t)b,
                       xor3((uint32_t)(a >> 32), c.w, k1), (uint32_t)a);
    }
    return c;
}

// Uniform ((r >> 9) + 1/2) 2^-23 in (0, 1), exact in binary32: the float
// 1 + m 2^-23 (m = r >> 9 as its mantissa) minus (1 - 2^-24) is
// (2m + 1) 2^-24, an exact difference.
__device__ __forceinline__ float word_to_uniform(uint32_t r)
{
    return __uint_as_float((r >> 9) | 0x3f800000u) - (1.0f - 0x1p-24f);
}

// Box-Muller pair: cosine branch (even tick) and sine branch (odd tick).
// v_sin/v_cos take their argument in revolutions, so theta = 2 pi u is u;
// v_log gives log2, and -2 ln u = (-2 ln 2) log2 u.  u >= 2^-24 is never
// denormal, so the hardware instructions need no range fix-ups.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float &zc, float &zs)
{
    constexpr float kMinus2Ln2 = -1.38629436111989061883f;
    const float rho =
        __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(word_to_uniform(a)));
    const float u = word_to_uniform(b);
    zc = rho * __builtin_amdgcn_cosf(u);
    zs = rho * __builtin_amdgcn_sinf(u);
}

// FP64 Box-Muller pair of the digitisation noise: the uniforms of the two
// words, rho = sqrt(-2 ln u_a), theta = 2 pi u_b, cosine branch (even column)
// and sine branch (odd column), all in double precision.
constexpr double kPi = 3.14159265358979323846;
__device__ __forceinline__ void box_muller_d(uint32_t a, uint32_t b, double &zc, double &zs)
{
    const double ua = ((double)(a >> 9) + 0.5) * 0x1p-23;
    const double ub = ((double)(b >> 9) + 0.5) * 0x1p-23;
    const double rho = sqrt(-2.0 * log(ua));
    const double theta = 2.0 * kPi * ub;
    double sn, cs;
    sincos(theta, &sn, &cs);
    zc = rho * cs;
    zs = rho * sn;
}

struct Win {
    double T;  // drift time to the response plane
    double mu_p, s_p, mu_t, s_t, q;
    int lo_p, lo_t, n_p, n_t;
    int status;  // 0 ok, 1 invalid, 2 misses the grid, 3 window too long
};

// Drift, diffusion and window of one depo.  FP64 with no contraction, in the
// order the definitions are written, so that the integer window bounds are
// reproducible bit for bit.
__device__ __forceinline__ Win depo_window(const wcsim_depo &dep, const PlaneParams &P)
{
#pragma clang fp contract(off)
    Win w;
    w.T = 0.0;
    w.status = 0;
    w.lo_p = w.lo_t = w.n_p = w.n_t = 0;
    const double x = dep.x, y = dep.y, z = dep.z, t = dep.t, q = dep.q;
    w.q = q;
    w.mu_p = w.s_p = w.mu_t = w.s_t = 0.0;
    if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !isfinite(t) || !isfinite(q) || q < 0.0 ||
        x < P.plane_x) {
        w.status = 1;
        return w;
    }
    // The drift speed changes linearly with drift time at the rate accel and
    // equals v on the response plane: the depo starts at v_s = sqrt(v^2 -
    // 2 accel L) and drifts for T = 2 L / (v + v_s) (T = L / v exactly when
    // accel = 0); a depo with v^2 - 2 accel L < 0 cannot reach the plane.
    const double L = x - P.plane_x;
    const double disc = P.v * P.v - 2.0 * P.accel * L;
    if (disc < 0.0) {
        w.status = 1;
        return w;
    }
    const double T = (2.0 * L) / (P.v + sqrt(disc));
    w.T = T;
    const double t_arr = t + T;
    const double sigma_p = sqrt(2.0 * P.DT * T);
    const double sigma_t = sqrt(2.0 * P.DL * T) / P.v;
    const double proj = y * P.dir_y + z * P.dir_z;
    w.mu_p = (proj - P.pitch_origin) / P.dp;
    w.s_p = sigma_p / P.dp;
    w.mu_t = (t_arr - P.t0) / P.tick;
    w.s_t = sigma_t / P.tick;
    const double lo_p = floor(w.mu_p - P.nsigma * w.s_p);
    const double hi_p = floor(w.mu_p + P.nsigma * w.s_p);
    const double lo_t = floor(w.mu_t - P.nsigma * w.s_t);
    const double hi_t = floor(w.mu_t + P.nsigma * w.s_t);
    if (hi_p < 0.0 || lo_p >= (double)P.Np || hi_t < 0.0 || lo_t >= (double)P.Nt) {
        w.status = 2;
        return w;
    }
    if (hi_p - lo_p + 1.0 > (double)kMaxWindow || hi_t - lo_t + 1.0 > (double)kMaxWindow) {
        w.status = 3;
        return w;
    }
    w.lo_p = (int)lo_p;
    w.lo_t = (int)lo_t;
    w.n_p = (int)hi_p - w.lo_p + 1;
    w.n_t = (int)hi_t - w.lo_t + 1;
    return w;
}

__device__ __forceinline__ double edge_erf(int lo, int k, double mu, double s)
{
    return erf(((double)(lo + k) - mu) / (kSqrt2 * s));
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int WIDTH>
__device__ __forceinline__ double seg_sum(double v)
{
#pragma unroll
    for (int m = WIDTH / 2; m > 0; m >>= 1)
        v += __shfl_xor(v, m, WIDTH);
    return v;
}

// q / S in FP64 for S > 0 of ordinary magnitude (a patch total): hardware
// reciprocal refined by two Newton steps, then the product, within a few FP64
// ulps of the quotient -- far below the float32 rounding the factor gets.
__device__ __forceinline__ double div_pos_d(double q, double S)
{
    double r = __builtin_amdgcn_rcp(S);
    r = fma(fma(-S, r, 1.0), r, r);
    r = fma(fma(-S, r, 1.0), r, r);
    return q * r;
}

// Inclusive prefix sum over the wavefront's lanes in FP64: within each row of
// 16 lanes by shifts of 1, 2, 4 and 8 lanes, then each row adds the last lane
// of the rows before it (row broadcasts of lanes 15 and 31).  Fixed order.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_shift_d(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)((uint64_t)b >> 32), CTRL, ROWS,
                                               0xf, true);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ __forceinline__ double wave_incl_scan_d(double v)
{
    v += dpp_shift_d<0x111, 0xf>(v);  // row_shr:1
    v += dpp_shift_d<0x112, 0xf>(v);  // row_shr:2
    v += dpp_shift_d<0x114, 0xf>(v);  // row_shr:4
    v += dpp_shift_d<0x118, 0xf>(v);  // row_shr:8
    v += dpp_shift_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_shift_d<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

__device__ __forceinline__ double readlane_d(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)b >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Electrons of a depo that survive the drift (electron lifetime tau; an
// extension beyond the paper, which starts from the drifted charge): each
// survives the drift time T with probability p = exp(-T / tau).  The depo
// keeps q p, or with fluctuation the normal approximation of Binomial(q, p),
// clamped at zero.  Absorption precedes the readout planes, so the deviate
// belongs to the depo alone: Philox under the lifetime key (no plane in it)
// at counter (0, 0, depo index in the event, event), the cosine branch of
// Box-Muller on words 0 and 1, all in FP64 (one draw per depo).
__device__ __forceinline__ double surviving_charge(const Win &w, const PlaneParams &P, int d,
                                                   uint32_t event)
{
    if (!(P.tau > 0.0))
        return w.q;
    const double p = exp(-w.T / P.tau);
    if (!P.fluct)
        return w.q * p;
    const uint4 r = philox4x32_10(make_uint4(0u, 0u, (uint32_t)d, event), P.lkey0, P.lkey1);
    const double ua = ((double)(r.x >> 9) + 0.5) * 0x1p-23;
    const double ub = ((double)(r.y >> 9) + 0.5) * 0x1p-23;
    const double z = sqrt(-2.0 * log(ua)) * cospi(2.0 * ub);
    const double F = w.q * p + z * sqrt(w.q * p * (1.0 - p));
    return (F < 0.0) ? 0.0 : F;
}

// Fluctuated bin value before rescaling: normal approximation of the binomial
// draw of q electrons with probability p, clamped at zero.
__device__ __forceinline__ float fluct_value(float q, float p, float z)
{
    const float qp = q * p;
    const float var = fmaf(-qp, p, qp);  // q p (1 - p)
    return fmaxf(0.0f, fmaf(z, __builtin_amdgcn_sqrtf(var), qp));
}

// The same value from the squared Box-Muller radius r2 = -2 ln u and the
// branch's cosine or sine c: z sqrt(var) = c sqrt(r2 var), as rho and the
// standard deviation are both non-negative (one square root instead of two
// per value pair).
__device__ __forceinline__ float fluct_value_r2(float q, float p, float r2, float c)
{
    const float qp = q * p;
    const float var = fmaf(-qp, p, qp);  // q p (1 - p)
    return fmaxf(0.0f, fmaf(c, __builtin_amdgcn_sqrtf(r2 * var), qp));
}

__device__ __forceinline__ int quad_of(int J) { return J >> 2; }  // floor(J / 4)

// ---------------------------------------------------------------------------
// Fill and Philox diagnostic kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_zero16(uint4 *p, size_t n16)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void k_fill_zero1(unsigned char *p, size_t n)
{
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0;
}

__global__ void k_philox(const uint4 *ctr, const uint2 *key, int64_t n, uint4 *out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = philox4x32_10(ctr[i], key[i].x, key[i].y);
}

// ---------------------------------------------------------------------------
// Exclusive scan (three phases: block sums, scan of block sums, add)
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256, kScanPer = 4, kScanBlock = kScanThreads * kScanPer;

template <typename T>
__device__ T block_exclusive_scan(T v, T *sh, T *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T u = __shfl_up(inc, o, 64);
        if (lane >= o)
            inc += u;
    }
    if (lane == 63)
        sh[wave] = inc;
    __syncthreads();
    T base = 0, tot = 0;
    for (int k = 0; k < kScanThreads / 64; ++k) {
        if (k < wave)
            base += sh[k];
        tot += sh[k];
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_local(T *data, int64_t n, T *block_sums)
{
    __shared__ T sh[kScanThreads / 64];
    const int64_t base = blockIdx.x * (int64_t)kScanBlock + threadIdx.x * kScanPer;
    T v[kScanPer];
    T sum = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = (base + k < n) ? data[base + k] : T(0);
        sum += v[k];
    }
    T total;
    T run = block_exclusive_scan<T>(sum, sh, &total);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n)
            data[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0)
        block_sums[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(T *sums, int64_t nb)
{
    __shared__ T sh[kScanThreads / 64];
    T carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        const int64_t i = b0 + threadIdx.x;
        T v = (i < nb) ? sums[i] : T(0);
        T total;
        T ex = block_exclusive_scan<T>(v, sh, &total);
        if (i < nb)
            sums[i] = ex + carry;
        carry += total;
    }
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_add(T *data, int64_t n, const T *sums)
{
    const int64_t base = blockIdx.x * (int64_t)kScanBlock + threadIdx.x * kScanPer;
    const T add = sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < n)
            data[base + k] += add;
}

template <typename T>
hipError_t exclusive_scan(T *data, int64_t n, void *scratch, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    T *sums = (T *)scratch;
    hipLaunchKernelGGL(k_scan_local<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, sums);
    hipLaunchKernelGGL(k_scan_sums<T>, dim3(1), dim3(kScanThreads), 0, s, sums, nb);
    hipLaunchKernelGGL(k_scan_add<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, sums);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Unfused path: patch sizes, flat patch values, flat scatter
// ---------------------------------------------------------------------------
__global__ void k_patch_sizes(const wcsim_depo *depos, int64_t n, PlaneParams P, int32_t *meta,
                              int64_t *sizes)
{
    const int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (d == 0)
        sizes[n] = 0;
    if (d >= n)
        return;
    const Win w = depo_window(depos[d], P);
    const bool ok = (w.status == 0);
    meta[4 * d + 0] = ok ? w.lo_p : 0;
    meta[4 * d + 1] = ok ? w.lo_t : 0;
    meta[4 * d + 2] = ok ? w.n_p : 0;
    meta[4 * d + 3] = ok ? w.n_t : 0;
    sizes[d] = ok ? (int64_t)w.n_p * w.n_t : 0;
}

template <int NT>
__device__ double block_sum_d(double v, double *red)
{
    v = seg_sum<64>(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
        red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k)
        s += red[k];
    return s;
}

// Window weights of one axis by a whole workgroup (any window up to
// kMaxWindow bins): erf at every edge into LDS, then differences and the sum.
template <int NT>
__device__ void block_axis_weights(int lo, int n, double mu, double s, float *W, double *E,
                                   double *red)
{
    for (int k = threadIdx.x; k <= n; k += NT)
        E[k] = (s > 0.0) ? edge_erf(lo, k, mu, s) : 0.0;
    __syncthreads();
    double part = 0.0;
    for (int i = threadIdx.x; i < n; i += NT)
        part += 0.5 * (E[i + 1] - E[i]);
    const double sum = block_sum_d<NT>(part, red);
    for (int i = threadIdx.x; i < n; i += NT)
        W[i] = (s > 0.0) ? (float)((0.5 * (E[i + 1] - E[i])) / sum) : (i == 0 ? 1.0f : 0.0f);
    __syncthreads();
}

// One workgroup per depo, any window size.  FLAT: write the patch at its
// offset in the flat value buffer.  Otherwise add it to the grid with float
// atomics (used for the few depos whose patch does not fit the LDS tiles).
// With fluctuation the rescaling needs the patch total before any value is
// final: FLAT stores the clamped draws and rescales them in place; the grid
// variant draws twice (same counters, same numbers).
template <int NT, bool FLAT, bool B>
__global__ __launch_bounds__(NT) void k_patch_generic(EventCtx e0, BatchTables bt,
                                                      const int32_t *index_list,
                                                      const int32_t *list_count, int64_t n_direct,
                                                      const int64_t *offsets, float *values)
{
    __shared__ float Wp[kMaxWindow], Wt[kMaxWindow];
    __shared__ double E[kMaxWindow + 1];
    __shared__ double red[NT / 64];
    const int64_t count = index_list ? (int64_t)*list_count : n_direct;
    for (int64_t k = blockIdx.x; k < count; k += gridDim.x) {
        const int gd = index_list ? index_list[k] : (int)k;
        const EventCtx &Ev = B ? bt.ev[find_event(bt.depo_base, bt.nev, gd)] : e0;
        const PlaneParams &P = Ev.kp;
        const uint32_t event = Ev.event;
        const gptr<float> grid = glb(Ev.grid);
        const int d = gd - (int)Ev.depo_base;  // index in the event's own depo array
        const wcsim_depo dep = glb(Ev.depos)[d];
        const Win w = depo_window(dep, P);
        if (w.status != 0)
            continue;
        block_axis_weights<NT>(w.lo_p, w.n_p, w.mu_p, w.s_p, Wp, E, red);
        block_axis_weights<NT>(w.lo_t, w.n_t, w.mu_t, w.s_t, Wt, E, red);
        const double qd = surviving_charge(w, P, d, event);
        const float qf = (float)qd;
        float *out = FLAT ? values + offsets[d] : nullptr;
        if (!P.fluct) {
            const int cnt = w.n_p * w.n_t;
            for (int it = threadIdx.x; it < cnt; it += NT) {
                const int i = it / w.n_t, j = it - i * w.n_t;
                const float v = qf * Wp[i] * Wt[j];
                if (FLAT) {
                    out[it] = v;
                } else {
                    const int I = w.lo_p + i, J = w.lo_t + j;
                    if ((unsigned)I < (unsigned)P.Np && (unsigned)J < (unsigned)P.Nt)
                        unsafeAtomicAdd(grid + (size_t)I * P.Nt + J, v);
                }
            }
        } else {
            const int qlo = quad_of(w.lo_t), nq = quad_of(w.lo_t + w.n_t - 1) - qlo + 1;
            const int items = w.n_p * nq;
            double S = 0.0;
            for (int it = threadIdx.x; it < items; it += NT) {
                const int i = it / nq, qd = qlo + (it - i * nq);
                const uint4 r = philox4x32_10(
                    make_uint4((uint32_t)qd, (uint32_t)(w.lo_p + i), (uint32_t)d, event), P.key0,
                    P.key1);
                float z[4];
                box_muller(r.x, r.y, z[0], z[1]);
                box_muller(r.z, r.w, z[2], z[3]);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int j = 4 * qd + m - w.lo_t;
                    if (j >= 0 && j < w.n_t) {
                        const float F = fluct_value(qf, Wp[i] * Wt[j], z[m]);
                        S += (double)F;
                        if (FLAT)
                            out[i * w.n_t + j] = F;
                    }
                }
            }
            S = block_sum_d<NT>(S, red);
            const float scale = (S > 0.0) ? (float)(qd / S) : 0.0f;
            for (int it = threadIdx.x; it < items; it += NT) {
                const int i = it / nq, qd = qlo + (it - i * nq);
                float z[4];
                if (!FLAT) {
                    const uint4 r = philox4x32_10(
                        make_uint4((uint32_t)qd, (uint32_t)(w.lo_p + i), (uint32_t)d, event),
                        P.key0, P.key1);
                    box_muller(r.x, r.y, z[0], z[1]);
                    box_muller(r.z, r.w, z[2], z[3]);
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int j = 4 * qd + m - w.lo_t;
                    if (j >= 0 && j < w.n_t) {
                        const float p = Wp[i] * Wt[j];
                        if (FLAT) {
                            float &o = out[i * w.n_t + j];
                            o = (S > 0.0) ? o * scale : qf * p;
                        } else {
                            const int I = w.lo_p + i, J = w.lo_t + j;
                            if ((unsigned)I < (unsigned)P.Np && (unsigned)J < (unsigned)P.Nt) {
                                const float v =
                                    (S > 0.0) ? fluct_value(qf, p, z[m]) * scale : qf * p;
                                unsafeAtomicAdd(grid + (size_t)I * P.Nt + J, v);
                            }
                        }
                    }
                }
            }
        }
        if (gridDim.x == 1)
            __threadfence();  // one workgroup: this patch's adds complete before the next's
        __syncthreads();
    }
}

// Flat patch set -> grid.  One wavefront per patch.
__global__ __launch_bounds__(256) void k_scatter_flat(int64_t n, const int32_t *meta,
                                                      const int64_t *offsets, const float *values,
                                                      float *grid, int Np, int Nt)
{
    const int lane = threadIdx.x & 63;
    const int64_t d = blockIdx.x * 4LL + (threadIdx.x >> 6);
    if (d >= n)
        return;
    const int lo_p = meta[4 * d], lo_t = meta[4 * d + 1], n_p = meta[4 * d + 2],
              n_t = meta[4 * d + 3];
    const float *v = values + offsets[d];
    const int cnt = n_p * n_t;
    for (int it = lane; it < cnt; it += 64) {
        const int i = it / n_t, j = it - i * n_t;
        const int I = lo_p + i, J = lo_t + j;
        if ((unsigned)I < (unsigned)Np && (unsigned)J < (unsigned)Nt)
            unsafeAtomicAdd(grid + (size_t)I * Nt + J, v[it]);
    }
}

// ---------------------------------------------------------------------------
// Fused path: tile binning and LDS-staged rasterization
// ---------------------------------------------------------------------------
constexpr int kHaloP = 32, kHaloT = 16;   // LDS region = tile + halo
constexpr int kRecP = kHaloP;             // longest pitch window of the tile path
constexpr int kRecT = kHaloT + 1;         // longest tick window of the tile path
constexpr int kRecQuads = (kRecT + 2) / 4 + 1;  // most tick quads such a window touches
constexpr int kRecWords = 64;             // floats per depo record (256 bytes)
constexpr int kRecWp = 8;                 // record offset of the pitch weights
constexpr int kRecWt = kRecWp + kRecP;    // record offset of the quad-aligned tick weights
static_assert(kRecWt % 4 == 0, "tick quads must be 16-byte aligned");
static_assert(kRecWt + 4 * kRecQuads <= kRecWords, "depo record overflow");
// Depos per tile work item (one wavefront).  Each work item flushes its own
// region cells with global atomics, and the regions of items sharing a track
// overlap, so longer chunks mean fewer atomics; at most 64, one window per
// lane for the bounding box.
constexpr int kChunk = 32;
static_assert(kChunk <= 64, "the chunk bounding box takes one patch window per lane");
constexpr int kFluctItems = 3;            // work items per lane held in registers
// A tile-path patch has at most kRecP * kRecQuads = 160 (row, quad) items.
static_assert(kRecP * kRecQuads <= 64 * kFluctItems, "patch items overflow");

struct TileGeom {
    int tp, tt, rp, rt, ntt;
};

__device__ __forceinline__ bool fits_tile(const Win &w, int p0, int t0, const TileGeom &g,
                                          const PlaneParams &P)
{
    if (w.n_p > kRecP || w.n_t > kRecT)
        return false;
    return min(w.lo_p + w.n_p, P.Np) <= p0 + g.rp && min(w.lo_t + w.n_t, P.Nt) <= t0 + g.rt;
}

__device__ __forceinline__ uint64_t lanemask_lt(int lane) { return (1ull << lane) - 1ull; }

// Mark the occupancy-map blocks that a window (status 0: it meets the grid)
// reaches.  Every writer stores the same value, so no atomics are needed.
__device__ __forceinline__ void mark_blocks(const Win &w, const PlaneParams &P, gptr<uint8_t> occ,
                                            int shift)
{
    const int p0 = max(w.lo_p, 0), p1 = min(w.lo_p + w.n_p, P.Np) - 1;
    const int t0 = max(w.lo_t, 0), t1 = min(w.lo_t + w.n_t, P.Nt) - 1;
    for (int b = p0 / kOccRows; b <= p1 / kOccRows; ++b)
        for (int c = t0 >> shift; c <= (t1 >> shift); ++c)
            occ[b * kOccCols + c] = 1;
}

// depo_tile of a depo whose patch does not fit a tile region (-1: no tile and
// no patch).
constexpr int32_t kTileLarge = -2;

// Window and tile of every depo.  Slots in a tile's list come from one atomic
// per distinct tile per wavefront (consecutive depos of a track share tiles).
// Depos and tiles carry global indices: in a batch, depo gd belongs to the
// event whose depo_base range holds it, and tile numbers continue across
// events from each event's tile_base.
template <bool B>
__global__ __launch_bounds__(256) void k_prep_bin(EventCtx e0, BatchTables bt, int64_t ntotal,
                                                  TileGeom g, int32_t *counters,
                                                  int32_t *tile_count, int32_t *depo_tile,
                                                  int32_t *depo_slot, int32_t *large)
{
    const int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int tile = -1;
    bool bad = false, big = false;
    if (d < ntotal) {
        const EventCtx &E = B ? bt.ev[find_event(bt.depo_base, bt.nev, (int)d)] : e0;
        const PlaneParams &P = E.kp;
        const int64_t dl = d - E.depo_base;
        // a batch reserves capacity per event; depos past its count are absent
        const Win w = (dl < E.n) ? depo_window(E.depos[dl], P) : Win{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 2};
        if (w.status == 1 || w.status == 3) {
            bad = true;
        } else if (w.status == 0) {
            mark_blocks(w, P, glb(E.occ), E.occ_shift);
            const int tp = min(max(w.lo_p, 0), P.Np - 1) / g.tp;
            const int tt = min(max(w.lo_t, 0), P.Nt - 1) / g.tt;
            if (fits_tile(w, tp * g.tp, tt * g.tt, g, P))
                tile = E.tile_base + tp * E.ntt + tt;
            else
                big = true;
        }
    }
    const uint64_t badm = __ballot(bad);
    if (lane == 0 && badm)
        atomicAdd(&counters[0], __popcll(badm));
    const uint64_t bigm = __ballot(big);
    if (bigm) {
        int base = 0;
        const int leader = __ffsll((unsigned long long)bigm) - 1;
        if (lane == leader)
            base = atomicAdd(&counters[1], __popcll(bigm));
        base = __shfl(base, leader);
        if (big)
            large[base + __popcll(bigm & lanemask_lt(lane))] = (int32_t)d;
    }
    int slot = 0;
    uint64_t active = __ballot(tile >= 0);
    while (active) {
        const int leader = __ffsll((unsigned long long)active) - 1;
        const int lt = __shfl(tile, leader);
        const uint64_t same = __ballot(tile == lt);
        int base = 0;
        if (lane == leader)
            base = atomicAdd(&tile_count[lt], __popcll(same));
        base = __shfl(base, leader);
        if (tile == lt)
            slot = base + __popcll(same & lanemask_lt(lane));
        active &= ~same;
    }
    if (d < ntotal) {
        depo_tile[d] = big ? kTileLarge : tile;
        depo_slot[d] = slot;
    }
}

// Tile schedule, two kernels over blocks of kSchedTiles tiles: per-tile depo
// counts -> exclusive list offsets (in place, ntiles + 1 entries, the scan of
// Sec. 4.3), and the list of work items {tile, first record, end record, 0}
// of at most kChunk depos each.  counters[2] = number of work items.
constexpr int kSchedThreads = 256, kSchedPer = 16, kSchedTiles = kSchedThreads * kSchedPer;

__device__ __forceinline__ int chunks_of(int count) { return (count + kChunk - 1) / kChunk; }

// Block totals of depos and of work items.
__global__ __launch_bounds__(kSchedThreads) void k_tile_sums(const int32_t *tile_count, int ntiles,
                                                            int2 *block_tot)
{
    __shared__ int sh[kSchedThreads / 64];
    const int first = blockIdx.x * kSchedTiles + threadIdx.x * kSchedPer;
    int st = 0, sc = 0;
#pragma unroll
    for (int k = 0; k < kSchedPer; ++k) {
        const int idx = first + k;
        const int c = (idx < ntiles) ? tile_count[idx] : 0;
        st += c;
        sc += chunks_of(c);
    }
    int tot_t, tot_c;
    block_exclusive_scan<int>(st, sh, &tot_t);
    block_exclusive_scan<int>(sc, sh, &tot_c);
    if (threadIdx.x == 0)
        block_tot[blockIdx.x] = make_int2(tot_t, tot_c);
}

// Exclusive scan of the block totals in place (one workgroup), so that each
// schedule block reads its two bases with one load.
__global__ __launch_bounds__(kSchedThreads) void k_scan_block_tot(int2 *block_tot, int nb)
{
    __shared__ int sh[kSchedThreads / 64];
    int carry_t = 0, carry_c = 0;
    for (int b0 = 0; b0 < nb; b0 += kSchedThreads) {
        const int i = b0 + threadIdx.x;
        const int2 v = (i < nb) ? block_tot[i] : make_int2(0, 0);
        int tot_t, tot_c;
        const int ex_t = block_exclusive_scan<int>(v.x, sh, &tot_t);
        const int ex_c = block_exclusive_scan<int>(v.y, sh, &tot_c);
        if (i < nb)
            block_tot[i] = make_int2(ex_t + carry_t, ex_c + carry_c);
        carry_t += tot_t;
        carry_c += tot_c;
    }
}

__global__ __launch_bounds__(kSchedThreads) void k_tile_schedule(int32_t *tile_count, int ntiles,
                                                                const int2 *block_base,
                                                                int4 *items, int32_t *counters)
{
    __shared__ int sh[kSchedThreads / 64];
    const int base_t = block_base[blockIdx.x].x, base_c = block_base[blockIdx.x].y;
    const int first = blockIdx.x * kSchedTiles + threadIdx.x * kSchedPer;
    int cnt[kSchedPer];
    int st = 0, sc = 0;
#pragma unroll
    for (int k = 0; k < kSchedPer; ++k) {
        const int idx = first + k;
        cnt[k] = (idx < ntiles) ? tile_count[idx] : 0;
        st += cnt[k];
        sc += chunks_of(cnt[k]);
    }
    int tot_t, tot_c;
    int off_t = block_exclusive_scan<int>(st, sh, &tot_t) + base_t;
    int off_c = block_exclusive_scan<int>(sc, sh, &tot_c) + base_c;
#pragma unroll
    for (int k = 0; k < kSchedPer; ++k) {
        const int idx = first + k;
        if (idx <= ntiles)
            tile_count[idx] = off_t;
        const int nch = chunks_of(cnt[k]);
        for (int j = 0; j < nch; ++j) {
            const int b = off_t + j * kChunk;
            items[off_c + j] = make_int4(idx, b, min(b + kChunk, off_t + cnt[k]), 0);
        }
        off_t += cnt[k];
        off_c += nch;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kSchedThreads - 1)
        counters[2] = off_c;
}

// ---------------------------------------------------------------------------
// Tile lists in depo order (reproducible sums).  The slots that binning takes
// by atomics order a tile's depos as the wavefronts happened to run; a stable
// least-significant-digit radix sort of the keys (tile; kTileLarge depos after
// the last tile; depos without a patch last) over the depo indices gives every
// depo its rank in its tile's list by index, and the large-patch list in index
// order.  Blocks of kSortBlock keys; 8-bit digits, one count / offsets /
// scatter triple per digit.
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256, kSortPer = 16, kSortBlock = kSortThreads * kSortPer;
static_assert(kSortThreads == kScanThreads, "the sort uses the block scan");

__global__ __launch_bounds__(256) void k_sort_keys(const int32_t *depo_tile, int64_t n,
                                                   uint32_t ntiles, uint32_t *keys,
                                                   int32_t *vals)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int t = depo_tile[i];
    keys[i] = (t >= 0) ? (uint32_t)t : (t == kTileLarge ? ntiles : ntiles + 1u);
    vals[i] = (int32_t)i;
}

// counts[b][d]: keys of block b with digit d; totals[d] += the block's count.
__global__ __launch_bounds__(kSortThreads) void k_sort_count(const uint32_t *keys, int64_t n,
                                                            int shift, int32_t *counts,
                                                            int32_t *totals)
{
    __shared__ int hist[256];
    const int tid = threadIdx.x;
    hist[tid] = 0;
    __syncthreads();
    const int64_t b0 = blockIdx.x * (int64_t)kSortBlock;
#pragma unroll 4
    for (int k = 0; k < kSortPer; ++k) {
        const int64_t i = b0 + k * kSortThreads + tid;
        if (i < n)
            atomicAdd(&hist[(keys[i] >> shift) & 255], 1);
    }
    __syncthreads();
    const int c = hist[tid];
    counts[(int64_t)blockIdx.x * 256 + tid] = c;
    if (c)
        atomicAdd(&totals[tid], c);
}

// One workgroup, thread d: the first output position of digit d in each block
// (the keys of smaller digits plus those of digit d in earlier blocks), in
// place; the totals are cleared for the next digit.
__global__ __launch_bounds__(kSortThreads) void k_sort_offsets(int32_t *counts, int nblk,
                                                              int32_t *totals)
{
    __shared__ int sh[kSortThreads / 64];
    const int d = threadIdx.x;
    int all;
    int run = block_exclusive_scan<int>(totals[d], sh, &all);
    totals[d] = 0;
    int b = 0;
    for (; b + 8 <= nblk; b += 8) {
        int c[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            c[u] = counts[(int64_t)(b + u) * 256 + d];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            counts[(int64_t)(b + u) * 256 + d] = run;
            run += c[u];
        }
    }
    for (; b < nblk; ++b) {
        const int c = counts[(int64_t)b * 256 + d];
        counts[(int64_t)b * 256 + d] = run;
        run += c;
    }
}

// Stable scatter of one block: its keys are taken in rounds of kSortThreads
// consecutive keys; a key's position is its digit's next free slot plus the
// keys of the same digit before it in the round (earlier wavefronts, then
// lower lanes of its own).
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const uint32_t *kin,
                                                              const int32_t *vin, int64_t n,
                                                              int shift, const int32_t *offsets,
                                                              uint32_t *kout, int32_t *vout)
{
    constexpr int NW = kSortThreads / 64;
    __shared__ int next[256];
    __shared__ int wcnt[NW][256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    next[tid] = offsets[(int64_t)blockIdx.x * 256 + tid];
#pragma unroll
    for (int u = 0; u < NW; ++u)
        wcnt[u][tid] = 0;
    __syncthreads();
    const int64_t b0 = blockIdx.x * (int64_t)kSortBlock;
    for (int k = 0; k < kSortPer; ++k) {
        const int64_t i = b0 + k * kSortThreads + tid;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const int32_t val = valid ? vin[i] : 0;
        const int dg = (int)((key >> shift) & 255u);
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t m = __ballot((dg >> bit) & 1);
            same &= ((dg >> bit) & 1) ? m : ~m;
        }
        const int rank = __popcll(same & lanemask_lt(lane));
        if (valid && rank == 0)
            wcnt[w][dg] = __popcll(same);
        __syncthreads();
        if (valid) {
            int pos = next[dg] + rank;
            for (int u = 0; u < w; ++u)
                pos += wcnt[u][dg];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();  // every position is formed before the counts move on
        int add = 0;
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            add += wcnt[u][tid];
            wcnt[u][tid] = 0;
        }
        next[tid] += add;
        __syncthreads();
    }
}

// From the sorted keys: each tile-listed depo's slot (its rank in the tile's
// list) and the large-patch list in depo order.  tile_off: the tiles'
// exclusive list offsets, ntiles + 1 entries.
__global__ __launch_bounds__(256) void k_sort_slots(const uint32_t *keys, const int32_t *vals,
                                                    int64_t n, uint32_t ntiles,
                                                    const int32_t *tile_off, int32_t *depo_slot,
                                                    int32_t *large)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t key = keys[i];
    if (key < ntiles)
        depo_slot[vals[i]] = (int32_t)(i - tile_off[key]);
    else if (key == ntiles)
        large[i - tile_off[ntiles]] = vals[i];
}

// Weights of one axis computed by one thread into a record, in FP64: the
// Gaussian's integral over each bin, normalised by the window total, rounded
// once to float32.  The edge arguments are x_k = (lo + k - mu) / (sqrt(2) s);
// the integrals come from the complementary error function of |x_k|,
// c_k = erfc(|x_k|), with erf(x) = sign(x) (1 - c): a bin on one side of the
// centre is the difference c_a - c_b of two tail values (no cancellation of
// values near 1, so tail bins keep their full relative precision), a bin
// holding the centre is 2 - c_a - c_b.  The window total is the same
// difference taken between the window's outer edges.
// erfc(x) for x >= 0 in FP64 without branches: exp(-x^2) erfcx(x), with
// erfcx(x) = exp(x^2) erfc(x) a polynomial of degree 18 in
// u = 9 / (3 + x) - 2 (the interval [0, 6] of x mapped onto [-1, 1]).  The
// polynomial is a Chebyshev expansion fitted by weighted least squares at 300
// Chebyshev nodes in 40-digit arithmetic, turned into powers of u in 50-digit
// arithmetic; the magnitudes of its coefficients sum to 1.0003, so Horner's
// rule loses nothing to cancellation: at most 2e-15 relative to the library
// erfc on [0, 6].  Beyond x = 6 erfcx is held at its value at 6 (erfc(6) =
// 2.2e-17: the absolute error stays below 1e-17).  The library erfc branches
// over three ranges of x here, and the lanes of a wavefront take all three.
__constant__ const double kErfcxPoly[19] = {
    0.32158541645431749, 0.36815156489826012, 0.2014388568192258,
    0.081626845134045015, 0.023308261232626117, 0.003956151636291854,
    7.0125313652629907e-05, -0.00012716419781459492, -1.5153801949992285e-05,
    4.532602482660329e-06, 8.1181436388616683e-07, -2.2753363747095745e-07,
    -3.482226636786867e-08, 1.44452931474044e-08, 8.4853769242305189e-10,
    -9.2921436560768322e-10, 4.7966663774361644e-11, 4.402449211974955e-11,
    -6.2047195508566893e-12};

// 1 / d for d in [3, 9] (no scaling or special cases needed): the hardware
// reciprocal refined by two Newton steps, each squaring the relative error.
__device__ __forceinline__ double recip_3_9(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    return fma(r, fma(-d, r, 1.0), r);
}

__device__ __forceinline__ double erfc_tail(double x)
{
    const double u = fma(9.0, recip_3_9(3.0 + fmin(x, 6.0)), -2.0);
    double p = kErfcxPoly[18];
#pragma unroll
    for (int k = 17; k >= 0; --k)
        p = fma(p, u, kErfcxPoly[k]);
    return exp(-x * x) * p;
}

__device__ __forceinline__ double edge_tail(int lo, int k, double mu, double inv, bool &neg)
{
    const double x = ((double)(lo + k) - mu) * inv;
    neg = x < 0.0;
    return erfc_tail(fabs(x));
}

__device__ __forceinline__ double bin_integral(double ca, bool na, double cb, bool nb)
{
    // erf(b) - erf(a) for edges a < b
    if (!na)
        return ca - cb;
    if (nb)
        return cb - ca;
    return (2.0 - ca) - cb;
}

__device__ __forceinline__ void thread_axis_weights(int lo, int n, double mu, double s, float *W)
{
    if (s == 0.0) {
        W[0] = 1.0f;
        return;
    }
    const double inv = 1.0 / (kSqrt2 * s);
    bool n0, nn;
    double c_lo = edge_tail(lo, 0, mu, inv, n0);
    const double c_n = edge_tail(lo, n, mu, inv, nn);
    const double rtot = 1.0 / bin_integral(c_lo, n0, c_n, nn);
    bool n_lo = n0;
    for (int i = 0; i + 1 < n; ++i) {
        bool n_hi;
        const double c_hi = edge_tail(lo, i + 1, mu, inv, n_hi);
        W[i] = (float)(bin_integral(c_lo, n_lo, c_hi, n_hi) * rtot);
        c_lo = c_hi;
        n_lo = n_hi;
    }
    W[n - 1] = (float)(bin_integral(c_lo, n_lo, c_n, nn) * rtot);  // the last edge is c_n
}

// floor(a / b) for 0 <= a < 4096 and 1 <= b <= 64 by a multiply-shift with
// m = ceil(2^20 / b): the error term a (m b - 2^20) / (b 2^20) stays below 1/b.
__device__ __forceinline__ int div_small(int a, int m) { return (int)(__umul24(a, m) >> 20); }
__device__ __forceinline__ int magic_small(int b) { return ((1 << 20) + b - 1) / b; }

// Depo records in tile-list order.  Header words: lo_p, lo_t, n_p, n_t, depo
// index, charge (FP64, two words) and the division magic of the tick quad
// count; then
// the pitch weights, and the tick weights placed by tick quad: entry
// 4 (floor(J / 4) - floor(lo_t / 4)) + J mod 4 holds the weight of tick J, and
// the entries of the first and last quad outside the window hold zero.
enum { kHLoP, kHLoT, kHNp, kHNt, kHDepo, kHQlo, kHQhi, kHMq, kHeaderWords };
static_assert(kHeaderWords <= kRecWp, "record header overflow");
constexpr int kStageStride = kRecWords + 1;  // odd: one LDS bank per lane

// Zero the blocks of one band of kOccRows grid rows whose bits are set in
// `m` (bit c: ticks c 2^shift .. (c + 1) 2^shift - 1), by one wavefront.
__device__ __forceinline__ void clear_blocks(gptr<float> grid, int Np, int Nt, int band,
                                             uint64_t m, int shift, int lane)
{
    const int r0 = band * kOccRows, nr = min(kOccRows, Np - r0);
    while (m) {
        const int c = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const int c0 = c << shift, c1 = min(c0 + (1 << shift), Nt);
        if ((Nt & 3) == 0) {  // rows of whole float4 words
            const int nc = (c1 - c0) >> 2;
            for (int i = lane; i < nr * nc; i += 64) {
                const int r = i / nc;
                *(gptr<float4>)(grid + (int64_t)(r0 + r) * Nt + c0 + 4 * (i - r * nc)) =
                    make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
        } else {
            const int nc = c1 - c0;
            for (int i = lane; i < nr * nc; i += 64) {
                const int r = i / nc;
                grid[(int64_t)(r0 + r) * Nt + c0 + (i - r * nc)] = 0.0f;
            }
        }
    }
}

// Two wavefronts per block of 64 depos: lane l of the first computes depo
// l's header and pitch weights into LDS, lane l of the second its tick
// weights (two FP64 chains per depo in flight instead of one, for the same
// LDS), then the block writes the records out one 256-byte row at a time.
// The first `nclr` blocks instead clear the occupied blocks of the grids, one
// band of kOccRows rows per wavefront at a time (nbands bands over all
// events): the clear is bound by HBM writes and the records by FP64
// arithmetic, so one launch runs both side by side.
template <bool B>
__global__ __launch_bounds__(128) void k_fill_records(EventCtx e0, BatchTables bt, int64_t ntotal,
                                                     const int32_t *depo_tile,
                                                     const int32_t *depo_slot,
                                                     const int32_t *tile_off, float *records,
                                                     int nbands, int nclr)
{
    __shared__ float stage[64 * kStageStride];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if ((int)blockIdx.x < nclr) {
        for (int gb = 2 * blockIdx.x + wv; gb < nbands; gb += 2 * nclr) {
            const int e = B ? find_event(bt.band_base, bt.nev, gb) : 0;
            const EventCtx &E = B ? bt.ev[e] : e0;
            const int band = B ? gb - bt.band_base[e] : gb;
            const uint64_t m = __ballot(glb(E.occ)[band * kOccCols + lane] != 0);
            clear_blocks(glb(E.grid), E.kp.Np, E.kp.Nt, band, m, E.occ_shift, lane);
        }
        return;
    }
    const int64_t gd = (blockIdx.x - nclr) * (int64_t)64 + lane;
    int pos = -1;
    const int t = (gd < ntotal) ? depo_tile[gd] : -1;
    if (t >= 0) {
        const EventCtx &E = B ? bt.ev[find_event(bt.depo_base, bt.nev, (int)gd)] : e0;
        const int64_t d = gd - E.depo_base;  // index in the event's own depo array
        pos = tile_off[t] + depo_slot[gd];
        const Win w = depo_window(E.depos[d], E.kp);
        float *rec = stage + lane * kStageStride;
        int *h = (int *)rec;
        const int off = w.lo_t & 3;
        const int nq = quad_of(w.lo_t + w.n_t - 1) - quad_of(w.lo_t) + 1;
        if (wv == 0) {  // header and pitch weights
            h[kHLoP] = w.lo_p;
            h[kHLoT] = w.lo_t;
            h[kHNp] = w.n_p;
            h[kHNt] = w.n_t;
            h[kHDepo] = (int)d;
            const double qs = surviving_charge(w, E.kp, (int)d, E.event);
            h[kHQlo] = (int)(uint32_t)__double_as_longlong(qs);
            h[kHQhi] = (int)(uint32_t)((uint64_t)__double_as_longlong(qs) >> 32);
            h[kHMq] = magic_small(nq);
            thread_axis_weights(w.lo_p, w.n_p, w.mu_p, w.s_p, rec + kRecWp);
        } else {  // tick weights
            float *Wt = rec + kRecWt;
            for (int k = 0; k < off; ++k)
                Wt[k] = 0.0f;
            for (int k = off + w.n_t; k < 4 * nq; ++k)
                Wt[k] = 0.0f;
            thread_axis_weights(w.lo_t, w.n_t, w.mu_t, w.s_t, Wt + off);
        }
    }
    __syncthreads();
    for (int r = wv; r < 64; r += 2) {
        const int pr = __builtin_amdgcn_readlane(pos, r);
        if (pr >= 0)
            records[(int64_t)pr * kRecWords + lane] = stage[r * kStageStride + lane];
    }
}

// Region columns start at the tile's first tick (a multiple of four) and rows
// are a multiple of four floats, so that a tick quad (four ticks 4k .. 4k + 3,
// the unit one Philox block covers) is one aligned 16-byte LDS access.  A
// window starts inside its tile and spans at most kHaloT + 1 ticks, so its
// last quad ends before column TT + kHaloT.  A quad's ticks outside the window
// carry weight zero, hence deposit zero; quads before tick 0 (windows of the
// first tile that start before the grid) are dropped, and cells outside the
// grid are never flushed.
template <int TT>
constexpr int region_cols()
{
    return TT + kHaloT;
}

// Patches per batch of items: consecutive patches of a work item whose (row,
// tick quad) items number at most kBatchItems are drawn together, their
// items laid out flat over kBatchItems / 64 passes of the wavefront, so that
// the lanes of a pass serve several small patches instead of one.
constexpr int kBatchItems = 64 * kFluctItems;

// One wavefront per work item (tile, chunk of <= kChunk depos), rasterizing
// its patches into its own LDS copy of the tile region (tile + halo).  The
// patches are taken in batches of consecutive patches whose (row, tick quad)
// items fit kFluctItems passes of 64 lanes; the items of a batch are laid out
// flat (patch after patch), each lane finds its item's patch from the
// patches' item offsets, reads the patch's header from the lane that holds it
// (lane k holds patch k) and its weights from the depo record.  With
// fluctuation every item's four values are added, in FP64, to its patch's
// total in LDS; once the batch is drawn, each patch's factor q / S is formed
// in FP64 by the lane holding it, and every value is rescaled and deposited.
// The bins of one patch are distinct, so depositing the batch one patch at a
// time makes every deposit a plain read-add-write LDS access (two patches of
// a batch may cover the same cell).  No other wavefront touches the region.
// The region's non-zero cells are then added to the grid with float atomics.
// OWN: the caller clears the whole region before the tile's first item and
// flushes it after the last (the owner flush); the item neither clears nor
// flushes.
template <int TP, int TT, bool B, bool FLUCT, bool OWN = false>
__device__ __forceinline__ void raster_item(float4 *acc4, double *xsum, const int4 item,
                                            const float *__restrict__ records,
                                            const EventCtx &e0, const BatchTables &bt)
{
    constexpr int RT = region_cols<TT>();
    constexpr int RP = TP + kHaloP;
    const int tile = item.x, beg = item.y, end = item.z;
    const int K = end - beg;  // patches of the work item (<= kChunk)
    const int lane = threadIdx.x & 63;  // the item's wavefront (one of OWN's workgroup)
    // lane k < K holds the header of patch k: window, depo index, charge
    int4 win = make_int4(INT_MAX, INT_MAX, 0, 0), hdr = make_int4(0, 0, 0, 0);
    if (lane < K) {
        const int4 *rec = (const int4 *)(records + (int64_t)(beg + lane) * kRecWords);
        win = rec[0];  // lo_p lo_t n_p n_t
        hdr = rec[1];  // depo, q low word, q high word, quad-count magic
    }
    const EventCtx &E = B ? bt.ev[find_event(bt.tile_base, bt.nev, tile)] : e0;
    const PlaneParams P = E.kp;
    const int local = tile - E.tile_base;
    const int p0 = (local / E.ntt) * TP, t0 = (local % E.ntt) * TT;
    const int c0 = t0;  // grid tick of region column 0
    // Only the bounding box of the chunk's patches (in region rows and tick
    // quads, within the grid) is cleared and flushed; deposits outside the
    // grid land outside it and are never read.
    int rlo = win.x, rhi = (win.z > 0) ? win.x + win.z : INT_MIN;
    int qlo = quad_of(win.y), qhi = (win.z > 0) ? quad_of(win.y + win.w - 1) + 1 : INT_MIN;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        rlo = min(rlo, __shfl_xor(rlo, m, 64));
        rhi = max(rhi, __shfl_xor(rhi, m, 64));
        qlo = min(qlo, __shfl_xor(qlo, m, 64));
        qhi = max(qhi, __shfl_xor(qhi, m, 64));
    }
    const int br0 = max(rlo, p0) - p0;
    const int br1 = min(min(rhi, (int)P.Np), p0 + RP) - p0;
    const int bq0 = max(4 * max(qlo, 0) - c0, 0) >> 2;
    const int bq1 = min(4 * min(qhi, quad_of((int)P.Nt - 1) + 1) - c0, RT) >> 2;
    const int bnq = max(bq1 - bq0, 0), bcells = max(br1 - br0, 0) * bnq;
    const int bmagic = magic_small(max(bnq, 1));
    for (int x = lane; x < (OWN ? 0 : bcells); x += 64) {
        const int r = div_small(x, bmagic);
        acc4[r * (RT / 4) + bq0 + br0 * (RT / 4) + (x - r * bnq)] =
            make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    // per-patch item counts and their inclusive prefix over the lanes
    const int pqlo = quad_of(win.y);
    const int pnq = (lane < K) ? quad_of(win.y + win.w - 1) - pqlo + 1 : 0;
    const int pitems = (lane < K) ? win.z * pnq : 0;
    int incl = pitems;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o, 64);
        if (lane >= o)
            incl += u;
    }
    const double pq = __longlong_as_double(
        (long long)(((uint64_t)(uint32_t)hdr.z << 32) | (uint32_t)hdr.y));  // patch charge, FP64
    const float pqf = (float)pq;

    wave_lds_sync();  // the cleared region is visible to every lane

    int kb = 0;  // first patch of the batch (uniform)
    while (kb < K) {
        const int base = __builtin_amdgcn_readlane(incl - pitems, kb);
        // the batch: patches kb .. ke, the longest run whose items fit
        const uint64_t fits = __ballot(lane >= kb && lane < K && incl - base <= kBatchItems);
        const int ke = 63 - __builtin_clzll(fits);
        const int nitems = __builtin_amdgcn_readlane(incl, ke) - base;
        const int npass = (nitems + 63) >> 6;
        float F[kFluctItems][4];
        int cell[kFluctItems], kk[kFluctItems];
        double carry = 0.0;  // total of the batch's earlier passes (uniform)
        // each item's patch: kb plus the patch ends at or below its flat index
        // (one pass over the batch's patch ends serves the lane's items)
#pragma unroll
        for (int b = 0; b < kFluctItems; ++b)
            kk[b] = kb;
        for (int j = kb; j < ke; ++j) {
            const int e = __builtin_amdgcn_readlane(incl, j) - base;
#pragma unroll
            for (int b = 0; b < kFluctItems; ++b)
                kk[b] += (64 * b + lane >= e) ? 1 : 0;
        }
#pragma unroll
        for (int b = 0; b < kFluctItems; ++b) {
            cell[b] = -1;
            if (b < npass) {
                const int g = 64 * b + lane;  // flat item index within the batch
                const bool valid = g < nitems;
                const int k = kk[b];
                // the patch's header, from the lane holding it
                const int lo_p = __shfl(win.x, k, 64), lo_t = __shfl(win.y, k, 64);
                const int d = __shfl(hdr.x, k, 64), m = __shfl(hdr.w, k, 64);
                const int nq = __shfl(pnq, k, 64);
                const int first = __shfl(incl - pitems, k, 64) - base;
                const float q = __shfl(pqf, k, 64);
                const int it = valid ? g - first : 0;
                const int i = div_small(it, m);
                const int qq = it - (int)__umul24(i, nq);
                const int qd = quad_of(lo_t) + qq;
                const int r = lo_p + i - p0, c = 4 * qd - c0;
                cell[b] = (valid && (unsigned)r < (unsigned)RP && (unsigned)c <= (unsigned)(RT - 4))
                              ? (r * RT + c) >> 2
                              : -1;
                const float *rec = records + (int64_t)(beg + k) * kRecWords;
                const float wp = valid ? rec[kRecWp + i] : 0.0f;
                const float4 wt = *(const float4 *)(rec + kRecWt + 4 * qq);
                const float w4[4] = {wt.x, wt.y, wt.z, wt.w};
                if constexpr (FLUCT) {
                    const uint4 rr = philox4x32_10(
                        make_uint4((uint32_t)qd, (uint32_t)(lo_p + i), (uint32_t)d, E.event),
                        P.key0, P.key1);
                    constexpr float kMinus2Ln2 = -1.38629436111989061883f;
                    const float r2a = kMinus2Ln2 * __builtin_amdgcn_logf(word_to_uniform(rr.x));
                    const float r2b = kMinus2Ln2 * __builtin_amdgcn_logf(word_to_uniform(rr.z));
                    const float ua = word_to_uniform(rr.y), ub = word_to_uniform(rr.w);
                    const float r2[4] = {r2a, r2a, r2b, r2b};
                    const float c[4] = {__builtin_amdgcn_cosf(ua), __builtin_amdgcn_sinf(ua),
                                        __builtin_amdgcn_cosf(ub), __builtin_amdgcn_sinf(ub)};
#pragma unroll
                    for (int mm = 0; mm < 4; ++mm)
                        F[b][mm] = fluct_value_r2(q, wp * w4[mm], r2[mm], c[mm]);
                    // the item's total in FP64, and its prefix over the batch
                    const double t = valid ? ((double)F[b][0] + (double)F[b][1]) +
                                                 ((double)F[b][2] + (double)F[b][3])
                                           : 0.0;
                    const double x = wave_incl_scan_d(t) + carry;
                    xsum[g] = x;
                    carry = readlane_d(x, 63);
                } else {
#pragma unroll
                    for (int mm = 0; mm < 4; ++mm)
                        F[b][mm] = q * (wp * w4[mm]);
                }
            }
        }
        if constexpr (FLUCT) {
            // the lane of each patch of the batch forms its total S as the
            // difference of the prefix sums at its last item and before its
            // first, and its factor q / S, in FP64 (negative when the clamped
            // total is zero: the patch keeps its mean)
            wave_lds_sync();
            float scale = 0.0f;
            if (lane >= kb && lane <= ke) {
                const int s0 = incl - pitems - base, s1 = incl - base;
                const double S = xsum[s1 - 1] - (s0 > 0 ? xsum[s0 - 1] : 0.0);
                scale = (S > 0.0) ? (float)div_pos_d(pq, S) : -1.0f;
            }
            wave_lds_sync();  // the next batch may overwrite the prefix sums
#pragma unroll
            for (int b = 0; b < kFluctItems; ++b) {
                const float sc = __shfl(scale, kk[b], 64);
                if (b < npass && cell[b] >= 0) {
                    if (sc >= 0.0f) {
#pragma unroll
                        for (int mm = 0; mm < 4; ++mm)
                            F[b][mm] *= sc;
                    } else {
                        // rare: every fluctuated bin of the patch is zero
                        const int k = kk[b];
                        const int g = 64 * b + lane;
                        const int first = __shfl(incl - pitems, k, 64) - base;
                        const int it = g - first;
                        const int i = div_small(it, __shfl(hdr.w, k, 64));
                        const int qq = it - (int)__umul24(i, __shfl(pnq, k, 64));
                        const float *rec = records + (int64_t)(beg + k) * kRecWords;
                        const float wp = rec[kRecWp + i];
                        const float4 wt = *(const float4 *)(rec + kRecWt + 4 * qq);
                        const float q = __shfl(pqf, k, 64);
                        F[b][0] = q * (wp * wt.x);
                        F[b][1] = q * (wp * wt.y);
                        F[b][2] = q * (wp * wt.z);
                        F[b][3] = q * (wp * wt.w);
                    }
                }
            }
        }
        // Deposit, one patch of the batch at a time: the bins of one patch are
        // distinct, but two patches of a batch may share cells.  A wavefront's
        // LDS accesses complete in program order, so each round reads what the
        // previous one wrote.
        for (int k = kb; k <= ke; ++k) {
#pragma unroll
            for (int b = 0; b < kFluctItems; ++b) {
                if (b < npass && cell[b] >= 0 && kk[b] == k) {
                    float4 a4 = acc4[cell[b]];
                    a4.x += F[b][0];
                    a4.y += F[b][1];
                    a4.z += F[b][2];
                    a4.w += F[b][3];
                    acc4[cell[b]] = a4;
                }
            }
        }
        kb = ke + 1;
    }
    wave_lds_sync();  // every deposit lands before the flush reads the region
    if constexpr (OWN)
        return;
    // Flush: consecutive lanes take consecutive ticks of a row, so that one
    // atomic instruction covers 256 contiguous bytes (few L2 lines) rather
    // than 16-byte pieces of many lines.
    const gptr<float> grid = glb(E.grid);
    const float *acc = (const float *)acc4;
    const int W = 4 * bnq;  // floats per bounding-box row
    const int nrows = max(br1 - br0, 0);
    auto flush_one = [&](int r, int col) {
        const float v = acc[(br0 + r) * RT + 4 * bq0 + col];
        const int J = c0 + 4 * bq0 + col;
        if (v != 0.0f && (unsigned)J < (unsigned)P.Nt)
            unsafeAtomicAdd(grid + (size_t)(p0 + br0 + r) * P.Nt + J, v);
    };
    if (W > 0 && W <= 64) {
        const int per = 64 / W, r_l = lane / W, col = lane - r_l * W;
        if (r_l < per)
            for (int r = r_l; r < nrows; r += per)
                flush_one(r, col);
    } else if (W > 64) {
        for (int r = 0; r < nrows; ++r)
            for (int col = lane; col < W; col += 64)
                flush_one(r, col);
    }
}

// FLUCT: the planes fluctuate (a template argument, so that no branch on it
// separates a pass's weight loads from the Philox rounds that need no weight).
template <int TP, int TT, bool B, bool FLUCT>
__global__ __launch_bounds__(64) void k_raster_tiles(const float *__restrict__ records,
                                                     const int4 *__restrict__ items,
                                                     const int32_t *__restrict__ counters,
                                                     EventCtx e0, BatchTables bt)
{
    constexpr int RP = TP + kHaloP, RT = region_cols<TT>();
    static_assert(RT % 4 == 0, "region rows must hold whole quads");
    __shared__ float4 acc4[RP * RT / 4];
    __shared__ double xsum[kBatchItems];  // prefix sums of a batch's fluctuated item totals
    // The launch has at most as many wavefronts as a typical work list has
    // items (the count is known only on the device); a wavefront takes items
    // blockIdx.x, + gridDim.x, ... so that every item is drawn.
    const int nitems_all = counters[2];
    for (int itm = blockIdx.x; itm < nitems_all; itm += gridDim.x)
        raster_item<TP, TT, B, FLUCT>(acc4, xsum, items[itm], records, e0, bt);
}

// Owner flush (reproducible sums).  Tiles are coloured by (tile row mod CP,
// tile column mod CT), with CP TP >= RP and CT TT >= RT, so that the LDS
// regions of two tiles of one colour never share a grid cell; one launch per
// colour, in a fixed order.  In a launch each tile of the colour is owned by
// one workgroup of kOwnerWaves wavefronts: wavefront w draws the tile's work
// items w, w + kOwnerWaves, ... (in list order) into its own copy of the
// region, and the workgroup adds the sum of the copies to the grid with plain
// read-add-writes.  Every cell receives its sums in the same order on every
// run.  The launch is persistent over the colour's list of tiles (the items
// that open them), one workgroup per resident slot.
constexpr int kOwnerWaves = 2;
constexpr int kColourCount = 3, kColourNext = 9;  // counters: tiles per colour, places handed out

template <int TP, int TT>
constexpr int owner_colours_p()
{
    return (TP + kHaloP + TP - 1) / TP;
}
template <int TT>
constexpr int owner_colours_t()
{
    return (region_cols<TT>() + TT - 1) / TT;
}

// Add a complete region to the grid (one workgroup of NT threads, exclusive
// owner of the region's cells): quads wholly inside the grid as 16-byte
// read-add-writes when rows are whole float4 words, the others cell by cell.
// The region is the sum of the NW wavefronts' copies, taken in wavefront
// order.  Each thread's grid values are all loaded before any is stored, so
// that the loads are in flight together.
template <int RP, int RT, int NW, int NT>
__device__ __forceinline__ void owner_flush(const float4 *acc4, gptr<float> grid, int Np, int Nt,
                                            int p0, int c0)
{
    constexpr int RQ = RT / 4, NQ = (RP * RQ + NT - 1) / NT;
    const bool vec = (Nt & 3) == 0;
    float4 a[NQ], g[NQ];
    int64_t off[NQ];
    bool whole[NQ], any[NQ];
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        const int x = threadIdx.x + NT * u;
        const int r = x / RQ, q = x - r * RQ;
        const int I = p0 + r, J = c0 + 4 * q;
        const bool in = x < RP * RQ && I < Np && J < Nt;
        a[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (in) {
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const float4 v = acc4[w * RP * RQ + x];
                a[u] = make_float4(a[u].x + v.x, a[u].y + v.y, a[u].z + v.z, a[u].w + v.w);
            }
        }
        any[u] = in && (a[u].x != 0.0f || a[u].y != 0.0f || a[u].z != 0.0f || a[u].w != 0.0f);
        whole[u] = vec && J + 3 < Nt;
        off[u] = (int64_t)I * Nt + J;
        g[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (any[u] && whole[u])
            g[u] = *(const gptr<float4>)(grid + off[u]);
    }
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        if (!any[u])
            continue;
        if (whole[u]) {
            *(gptr<float4>)(grid + off[u]) =
                make_float4(g[u].x + a[u].x, g[u].y + a[u].y, g[u].z + a[u].z, g[u].w + a[u].w);
        } else {
            const int J = (int)(off[u] % Nt);
            const float v[4] = {a[u].x, a[u].y, a[u].z, a[u].w};
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (v[m] != 0.0f && J + m < Nt)
                    grid[off[u] + m] = grid[off[u] + m] + v[m];
        }
    }
}

// Lists of the items that open a tile, by colour: counts (counters[kColourCount
// + c]), then each item's place behind the counts of the smaller colours
// (counters[kColourNext + c] hands out places; the order within a colour does
// not matter: its tiles are independent).
template <int TP, int TT, bool B, bool SCATTER>
__global__ __launch_bounds__(256) void k_owner_lists(const int4 *__restrict__ items,
                                                     int32_t *counters,
                                                     const int32_t *__restrict__ tile_off,
                                                     EventCtx e0, BatchTables bt,
                                                     int32_t *colour_list)
{
    constexpr int CP = owner_colours_p<TP, TT>(), CT = owner_colours_t<TT>();
    const int nitems_all = counters[2];
    const int lane = threadIdx.x & 63;
    const int stride = gridDim.x * blockDim.x;
    // whole wavefronts iterate together: one atomic per colour per wavefront
    for (int i0 = blockIdx.x * blockDim.x + (threadIdx.x & ~63); i0 < nitems_all; i0 += stride) {
        const int itm = i0 + lane;
        int c = -1;
        if (itm < nitems_all) {
            const int4 it = items[itm];
            if (it.y == tile_off[it.x]) {  // the tile's first item
                const EventCtx &E = B ? bt.ev[find_event(bt.tile_base, bt.nev, it.x)] : e0;
                const int local = it.x - E.tile_base;
                const int tp = local / E.ntt, tt = local - tp * E.ntt;
                c = (tp % CP) * CT + tt % CT;
            }
        }
        int base = 0;
        if (SCATTER)
            for (int u = 0; u < CP * CT; ++u)
                base += (u < c) ? counters[kColourCount + u] : 0;
        for (int u = 0; u < CP * CT; ++u) {
            const uint64_t m = __ballot(c == u);
            if (!m)
                continue;
            const int leader = __ffsll((unsigned long long)m) - 1;
            int first = 0;
            if (lane == leader)
                first = atomicAdd(&counters[(SCATTER ? kColourNext : kColourCount) + u],
                                  __popcll(m));
            first = __shfl(first, leader);
            if (SCATTER && c == u)
                colour_list[base + first + __popcll(m & lanemask_lt(lane))] = itm;
        }
    }
}

template <int TP, int TT, bool B, bool FLUCT>
__global__ __launch_bounds__(64 * kOwnerWaves) void k_raster_owner(
    const float *__restrict__ records, const int4 *__restrict__ items,
    const int32_t *__restrict__ counters, const int32_t *__restrict__ colour_list, EventCtx e0,
    BatchTables bt, int colour_p, int colour_t)
{
    constexpr int RP = TP + kHaloP, RT = region_cols<TT>(), NW = kOwnerWaves;
    constexpr int CP = owner_colours_p<TP, TT>(), CT = owner_colours_t<TT>();
    static_assert(CP * TP >= RP && CT * TT >= RT, "regions of one colour must be disjoint");
    constexpr int RQ4 = RP * RT / 4;
    __shared__ float4 acc4[NW * RQ4];
    __shared__ double xsum[NW * kBatchItems];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nitems_all = counters[2];
    const int colour = colour_p * CT + colour_t;
    int base = 0;
    for (int c = 0; c < colour; ++c)
        base += counters[kColourCount + c];
    const int ntiles_c = counters[kColourCount + colour];
    for (int k = blockIdx.x; k < ntiles_c; k += gridDim.x) {
        const int itm = colour_list[base + k];
        const int tile = items[itm].x;
        const EventCtx &E = B ? bt.ev[find_event(bt.tile_base, bt.nev, tile)] : e0;
        const int local = tile - E.tile_base;
        const int tp = local / E.ntt, tt = local - tp * E.ntt;
        float4 *mine = acc4 + w * RQ4;
        for (int x = lane; x < RQ4; x += 64)
            mine[x] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        wave_lds_sync();
        for (int j = itm + w; j < nitems_all; j += NW) {
            const int4 it = items[j];
            if (it.x != tile)
                break;
            raster_item<TP, TT, B, FLUCT, true>(mine, xsum + w * kBatchItems, it, records, e0, bt);
        }
        __syncthreads();  // every copy of the region is complete
        owner_flush<RP, RT, NW, 64 * NW>(acc4, glb(E.grid), E.kp.Np, E.kp.Nt, tp * TP, tt * TT);
        __syncthreads();  // the copies are read before the next tile clears them
    }
}

// Descriptor of a single event (kernel argument; no table lookups).
EventCtx single_event(const wcsim_plane *pl, const wcsim_depo *depos, int64_t n,
                      uint64_t event_id, float *grid, uint8_t *occ = nullptr)
{
    EventCtx e{};
    e.kp = pl->kp;
    e.depos = depos;
    e.grid = grid;
    e.occ = occ;
    e.occ_shift = occ_shift_of(pl->Nt);
    e.depo_base = 0;
    e.n = (int32_t)n;
    e.event = (uint32_t)event_id;
    e.tile_base = 0;
    e.ntt = pl->ntt;
    return e;
}

unsigned blocks_for(int64_t n, int threads)
{
    return (unsigned)((n + threads - 1) / threads);
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
TileShape tile_shape(int id)
{
    switch (id) {
    case 1:
        return {32, 32, kHaloP, kHaloT};
    case 2:
        return {64, 8, kHaloP, kHaloT};
    default:
        return {32, 8, kHaloP, kHaloT};
    }
}

hipError_t launch_fill_zero(void *ptr, size_t bytes, hipStream_t s)
{
    if (bytes == 0)
        return hipSuccess;
    const size_t n16 = bytes / 16;
    if (n16) {
        const unsigned blocks = (unsigned)std::min<size_t>((n16 + 255) / 256, 8192);
        hipLaunchKernelGGL(k_fill_zero16, dim3(blocks), dim3(256), 0, s, (uint4 *)ptr, n16);
    }
    const size_t rem = bytes - n16 * 16;
    if (rem)
        hipLaunchKernelGGL(k_fill_zero1, dim3(1), dim3(16), 0, s, (unsigned char *)ptr + n16 * 16,
                           rem);
    return hipGetLastError();
}

// One thread per four consecutive samples of a row (one Philox call).  The
// deviates are evaluated in FP64 and rounded once to float32, the decision is
// taken in float32 in the order the definition states.
__global__ __launch_bounds__(256) void k_digitize(const float *__restrict__ wave, int64_t nrows,
                                                  int64_t ncols, float gain, float pedestal,
                                                  float sigma, float top, uint32_t k0, uint32_t k1,
                                                  uint32_t event, uint16_t *__restrict__ adc)
{
#pragma clang fp contract(off)
    const int64_t nq = (ncols + 3) / 4;
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= nrows * nq)
        return;
    const int64_t row = g / nq, q = g - row * nq;
    float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (sigma > 0.0f) {
        const uint4 r = philox4x32_10(make_uint4((uint32_t)q, (uint32_t)row, 0u, event), k0, k1);
        double zd[4];
        box_muller_d(r.x, r.y, zd[0], zd[1]);
        box_muller_d(r.z, r.w, zd[2], zd[3]);
#pragma unroll
        for (int m = 0; m < 4; ++m)
            z[m] = (float)zd[m];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int64_t col = 4 * q + m;
        if (col < ncols) {
            const int64_t i = row * ncols + col;
            float v = wave[i] * gain;
            v = v + pedestal;
            v = v + sigma * z[m];
            v = fminf(fmaxf(rintf(v), 0.0f), top);
            adc[i] = (uint16_t)v;
        }
    }
}

hipError_t launch_digitize(const float *wave, int64_t nrows, int64_t ncols, float gain,
                           float pedestal, float sigma, int bits, uint64_t seed, uint32_t event,
                           uint16_t *adc, hipStream_t s)
{
    const int64_t n = nrows * ((ncols + 3) / 4);
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_digitize, dim3(blocks_for(n, 256)), dim3(256), 0, s, wave, nrows, ncols,
                       gain, pedestal, sigma, (float)((1 << bits) - 1),
                       (uint32_t)seed ^ 0x6e6f6973u, (uint32_t)(seed >> 32), event, adc);
    return hipGetLastError();
}

// Coloured noise: a workgroup takes 1024 columns of one row, draws the white
// deviates of those columns and of the nfir - 1 before them into LDS in FP64
// (one Philox call per quad, as k_digitize), then each thread filters four of
// the columns (FP64 taps and sums in LDS and registers), rounds the filtered
// noise once to float32 and digitises.
constexpr int kFirCols = 1024;
__global__ __launch_bounds__(256) void k_digitize_fir(const float *__restrict__ wave, int64_t nrows,
                                                      int64_t ncols, float gain, float pedestal,
                                                      float sigma, const float *__restrict__ fir,
                                                      int nfir, float top, uint32_t k0,
                                                      uint32_t k1, uint32_t event,
                                                      uint16_t *__restrict__ adc)
{
#pragma clang fp contract(off)
    __shared__ double h[kMaxFir];
    __shared__ double z[kFirCols + kMaxFir + 4];
    const int64_t tiles = (ncols + kFirCols - 1) / kFirCols;
    const int64_t row = blockIdx.x / tiles;
    const int64_t t0 = (blockIdx.x - row * tiles) * kFirCols;
    // z[i] holds the deviate of column base + i; base is a multiple of four
    const int64_t first = t0 - (nfir - 1);
    const int64_t base = (first >= 0) ? (first & ~(int64_t)3) : -((-first + 3) & ~(int64_t)3);
    const int64_t end = min(t0 + kFirCols, ncols);
    const int nz = (int)(end - base);
    for (int k = threadIdx.x; k < nfir; k += blockDim.x)
        h[k] = (double)fir[k];
    for (int qi = threadIdx.x; 4 * qi < nz; qi += blockDim.x) {
        const int64_t c = base + 4 * qi;  // first column of the quad
        double zz[4] = {0.0, 0.0, 0.0, 0.0};
        if (c >= 0 && sigma > 0.0f) {
            const uint4 r =
                philox4x32_10(make_uint4((uint32_t)(c >> 2), (uint32_t)row, 0u, event), k0, k1);
            box_muller_d(r.x, r.y, zz[0], zz[1]);
            box_muller_d(r.z, r.w, zz[2], zz[3]);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
            z[4 * qi + m] = zz[m];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kFirCols / 256; ++m) {
        const int64_t col = t0 + threadIdx.x + 256 * m;
        if (col >= ncols)
            break;
        double n = 0.0;
        const int kmax = (int)min((int64_t)nfir - 1, col);
        const int zi = (int)(col - base);
        for (int k = 0; k <= kmax; ++k)
            n = fma(h[k], z[zi - k], n);
        const int64_t i = row * ncols + col;
        float v = wave[i] * gain;
        v = v + pedestal;
        v = v + sigma * (float)n;
        v = fminf(fmaxf(rintf(v), 0.0f), top);
        adc[i] = (uint16_t)v;
    }
}

hipError_t launch_digitize_fir(const float *wave, int64_t nrows, int64_t ncols, float gain,
                               float pedestal, float sigma, const float *fir, int nfir, int bits,
                               uint64_t seed, uint32_t event, uint16_t *adc, hipStream_t s)
{
    const int64_t blocks = nrows * ((ncols + kFirCols - 1) / kFirCols);
    if (blocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_digitize_fir, dim3((unsigned)blocks), dim3(256), 0, s, wave, nrows, ncols,
                       gain, pedestal, sigma, fir, nfir, (float)((1 << bits) - 1),
                       (uint32_t)seed ^ 0x6e6f6973u, (uint32_t)(seed >> 32), event, adc);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, const uint32_t *key, int64_t n, uint32_t *out,
                         hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3(blocks_for(n, 256)), dim3(256), 0, s, (const uint4 *)ctr,
                       (const uint2 *)key, n, (uint4 *)out);
    return hipGetLastError();
}

size_t scan_scratch_bytes(int64_t n)
{
    return align_up(sizeof(int64_t) * (size_t)((n + kScanBlock - 1) / kScanBlock + 1));
}

hipError_t launch_exclusive_scan_i64(int64_t *data, int64_t n, void *scratch, hipStream_t s)
{
    return exclusive_scan<int64_t>(data, n, scratch, s);
}

hipError_t launch_exclusive_scan_i32(int32_t *data, int64_t n, void *scratch, hipStream_t s)
{
    return exclusive_scan<int32_t>(data, n, scratch, s);
}

hipError_t launch_patch_sizes(const wcsim_plane *pl, const wcsim_depo *depos, int64_t n,
                              int32_t *meta, int64_t *sizes, hipStream_t s)
{
    hipLaunchKernelGGL(k_patch_sizes, dim3(blocks_for(std::max<int64_t>(n, 1), 256)), dim3(256), 0,
                       s, depos, n, pl->kp, meta, sizes);
    return hipGetLastError();
}

hipError_t launch_patch_values(const wcsim_plane *pl, const wcsim_depo *depos, int64_t n,
                               uint64_t event_id, const int32_t *meta, const int64_t *offsets,
                               float *values, hipStream_t s)
{
    (void)meta;
    if (n <= 0)
        return hipSuccess;
    const unsigned grid = (unsigned)std::min<int64_t>(n, 1 << 20);
    const EventCtx e0 = single_event(pl, depos, n, event_id, nullptr);
    hipLaunchKernelGGL((k_patch_generic<64, true, false>), dim3(grid), dim3(64), 0, s, e0,
                       BatchTables{}, nullptr, nullptr, n, offsets, values);
    return hipGetLastError();
}

hipError_t launch_scatter_flat(const wcsim_plane *pl, int64_t n, const int32_t *meta,
                               const int64_t *offsets, const float *values, float *grid,
                               hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_scatter_flat, dim3(blocks_for(n, 4)), dim3(256), 0, s, n, meta, offsets,
                       values, grid, (int)pl->Np, (int)pl->Nt);
    return hipGetLastError();
}

// Blocks of the record kernel that clear the occupied blocks of the grids:
// one per band of grid rows (300 for a 9600-row plane), at most this many.
constexpr int kMaxClearBlocks = 4096;

static size_t sched_blocks_of(int64_t ntiles)
{
    return (size_t)((ntiles + 1 + kSchedTiles - 1) / kSchedTiles);
}

static size_t items_cap(int64_t ntiles, int64_t n)
{
    return (size_t)ntiles + (size_t)(std::max<int64_t>(n, 1) / kChunk) + 1;
}

// Wavefronts of the raster launch: enough for the work lists of track-like
// and uniform depo sets (a work item holds up to kChunk depos of one tile;
// the collection plane's 500,000 depos make 29,129 items), never more than
// the worst case; any further items are taken by a second round.
static unsigned raster_grid(int64_t ntiles, int64_t n)
{
    return (unsigned)std::min<size_t>(items_cap(ntiles, n), (size_t)(n / 8) + 4096);
}

// Counters: [0..2] as RasterWork states, then the sort's digit totals.
constexpr int kCounterWords = 64;
constexpr size_t kCounterBytes = sizeof(int32_t) * (kCounterWords + 256);

// The tile-list sort works in the record area before the records are written:
// keys and depo indices twice (ping-pong) and the per-block digit counts.
static size_t sort_blocks_of(size_t n) { return (n + kSortBlock - 1) / kSortBlock; }
static size_t sort_bytes(size_t n)
{
    return 4 * align_up(sizeof(int32_t) * n) + align_up(sizeof(int32_t) * 256 * sort_blocks_of(n));
}

size_t raster_work_bytes_batch(const wcsim_plane *pl, int64_t n, int64_t ntiles, int64_t nbands)
{
    (void)pl;
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    return align_up(kCounterBytes) + align_up(sizeof(int32_t) * (size_t)(ntiles + 1)) +
           align_up((size_t)kOccCols * (size_t)nbands) +
           align_up(sizeof(int2) * sched_blocks_of(ntiles)) +
           align_up(sizeof(int4) * items_cap(ntiles, n)) + 3 * align_up(sizeof(int32_t) * nn) +
           align_up(std::max(sizeof(float) * kRecWords * nn, sort_bytes(nn)));
}

RasterWork raster_work_carve_batch(const wcsim_plane *pl, int64_t n, int64_t ntiles,
                                   int64_t nbands, void *base)
{
    (void)pl;
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    char *p = (char *)base;
    RasterWork w;
    w.counters = (int32_t *)p;
    w.sort_tot = w.counters + kCounterWords;
    p += align_up(kCounterBytes);
    w.tile_count = (int32_t *)p;
    p += align_up(sizeof(int32_t) * (size_t)(ntiles + 1));
    w.occ = (uint8_t *)p;  // adjacent to the counters: cleared together
    p += align_up((size_t)kOccCols * (size_t)nbands);
    w.block_tot = (int2 *)p;
    p += align_up(sizeof(int2) * sched_blocks_of(ntiles));
    w.items = (int4 *)p;
    p += align_up(sizeof(int4) * items_cap(ntiles, n));
    w.depo_tile = (int32_t *)p;
    p += align_up(sizeof(int32_t) * nn);
    w.depo_slot = (int32_t *)p;
    p += align_up(sizeof(int32_t) * nn);
    w.large = (int32_t *)p;
    p += align_up(sizeof(int32_t) * nn);
    w.records = (float *)p;
    return w;
}

size_t raster_work_bytes(const wcsim_plane *pl, int64_t n)
{
    return raster_work_bytes_batch(pl, n, pl->ntiles, occ_bands(pl->Np));
}

RasterWork raster_work_carve(const wcsim_plane *pl, int64_t n, void *base)
{
    return raster_work_carve_batch(pl, n, pl->ntiles, occ_bands(pl->Np), base);
}

// Compute units of the current device (cached per device).
static int device_cus()
{
    static std::atomic<int> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 256;
    int v = cus[dev].load(std::memory_order_relaxed);
    if (v <= 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            v <= 0)
            v = 256;
        cus[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

// The colour lists (in depo_tile, free once the records are written: a tile
// list has at most n items), then one launch per colour of the owner flush,
// colours in row-major order, each with as many workgroups as the device
// holds at once (LDS-bound).
template <int TP, int TT, bool B, bool FLUCT>
static void launch_owner_phases(unsigned items_grid, const RasterWork &w, const EventCtx &e0,
                                const BatchTables &bt, hipStream_t s)
{
    const unsigned lg = std::max(1u, std::min(items_grid / 4, 2048u));
    hipLaunchKernelGGL((k_owner_lists<TP, TT, B, false>), dim3(lg), dim3(256), 0, s, w.items,
                       w.counters, w.tile_count, e0, bt, w.depo_tile);
    hipLaunchKernelGGL((k_owner_lists<TP, TT, B, true>), dim3(lg), dim3(256), 0, s, w.items,
                       w.counters, w.tile_count, e0, bt, w.depo_tile);
    constexpr size_t lds = sizeof(float4) * kOwnerWaves * (TP + kHaloP) * region_cols<TT>() / 4 +
                           sizeof(double) * kOwnerWaves * kBatchItems;
    const unsigned per_cu = (unsigned)std::max<size_t>(1, (160 * 1024) / lds);
    const unsigned grid = (unsigned)device_cus() * per_cu;
    for (int cp = 0; cp < owner_colours_p<TP, TT>(); ++cp)
        for (int ct = 0; ct < owner_colours_t<TT>(); ++ct)
            hipLaunchKernelGGL((k_raster_owner<TP, TT, B, FLUCT>), dim3(grid),
                               dim3(64 * kOwnerWaves), 0, s, w.records, w.items, w.counters,
                               w.depo_tile, e0, bt, cp, ct);
}

template <bool B, bool FLUCT>
static void launch_raster_owner(int tile, unsigned grid, const RasterWork &w, const EventCtx &e0,
                                const BatchTables &bt, hipStream_t s)
{
    switch (tile) {
    case 1:
        launch_owner_phases<32, 32, B, FLUCT>(grid, w, e0, bt, s);
        break;
    case 2:
        launch_owner_phases<64, 8, B, FLUCT>(grid, w, e0, bt, s);
        break;
    default:
        launch_owner_phases<32, 8, B, FLUCT>(grid, w, e0, bt, s);
        break;
    }
}

// Tile lists in depo order: sort, then slots and the ordered large-patch list.
static void launch_tile_list_sort(int64_t n, int64_t ntiles, const RasterWork &w, hipStream_t s)
{
    const size_t nn = (size_t)n;
    char *p = (char *)w.records;
    uint32_t *kA = (uint32_t *)p;
    p += align_up(sizeof(int32_t) * nn);
    uint32_t *kB = (uint32_t *)p;
    p += align_up(sizeof(int32_t) * nn);
    int32_t *vA = (int32_t *)p;
    p += align_up(sizeof(int32_t) * nn);
    int32_t *vB = (int32_t *)p;
    p += align_up(sizeof(int32_t) * nn);
    int32_t *counts = (int32_t *)p;
    const unsigned nblk = (unsigned)sort_blocks_of(nn);
    const uint32_t nt = (uint32_t)ntiles;
    int bits = 1;
    while (bits < 32 && ((uint64_t)nt + 1) >> bits)
        ++bits;
    hipLaunchKernelGGL(k_sort_keys, dim3(blocks_for(n, 256)), dim3(256), 0, s, w.depo_tile, n, nt,
                       kA, vA);
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_sort_count, dim3(nblk), dim3(kSortThreads), 0, s, kA, n, shift,
                           counts, w.sort_tot);
        hipLaunchKernelGGL(k_sort_offsets, dim3(1), dim3(kSortThreads), 0, s, counts, (int)nblk,
                           w.sort_tot);
        hipLaunchKernelGGL(k_sort_scatter, dim3(nblk), dim3(kSortThreads), 0, s, kA, vA, n, shift,
                           counts, kB, vB);
        std::swap(kA, kB);
        std::swap(vA, vB);
    }
    hipLaunchKernelGGL(k_sort_slots, dim3(blocks_for(n, 256)), dim3(256), 0, s, kA, vA, n, nt,
                       w.tile_count, w.depo_slot, w.large);
}

template <bool B, bool FLUCT>
static void launch_raster_tiles(int tile, unsigned grid, const RasterWork &w, const EventCtx &e0,
                                const BatchTables &bt, hipStream_t s)
{
    switch (tile) {
    case 1:
        hipLaunchKernelGGL((k_raster_tiles<32, 32, B, FLUCT>), dim3(grid), dim3(64), 0, s,
                           w.records, w.items, w.counters, e0, bt);
        break;
    case 2:
        hipLaunchKernelGGL((k_raster_tiles<64, 8, B, FLUCT>), dim3(grid), dim3(64), 0, s,
                           w.records, w.items, w.counters, e0, bt);
        break;
    default:
        hipLaunchKernelGGL((k_raster_tiles<32, 8, B, FLUCT>), dim3(grid), dim3(64), 0, s,
                           w.records, w.items, w.counters, e0, bt);
        break;
    }
}

// The launch sequence shared by single events and batches: clear counters,
// window + tile per depo, tile schedule, depo records, LDS-tiled raster,
// large-patch raster.  `ev` (single events only) receives three stage marks.
template <bool B>
static hipError_t raster_sequence(const wcsim_plane *pl, const EventCtx &e0,
                                  const BatchTables &bt, int64_t n, int64_t ntiles,
                                  int64_t nbands, const RasterWork &w, hipStream_t s,
                                  const hipEvent_t *ev)
{
    hipError_t e;
    auto mark = [&](int i) { return ev ? hipEventRecord(ev[i], s) : hipSuccess; };
    // counters, tile counts and occupancy maps are adjacent: one clear
    const size_t clear = (size_t)((char *)w.occ - (char *)w.counters) +
                         (size_t)kOccCols * (size_t)nbands;
    if ((e = launch_fill_zero(w.counters, align_up(clear, 16), s)) != hipSuccess)
        return e;
    if (n <= 0) {  // an empty map: nothing of the grid is read
        for (int i = 0; i < 3; ++i)
            if ((e = mark(i)) != hipSuccess)
                return e;
        return hipSuccess;
    }
    TileGeom g;
    g.tp = pl->ts.tp;
    g.tt = pl->ts.tt;
    g.rp = pl->ts.tp + kHaloP;
    g.rt = pl->ts.tt + kHaloT;
    g.ntt = pl->ntt;
    hipLaunchKernelGGL(k_prep_bin<B>, dim3(blocks_for(n, 256)), dim3(256), 0, s, e0, bt, n, g,
                       w.counters, w.tile_count, w.depo_tile, w.depo_slot, w.large);
    const unsigned sched_blocks = (unsigned)sched_blocks_of(ntiles);
    hipLaunchKernelGGL(k_tile_sums, dim3(sched_blocks), dim3(kSchedThreads), 0, s, w.tile_count,
                       (int)ntiles, w.block_tot);
    hipLaunchKernelGGL(k_scan_block_tot, dim3(1), dim3(kSchedThreads), 0, s, w.block_tot,
                       (int)sched_blocks);
    hipLaunchKernelGGL(k_tile_schedule, dim3(sched_blocks), dim3(kSchedThreads), 0, s,
                       w.tile_count, (int)ntiles, w.block_tot, w.items, w.counters);
    if (pl->det)
        launch_tile_list_sort(n, ntiles, w, s);
    // clearing blocks: one per band of grid rows, at most kMaxClearBlocks
    const int nclr = (int)std::min<int64_t>(kMaxClearBlocks, nbands);
    hipLaunchKernelGGL(k_fill_records<B>, dim3(blocks_for(n, 64) + nclr), dim3(128), 0, s, e0, bt,
                       n, w.depo_tile, w.depo_slot, w.tile_count, w.records, (int)nbands, nclr);
    if ((e = hipGetLastError()) != hipSuccess || (e = mark(0)) != hipSuccess)
        return e;
    const unsigned grid_items = raster_grid(ntiles, n);
    if (pl->det && pl->kp.fluct)
        launch_raster_owner<B, true>(pl->tile, grid_items, w, e0, bt, s);
    else if (pl->det)
        launch_raster_owner<B, false>(pl->tile, grid_items, w, e0, bt, s);
    else if (pl->kp.fluct)
        launch_raster_tiles<B, true>(pl->tile, grid_items, w, e0, bt, s);
    else
        launch_raster_tiles<B, false>(pl->tile, grid_items, w, e0, bt, s);
    if ((e = hipGetLastError()) != hipSuccess || (e = mark(1)) != hipSuccess)
        return e;
    // Depos whose patch does not fit a tile region: one workgroup each, direct
    // atomics.  The grid is persistent over the device-side count, one
    // workgroup per CU (most workloads have no such depo, and each workgroup
    // holds 17 KB of LDS while it looks).  With reproducible sums one
    // workgroup adds the patches one after another in depo order (a patch's
    // bins are distinct; its atomics complete before the next patch's).
    const unsigned lg = pl->det ? 1u : (unsigned)std::min<int64_t>(n, 256);
    hipLaunchKernelGGL((k_patch_generic<256, false, B>), dim3(lg), dim3(256), 0, s, e0, bt,
                       w.large, w.counters + 1, (int64_t)0, nullptr, nullptr);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    return mark(2);
}

hipError_t launch_raster_fused(const wcsim_plane *pl, const wcsim_depo *depos, int64_t n,
                               uint64_t event_id, const RasterWork &w, float *grid, hipStream_t s,
                               const hipEvent_t *ev)
{
    const EventCtx e0 = single_event(pl, depos, n, event_id, grid, w.occ);
    return raster_sequence<false>(pl, e0, BatchTables{}, n, pl->ntiles, occ_bands(pl->Np), w, s,
                                  ev);
}

hipError_t launch_raster_batch(const wcsim_plane *pl, const BatchTables &bt, int64_t n_total,
                               int64_t ntiles_total, int64_t nbands_total, const RasterWork &w,
                               hipStream_t s, const hipEvent_t *ev)
{
    return raster_sequence<true>(pl, EventCtx{}, bt, n_total, ntiles_total, nbands_total, w, s,
                                 ev);
}

// Zero the blocks that the occupancy map leaves unmarked (one wavefront per
// band of rows), so that the whole grid holds the event.
__global__ __launch_bounds__(64) void k_clear_unoccupied(float *grid, int Np, int Nt,
                                                         const uint8_t *occ, int shift)
{
    const int band = blockIdx.x, lane = threadIdx.x;
    const int nb = (Nt + (1 << shift) - 1) >> shift;
    const uint64_t valid = (nb >= 64) ? ~0ull : ((1ull << nb) - 1ull);
    const uint64_t m = __ballot(occ[band * kOccCols + lane] != 0);
    clear_blocks(glb(grid), Np, Nt, band, ~m & valid, shift, lane);
}

hipError_t launch_clear_unoccupied(float *grid, int Np, int Nt, const uint8_t *occ, int shift,
                                   hipStream_t s)
{
    if (Np <= 0 || Nt <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_clear_unoccupied, dim3((unsigned)occ_bands(Np)), dim3(64), 0, s, grid,
                       Np, Nt, occ, shift);
    return hipGetLastError();
}

}  // namespace wcs
