// FFT convolution of the plane grid with the detector response on gfx950
// (arXiv:2304.01841, Sec. 2 step 3, where the transforms carry the bulk of the
// convolution's work; the tick-axis inverse is a complex-to-real transform
// along axis 1, the idft_cr of Sec. 4.2).
//
// The grid is [Np][Nt] float32 (ticks contiguous).  The linear convolution
// out[p][t] = sum_r sum_s R[r][s] G[p + r0 - r][t - s] runs in three passes,
// each one HBM read and one HBM write of its operand:
//   A  tick-axis real FFT of every pitch row, zero-padded to N' = 2 N2 >=
//      Nt + Rt - 1 (no wrap-around), written as column chunks [C][Np][F] of
//      F consecutive frequencies so that the next pass reads whole chunks;
//   B  per frequency chunk and pitch block: overlap-save along pitch.  A block
//      of L rows (the V = L - Rp + 1 output rows plus Rp - 1 rows of history)
//      is transformed in LDS, multiplied by the resident response spectrum
//      K = DFT_{L x N'}(R) / (L N'), transformed back, and the V valid rows are
//      kept (all rows, or only each wire's centre impact row);
//   C  tick-axis inverse real FFT of every kept row, cropped to Nt ticks.
// No step is a dense contraction, so there is no MFMA: the transforms are
// mixed-radix (2, 3, 4, 5, 8) self-sorting Stockham passes over LDS, each pass
// staging its butterflies in registers between two barriers so one LDS buffer
// suffices.  Twiddles come from two small FP64-derived tables per transform
// size held in LDS (W^j = Hi[j / 64] Lo[j mod 64]), so no pass waits on global
// memory, and every global<->LDS copy issues its loads in batches.
#include <math.h>

#include <type_traits>
#include <vector>

#include "wcsim_internal.h"

namespace wcs {
namespace {

constexpr int kRegComplex = 32;  // complex values a thread stages per pass
constexpr int kTwLo = 64;        // low table of a two-level twiddle table

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }  // * (-i)
__device__ __forceinline__ float2 mul_pi(float2 a) { return make_float2(-a.y, a.x); }  // * (+i)
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// exp(-2 pi i j / n) from a two-level table in LDS: tab[0..63] = W^l,
// tab[64 + h] = W^(64 h).
__device__ __forceinline__ float2 tw_at(const float2 *tab, int j)
{
    return cmul(tab[kTwLo + (j >> 6)], tab[j & (kTwLo - 1)]);
}

// Forward DFTs of length R in registers: X_m = sum_t x_t exp(-2 pi i t m / R).
template <int R>
__device__ __forceinline__ void dft(float2 *x);

template <>
__device__ __forceinline__ void dft<2>(float2 *x)
{
    const float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
}

template <>
__device__ __forceinline__ void dft<4>(float2 *x)
{
    const float2 t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]);
    const float2 t2 = cadd(x[1], x[3]), t3 = mul_mi(csub(x[1], x[3]));
    x[0] = cadd(t0, t2);
    x[2] = csub(t0, t2);
    x[1] = cadd(t1, t3);
    x[3] = csub(t1, t3);
}

template <>
__device__ __forceinline__ void dft<8>(float2 *x)
{
    // Even outputs are the 4-point DFT of x_t + x_{t+4}; odd outputs the
    // 4-point DFT of (x_t - x_{t+4}) exp(-2 pi i t / 8).
    constexpr float c = 0.70710678118654752440f;
    float2 a[4], b[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        a[t] = cadd(x[t], x[t + 4]);
        b[t] = csub(x[t], x[t + 4]);
    }
    b[1] = make_float2(c * (b[1].x + b[1].y), c * (b[1].y - b[1].x));
    b[2] = mul_mi(b[2]);
    b[3] = make_float2(c * (b[3].y - b[3].x), -c * (b[3].x + b[3].y));
    dft<4>(a);
    dft<4>(b);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        x[2 * m] = a[m];
        x[2 * m + 1] = b[m];
    }
}

template <>
__device__ __forceinline__ void dft<3>(float2 *x)
{
    constexpr float h = 0.86602540378443864676f;  // sin(pi/3)
    const float2 s = cadd(x[1], x[2]);
    const float2 d = csub(x[1], x[2]);
    const float2 m = make_float2(x[0].x - 0.5f * s.x, x[0].y - 0.5f * s.y);
    const float2 r = make_float2(h * d.y, -h * d.x);  // -i sin(pi/3) d
    x[0] = cadd(x[0], s);
    x[1] = cadd(m, r);
    x[2] = csub(m, r);
}

template <>
__device__ __forceinline__ void dft<5>(float2 *x)
{
    constexpr float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
    constexpr float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
    constexpr float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
    constexpr float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
    const float2 b1 = cadd(x[1], x[4]), d1 = csub(x[1], x[4]);
    const float2 b2 = cadd(x[2], x[3]), d2 = csub(x[2], x[3]);
    const float2 x0 = x[0];
    const float2 e1 = make_float2(x0.x + c1 * b1.x + c2 * b2.x, x0.y + c1 * b1.y + c2 * b2.y);
    const float2 e2 = make_float2(x0.x + c2 * b1.x + c1 * b2.x, x0.y + c2 * b1.y + c1 * b2.y);
    // o1 = s1 d1 + s2 d2, o2 = s2 d1 - s1 d2; X1,4 = e1 -/+ i o1, X2,3 = e2 -/+ i o2
    const float2 o1 = make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y);
    const float2 o2 = make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y);
    x[0] = cadd(x0, cadd(b1, b2));
    x[1] = cadd(e1, mul_mi(o1));
    x[4] = csub(e1, mul_mi(o1));
    x[2] = cadd(e2, mul_mi(o2));
    x[3] = csub(e2, mul_mi(o2));
}

// 16 points as 4 x 4: t = 4 t1 + t2, m = m1 + 4 m2; 4-point DFTs over t1,
// the factors exp(-2 pi i t2 m1 / 16), then 4-point DFTs over t2.
template <>
__device__ __forceinline__ void dft<16>(float2 *x)
{
    constexpr float c1 = 0.92387953251128675613f;  // cos(pi/8)
    constexpr float s1 = 0.38268343236508977173f;  // sin(pi/8)
    constexpr float h = 0.70710678118654752440f;   // cos(pi/4)
    float2 a[4][4];
#pragma unroll
    for (int t2 = 0; t2 < 4; ++t2) {
        a[t2][0] = x[t2];
        a[t2][1] = x[4 + t2];
        a[t2][2] = x[8 + t2];
        a[t2][3] = x[12 + t2];
        dft<4>(a[t2]);
    }
    // a[t2][m1] *= W^(t2 m1), W = exp(-2 pi i / 16)
    auto w1 = [&](float2 v) { return make_float2(c1 * v.x + s1 * v.y, c1 * v.y - s1 * v.x); };
    auto w2 = [&](float2 v) { return make_float2(h * (v.x + v.y), h * (v.y - v.x)); };
    auto w3 = [&](float2 v) { return make_float2(s1 * v.x + c1 * v.y, s1 * v.y - c1 * v.x); };
    auto w6 = [&](float2 v) { return make_float2(h * (v.y - v.x), -h * (v.x + v.y)); };
    auto w9 = [&](float2 v) { return make_float2(-c1 * v.x - s1 * v.y, s1 * v.x - c1 * v.y); };
    a[1][1] = w1(a[1][1]);
    a[1][2] = w2(a[1][2]);
    a[1][3] = w3(a[1][3]);
    a[2][1] = w2(a[2][1]);
    a[2][2] = mul_mi(a[2][2]);  // W^4 = -i
    a[2][3] = w6(a[2][3]);
    a[3][1] = w3(a[3][1]);
    a[3][2] = w6(a[3][2]);
    a[3][3] = w9(a[3][3]);
#pragma unroll
    for (int m1 = 0; m1 < 4; ++m1) {
        float2 b[4] = {a[0][m1], a[1][m1], a[2][m1], a[3][m1]};
        dft<4>(b);
#pragma unroll
        for (int m2 = 0; m2 < 4; ++m2)
            x[m1 + 4 * m2] = b[m2];
    }
}

// Multiply x_t by w^t, t = 1..R-1 (powers by repeated products: a few ulp,
// far below the float32 transform error).
template <int R>
__device__ __forceinline__ void twiddle_powers(float2 *x, float2 w)
{
    float2 wt = w;
#pragma unroll
    for (int t = 1; t < R; ++t) {
        x[t] = cmul(x[t], wt);
        if (t + 1 < R)
            wt = (t == 1) ? cmul(w, w) : cmul(wt, w);
    }
}

// One self-sorting Stockham pass of radix R over `nseq` sequences of length N
// held in LDS (element x of sequence s at s*sstride + x*estride).  Sequence s
// of butterfly g is g mod nseq (nseq a power of two), so neighbouring threads
// touch neighbouring sequences.  With p the product of the radices already
// applied: butterfly i (k = i mod p) reads x[i + t N/R], multiplies by
// exp(-2 pi i t k / (p R)), runs the R-point DFT and writes y[(i-k) R + k + t p].
template <int R, int MAXB>
__device__ __forceinline__ void stockham_pass(float2 *buf, int N, int p, int nseq_shift,
                                              int sstride, int estride, const float2 *tab)
{
    const int nb = N / R;
    const int total = nb << nseq_shift;
    const int twstep = N / (p * R);
    const int nseq_mask = (1 << nseq_shift) - 1;
    float2 v[MAXB][R];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int g = threadIdx.x + b * blockDim.x;
        if (g < total) {
            const int s = g & nseq_mask, i = g >> nseq_shift;
            const float2 *src = buf + s * sstride + i * estride;
#pragma unroll
            for (int t = 0; t < R; ++t)
                v[b][t] = src[t * nb * estride];
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int g = threadIdx.x + b * blockDim.x;
        if (g < total) {
            const int s = g & nseq_mask, i = g >> nseq_shift;
            const int k = i % p;
            if (k != 0)
                twiddle_powers<R>(v[b], tw_at(tab, k * twstep));
            dft<R>(v[b]);
            float2 *dst = buf + s * sstride + ((i - k) * R + k) * estride;
#pragma unroll
            for (int t = 0; t < R; ++t)
                dst[t * p * estride] = v[b][t];
        }
    }
    __syncthreads();
}

// Forward transform of every sequence with a runtime plan.
__device__ void fft_lds(float2 *buf, const FftPlan &plan, int nseq_shift, int sstride,
                        int estride, const float2 *tab)
{
    int p = 1;
    for (int q = 0; q < plan.npass; ++q) {
        const int R = plan.radix[q];
        switch (R) {
        case 8:
            stockham_pass<8, kRegComplex / 8>(buf, plan.n, p, nseq_shift, sstride, estride, tab);
            break;
        case 4:
            stockham_pass<4, kRegComplex / 4>(buf, plan.n, p, nseq_shift, sstride, estride, tab);
            break;
        case 2:
            stockham_pass<2, kRegComplex / 2>(buf, plan.n, p, nseq_shift, sstride, estride, tab);
            break;
        case 5:
            stockham_pass<5, kRegComplex / 5>(buf, plan.n, p, nseq_shift, sstride, estride, tab);
            break;
        default:
            stockham_pass<3, kRegComplex / 3>(buf, plan.n, p, nseq_shift, sstride, estride, tab);
            break;
        }
        p *= R;
    }
}

// Marker for the default operand of a transform's first pass (input) or last
// pass (output): the LDS buffer itself.
struct InLds {};

// Runtime-plan transform as a policy object (any supported size).
struct FftRt {
    static constexpr int kMaxThreads = 1024;
    FftPlan plan;
    int nseq_shift, sstride, estride;
    __device__ __forceinline__ void run(float2 *buf, const float2 *tab) const
    {
        fft_lds(buf, plan, nseq_shift, sstride, estride, tab);
    }
    // Same contract as FftCt::run_io, by plain copies around run().
    template <class Load, class Store>
    __device__ __forceinline__ void run_io(float2 *buf, const float2 *tab, Load load,
                                           Store store) const
    {
        const int total = plan.n << nseq_shift, mask = (1 << nseq_shift) - 1;
        if constexpr (!std::is_same<Load, InLds>::value) {
            for (int g = threadIdx.x; g < total; g += blockDim.x)
                buf[(g & mask) * sstride + (g >> nseq_shift) * estride] =
                    load(g & mask, g >> nseq_shift);
            __syncthreads();
        }
        run(buf, tab);
        if constexpr (!std::is_same<Store, InLds>::value) {
            for (int g = threadIdx.x; g < total; g += blockDim.x)
                store(g & mask, g >> nseq_shift,
                      buf[(g & mask) * sstride + (g >> nseq_shift) * estride]);
        }
    }
};

// Compile-time Stockham pass: sizes, strides and the radix are constants, so
// the index arithmetic folds and the butterflies unroll.  With GLOAD the pass
// takes its inputs from load(s, n) (element n of sequence s) instead of LDS:
// the first pass of a transform reads global memory directly, all of its loads
// in flight together, with no separate copy into LDS.  With GSTORE it hands its
// outputs to store(s, n, value) instead of writing LDS; the caller then
// synchronises before LDS is used again.
// A store functor with a prefetch(s, n) member takes, besides the value, an
// operand it named in advance (a response-spectrum factor): the last pass
// issues those loads right after its read barrier, so that they are in
// flight during the butterflies instead of after them.
template <class S, class = void>
struct HasPrefetch : std::false_type {};
template <class S>
struct HasPrefetch<S, std::void_t<decltype(&S::prefetch)>> : std::true_type {};

template <int N, int R, int P, int NSS, int SS, int ES, int NT, bool GLOAD, bool GSTORE,
          class Load, class Store>
__device__ __forceinline__ void ct_pass(float2 *buf, const float2 *tab, Load &load, Store &store)
{
    constexpr int NB = N / R;
    constexpr int TOTAL = NB << NSS;
    constexpr int MAXB = (TOTAL + NT - 1) / NT;
    constexpr int TWSTEP = N / (P * R);
    constexpr int MASK = (1 << NSS) - 1;
    // Unguarded loads when at most 1/8 of them would be discarded.
    constexpr bool kLoadAll = 8 * (MAXB * NT - TOTAL) <= MAXB * NT;
    static_assert(!GLOAD || P == 1, "only the first pass reads its inputs from a loader");
    const int tid = threadIdx.x;
    float2 v[MAXB][R];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        if constexpr (GLOAD && kLoadAll) {
            // Threads past the last butterfly load a valid one's inputs and
            // discard them: no branch separates the loads of the MAXB
            // butterflies, so all of them are in flight together (loaders
            // select their padding instead of branching).
            const int g = min(tid + b * NT, TOTAL - 1);
            const int s = g & MASK, i = g >> NSS;
#pragma unroll
            for (int t = 0; t < R; ++t)
                v[b][t] = load(s, i + t * NB);
        } else {
            const int g = tid + b * NT;
            if ((TOTAL % NT) == 0 || g < TOTAL) {
                const int s = g & MASK, i = g >> NSS;
                if constexpr (GLOAD) {
#pragma unroll
                    for (int t = 0; t < R; ++t)
                        v[b][t] = load(s, i + t * NB);
                } else {
                    const float2 *src = buf + s * SS + i * ES;
#pragma unroll
                    for (int t = 0; t < R; ++t)
                        v[b][t] = src[t * NB * ES];
                }
            }
        }
    }
    if constexpr (!GLOAD)
        __syncthreads();  // every input is read before any output lands in LDS
    constexpr bool kPre = GSTORE && HasPrefetch<Store>::value;
    float2 pre[kPre ? MAXB : 1][kPre ? R : 1];
    if constexpr (kPre) {
#pragma unroll
        for (int b = 0; b < MAXB; ++b) {
            const int g = tid + b * NT;
            if ((TOTAL % NT) == 0 || g < TOTAL) {
                const int s = g & MASK, i = g >> NSS;
                const int k = (P == 1) ? 0 : i % P;
                const int n0 = (i - k) * R + k;
#pragma unroll
                for (int t = 0; t < R; ++t)
                    pre[b][t] = store.prefetch(s, n0 + t * P);
            }
        }
    }
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int g = tid + b * NT;
        if ((TOTAL % NT) == 0 || g < TOTAL) {
            const int s = g & MASK, i = g >> NSS;
            const int k = (P == 1) ? 0 : i % P;
            if (P > 1)
                twiddle_powers<R>(v[b], tw_at(tab, k * TWSTEP));
            dft<R>(v[b]);
            const int n0 = (i - k) * R + k;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                if constexpr (kPre)
                    store(s, n0 + t * P, v[b][t], pre[b][t]);
                else if constexpr (GSTORE)
                    store(s, n0 + t * P, v[b][t]);
                else
                    buf[s * SS + (n0 + t * P) * ES] = v[b][t];
            }
        }
    }
    if constexpr (!GSTORE)
        __syncthreads();
}

template <int N, int NSS, int SS, int ES, int NT, int P, class Load, class Store, int R,
          int... Rest>
__device__ __forceinline__ void ct_fft(float2 *buf, const float2 *tab, Load &load, Store &store)
{
    constexpr bool kLast = sizeof...(Rest) == 0;
    constexpr bool kLoad = P == 1 && !std::is_same<Load, InLds>::value;
    constexpr bool kStore = kLast && !std::is_same<Store, InLds>::value;
    ct_pass<N, R, P, NSS, SS, ES, NT, kLoad, kStore>(buf, tab, load, store);
    if constexpr (!kLast)
        ct_fft<N, NSS, SS, ES, NT, P * R, Load, Store, Rest...>(buf, tab, load, store);
}

// Compile-time transform as a policy object.  run(): LDS in, LDS out.
// run_io(load, store): either end may be a functor or InLds.
template <int N, int NSS, int SS, int ES, int NT, int... Rs>
struct FftCt {
    static constexpr int kThreads = NT;
    static constexpr int kMaxThreads = NT;
    __device__ __forceinline__ void run(float2 *buf, const float2 *tab) const
    {
        InLds in, out;
        ct_fft<N, NSS, SS, ES, NT, 1, InLds, InLds, Rs...>(buf, tab, in, out);
    }
    template <class Load, class Store>
    __device__ __forceinline__ void run_io(float2 *buf, const float2 *tab, Load load,
                                           Store store) const
    {
        ct_fft<N, NSS, SS, ES, NT, 1, Load, Store, Rs...>(buf, tab, load, store);
    }
};

// Copy loop with the global accesses of kBatch iterations issued together:
// value i = load(i) for i < total, then store(i, value).  A plain loop would
// wait for each load before the LDS store of the same iteration and expose the
// full memory latency once per iteration.
constexpr int kBatch = 8;
template <class LoadF, class StoreF>
__device__ __forceinline__ void batched_copy(int total, LoadF load, StoreF store)
{
    for (int i0 = threadIdx.x; i0 < total; i0 += kBatch * blockDim.x) {
        float2 v[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int i = i0 + b * blockDim.x;
            if (i < total)
                v[b] = load(i);
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int i = i0 + b * blockDim.x;
            if (i < total)
                store(i, v[b]);
        }
    }
}

// Twiddle tables (global) of a kernel, copied into LDS.  Both tables have at
// most blockDim.x entries (checked on the host).
struct TwTables {
    const float2 *a;
    int na;
    const float2 *b;
    int nb;
};

__device__ __forceinline__ void load_tables(const TwTables &t, float2 *la, float2 *lb)
{
    const int tid = threadIdx.x;
    const float2 va = (tid < t.na) ? t.a[tid] : make_float2(0.0f, 0.0f);
    const float2 vb = (t.b && tid < t.nb) ? t.b[tid] : make_float2(0.0f, 0.0f);
    if (tid < t.na)
        la[tid] = va;
    if (t.b && tid < t.nb)
        lb[tid] = vb;
}

// ---------------------------------------------------------------------------
// Pass A: tick-axis real FFT of rows.  Real rows of length ncols (zero padded
// to 2 N2) are packed as z_n = x_{2n} + i x_{2n+1}; Z = FFT_N2(z) gives
// X_k = E_k - i w^k D_k and X_{N2-k} = conj(E_k + i w^k D_k), with
// E_k = (Z_k + conj Z_{N2-k}) / 2, D_k = (Z_k - conj Z_{N2-k}) / 2 and
// w = exp(-2 pi i / N').  Output chunk layout X[c][row][f], k = c F + f,
// frequencies above N2 zero.
// LDS: rows [RPW][N2 + 1], then the N2 table, then the N' table.
// ---------------------------------------------------------------------------
// Rows of one tick-axis forward launch; in a batch, taken from the event that
// owns the workgroup.
struct R2CIo {
    const float *in;
    int nrows, ncols;
    int64_t in_stride;
    float2 *X;
    const uint8_t *occ;  // occupancy map of `in` (nullptr: every block is read)
    int occ_shift;
};

// Loads of grid blocks that the occupancy map leaves unmarked read this pair
// of zeros instead (one cached line for the whole launch).
__device__ const float2 g_zero_pair[1] = {};

template <class FFT, bool BATCH>
__global__ __launch_bounds__(FFT::kMaxThreads) void k_rows_r2c(R2CIo io, BatchTables bt, int N2,
                                                              FFT fft, TwTables tw, int F_shift,
                                                              int C, int rpw_shift)
{
    extern __shared__ float2 lds[];
    int blk = blockIdx.x;
    if (BATCH) {
        const int e = find_event(bt.rblk_base, bt.nev, blk);
        const EventCtx &E = bt.ev[e];
        io.in = E.grid;
        io.nrows = E.kp.Np;
        io.ncols = E.kp.Nt;
        io.in_stride = E.kp.Nt;
        io.X = E.X;
        io.occ = E.occ;
        io.occ_shift = E.occ_shift;
        blk -= bt.rblk_base[e];
    }
    const gptr<const float> in = glb(io.in);
    const int nrows = io.nrows, ncols = io.ncols;
    const int64_t in_stride = io.in_stride;
    const gptr<float2> X = glb(io.X);
    const int RPW = 1 << rpw_shift;
    const int S = N2 + 1;
    float2 *tabN2 = lds + RPW * S;
    float2 *tabH = tabN2 + tw.na;
    load_tables(tw, tabN2, tabH);
    const int row0 = blk * RPW;
    // Bit c of occ_m: ticks c 2^osh .. (c + 1) 2^osh - 1 of this workgroup's
    // band of rows are occupied (every bit set without a map; a shift of 31
    // sends every tick to bit 0).
    uint64_t occ_m = ~0ull;
    int osh = 31;
    if (io.occ) {
        occ_m = __ballot(io.occ[(row0 / kOccRows) * kOccCols + (threadIdx.x & 63)] != 0);
        osh = io.occ_shift;
        if (occ_m == 0) {  // no depo reaches this band of rows: zero spectra
            const int fmask = (1 << F_shift) - 1, cf = C << F_shift;
            for (int s = 0; s < RPW && row0 + s < nrows; ++s)
                for (int k = threadIdx.x; k < cf; k += blockDim.x)
                    X[(((int64_t)(k >> F_shift) * nrows + row0 + s) << F_shift) + (k & fmask)] =
                        make_float2(0.0f, 0.0f);
            return;
        }
    }
    // z_n of row s straight from global memory into the first pass.  Every
    // load is issued unconditionally from a clamped (valid) address and the
    // padding is selected afterwards, so the loads of a pass stay in flight
    // together instead of waiting on each other across branches.  Loads in
    // unoccupied blocks read the zero pair instead (the two ticks of a load
    // share a block: blocks are at least 64 ticks and t is even).
    auto load2 = [&](int s, int n) {  // even ncols and stride: one 8-byte load
        const int row = row0 + s, t = 2 * n;
        const int tc = min(t, ncols - 2);
        const gptr<const float> src = in + (int64_t)min(row, nrows - 1) * in_stride + tc;
        const bool occ = (occ_m >> (tc >> osh)) & 1ull;
        const float2 v = *(occ ? (gptr<const float2>)src : glb(g_zero_pair));
        const bool ok = row < nrows && t < ncols;
        return ok ? v : make_float2(0.0f, 0.0f);
    };
    auto load1 = [&](int s, int n) {
        const int row = row0 + s, t = 2 * n;
        const gptr<const float> src = in + (int64_t)min(row, nrows - 1) * in_stride;
        const int ta = min(t, ncols - 1), tb = min(t + 1, ncols - 1);
        const bool occ = (occ_m >> (ta >> osh)) & 1ull;
        const gptr<const float> zf = (gptr<const float>)glb(g_zero_pair);
        const float a = *(occ ? src + ta : zf), b = *(occ ? src + tb : zf);
        const bool ok = row < nrows;
        return make_float2((ok && t < ncols) ? a : 0.0f, (ok && t + 1 < ncols) ? b : 0.0f);
    };
    if ((ncols & 1) == 0 && (in_stride & 1) == 0)
        fft.run_io(lds, tabN2, load2, InLds{});
    else
        fft.run_io(lds, tabN2, load1, InLds{});
    // Unpacking straight to the output: the pair (k, N2 - k) goes from LDS to
    // its two chunk slots, and the padding frequencies above N2 get zeros.
    const int half = N2 / 2;
    const int F = 1 << F_shift;
    const int CF = C << F_shift;
    for (int s = 0; s < RPW; ++s) {
        const int row = row0 + s;
        if (row >= nrows)
            break;
        const float2 *b = lds + s * S;
        auto put = [&](int k, float2 v) {
            X[(((int64_t)(k >> F_shift) * nrows + row) << F_shift) + (k & (F - 1))] = v;
        };
        for (int k = threadIdx.x; k <= half; k += blockDim.x) {
            const int kn = (k == 0) ? 0 : N2 - k;
            const float2 Zk = b[k], Zn = b[kn];
            const float2 E = make_float2(0.5f * (Zk.x + Zn.x), 0.5f * (Zk.y - Zn.y));
            const float2 D = make_float2(0.5f * (Zk.x - Zn.x), 0.5f * (Zk.y + Zn.y));
            const float2 wD = cmul(tw_at(tabH, k), D);
            put(k, csub(E, mul_pi(wD)));
            put((k == 0) ? N2 : kn, conjf2(cadd(E, mul_pi(wD))));
        }
        for (int k = N2 + 1 + threadIdx.x; k < CF; k += blockDim.x)
            put(k, make_float2(0.0f, 0.0f));
    }
}

// ---------------------------------------------------------------------------
// Pass C: tick-axis inverse real FFT of rows, cropped to ncols ticks.
// Z_k = A_k + i conj(w^k) B_k with A_k = X_k + conj X_{N2-k},
// B_k = X_k - conj X_{N2-k}; the unnormalised inverse FFT_N2 of Z gives
// z_n = x_{2n} + i x_{2n+1}.  The inverse runs as a forward transform of
// conj(Z) (conj of the result).
// ---------------------------------------------------------------------------
struct C2RIo {
    const float2 *Y;
    int nrows;
    float *out;
    int ncols;
    int64_t out_stride;
};

template <class FFT, bool BATCH>
__global__ __launch_bounds__(FFT::kMaxThreads) void k_rows_c2r(C2RIo io, BatchTables bt, int N2,
                                                              FFT fft, TwTables tw, int F_shift,
                                                              int C, int rpw_shift)
{
    extern __shared__ float2 lds[];
    int blk = blockIdx.x;
    if (BATCH) {
        const int e = find_event(bt.cblk_base, bt.nev, blk);
        const EventCtx &E = bt.ev[e];
        io.Y = E.Y;
        io.nrows = E.nout;
        io.out = E.out;
        io.ncols = E.kp.Nt;
        io.out_stride = E.kp.Nt;
        blk -= bt.cblk_base[e];
    }
    const gptr<const float2> Y = glb(io.Y);
    const int nrows = io.nrows, ncols = io.ncols;
    const gptr<float> out = glb(io.out);
    const int64_t out_stride = io.out_stride;
    const int RPW = 1 << rpw_shift;
    const int S = N2 + 1;
    float2 *tabN2 = lds + RPW * S;
    float2 *tabH = tabN2 + tw.na;
    load_tables(tw, tabN2, tabH);
    const int row0 = blk * RPW;
    const int F = 1 << F_shift;
    const int total = C << (F_shift + rpw_shift);
    batched_copy(
        total,
        [&](int g) {
            const int f = g & (F - 1);
            const int s = (g >> F_shift) & (RPW - 1);
            const int c = g >> (F_shift + rpw_shift);
            const int row = row0 + s;
            if (row >= nrows)
                return make_float2(0.0f, 0.0f);
            const float2 v = Y[(((int64_t)c * nrows + row) << F_shift) + f];
            return v;
        },
        [&](int g, float2 v) {
            const int f = g & (F - 1);
            const int s = (g >> F_shift) & (RPW - 1);
            const int k = ((g >> (F_shift + rpw_shift)) << F_shift) + f;
            if (k <= N2)
                lds[s * S + k] = v;
        });
    __syncthreads();
    const int half = N2 / 2;
    for (int s = 0; s < RPW; ++s) {
        float2 *b = lds + s * S;
        for (int k = threadIdx.x; k <= half; k += blockDim.x) {
            const int kn = (k == 0) ? N2 : N2 - k;
            const float2 Xk = b[k], Xn = b[kn];
            const float2 A = make_float2(Xk.x + Xn.x, Xk.y - Xn.y);
            const float2 B = make_float2(Xk.x - Xn.x, Xk.y + Xn.y);
            const float2 wB = cmul(conjf2(tw_at(tabH, k)), B);
            b[k] = conjf2(cadd(A, mul_pi(wB)));
            if (k != 0)
                b[kn] = csub(A, mul_pi(wB));  // conj of conj(A - i conj(w) B)
        }
    }
    __syncthreads();
    const bool vec2 = ((ncols & 1) == 0) && ((out_stride & 1) == 0);
    // the last pass writes x_{2n}, x_{2n+1} of row s straight to global memory
    auto store = [&](int s, int n, float2 z) {
        const int row = row0 + s, t = 2 * n;
        if (row >= nrows || t >= ncols)
            return;
        const gptr<float> dst = out + (int64_t)row * out_stride;
        if (vec2) {
            *(gptr<float2>)(dst + t) = make_float2(z.x, -z.y);
        } else {
            dst[t] = z.x;
            if (t + 1 < ncols)
                dst[t + 1] = -z.y;
        }
    };
    fft.run_io(lds, tabN2, InLds{}, store);
}

// ---------------------------------------------------------------------------
// Pass B: pitch-axis overlap-save convolution of one frequency chunk.
//   mode 0: output every pitch row; mode 1: only row w*nimpact + nimpact/2 of
//   each wire (output row w); mode 2: response spectrum (forward transform of
//   rows 0..nrows_in-1 zero-padded to L, scaled, written as [c][L][F]).
// A workgroup takes Fb of the chunk's F columns (Fb < F when an L x F block
// would not leave room for two workgroups per CU).
// Workgroups are mapped XCD-major: workgroup b runs on XCD b mod 8, and the
// workgroups of one XCD walk the pitch blocks of one chunk before the next,
// the column parts of a block one after the other, so the chunk's response
// spectrum, the rows shared by neighbouring blocks and the other part of each
// row segment are re-read from that XCD's L2.
// Wire output with D = nimpact dividing L folds the inverse: the kept rows of
// a block are n = n0 + D w (n0 fixed by the block's first row), and
//   y[n0 + D w] = sum_{k'<L/D} Z[k'] exp(2 pi i k' w / (L/D)),
//   Z[k'] = exp(2 pi i k' n0 / L) sum_{j<D} P[k' + j L/D] exp(2 pi i j n0 / D),
// P the block spectrum times the response spectrum (which carries 1/(L N')).
// So the inverse runs at length L/D on the folded spectrum instead of L.
// LDS: the block [L][Fb], the folded block [L/D][Fb] (fold only), then the L
// table and the L/D table.
// ---------------------------------------------------------------------------
struct PitchIo {
    const float2 *X;
    int nrows_in;
    const float2 *K;
    float2 *Y;
    int nrows_out, nblocks, mode;
};

// Last forward pass of a pitch block: the value times the resident response
// spectrum (conjugated when the inverse runs as a forward transform), into LDS.
template <bool CONJ>
struct KMulStore {
    float2 *lds;
    const float2 *Kc;
    int F_shift, Fb_shift;
    __device__ __forceinline__ float2 prefetch(int s, int n) const
    {
        return Kc[(n << F_shift) + s];
    }
    __device__ __forceinline__ void operator()(int s, int n, float2 v, float2 k) const
    {
        const float2 r = cmul(v, k);
        lds[(n << Fb_shift) + s] = CONJ ? conjf2(r) : r;
    }
    __device__ __forceinline__ void operator()(int s, int n, float2 v) const
    {
        (*this)(s, n, v, prefetch(s, n));
    }
};

template <class FFT, class FFT2, bool BATCH>
__global__ __launch_bounds__(FFT::kMaxThreads) void k_pitch_conv(PitchIo io, BatchTables bt, int L,
                                                                int V, int Rp, int r0, int C,
                                                                int F_shift, int Fb_shift,
                                                                FFT fft, FFT2 fft2, TwTables tw,
                                                                int nimpact, int fold_ok,
                                                                float scale)
{
    extern __shared__ float2 lds[];
    int gblk = blockIdx.x;
    if (BATCH) {
        // every event's range is a multiple of 8 workgroups, so the XCD of a
        // workgroup is the same in global and event-local numbering
        const int e = find_event(bt.pblk_base, bt.nev, gblk);
        const EventCtx &E = bt.ev[e];
        io.X = E.X;
        io.nrows_in = E.kp.Np;
        io.K = E.K;
        io.Y = E.Y;
        io.nrows_out = E.nout;
        io.nblocks = E.nblocks;
        io.mode = E.mode;
        gblk -= bt.pblk_base[e];
    }
    const float2 *__restrict__ X = io.X;
    const int nrows_in = io.nrows_in, nrows_out = io.nrows_out, nblocks = io.nblocks;
    const int mode = io.mode;
    const float2 *__restrict__ K = io.K;
    float2 *__restrict__ Y = io.Y;
    const int parts_shift = F_shift - Fb_shift;  // parts of Fb columns per chunk
    const int xcd = gblk & 7, slot = gblk >> 3;
    const int hf = slot & ((1 << parts_shift) - 1), rest = slot >> parts_shift;
    const int lc = rest / nblocks, blk = rest - lc * nblocks;
    const int c = lc * 8 + xcd;
    if (c >= C)
        return;
    const int D = nimpact, L10 = L / D;
    const bool fold = fold_ok && mode == 1;
    const int LFb = L << Fb_shift;
    float2 *Z = lds + LFb;
    float2 *tabL = Z + (fold_ok ? (L10 << Fb_shift) : 0);
    float2 *tab2 = tabL + tw.na;
    float2 *wfold = tab2 + tw.nb;  // D fold twiddles when folding
    load_tables(tw, tabL, tab2);
    const int P0 = blk * V;
    // block row n0 is the first kept row (grid row = centre impact of a wire)
    const int n0 = ((D / 2 - P0 + Rp - 1) % D + D) % D;
    if (fold && (int)threadIdx.x < D) {
        // exp(+2 pi i (j n0 mod D) / D) for j = threadIdx.x, from FP64
        double sv, cv;
        sincospi(2.0 * (double)((threadIdx.x * n0) % D) / (double)D, &sv, &cv);
        wfold[threadIdx.x] = make_float2((float)cv, (float)sv);
    }
    const int in0 = (mode == 2) ? 0 : P0 + r0 - (Rp - 1);
    const int col0 = hf << Fb_shift;
    const float2 *src = X + ((int64_t)c * nrows_in << F_shift) + col0;
    // block row n, column s straight from global memory into the first pass
    auto load = [&](int s, int n) {
        const int row = in0 + n;
        return (row >= 0 && row < nrows_in) ? src[((int64_t)row << F_shift) + s]
                                            : make_float2(0.0f, 0.0f);
    };
    if (mode == 2) {
        float2 *dst = Y + ((int64_t)c * L << F_shift) + col0;
        fft.run_io(lds, tabL, load,
                   [&](int s, int n, float2 v) { dst[(n << F_shift) + s] = cscale(v, scale); });
        return;
    }
    const float2 *Kc = K + ((int64_t)c * L << F_shift) + col0;
    float2 *dst = Y + ((int64_t)c * nrows_out << F_shift) + col0;
    if (fold) {
        // forward transform times the response spectrum, then the fold
        fft.run_io(lds, tabL, load, KMulStore<false>{lds, Kc, F_shift, Fb_shift});
        __syncthreads();
        for (int t = threadIdx.x; t < (L10 << Fb_shift); t += blockDim.x) {
            const int kp = t >> Fb_shift, s = t & ((1 << Fb_shift) - 1);
            float2 acc = make_float2(0.0f, 0.0f);
            for (int j = 0; j < D; ++j)
                acc = cadd(acc, cmul(lds[((kp + j * L10) << Fb_shift) + s], wfold[j]));
            // conjugated: the inverse runs as a forward transform
            // (kp n0 < L10 D = L: no reduction needed)
            Z[t] = conjf2(cmul(acc, conjf2(tw_at(tabL, kp * n0))));
        }
        __syncthreads();
        // kept row n = n0 + D w is grid row p = P0 + n - (Rp - 1), output row
        // p / D = q0 + w (floor division, exact for every kept row)
        const int base = P0 + n0 - (Rp - 1);
        const int q0 = (base >= 0) ? base / D : -((D - 1 - base) / D);
        const int wmin = (Rp - 1 - n0 + D - 1) / D;  // first w with n >= Rp - 1
        const int wend = nrows_in - base;              // p < nrows_in  <=>  D w < wend
        fft2.run_io(Z, tab2, InLds{}, [&](int s, int w, float2 v) {
            if (w < wmin || D * w >= wend)
                return;
            dst[((int64_t)(q0 + w) << F_shift) + s] = conjf2(v);
        });
        return;
    }
    // forward transform; its last pass multiplies by the response spectrum and
    // conjugates (the inverse runs as a forward transform of the conjugate)
    fft.run_io(lds, tabL, load, KMulStore<true>{lds, Kc, F_shift, Fb_shift});
    __syncthreads();
    // inverse; its last pass writes the block's valid rows
    fft.run_io(lds, tabL, InLds{}, [&](int s, int n, float2 v) {
        const int p = P0 + n - (Rp - 1);
        if (n < Rp - 1 || p >= nrows_in)
            return;
        int o = p;
        if (mode == 1) {
            if (p % nimpact != nimpact / 2)
                return;
            o = p / nimpact;
        }
        dst[((int64_t)o << F_shift) + s] = conjf2(v);
    });
}

// ---------------------------------------------------------------------------
// Pass B for wire output, polyphase form.  With D = nimpact, wire w keeps grid
// row p = w D + D/2, and per tick frequency out[w] = sum_r K[r] X[p + r0 - r]
// (K: the response's tick spectrum, X: the grid's).  Split r = D a + b: with
// cw = D/2 + r0 and cw - b = D s_b + phi_b (0 <= phi_b < D),
//   out[w] = sum_b sum_a h_b[a] G_{phi_b}[w + s_b - a],
//   h_b[a] = K[D a + b] (A = ceil(Rp / D) taps), G_phi[m] = X[D m + phi]:
// D convolutions of wire-rate phase sequences with A-tap filters, summed.
// Overlap-save along wires with blocks of M = 128: block w0 takes
// x_b[j] = G_{phi_b}[w0 + s_b - (A - 1) + j] (j < M), forms
// Y(f) = sum_b H_b(f) DFT_M(x_b)(f) with H_b = DFT_M(h_b) / (M N') resident,
// and keeps y[j] = IDFT_M(Y)[j], j >= A - 1, as out[w0 + j - (A - 1)].
// A workgroup takes one block of V = M - A + 1 wires for all F columns of a
// chunk.  Per phase: a radix-8 pass from global memory into LDS, then a
// radix-16 pass whose outputs (frequencies i + 8 t of column s: the same for
// every phase) are multiplied by H_b and summed in registers; then the inverse
// (a forward transform of the conjugate).  Workgroups are mapped XCD-major as
// in k_pitch_conv.
// ---------------------------------------------------------------------------
constexpr int kPolyM = 128;
constexpr int kPolyMaxTaps = 64;  // A <= 64: at least 65 wires per block
struct PolyIo {
    const float2 *X;  // [C][Np][F]
    int Np;
    const float2 *H;  // [C][D][M][F]
    float2 *Y;        // [C][Nw][F]
    int Nw, nblocks;
};

template <int F, bool BATCH>
__global__ __launch_bounds__(8 * F) void k_pitch_poly(PolyIo io, BatchTables bt, int C, int D,
                                                      int A, int cw, const float2 *twM)
{
    constexpr int NT = 8 * F, M = kPolyM, NSS = (F == 16) ? 4 : 3;
    constexpr int NTAB = kTwLo + M / kTwLo + 1;  // two-level table of exp(-2 pi i j / M)
    __shared__ float2 buf[M * F];
    __shared__ float2 tab[NTAB];
    int gblk = blockIdx.x;
    if (BATCH) {
        const int e = find_event(bt.pblk_base, bt.nev, gblk);
        const EventCtx &E = bt.ev[e];
        io.X = E.X;
        io.Np = E.kp.Np;
        io.H = E.K;
        io.Y = E.Y;
        io.Nw = E.nout;
        io.nblocks = E.nblocks;
        gblk -= bt.pblk_base[e];
    }
    const int xcd = gblk & 7, slot = gblk >> 3;
    const int lc = slot / io.nblocks, blk = slot - lc * io.nblocks;
    const int c = lc * 8 + xcd;
    if (c >= C)
        return;
    for (int t = threadIdx.x; t < NTAB; t += NT)
        tab[t] = twM[t];
    const int V = M - A + 1, w0 = blk * V;
    const int tid = threadIdx.x, s = tid % F, i = tid / F;  // radix-16 butterfly i < 8 of column s
    const gptr<const float2> Xc = glb(io.X) + (int64_t)c * io.Np * F;
    const gptr<const float2> Hc = glb(io.H) + (int64_t)c * D * M * F;
    float2 acc[16];
#pragma unroll
    for (int t = 0; t < 16; ++t)
        acc[t] = make_float2(0.0f, 0.0f);
    InLds none;
    for (int b = 0; b < D; ++b) {
        const int phi = ((cw - b) % D + D) % D;
        const int m0 = w0 + (cw - b - phi) / D - (A - 1);
        // x_b[j] from global memory (zero outside the grid), from a clamped row
        auto load = [&](int col, int j) {
            const int q = (m0 + j) * D + phi;
            const int qc = min(max(q, 0), io.Np - 1);
            const float2 v = Xc[(int64_t)qc * F + col];
            return (q == qc) ? v : make_float2(0.0f, 0.0f);
        };
        ct_pass<M, 8, 1, NSS, 1, F, NT, true, false>(buf, tab, load, none);
        // radix-16 pass (p = 8) into registers, then times H_b, summed over b
        const gptr<const float2> Hb = Hc + (int64_t)b * M * F;
        float2 h[16], v[16];
#pragma unroll
        for (int t = 0; t < 16; ++t)
            h[t] = Hb[(i + 8 * t) * F + s];
#pragma unroll
        for (int t = 0; t < 16; ++t)
            v[t] = buf[(i + 8 * t) * F + s];
        twiddle_powers<16>(v, tw_at(tab, i));
        dft<16>(v);
#pragma unroll
        for (int t = 0; t < 16; ++t)
            acc[t] = cadd(acc[t], cmul(v[t], h[t]));
        __syncthreads();  // every read of this phase precedes the next phase's writes
    }
    // inverse: the forward transform of the conjugate, conjugated
#pragma unroll
    for (int t = 0; t < 16; ++t)
        buf[(i + 8 * t) * F + s] = conjf2(acc[t]);
    __syncthreads();
    const gptr<float2> Yc = glb(io.Y) + (int64_t)c * io.Nw * F;
    const int nw = io.Nw;
    auto store = [&](int col, int j, float2 val) {
        const int w = w0 + j - (A - 1);
        if (j < A - 1 || w >= nw)
            return;
        Yc[(int64_t)w * F + col] = conjf2(val);
    };
    ct_fft<M, NSS, 1, F, NT, 1, InLds, decltype(store), 8, 16>(buf, tab, none, store);
}

// Response spectra of the polyphase pass: H[c][b][f][s] = sum_{a < A, D a + b < Rp}
// XR[c][D a + b][s] exp(-2 pi i a f / M) / (M N'), from the tick spectra XR of
// the response rows (FP64 sums, once per plane).
__global__ void k_poly_spectrum(const float2 *XR, int Rp, int C, int F, int D, int A,
                                double scale, float2 *H)
{
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)C * D * kPolyM * F;
    if (idx >= total)
        return;
    const int sc = (int)(idx % F);
    int64_t r = idx / F;
    const int f = (int)(r % kPolyM);
    r /= kPolyM;
    const int b = (int)(r % D), c = (int)(r / D);
    double re = 0.0, im = 0.0;
    for (int a = 0; a < A && D * a + b < Rp; ++a) {
        const float2 x = XR[((int64_t)c * Rp + D * a + b) * F + sc];
        double sn, cs;
        sincospi(-2.0 * (double)((a * f) % kPolyM) / (double)kPolyM, &sn, &cs);
        re += (double)x.x * cs - (double)x.y * sn;
        im += (double)x.x * sn + (double)x.y * cs;
    }
    H[idx] = make_float2((float)(re * scale), (float)(im * scale));
}

int ilog2(int v)
{
    int s = 0;
    while ((1 << s) < v)
        ++s;
    return s;
}

// Threads for a transform of `nseq` sequences of length n so that every pass
// stages at most kRegComplex values per thread.
int threads_for(const FftPlan &plan, int nseq)
{
    int need = 64;
    for (int q = 0; q < plan.npass; ++q) {
        const int R = plan.radix[q];
        const int total = plan.n / R * nseq;
        const int maxb = kRegComplex / R;
        const int t = (total + maxb - 1) / maxb;
        need = std::max(need, t);
    }
    int threads = 64;
    while (threads < need)
        threads *= 2;
    return threads;
}

// Rows per workgroup in passes A and C.  One row keeps a workgroup's LDS at
// one row (25 KB for N2 = 3125), so six workgroups share a CU and the global
// loads of some overlap the transforms of others; two rows per workgroup
// halve that overlap and measured slower.
constexpr int kRowsShift = 0;
constexpr int kRowsPerBlock = 1 << kRowsShift;

// Compile-time transforms for the sizes the schedules use:
//   tick axis N2 = 3125 (N' = 6250, 6000-tick planes; 320 threads: two
//   radix-5 butterflies per thread and pass) and N2 = 600 (N' = 1200,
//   1000-tick planes);
//   pitch axis: L = 1024 or 640 or 960 over 8 columns, L = 512 over 16
//   columns.  A pitch block fills much of the LDS, so a CU holds two or three
//   workgroups; they get 512 threads to keep enough waves.
using TickCt3125 = FftCt<3125, kRowsShift, 3126, 1, 320, 5, 5, 5, 5, 5>;
using TickCt600 = FftCt<600, kRowsShift, 601, 1, 128, 8, 5, 5, 3>;
using PitchCt1024x8 = FftCt<1024, 3, 1, 8, 512, 16, 16, 4>;
using PitchCt512x16 = FftCt<512, 4, 1, 16, 512, 8, 8, 8>;
// Blocks a multiple of 10 rows long for the folded wire-output inverse, with
// the folded transforms of length L / 10.
using PitchCt640x8 = FftCt<640, 3, 1, 8, 512, 16, 8, 5>;
using PitchCt960x8 = FftCt<960, 3, 1, 8, 512, 8, 8, 5, 3>;
using FoldCt64x8 = FftCt<64, 3, 1, 8, 512, 8, 8>;
using FoldCt96x8 = FftCt<96, 3, 1, 8, 512, 8, 4, 3>;

int table_len(int m) { return kTwLo + (m + kTwLo - 1) / kTwLo; }

TwTables tick_tables(const wcsim_plane *pl)
{
    return {pl->twT, table_len(pl->N2), pl->twHalf, table_len(pl->N2 + 1)};
}

// `blocks` = workgroups of the launch; a batch passes its total and tables.
template <class FFT, bool B>
void launch_r2c(const wcsim_plane *pl, FFT fft, int threads, const R2CIo &io,
                const BatchTables &bt, unsigned blocks, hipStream_t s)
{
    const TwTables tw = tick_tables(pl);
    const size_t lds = sizeof(float2) * ((size_t)(pl->N2 + 1) * kRowsPerBlock + tw.na + tw.nb);
    hipLaunchKernelGGL((k_rows_r2c<FFT, B>), dim3(blocks), dim3(threads), lds, s, io, bt, pl->N2,
                       fft, tw, ilog2(pl->F), pl->C, kRowsShift);
}

template <class FFT, bool B>
void launch_c2r(const wcsim_plane *pl, FFT fft, int threads, const C2RIo &io,
                const BatchTables &bt, unsigned blocks, hipStream_t s)
{
    const TwTables tw = tick_tables(pl);
    const size_t lds = sizeof(float2) * ((size_t)(pl->N2 + 1) * kRowsPerBlock + tw.na + tw.nb);
    hipLaunchKernelGGL((k_rows_c2r<FFT, B>), dim3(blocks), dim3(threads), lds, s, io, bt, pl->N2,
                       fft, tw, ilog2(pl->F), pl->C, kRowsShift);
}

bool plan_is(const FftPlan &p, std::initializer_list<int> radices)
{
    if (p.npass != (int)radices.size())
        return false;
    int q = 0;
    for (int r : radices)
        if (p.radix[q++] != r)
            return false;
    return true;
}

FftRt runtime_fft(const FftPlan &plan, int nseq_shift, int sstride, int estride)
{
    FftRt f;
    f.plan = plan;
    f.nseq_shift = nseq_shift;
    f.sstride = sstride;
    f.estride = estride;
    return f;
}

int tick_threads(const wcsim_plane *pl)
{
    return std::min(1024, std::max(256, threads_for(pl->planT, kRowsPerBlock)));
}

int pitch_threads(const wcsim_plane *pl)
{
    return std::min(1024, std::max(256, threads_for(pl->planL, pl->Fb)));
}

template <bool B>
hipError_t rows_r2c_any(const wcsim_plane *pl, const R2CIo &io, const BatchTables &bt,
                        unsigned blocks, hipStream_t s)
{
    if (pl->N2 == 3125 && plan_is(pl->planT, {5, 5, 5, 5, 5}))
        launch_r2c<TickCt3125, B>(pl, TickCt3125(), TickCt3125::kThreads, io, bt, blocks, s);
    else if (pl->N2 == 600 && plan_is(pl->planT, {8, 5, 5, 3}))
        launch_r2c<TickCt600, B>(pl, TickCt600(), TickCt600::kThreads, io, bt, blocks, s);
    else
        launch_r2c<FftRt, B>(pl, runtime_fft(pl->planT, kRowsShift, pl->N2 + 1, 1),
                             tick_threads(pl), io, bt, blocks, s);
    return hipGetLastError();
}

template <bool B>
hipError_t rows_c2r_any(const wcsim_plane *pl, const C2RIo &io, const BatchTables &bt,
                        unsigned blocks, hipStream_t s)
{
    if (pl->N2 == 3125 && plan_is(pl->planT, {5, 5, 5, 5, 5}))
        launch_c2r<TickCt3125, B>(pl, TickCt3125(), TickCt3125::kThreads, io, bt, blocks, s);
    else if (pl->N2 == 600 && plan_is(pl->planT, {8, 5, 5, 3}))
        launch_c2r<TickCt600, B>(pl, TickCt600(), TickCt600::kThreads, io, bt, blocks, s);
    else
        launch_c2r<FftRt, B>(pl, runtime_fft(pl->planT, kRowsShift, pl->N2 + 1, 1),
                             tick_threads(pl), io, bt, blocks, s);
    return hipGetLastError();
}

hipError_t rows_r2c(const wcsim_plane *pl, const float *in, int nrows, int ncols,
                    int64_t in_stride, float2 *X, hipStream_t s, const uint8_t *occ = nullptr)
{
    static_assert(kOccRows % kRowsPerBlock == 0, "a tick-pass workgroup spans one map band");
    const R2CIo io = {in, nrows, ncols, in_stride, X, occ, occ ? occ_shift_of(ncols) : 0};
    return rows_r2c_any<false>(pl, io, BatchTables{}, (unsigned)rows_blocks(nrows), s);
}

hipError_t rows_c2r(const wcsim_plane *pl, const float2 *Y, int nrows, float *out, int ncols,
                    int64_t out_stride, hipStream_t s)
{
    const C2RIo io = {Y, nrows, out, ncols, out_stride};
    return rows_c2r_any<false>(pl, io, BatchTables{}, (unsigned)rows_blocks(nrows), s);
}

template <class FFT, class FFT2, bool B>
void launch_pitch(const wcsim_plane *pl, FFT fft, FFT2 fft2, int threads, const PitchIo &io,
                  const BatchTables &bt, unsigned blocks, float scale, hipStream_t s)
{
    const TwTables tw = {pl->twL, table_len(pl->L), pl->fold ? pl->twF : nullptr,
                         pl->fold ? table_len(pl->L10) : 0};
    const size_t lds =
        sizeof(float2) * ((size_t)pl->L * pl->Fb +
                          (pl->fold ? (size_t)pl->L10 * pl->Fb + pl->kp.nimpact : 0) + tw.na +
                          tw.nb);
    hipLaunchKernelGGL((k_pitch_conv<FFT, FFT2, B>), dim3(blocks), dim3(threads), lds, s, io, bt,
                       pl->L, pl->V, pl->Rp, pl->r0, pl->C, ilog2(pl->F), ilog2(pl->Fb), fft,
                       fft2, tw, (int)pl->kp.nimpact, pl->fold ? 1 : 0, scale);
}

template <bool B>
hipError_t pitch_any(const wcsim_plane *pl, const PitchIo &io, const BatchTables &bt,
                     unsigned blocks, float scale, hipStream_t s)
{
    const bool fold10 = pl->fold && pl->kp.nimpact == 10;
    if (pl->L == 1024 && pl->Fb == 8 && !pl->fold)
        launch_pitch<PitchCt1024x8, PitchCt1024x8, B>(pl, PitchCt1024x8(), PitchCt1024x8(),
                                                      PitchCt1024x8::kThreads, io, bt, blocks,
                                                      scale, s);
    else if (pl->L == 512 && pl->Fb == 16 && !pl->fold && plan_is(pl->planL, {8, 8, 8}))
        launch_pitch<PitchCt512x16, PitchCt512x16, B>(pl, PitchCt512x16(), PitchCt512x16(),
                                                      PitchCt512x16::kThreads, io, bt, blocks,
                                                      scale, s);
    else if (pl->L == 640 && pl->Fb == 8 && fold10 && plan_is(pl->planF, {8, 8}))
        launch_pitch<PitchCt640x8, FoldCt64x8, B>(pl, PitchCt640x8(), FoldCt64x8(),
                                                  PitchCt640x8::kThreads, io, bt, blocks, scale, s);
    else if (pl->L == 960 && pl->Fb == 8 && fold10 && plan_is(pl->planL, {8, 8, 5, 3}) &&
             plan_is(pl->planF, {8, 4, 3}))
        launch_pitch<PitchCt960x8, FoldCt96x8, B>(pl, PitchCt960x8(), FoldCt96x8(),
                                                  PitchCt960x8::kThreads, io, bt, blocks, scale, s);
    else
        launch_pitch<FftRt, FftRt, B>(pl, runtime_fft(pl->planL, ilog2(pl->Fb), 1, pl->Fb),
                                      runtime_fft(pl->fold ? pl->planF : pl->planL, ilog2(pl->Fb),
                                                  1, pl->Fb),
                                      pitch_threads(pl), io, bt, blocks, scale, s);
    return hipGetLastError();
}

hipError_t pitch_pass(const wcsim_plane *pl, const float2 *X, int nrows_in, const float2 *K,
                      float2 *Y, int nrows_out, int nblocks, int mode, float scale, hipStream_t s)
{
    const PitchIo io = {X, nrows_in, K, Y, nrows_out, nblocks, mode};
    const unsigned blocks = (unsigned)(8 * ((pl->C + 7) / 8) * nblocks * (pl->F / pl->Fb));
    return pitch_any<false>(pl, io, BatchTables{}, blocks, scale, s);
}

}  // namespace

// ---------------------------------------------------------------------------
// Plans and tables
// ---------------------------------------------------------------------------
bool make_plan(int n, FftPlan *plan)
{
    plan->n = n;
    plan->npass = 0;
    if (n < 2)
        return false;
    // Powers of two as radix-8 passes, with a trailing 2 * 8 = 16 split as
    // 4 * 4; then radices 5 and 3.
    int m = n, twos = 0;
    while (m % 2 == 0) {
        m /= 2;
        ++twos;
    }
    int eights = twos / 3, rest = twos % 3;
    if (rest == 1 && eights > 0) {
        --eights;
        rest = 4;  // 2^4 = 4 * 4
    }
    auto push = [&](int r) {
        if (plan->npass >= kMaxPass)
            return false;
        plan->radix[plan->npass++] = r;
        return true;
    };
    for (int k = 0; k < eights; ++k)
        if (!push(8))
            return false;
    if (rest == 4) {
        if (!push(4) || !push(4))
            return false;
    } else if (rest == 2) {
        if (!push(4))
            return false;
    } else if (rest == 1) {
        if (!push(2))
            return false;
    }
    for (int r : {5, 3}) {
        while (m % r == 0) {
            if (!push(r))
                return false;
            m /= r;
        }
    }
    return m == 1;
}

int smallest_smooth_even(int nmin)
{
    int n = std::max(4, nmin + (nmin & 1));
    for (;; n += 2) {
        FftPlan p;
        if (make_plan(n / 2, &p))
            return n;
    }
}

int twiddle_table_len(int m) { return table_len(m); }

int rows_blocks(int nrows) { return (nrows + kRowsPerBlock - 1) / kRowsPerBlock; }

int pitch_blocks_total(const wcsim_plane *pl)
{
    return 8 * ((pl->C + 7) / 8) * pl->nblocks * (pl->F / pl->Fb);
}

bool same_schedule_class(const wcsim_plane *a, const wcsim_plane *b)
{
    return a->Nfft == b->Nfft && a->L == b->L && a->F == b->F && a->Fb == b->Fb &&
           a->poly == b->poly && a->kp.fluct == b->kp.fluct &&
           a->fold == b->fold && a->Rp == b->Rp &&
           a->Rt == b->Rt && a->r0 == b->r0 && a->tile == b->tile && a->det == b->det &&
           a->Nt == b->Nt &&
           a->kp.nimpact == b->kp.nimpact && a->device == b->device;
}

int poly_blocks_total(const wcsim_plane *pl)
{
    return 8 * ((pl->C + 7) / 8) * pl->polyBlocks;
}

// The polyphase pitch pass of one plane (io set) or of a batch (tables).
template <bool B>
hipError_t poly_any(const wcsim_plane *pl, const PolyIo &io, const BatchTables &bt,
                    unsigned blocks, hipStream_t s)
{
    if (pl->F == 16)
        hipLaunchKernelGGL((k_pitch_poly<16, B>), dim3(blocks), dim3(128), 0, s, io, bt, pl->C,
                           (int)pl->kp.nimpact, pl->polyA, pl->polyCw, pl->twP);
    else
        hipLaunchKernelGGL((k_pitch_poly<8, B>), dim3(blocks), dim3(64), 0, s, io, bt, pl->C,
                           (int)pl->kp.nimpact, pl->polyA, pl->polyCw, pl->twP);
    return hipGetLastError();
}

hipError_t launch_convolve_batch_ab(const wcsim_plane *pl, const BatchTables &bt, int nblk_r,
                                    int nblk_p, bool poly, hipStream_t s, const hipEvent_t *ev,
                                    hipEvent_t after_a, hipEvent_t before_b)
{
    auto mark = [&](int i) { return ev ? hipEventRecord(ev[i], s) : hipSuccess; };
    hipError_t e;
    if ((e = rows_r2c_any<true>(pl, R2CIo{}, bt, (unsigned)nblk_r, s)) != hipSuccess ||
        (e = mark(0)) != hipSuccess ||
        (after_a && (e = hipEventRecord(after_a, s)) != hipSuccess) ||
        (before_b && (e = hipStreamWaitEvent(s, before_b, 0)) != hipSuccess))
        return e;
    if ((e = poly ? poly_any<true>(pl, PolyIo{}, bt, (unsigned)nblk_p, s)
                  : pitch_any<true>(pl, PitchIo{}, bt, (unsigned)nblk_p, 1.0f, s)) != hipSuccess)
        return e;
    return mark(1);
}

hipError_t launch_convolve_batch_c(const wcsim_plane *pl, const BatchTables &bt, int nblk_c,
                                   hipStream_t s)
{
    return rows_c2r_any<true>(pl, C2RIo{}, bt, (unsigned)nblk_c, s);
}

size_t conv_work_bytes(const wcsim_plane *pl, wcsim_out out_kind)
{
    const int64_t nout = (out_kind == WCSIM_OUT_WIRE) ? pl->Nw : pl->Np;
    return align_up(sizeof(float2) * (size_t)pl->C * pl->F * (size_t)pl->Np) +
           align_up(sizeof(float2) * (size_t)pl->C * pl->F * (size_t)nout);
}

hipError_t launch_convolve(const wcsim_plane *pl, const float *grid, float *out,
                           wcsim_out out_kind, void *work, hipStream_t s, const hipEvent_t *ev,
                           const uint8_t *occ)
{
    auto mark = [&](int i) { return ev ? hipEventRecord(ev[i], s) : hipSuccess; };
    const int64_t nout = (out_kind == WCSIM_OUT_WIRE) ? pl->Nw : pl->Np;
    float2 *X = (float2 *)work;
    float2 *Y = (float2 *)((char *)work +
                           align_up(sizeof(float2) * (size_t)pl->C * pl->F * (size_t)pl->Np));
    hipError_t e;
    if ((e = rows_r2c(pl, grid, (int)pl->Np, (int)pl->Nt, pl->Nt, X, s, occ)) != hipSuccess ||
        (e = mark(0)) != hipSuccess)
        return e;
    if (out_kind == WCSIM_OUT_WIRE && pl->poly) {
        const PolyIo io = {X, (int)pl->Np, pl->KP, Y, (int)pl->Nw, pl->polyBlocks};
        e = poly_any<false>(pl, io, BatchTables{}, (unsigned)poly_blocks_total(pl), s);
    } else {
        e = pitch_pass(pl, X, (int)pl->Np, pl->K, Y, (int)nout, pl->nblocks,
                       out_kind == WCSIM_OUT_WIRE ? 1 : 0, 1.0f, s);
    }
    if (e != hipSuccess || (e = mark(1)) != hipSuccess)
        return e;
    if ((e = rows_c2r(pl, Y, (int)nout, out, (int)pl->Nt, pl->Nt, s)) != hipSuccess)
        return e;
    return mark(2);
}

size_t response_work_bytes(const wcsim_plane *pl)
{
    return align_up(sizeof(float2) * (size_t)pl->C * pl->F * (size_t)pl->Rp);
}

// Response spectrum K[c][l][f] = sum_{i<Rp} sum_{s<Rt} R[i][s]
//   exp(-2 pi i (l i / L + k s / N')) / (L N'), k = c F + f.
// Response combined with the electronics response along ticks:
// out[r][t] = sum_s R[r][s] E[t - s], t < Rt0 + Ne - 1 (FP64 sums).  Runs once
// per plane creation.
__global__ void k_combine_response(const float *R, int Rp, int Rt0, const float *E, int Ne,
                                   float *out)
{
    const int Rt = Rt0 + Ne - 1;
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= (int64_t)Rp * Rt)
        return;
    const int r = (int)(g / Rt), t = (int)(g - (int64_t)r * Rt);
    double acc = 0.0;
    for (int s = max(0, t - Ne + 1); s <= min(Rt0 - 1, t); ++s)
        acc += (double)R[(int64_t)r * Rt0 + s] * (double)E[t - s];
    out[g] = (float)acc;
}

hipError_t launch_combine_response(const float *R, int Rp, int Rt0, const float *E, int Ne,
                                   float *out, hipStream_t s)
{
    const int64_t n = (int64_t)Rp * (Rt0 + Ne - 1);
    hipLaunchKernelGGL(k_combine_response, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, R,
                       Rp, Rt0, E, Ne, out);
    return hipGetLastError();
}

hipError_t build_response_spectrum(wcsim_plane *pl, const float *resp_dev, void *work,
                                   hipStream_t s)
{
    float2 *XR = (float2 *)work;
    hipError_t e;
    if ((e = rows_r2c(pl, resp_dev, pl->Rp, pl->Rt, pl->Rt, XR, s)) != hipSuccess)
        return e;
    const float scale = (float)(1.0 / ((double)pl->L * (double)pl->Nfft));
    if ((e = pitch_pass(pl, XR, pl->Rp, nullptr, pl->K, pl->L, 1, 2, scale, s)) != hipSuccess)
        return e;
    if (!pl->poly)
        return hipSuccess;
    const int64_t total = (int64_t)pl->C * pl->kp.nimpact * kPolyM * pl->F;
    hipLaunchKernelGGL(k_poly_spectrum, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, XR,
                       pl->Rp, pl->C, pl->F, (int)pl->kp.nimpact, pl->polyA,
                       1.0 / ((double)kPolyM * (double)pl->Nfft), pl->KP);
    return hipGetLastError();
}

int poly_block_rows() { return kPolyM; }
int poly_max_taps() { return kPolyMaxTaps; }

}  // namespace wcs
