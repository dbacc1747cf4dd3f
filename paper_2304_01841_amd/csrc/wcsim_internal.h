// Internal declarations of libwcsim: kernel-side parameter blocks, the plane
// object and the launch helpers shared by the raster and FFT translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "wcsim.h"

namespace wcs {

// ---------------------------------------------------------------------------
// Status plumbing
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
wcsim_status fail(wcsim_status st, const std::string &msg);
wcsim_status check_hip(hipError_t e, const char *what);

#define WCS_HIP(expr)                                                      \
    do {                                                                   \
        hipError_t _e = (expr);                                            \
        if (_e != hipSuccess)                                              \
            return ::wcs::check_hip(_e, #expr);                            \
    } while (0)

// ---------------------------------------------------------------------------
// Kernel-side view of a plane's geometry and physics.  Every double here is
// derived on the host exactly as the definitions read (dp = pitch / nimpact),
// so that the device reproduces the window bounds operation by operation.
// ---------------------------------------------------------------------------
struct PlaneParams {
    double v, DL, DT, nsigma;
    double dp, tick, t0, plane_x, dir_y, dir_z, pitch_origin;
    int32_t Np, Nt, nimpact, plane_id;
    uint32_t key0, key1;  // Philox key of the bin draws: seed low word, seed high word ^ plane_id
    uint32_t lkey0, lkey1;  // Philox key of the lifetime draw: seed low word ^ 0x6c696665, seed high word
    int32_t fluct;
    int32_t pad_;
    double tau;    // electron lifetime (us), 0: no absorption
    double accel;  // rate of change of the drift speed with drift time (mm/us^2)
};

// Maximum window length per axis handled anywhere in the library.
constexpr int kMaxWindow = 1024;

// Occupancy map of a plane grid: one byte per block of kOccRows pitch rows x
// 2^shift ticks, kOccCols bytes per band of kOccRows rows (at most 64 tick
// blocks per band: shift >= 6 is the least with ceil(Nt / 2^shift) <= 64).  A
// byte is non-zero when some depo window reaches the block; blocks never
// reached are neither cleared nor read (the tick-axis pass takes them as zero).
constexpr int kOccRows = 32, kOccCols = 64;
inline int occ_shift_of(int64_t Nt)
{
    int s = 6;
    while (((Nt + (1LL << s) - 1) >> s) > kOccCols)
        ++s;
    return s;
}
inline int64_t occ_bands(int64_t Np) { return (Np + kOccRows - 1) / kOccRows; }

// ---------------------------------------------------------------------------
// Batched execution: one descriptor per event in device memory, and prefix
// bases (nev + 1 entries each) that map a global index of each kind of work
// to its event: depos, tiles, and the workgroups of the three FFT passes.
// ---------------------------------------------------------------------------
struct EventCtx {
    PlaneParams kp;
    const wcsim_depo *depos;
    float *grid;       // [Np][Nt]
    const float2 *K;   // response spectrum of the event's plane
    float2 *X;         // [C][Np][F]
    float2 *Y;         // [C][nout][F]
    float *out;        // [nout][Nt]
    uint8_t *occ;      // occupancy map of the grid (occ_bands(Np) x kOccCols bytes)
    int64_t depo_base;
    int32_t n;
    uint32_t event;
    int32_t tile_base, ntt;
    int32_t nout, nblocks, mode;
    int32_t occ_shift;  // tick blocks of the map are 2^occ_shift ticks
};

struct BatchTables {
    const EventCtx *ev;
    const int32_t *depo_base;  // global depo index of each event's depo 0 (fits int32: < 2^31)
    const int32_t *tile_base;
    const int32_t *rblk_base;  // tick-axis forward pass workgroups
    const int32_t *pblk_base;  // pitch-axis pass workgroups
    const int32_t *cblk_base;  // tick-axis inverse pass workgroups
    const int32_t *band_base;  // bands of kOccRows grid rows (occupancy map)
    int32_t nev;
};

// A pointer read from memory (an event's table entry) has no address space
// for the compiler, which then emits flat instructions for its accesses; those
// count against the LDS wait counter too, so each LDS wait in the kernel also
// waits for the HBM loads and atomics in flight.  Every pointer the kernels
// take addresses device memory: this cast lets the compiler emit global ones.
// (The host pass, which only checks the kernels' bodies, has no such space.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T> using gptr = __attribute__((address_space(1))) T *;
#else
template <class T> using gptr = T *;
#endif
template <class T> __device__ __forceinline__ gptr<T> glb(T *p) { return (gptr<T>)p; }

// Largest e with base[e] <= key (base ascending, base[0] = 0).
__device__ __forceinline__ int find_event(const int32_t *base, int nev, int key)
{
    int lo = 0, hi = nev - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= key)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// FFT plans
// ---------------------------------------------------------------------------
constexpr int kMaxPass = 12;
struct FftPlan {
    int32_t n;
    int32_t npass;
    int32_t radix[kMaxPass];
};

bool make_plan(int n, FftPlan *plan);     // factor n into radices {8,4,2,5,3}
int twiddle_table_len(int count);         // entries of a two-level twiddle table
int smallest_smooth_even(int nmin);      // smallest even n >= nmin with n/2 plannable

// Raster tile shapes (pitch x tick tile; the LDS region adds a halo).
struct TileShape {
    int tp, tt, hp, ht;
};
constexpr int kNumTileShapes = 3;
TileShape tile_shape(int id);

}  // namespace wcs

// ---------------------------------------------------------------------------
// Plane object
// ---------------------------------------------------------------------------
struct wcsim_plane {
    wcsim_plane_desc desc;  // response pointer cleared (host copy not kept)
    wcsim_physics phys;
    wcs::PlaneParams kp;
    int device;
    int64_t Np, Nt, Nw;
    // FFT schedule: tick axis N' = 2 N2 (real), pitch axis overlap-save blocks
    // of length L with V = L - Rp + 1 valid rows each.
    int Nfft, N2, H, F, C, L, V, nblocks;
    // Fb: columns per pitch-pass workgroup (divides F); fold: wire output
    // folds the inverse to length L10 = L / nimpact (nimpact divides L)
    int Fb, L10;
    bool fold;
    int Rp, Rt, r0;
    wcs::FftPlan planT, planL, planF;
    float2 *twT;     // two-level table of exp(-2 pi i j / N2), j < N2
    float2 *twHalf;  // two-level table of exp(-2 pi i k / N'), k <= N2
    float2 *twL;     // two-level table of exp(-2 pi i j / L), j < L
    float2 *twF;     // two-level table of exp(-2 pi i j / L10), j < L10 (fold only)
    float2 *K;       // response spectrum [C][L][F], scaled by 1/(L N')
    // polyphase wire-output pitch pass (poly): response spectra KP[C][D][M][F]
    // of the D phase filters of polyA = ceil(Rp / D) taps, scaled by
    // 1/(M N'); blocks of polyV = M - polyA + 1 wires; polyCw = D/2 + r0
    bool poly;
    int polyA, polyV, polyBlocks, polyCw;
    float2 *KP;
    float2 *twP;     // two-level table of exp(-2 pi i j / M), j < M
    // owner of K and the twiddle tables; planes with the same response and
    // transform sizes share one
    std::shared_ptr<struct wcs_spectrum> spectrum;
    int tile;
    bool det;  // reproducible sums: sorted tile lists, owner flush, ordered large patches
    wcs::TileShape ts;
    int ntp, ntt;
    int64_t ntiles;
};

struct wcsim_patches {
    int64_t n;
    int64_t nvalues;
    int32_t *meta;     // [n][4]
    int64_t *offsets;  // [n+1]
    float *values;
    wcsim_depo *staged;  // device copy of host depos (owned) or nullptr
    int device;
};

namespace wcs {

// ---------------------------------------------------------------------------
// Launch helpers (defined in raster.hip / fft.hip)
// ---------------------------------------------------------------------------
hipError_t launch_fill_zero(void *ptr, size_t bytes, hipStream_t s);

hipError_t launch_combine_response(const float *R, int Rp, int Rt0, const float *E, int Ne,
                                   float *out, hipStream_t s);
hipError_t launch_digitize(const float *wave, int64_t nrows, int64_t ncols, float gain,
                           float pedestal, float sigma, int bits, uint64_t seed, uint32_t event,
                           uint16_t *adc, hipStream_t s);
constexpr int kMaxFir = 1024;
hipError_t launch_digitize_fir(const float *wave, int64_t nrows, int64_t ncols, float gain,
                               float pedestal, float sigma, const float *fir, int nfir, int bits,
                               uint64_t seed, uint32_t event, uint16_t *adc, hipStream_t s);
hipError_t launch_philox(const uint32_t *ctr, const uint32_t *key, int64_t n, uint32_t *out,
                         hipStream_t s);

// unfused rasterize: per-depo sizes, scan, values
hipError_t launch_patch_sizes(const wcsim_plane *pl, const wcsim_depo *depos, int64_t n,
                              int32_t *meta, int64_t *sizes, hipStream_t s);
size_t scan_scratch_bytes(int64_t n);
hipError_t launch_exclusive_scan_i64(int64_t *data, int64_t n, void *scratch, hipStream_t s);
hipError_t launch_exclusive_scan_i32(int32_t *data, int64_t n, void *scratch, hipStream_t s);
hipError_t launch_patch_values(const wcsim_plane *pl, const wcsim_depo *depos, int64_t n,
                               uint64_t event_id, const int32_t *meta, const int64_t *offsets,
                               float *values, hipStream_t s);
hipError_t launch_scatter_flat(const wcsim_plane *pl, int64_t n, const int32_t *meta,
                               const int64_t *offsets, const float *values, float *grid,
                               hipStream_t s);

// fused raster + LDS-staged scatter
struct RasterWork {
    int32_t *counters;    // [0] invalid depos, [1] large-patch depos, [2] tile work items
    int32_t *tile_count;  // [ntiles + 1] counts -> exclusive list offsets
    int2 *block_tot;      // per schedule block: depos and work items
    int4 *items;          // work items {tile, first record, end record, 0}
    int32_t *depo_tile;   // [n] tile of each depo (-1: none)
    int32_t *depo_slot;   // [n] position in its tile's list
    int32_t *large;       // [n] depos of the large-patch path
    float *records;       // [n][64] depo records in tile-list order
    uint8_t *occ;         // occupancy maps of the grids (bands x kOccCols bytes)
    int32_t *sort_tot;    // [256] digit totals of the tile-list sort (zero between passes)
};
size_t raster_work_bytes(const wcsim_plane *pl, int64_t n);
RasterWork raster_work_carve(const wcsim_plane *pl, int64_t n, void *base);
// `ev` (nullable): 3 events recorded after binning, after the LDS-tiled
// raster kernel and after the large-patch kernel.
// The sequence clears the occupancy map w.occ and the grid's occupied blocks;
// the others keep whatever they held.
hipError_t launch_raster_fused(const wcsim_plane *pl, const wcsim_depo *depos, int64_t n,
                               uint64_t event_id, const RasterWork &w, float *grid,
                               hipStream_t s, const hipEvent_t *ev = nullptr);
// Batched: events of planes sharing one schedule class (pl = any of them);
// n_total depos, ntiles_total tiles and nbands_total map bands over all events.
size_t raster_work_bytes_batch(const wcsim_plane *pl, int64_t n_total, int64_t ntiles_total,
                               int64_t nbands_total);
RasterWork raster_work_carve_batch(const wcsim_plane *pl, int64_t n_total, int64_t ntiles_total,
                                   int64_t nbands_total, void *base);
// Each event's map (EventCtx::occ, inside w.occ) and the occupied blocks of
// its grid are cleared by the sequence itself.
// `ev` (nullable): 3 stage marks as for launch_raster_fused.
hipError_t launch_raster_batch(const wcsim_plane *pl, const BatchTables &bt, int64_t n_total,
                               int64_t ntiles_total, int64_t nbands_total, const RasterWork &w,
                               hipStream_t s, const hipEvent_t *ev = nullptr);
// Zero the blocks of a grid that its occupancy map marks as not reached.
hipError_t launch_clear_unoccupied(float *grid, int Np, int Nt, const uint8_t *occ, int shift,
                                   hipStream_t s);

// FFT convolution passes
size_t conv_work_bytes(const wcsim_plane *pl, wcsim_out out_kind);
// `ev` (nullable): 3 events recorded after passes A, B and C.  `occ`
// (nullable): the grid's occupancy map; blocks it does not mark are read as
// zero.
hipError_t launch_convolve(const wcsim_plane *pl, const float *grid, float *out,
                           wcsim_out out_kind, void *work, hipStream_t s,
                           const hipEvent_t *ev = nullptr, const uint8_t *occ = nullptr);
hipError_t build_response_spectrum(wcsim_plane *pl, const float *resp_dev, void *work,
                                   hipStream_t s);
size_t response_work_bytes(const wcsim_plane *pl);
// Batched convolution over every event of the tables, in two parts that may
// run on different streams: passes A and B, then pass C.  nblk_* = total
// workgroups of each pass (the last entries of the bases).  `ev` (nullable):
// 2 events recorded after passes A and B; `after_a` (nullable) is recorded
// after pass A as well, and pass B waits for `before_b` (nullable).
// `poly`: wire output through the polyphase pitch pass (pl->poly), whose
// workgroup counts are in the tables' pblk_base.
hipError_t launch_convolve_batch_ab(const wcsim_plane *pl, const BatchTables &bt, int nblk_r,
                                    int nblk_p, bool poly, hipStream_t s, const hipEvent_t *ev,
                                    hipEvent_t after_a, hipEvent_t before_b);
hipError_t launch_convolve_batch_c(const wcsim_plane *pl, const BatchTables &bt, int nblk_c,
                                   hipStream_t s);
int rows_blocks(int nrows);                       // workgroups of a tick-axis pass
int pitch_blocks_total(const wcsim_plane *pl);    // workgroups of the pitch pass
int poly_blocks_total(const wcsim_plane *pl);     // workgroups of the polyphase pitch pass
int poly_block_rows();                            // M, the polyphase block transform length
int poly_max_taps();                              // longest phase filter of the polyphase pass
bool same_schedule_class(const wcsim_plane *a, const wcsim_plane *b);

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

}  // namespace wcs
