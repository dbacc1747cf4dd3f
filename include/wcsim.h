/*
 * wcsim.h -- C ABI of the MI355X LArTPC signal-simulation hot path.
 *
 * The library computes the three steps the paper's DepoTransform holds
 * (arXiv:2304.01841, Sec. 2):
 *   1. Rasterization: every group of ionization electrons (a depo) is drifted to
 *      the response plane, diffused into 2-D Gaussian widths and binned into a
 *      patch of (pitch-impact bin x time tick) weights, optionally with
 *      statistical fluctuation (Sec. 2 step 1; random numbers Sec. 4.1);
 *   2. Scatter-Add: patches are summed into a plane grid with atomic adds
 *      (Sec. 2 step 2);
 *   3. Convolution: the grid is convolved with the detector response by FFT
 *      (Sec. 2 step 3; inverse real transform along the tick axis as in the
 *      idft_cr example of Sec. 4.2).
 *
 * Units: mm, us, electrons.  Diffusion constants in mm^2/us (1 cm^2/s =
 * 1e-4 mm^2/us).
 *
 * Conventions shared by every entry point:
 *   - Every call returns a wcsim_status; no C++ exception crosses the ABI.
 *     On failure, wcsim_last_error() gives a message (thread-local, valid until
 *     the next wcsim_* call on the same thread).
 *   - Validation failures return WCSIM_E_INVALID with nothing launched and
 *     outputs untouched.  HIP runtime failures return WCSIM_E_DEVICE,
 *     allocation failures WCSIM_E_NOMEM.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous on it, except wcsim_plane_create/destroy, the patch-set
 *     calls that allocate or copy to the host, and every path that reads or
 *     writes host memory, which synchronise the stream before returning.
 *   - A wcsim_plane is immutable after creation and may be shared by
 *     concurrent calls on different streams; calls that share a workspace
 *     must be ordered by the caller.
 *   - Device pointers must be device (or managed) memory of the current HIP
 *     device; the caller owns every buffer it passes in.
 */
#ifndef WCSIM_H
#define WCSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WCSIM_OK = 0,
    WCSIM_E_INVALID = -1, /* bad argument; nothing launched */
    WCSIM_E_NOMEM = -2,   /* allocation failed / workspace too small */
    WCSIM_E_DEVICE = -3,  /* HIP runtime error */
    WCSIM_E_STATE = -4    /* object used in a wrong state (e.g. NULL handle) */
} wcsim_status;

typedef enum { WCSIM_MEM_HOST = 0, WCSIM_MEM_DEVICE = 1 } wcsim_mem;

typedef enum {
    WCSIM_OUT_WIRE = 0, /* [nwires][nticks]: impact row nimpact/2 of each wire cell */
    WCSIM_OUT_PITCH = 1 /* [nwires*nimpact][nticks]: every pitch-impact row */
} wcsim_out;

/* One depo (Sec. 2 step 1: a group of ionization electrons): x is the drift
 * coordinate, (y, z) the transverse position, t the deposition time and q the
 * number of electrons (q >= 0).  Array of structures, 40 bytes per depo. */
typedef struct {
    double x, y, z, t, q;
} wcsim_depo;

/* Drift and diffusion constants and fluctuation switch. */
typedef struct {
    double drift_speed; /* mm/us, > 0 */
    double DL, DT;      /* longitudinal / transverse diffusion, mm^2/us, >= 0 */
    double nsigma;      /* patch half-extent in Gaussian widths, >= 0 */
    int32_t fluctuate;  /* 0: mean patch; 1: binomial fluctuation */
    int32_t reserved;   /* must be 0 */
    uint64_t seed;      /* Philox key (mixed with plane_id) */
    double lifetime;    /* electron lifetime tau, us, >= 0; 0: no absorption.  An
                         * extension beyond the paper, which starts from the drifted
                         * charge: each electron survives the drift time T with
                         * probability exp(-T / tau); the depo keeps the mean q p,
                         * or with fluctuation a normal-approximated binomial count
                         * drawn from Philox under the key (seed low word XOR
                         * 0x6c696665, seed high word) at counter (0, 0, depo,
                         * event).  No plane enters that draw: every plane of an
                         * event sees the same surviving charge. */
    double drift_accel; /* mm/us^2, finite; 0: constant drift speed.  An extension
                         * beyond the paper: the drift speed changes linearly with
                         * drift time at this rate and equals drift_speed on the
                         * response plane, so a depo at distance L from the plane
                         * starts at v_s = sqrt(v^2 - 2 a L) and drifts for
                         * T = 2 L / (v + v_s); a depo with v^2 - 2 a L < 0 cannot
                         * reach the plane and is invalid. */
} wcsim_physics;

/* Plane geometry and response (Sec. 2 steps 2-3).  The grid has
 * nwires*nimpact pitch bins of pitch/nimpact mm, starting at pitch coordinate
 * pitch_origin, and nticks ticks of `tick` us starting at t0.  The pitch
 * coordinate of a depo is y*dir_y + z*dir_z.  The response is
 * [resp_npitch][resp_nticks] float32 in host memory, row-major; response row
 * resp_origin is aligned with the output row and tick 0 of the response is
 * the output tick itself (causal):
 *   out[p][t] = sum_r sum_s response[r][s] grid[p + resp_origin - r][t - s]. */
typedef struct {
    int32_t plane_id, nwires, nimpact, nticks;
    double pitch, tick, t0;
    double plane_x, dir_y, dir_z, pitch_origin;
    int32_t resp_npitch, resp_nticks, resp_origin, reserved;
    const float *response;
    /* Electronics response (an extension beyond the paper, which stops at the
     * induced current): elec_nticks samples, host memory, copied; 0 = none.
     * The plane convolves with R (x) E, each response row convolved along
     * ticks with E (starting at tick 0), so the effective response is
     * resp_npitch x (resp_nticks + elec_nticks - 1) and the tick transform
     * must cover nticks + that length - 1.  At most 8192 samples, finite. */
    int32_t elec_nticks, reserved2; /* reserved2 must be 0 */
    const float *elec_response;
} wcsim_plane_desc;

/* Execution schedule of a plane; 0 in a field means "choose".  The result of
 * the simulation does not depend on it (up to float32 rounding). */
typedef struct {
    int32_t fft_ticks;  /* even padded tick-axis transform length N' >= nticks + resp_nticks - 1,
                         * N'/2 a product of 2, 3 and 5; one row of N'/2 + 1 complex
                         * values and its twiddle tables must fit a workgroup's LDS,
                         * so N' <= 20000 (else WCSIM_E_INVALID) */
    int32_t fft_pitch;  /* pitch-axis overlap-save block transform length L > resp_npitch - 1 */
    int32_t freq_chunk; /* spectrum columns per chunk (8 or 16) */
    int32_t tile;       /* raster tile shape id, pitch bins x ticks of a tile: 0 = 32 x 8
                         * (default), 1 = 32 x 32, 2 = 64 x 8; each wavefront's LDS
                         * region adds a 32-bin x 16-tick halo */
    int32_t wire_mode;  /* pitch pass of wire output (Sec. 2 step 3): 1 = polyphase
                         * (per tick frequency, the nimpact phases of the grid rows at
                         * wire rate, each convolved with its ceil(resp_npitch /
                         * nimpact)-tap slice of the response through 128-point
                         * transforms and summed; needs nimpact > 1 and at most 64
                         * taps), 2 = overlap-save blocks of fft_pitch rows; 0 =
                         * polyphase where it applies, else blocks */
    int32_t deterministic; /* 1: the simulated grid and output are reproducible bit for
                         * bit (Sec. 2 step 2 sums in a fixed order): depos are
                         * listed per tile in index order, tiles are flushed in
                         * colour phases whose LDS regions are disjoint with plain
                         * read-add-writes, and depos too large for a tile are
                         * added one after another in index order; 0 (default) =
                         * float atomics, whose order of addition varies from run
                         * to run.  Applies to the fused simulate entry points
                         * (single events and batches). */
} wcsim_schedule;

/* Derived sizes of a plane (read-only). */
typedef struct {
    int64_t npitch, nticks, nwires, nimpact;
    int32_t fft_ticks, fft_pitch, freq_chunk, tile;
    int32_t nchunks;        /* spectrum column chunks */
    int32_t pitch_blocks;   /* overlap-save blocks along pitch */
    int32_t tile_pitch, tile_ticks;
    int64_t ntiles;
    int64_t spectrum_bytes; /* resident response spectrum */
    int32_t pitch_cols;     /* spectrum columns per pitch-pass workgroup (divides freq_chunk) */
    int32_t wire_fold;      /* 1: wire output folds the pitch inverse to fft_pitch / nimpact */
    int32_t wire_polyphase; /* 1: wire output uses the polyphase pitch pass */
    int32_t wire_blocks;    /* polyphase blocks along the wires (0 without) */
    int32_t deterministic;  /* 1: reproducible sums (wcsim_schedule.deterministic) */
} wcsim_plane_info;

typedef struct wcsim_plane wcsim_plane;
typedef struct wcsim_patches wcsim_patches;

/* Create a plane: validates the descriptor and physics, copies the response,
 * chooses a schedule and computes the resident response spectrum on the GPU
 * (Sec. 2 step 3: the response is transformed once per plane).  Synchronises
 * `stream`.  Errors: WCSIM_E_INVALID for NULL pointers, non-positive sizes,
 * nimpact < 1, resp_origin outside [0, resp_npitch), non-finite or
 * out-of-range constants, or a non-unit pitch direction; WCSIM_E_NOMEM when
 * device memory runs out.  The plane owns its device memory until
 * wcsim_plane_destroy. */
wcsim_status wcsim_plane_create(const wcsim_plane_desc *desc, const wcsim_physics *phys,
                                void *stream, wcsim_plane **out);

/* Same with an explicit schedule (fields 0 = choose).  WCSIM_E_INVALID when a
 * requested schedule is not supported for the plane. */
wcsim_status wcsim_plane_create_with_schedule(const wcsim_plane_desc *desc,
                                              const wcsim_physics *phys,
                                              const wcsim_schedule *sched, void *stream,
                                              wcsim_plane **out);

/* Same as wcsim_plane_create, but when `donor` has the same response (shape,
 * origin and values) and a tick-axis transform long enough for this plane,
 * the new plane takes the donor's transform sizes and shares its resident
 * response spectrum (reference counted) instead of building one: planes of
 * any wire count with one response then cost no spectrum memory or set-up
 * (the spectrum does not depend on the number of wires).  Otherwise it
 * builds its own.  WCSIM_E_INVALID for a NULL donor. */
wcsim_status wcsim_plane_create_sharing(const wcsim_plane_desc *desc, const wcsim_physics *phys,
                                        const wcsim_plane *donor, void *stream,
                                        wcsim_plane **out);

/* Frees the plane (synchronises the device first).  NULL is ignored. */
void wcsim_plane_destroy(wcsim_plane *plane);

wcsim_status wcsim_plane_get_info(const wcsim_plane *plane, wcsim_plane_info *info);

/* Rasterization (Sec. 2 step 1): one patch per depo.
 *   depos: n depos in host (mem = WCSIM_MEM_HOST) or device memory.
 *   event_id: mixed into the fluctuation random numbers (low 32 bits).
 * A patch covers the inclusive window floor(mu - nsigma s) ..
 * floor(mu + nsigma s) along pitch and ticks.  Depos whose window misses the
 * grid, and invalid depos, get an empty patch.  Host depos are validated on
 * the host (non-finite field, q < 0, x < plane_x or a depo that cannot reach
 * the plane under drift_accel -> WCSIM_E_INVALID);
 * invalid device depos contribute nothing.  A window longer than 1024 bins on
 * either axis is rejected (host) or dropped (device).
 * The patch set is allocated by the library (the call synchronises `stream`
 * to size it) and owned by the caller through *out until
 * wcsim_patches_destroy. */
wcsim_status wcsim_rasterize(const wcsim_plane *plane, const wcsim_depo *depos, int64_t n,
                             wcsim_mem mem, uint64_t event_id, void *stream,
                             wcsim_patches **out);

/* Number of depos and of patch values in a patch set. */
wcsim_status wcsim_patches_count(const wcsim_patches *patches, int64_t *ndepos, int64_t *nvalues);

/* Device views of a patch set (valid until wcsim_patches_destroy):
 *   meta    [ndepos][4] int32 = lo_p, lo_t, n_p, n_t (absolute first bin and
 *           window lengths; n_p = n_t = 0 for an empty patch),
 *   offsets [ndepos + 1] int64 exclusive prefix sum of n_p*n_t (the scan of
 *           patch sizes, Sec. 4.3),
 *   values  [nvalues] float32, patch d row-major n_p x n_t at offsets[d]. */
wcsim_status wcsim_patches_device(const wcsim_patches *patches, const int32_t **meta,
                                  const int64_t **offsets, const float **values);

/* Copy a patch set to host arrays of the sizes above (synchronous). */
wcsim_status wcsim_patches_copy_to_host(const wcsim_patches *patches, int32_t *meta,
                                        int64_t *offsets, float *values);

void wcsim_patches_destroy(wcsim_patches *patches);

/* Scatter-Add (Sec. 2 step 2): grid[p][t] += patch value for every patch bin
 * inside the [npitch][nticks] float32 device grid; bins outside are dropped.
 * zero_first != 0 clears the grid first.  Atomic float adds: the summation
 * order is unspecified. */
wcsim_status wcsim_scatter_add(const wcsim_plane *plane, const wcsim_patches *patches,
                               float *grid, int32_t zero_first, void *stream);

/* Workspace (device bytes) that wcsim_convolve needs for an output kind. */
size_t wcsim_convolve_workspace_bytes(const wcsim_plane *plane, wcsim_out out_kind);

/* Convolution (Sec. 2 step 3): out = grid (*) response, cropped to the grid
 * (see wcsim_plane_desc), as [npitch][nticks] (WCSIM_OUT_PITCH) or
 * [nwires][nticks] (WCSIM_OUT_WIRE) float32 in device memory.  `grid` is the
 * [npitch][nticks] float32 device grid.  `workspace` is device memory of at
 * least wcsim_convolve_workspace_bytes bytes, aligned to 256 bytes. */
wcsim_status wcsim_convolve(const wcsim_plane *plane, const float *grid, float *out,
                            wcsim_out out_kind, void *workspace, void *stream);

/* Workspace (device bytes) for wcsim_simulate_event with up to n depos. */
size_t wcsim_simulate_workspace_bytes(const wcsim_plane *plane, int64_t n, wcsim_out out_kind);

/* The whole DepoTransform (Sec. 2 steps 1-3) for one event: rasterize with
 * fluctuation as configured, scatter into the plane grid through LDS-staged
 * tiles, convolve, and write `out` ([nwires][nticks] or [npitch][nticks]
 * float32, in host or device memory per out_mem).  Depos follow the rules of
 * wcsim_rasterize.  `workspace`: device memory of at least
 * wcsim_simulate_workspace_bytes(plane, n, out_kind) bytes, 256-byte aligned;
 * after the call it also holds the plane grid (see wcsim_workspace_grid) and
 * the count of invalid device depos (wcsim_workspace_invalid_count). */
wcsim_status wcsim_simulate_event(const wcsim_plane *plane, const wcsim_depo *depos, int64_t n,
                                  wcsim_mem depo_mem, uint64_t event_id, float *out,
                                  wcsim_out out_kind, wcsim_mem out_mem, void *workspace,
                                  void *stream);

/* Allocation-free variant of wcsim_simulate_event, for callers that cannot
 * allocate device memory or pass a workspace of their own (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * workspace is a fixed device array of WCSIM_NOALLOC_SCRATCH_BYTES bytes that
 * the library holds on every GPU it runs on until the process ends; the call
 * makes no allocation of any kind.  Depos and output are device memory (the
 * caller's, as in wcsim_simulate_event with WCSIM_MEM_DEVICE for both); the
 * current device must be the plane's.  Same results as wcsim_simulate_event.
 * Errors: WCSIM_E_INVALID when the event needs more workspace than the array
 * holds (wcsim_simulate_workspace_bytes(plane, n, out_kind) >
 * WCSIM_NOALLOC_SCRATCH_BYTES) or for bad arguments, with nothing launched.
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents (each call clears what it needs): calls whose executions
 * overlap on one GPU (other streams, other threads) race and must not be
 * issued; calls in order on one stream are safe. */
#define WCSIM_NOALLOC_SCRATCH_BYTES (64u << 20)
wcsim_status wcsim_simulate_event_noalloc(const wcsim_plane *plane, const wcsim_depo *depos,
                                          int64_t n, uint64_t event_id, float *out,
                                          wcsim_out out_kind, void *stream);

/* wcsim_simulate_event with stage timing, for measuring each kernel on the
 * stream it runs on (the paper times Rasterization, Scatter-Add and FFT
 * separately, Sec. 5.2).  `events` holds WCSIM_NUM_STAGE_EVENTS hipEvent_t
 * handles created by the caller; they are recorded on `stream` at:
 *   [0] start, [1] grid cleared, [2] depos binned to tiles,
 *   [3] LDS-tiled raster + scatter done, [4] large-patch raster done,
 *   [5] tick-axis FFT done, [6] pitch-axis convolution done,
 *   [7] inverse tick-axis FFT done (end).
 * Same results and errors as wcsim_simulate_event; WCSIM_E_INVALID if
 * `events` or one of its entries is NULL. */
#define WCSIM_NUM_STAGE_EVENTS 8
wcsim_status wcsim_simulate_event_profiled(const wcsim_plane *plane, const wcsim_depo *depos,
                                           int64_t n, wcsim_mem depo_mem, uint64_t event_id,
                                           float *out, wcsim_out out_kind, wcsim_mem out_mem,
                                           void *workspace, void *stream, void *const *events);

/* Schedule tuning (the paper treats launch geometry as a tuning parameter,
 * Sec. 5.3): times wcsim_simulate_event of one plane under each of `ncand`
 * candidate schedules on the caller's `n` device depos.  For each candidate
 * a plane is created from desc/phys (its response spectrum included), two
 * untimed events are run, then `reps` timed events (HIP events on `stream`);
 * ms[i] receives the median time per event in milliseconds, or -1 when
 * candidate i is not a valid schedule for this plane.  Allocates and frees
 * its own device workspace and output; synchronises `stream`.  Errors:
 * WCSIM_E_INVALID for bad arguments or when no candidate is valid,
 * WCSIM_E_NOMEM, WCSIM_E_DEVICE.  Results do not depend on the schedule
 * (within the stated tolerances); only the time does. */
wcsim_status wcsim_tune_schedules(const wcsim_plane_desc *desc, const wcsim_physics *phys,
                                  const wcsim_schedule *cands, int32_t ncand,
                                  const wcsim_depo *depos, int64_t n, wcsim_out out_kind,
                                  int32_t reps, void *stream, float *ms);

/* Device pointer to the [npitch][nticks] grid inside a simulate workspace.
 * After wcsim_simulate_event it holds the event's grid (Sec. 2 step 2) in
 * every block of 32 pitch rows x 2^k ticks (the least k >= 6 with at most 64
 * blocks per row) that a depo window reaches; the other blocks are neither
 * cleared nor read by the event (the convolution takes them as zero) and
 * keep whatever they held.  Call wcsim_workspace_grid_complete to zero them
 * when the whole grid is wanted. */
float *wcsim_workspace_grid(const wcsim_plane *plane, void *workspace, int64_t n);

/* Zero, on `stream`, the blocks of the workspace grid that the last
 * wcsim_simulate_event with this workspace, plane and depo count n did not
 * reach, so that the whole grid (wcsim_workspace_grid) is that event's.
 * Errors: WCSIM_E_STATE for a NULL plane, WCSIM_E_INVALID for a NULL or
 * misaligned workspace or n < 0, WCSIM_E_DEVICE. */
wcsim_status wcsim_workspace_grid_complete(const wcsim_plane *plane, void *workspace, int64_t n,
                                           void *stream);

/* Number of invalid depos dropped by the last wcsim_simulate_event that used
 * this workspace (synchronises `stream`). */
wcsim_status wcsim_workspace_invalid_count(const void *workspace, void *stream, int64_t *count);

/* Batched form: nevents events, each with its own plane (planes may repeat),
 * depos (device memory), event id and output (device memory), run as chunks
 * of launch sequences whose kernels each cover every event of a chunk (see
 * wcsim_batch_chunk_count).  Asynchronous on `stream`: the batch is complete
 * in `stream`'s order.  `workspace`: device memory of at least
 * wcsim_batch_workspace_bytes bytes. */
size_t wcsim_batch_workspace_bytes(const wcsim_plane *const *planes, const int64_t *n,
                                   int32_t nevents, wcsim_out out_kind);
wcsim_status wcsim_simulate_batch(const wcsim_plane *const *planes,
                                  const wcsim_depo *const *depos, const int64_t *n,
                                  const uint64_t *event_ids, int32_t nevents,
                                  float *const *outs, wcsim_out out_kind, void *workspace,
                                  void *stream);

/* Number of chunks wcsim_simulate_batch cuts these events into: the events
 * are grouped by schedule class (planes whose kernels can share a launch) and
 * each class is cut into chunks of at most 16 events, in the callers' order.
 * A chunk's rasterization (binning, records, LDS-tiled raster) runs as one
 * launch sequence on `stream`, its three FFT passes as another on a second
 * stream of the library's, so that one chunk's rasterization overlaps the
 * previous chunk's passes; chunk data alternate between two halves of the
 * workspace.  0 for bad arguments. */
int32_t wcsim_batch_chunk_count(const wcsim_plane *const *planes, const int64_t *n,
                                int32_t nevents, wcsim_out out_kind);

/* wcsim_simulate_batch with stage timing (the paper's per-kernel timers,
 * Sec. 5.2): `events` holds WCSIM_BATCH_STAGE_EVENTS hipEvent_t handles per
 * chunk (nevents_events = chunks * WCSIM_BATCH_STAGE_EVENTS), recorded for
 * chunk c (base b = 9c) at [b + 0] start of its rasterization, [b + 1] depos
 * binned and records built, [b + 2] LDS-tiled raster done, [b + 3]
 * large-patch raster done (on `stream`), [b + 4] start of its tick-axis and
 * pitch-axis passes, [b + 5] tick-axis FFT done, [b + 6] pitch-axis
 * convolution done (on the library's second stream), [b + 8] start and
 * [b + 7] end of its inverse tick-axis FFT (on `stream`, after the next
 * chunk's rasterization).  WCSIM_E_INVALID when the count does not match or
 * an entry is NULL. */
#define WCSIM_BATCH_STAGE_EVENTS 9
wcsim_status wcsim_simulate_batch_profiled(const wcsim_plane *const *planes,
                                           const wcsim_depo *const *depos, const int64_t *n,
                                           const uint64_t *event_ids, int32_t nevents,
                                           float *const *outs, wcsim_out out_kind,
                                           void *workspace, void *stream, void *const *events,
                                           int32_t nevents_events);

/* Captured batch (hipGraph): the launch sequence of a batch of up to
 * capacity[e] depos per event on the given planes is captured once; each run
 * then uploads only the event descriptors (depo pointers and counts, event ids,
 * outputs) and replays the graph, so repeated batches of this shape pay no
 * per-kernel launch cost and no re-capture.  `workspace` (device, at least
 * wcsim_batch_workspace_bytes(planes, capacity, nevents, out_kind) bytes,
 * 256-byte aligned) stays bound to the batch until wcsim_batch_destroy.
 * Runs on one batch object are serialised (a run waits until the previous
 * run's descriptors have been uploaded).  Errors: WCSIM_E_INVALID for bad
 * arguments or counts above capacity. */
typedef struct wcsim_batch wcsim_batch;
wcsim_status wcsim_batch_create(const wcsim_plane *const *planes, const int64_t *capacity,
                                int32_t nevents, wcsim_out out_kind, void *workspace,
                                wcsim_batch **out);
wcsim_status wcsim_batch_run(wcsim_batch *batch, const wcsim_depo *const *depos,
                             const int64_t *n, const uint64_t *event_ids, float *const *outs,
                             void *stream);
void wcsim_batch_destroy(wcsim_batch *batch);

/* Digitisation with white noise: an extension beyond the paper, which ends at
 * the current induced on the wires (Sec. 2).  Each sample w of a waveform
 * `wave` [nrows][ncols] float32 (device memory; e.g. a simulate_event output)
 * becomes the ADC code
 *   adc = min(max(rint(((w * gain) + pedestal) + sigma * z), 0), 2^bits - 1)
 * stored as uint16 in `adc` [nrows][ncols] (device memory, caller-owned).  The
 * arithmetic is float32 in exactly that order with no fused multiply-add,
 * rint rounds half to even.  z is a standard normal deviate per sample (white
 * noise of sigma ADC counts; sigma = 0: none) from Philox4x32-10 under the key
 * (seed low word XOR 0x6e6f6973, seed high word) at counter (floor(col / 4),
 * row, 0, event_id low word): one call serves four consecutive columns, words
 * (0,1) the columns with col mod 4 in {0,1} and words (2,3) the others, each
 * pair through Box-Muller with the cosine branch to the even column; the
 * uniform of a word r is ((r >> 9) + 1/2) 2^-23 and the transform is evaluated
 * in FP64 (rho = sqrt(-2 ln u_a), theta = 2 pi u_b), z rounded once to
 * float32.
 * Requires nrows, ncols >= 0, 1 <= bits <= 16, finite gain and pedestal,
 * finite sigma >= 0; otherwise WCSIM_E_INVALID.  Asynchronous on `stream`. */
wcsim_status wcsim_digitize(const float *wave, int64_t nrows, int64_t ncols, float gain,
                            float pedestal, float sigma, int32_t bits, uint64_t seed,
                            uint64_t event_id, uint16_t *adc, void *stream);

/* Digitisation with coloured noise (same extension): as wcsim_digitize, with
 * the white deviates z filtered by the causal FIR filter fir[0..nfir) (device
 * memory, float32) before scaling by sigma:
 *   n[row][col] = sum_{k < nfir, k <= col} fir[k] z[row][col - k]
 * with z the FP64 deviates and the sum in FP64, n rounded once to float32:
 *   adc = min(max(rint(((w * gain) + pedestal) + sigma * n), 0), 2^bits - 1),
 * the noise spectrum being |DFT(fir)|^2 (white noise before column 0 is
 * zero).  z is the deviate wcsim_digitize uses, so fir = {1} reproduces it.
 * 1 <= nfir <= 1024; other requirements and errors as wcsim_digitize. */
wcsim_status wcsim_digitize_coloured(const float *wave, int64_t nrows, int64_t ncols, float gain,
                                     float pedestal, float sigma, const float *fir, int32_t nfir,
                                     int32_t bits, uint64_t seed, uint64_t event_id, uint16_t *adc,
                                     void *stream);

/* Diagnostic: the Philox4x32-10 generator the fluctuation uses (Sec. 4.1,
 * random123), evaluated on the GPU: out[i] = Philox4x32-10(ctr[i], key[i]).
 * ctr/out: n x 4 uint32, key: n x 2 uint32, all device memory. */
wcsim_status wcsim_philox4x32_10(const uint32_t *ctr, const uint32_t *key, int64_t n,
                                 uint32_t *out, void *stream);

const char *wcsim_last_error(void);

/* Library version (major*10000 + minor*100 + patch): 10400. */
int32_t wcsim_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WCSIM_H */
