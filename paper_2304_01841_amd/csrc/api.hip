// C ABI of libwcsim (declared in include/wcsim.h): argument validation,
// plane objects with their resident response spectra, patch sets, workspace
// carving and the launch sequences of the DepoTransform steps
// (arXiv:2304.01841, Sec. 2).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "wcsim_internal.h"

// Device buffers of a response spectrum and its twiddle tables, with the
// host response they were built from (to recognise a compatible donor).
struct wcs_spectrum {
    float2 *K = nullptr, *twT = nullptr, *twHalf = nullptr, *twL = nullptr, *twF = nullptr;
    float2 *H = nullptr, *twP = nullptr;  // polyphase spectra and table (poly planes)
    std::vector<float> response, elec;
    int Rp = 0, Rt = 0, r0 = 0, Nfft = 0, L = 0, F = 0, device = -1;
    bool poly = false;
    ~wcs_spectrum()
    {
        (void)hipFree(H);
        (void)hipFree(twP);
        (void)hipFree(K);
        (void)hipFree(twT);
        (void)hipFree(twHalf);
        (void)hipFree(twL);
        (void)hipFree(twF);
    }
};

namespace wcs {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

wcsim_status fail(wcsim_status st, const std::string &msg)
{
    set_error(msg);
    return st;
}

wcsim_status check_hip(hipError_t e, const char *what)
{
    set_error(std::string("HIP error in ") + what + ": " + hipGetErrorString(e));
    return (e == hipErrorOutOfMemory) ? WCSIM_E_NOMEM : WCSIM_E_DEVICE;
}

namespace {

bool finite_all(std::initializer_list<double> v)
{
    for (double x : v)
        if (!std::isfinite(x))
            return false;
    return true;
}

// Tick extent of the response a plane convolves with: the caller's response
// convolved along ticks with the electronics response, if there is one.
int effective_resp_nticks(const wcsim_plane_desc *d)
{
    return d->resp_nticks + (d->elec_nticks > 0 ? d->elec_nticks - 1 : 0);
}

wcsim_status validate_plane(const wcsim_plane_desc *d, const wcsim_physics *ph)
{
    if (!d || !ph)
        return fail(WCSIM_E_INVALID, "NULL plane descriptor or physics");
    if (d->nwires <= 0 || d->nimpact < 1 || d->nticks <= 0)
        return fail(WCSIM_E_INVALID, "nwires, nimpact and nticks must be positive");
    if ((int64_t)d->nwires * d->nimpact > (1LL << 30) || d->nticks > (1 << 24))
        return fail(WCSIM_E_INVALID, "plane too large");
    if (!finite_all({d->pitch, d->tick, d->t0, d->plane_x, d->dir_y, d->dir_z, d->pitch_origin}))
        return fail(WCSIM_E_INVALID, "non-finite plane geometry");
    if (!(d->pitch > 0.0) || !(d->tick > 0.0))
        return fail(WCSIM_E_INVALID, "pitch and tick must be positive");
    const double norm = d->dir_y * d->dir_y + d->dir_z * d->dir_z;
    if (fabs(norm - 1.0) > 1e-6)
        return fail(WCSIM_E_INVALID, "pitch direction must be a unit vector");
    if (d->resp_npitch <= 0 || d->resp_nticks <= 0 || !d->response)
        return fail(WCSIM_E_INVALID, "response must be non-empty");
    if (d->resp_origin < 0 || d->resp_origin >= d->resp_npitch)
        return fail(WCSIM_E_INVALID, "resp_origin outside [0, resp_npitch)");
    if (d->resp_npitch > 4096 || d->resp_nticks > 8192)
        return fail(WCSIM_E_INVALID, "response too large");
    for (int64_t i = 0; i < (int64_t)d->resp_npitch * d->resp_nticks; ++i)
        if (!std::isfinite(d->response[i]))
            return fail(WCSIM_E_INVALID, "non-finite response value");
    if (d->elec_nticks < 0 || d->elec_nticks > 8192 || (d->elec_nticks > 0 && !d->elec_response))
        return fail(WCSIM_E_INVALID, "electronics response: 0..8192 samples");
    for (int i = 0; i < d->elec_nticks; ++i)
        if (!std::isfinite(d->elec_response[i]))
            return fail(WCSIM_E_INVALID, "non-finite electronics response value");
    if (!finite_all({ph->drift_speed, ph->DL, ph->DT, ph->nsigma, ph->lifetime, ph->drift_accel}))
        return fail(WCSIM_E_INVALID, "non-finite physics constant");
    if (ph->lifetime < 0.0)
        return fail(WCSIM_E_INVALID, "lifetime must be >= 0");
    if (!(ph->drift_speed > 0.0) || ph->DL < 0.0 || ph->DT < 0.0 || ph->nsigma < 0.0)
        return fail(WCSIM_E_INVALID, "drift speed must be > 0 and DL, DT, nsigma >= 0");
    if (ph->fluctuate != 0 && ph->fluctuate != 1)
        return fail(WCSIM_E_INVALID, "fluctuate must be 0 or 1");
    if (ph->reserved != 0 || d->reserved != 0 || d->reserved2 != 0)
        return fail(WCSIM_E_INVALID, "reserved fields must be 0");
    return WCSIM_OK;
}

int pow2_at_least(int v)
{
    int p = 1;
    while (p < v)
        p *= 2;
    return p;
}

// Two-level table of W = exp(-2 pi i / n) for exponents j < count, rounded
// from FP64: entries 0..63 hold W^l, entry 64 + h holds W^(64 h), so that
// W^j = T[64 + j / 64] T[j mod 64].
std::vector<float2> twiddles(int n, int count)
{
    std::vector<float2> t((size_t)twiddle_table_len(count));
    auto w = [n](int64_t j) {
        const double a = -2.0 * M_PI * (double)(j % n) / (double)n;
        return make_float2((float)cos(a), (float)sin(a));
    };
    for (int l = 0; l < 64; ++l)
        t[(size_t)l] = w(l);
    for (size_t h = 64; h < t.size(); ++h)
        t[h] = w(64 * (int64_t)(h - 64));
    return t;
}

void free_plane(wcsim_plane *p)
{
    delete p;  // device buffers belong to the (possibly shared) spectrum
}

constexpr size_t kLdsBytes = 160 * 1024;

wcsim_status choose_schedule(wcsim_plane *pl, const wcsim_schedule *sc)
{
    const int nmin = (int)(pl->Nt + pl->Rt - 1);
    int nfft = (sc && sc->fft_ticks) ? sc->fft_ticks : smallest_smooth_even(nmin);
    if (nfft < nmin || (nfft & 1))
        return fail(WCSIM_E_INVALID, "fft_ticks must be even and >= nticks + resp_nticks - 1");
    pl->Nfft = nfft;
    pl->N2 = nfft / 2;
    if (!make_plan(pl->N2, &pl->planT))
        return fail(WCSIM_E_INVALID, "fft_ticks/2 must factor into 2, 3 and 5");
    if (sizeof(float2) * ((size_t)(pl->N2 + 1) * 2 + twiddle_table_len(pl->N2) +
                          twiddle_table_len(pl->N2 + 1)) > kLdsBytes ||
        twiddle_table_len(pl->N2 + 1) > 256)
        return fail(WCSIM_E_INVALID, "tick-axis transform too long for LDS");
    // Default pitch block: about four response lengths (the overlap-save
    // history is Rp - 1 of the L rows), in 8-column chunks from L = 1024 on so
    // that a block fits 64 KB of LDS.
    int L = (sc && sc->fft_pitch) ? sc->fft_pitch
                                  : std::min(2048, std::max(256, pow2_at_least(4 * pl->Rp)));
    pl->F = (sc && sc->freq_chunk) ? sc->freq_chunk : (L >= 1024 ? 8 : 16);
    if (pl->F != 8 && pl->F != 16)
        return fail(WCSIM_E_INVALID, "freq_chunk must be 8 or 16");
    if (L < pl->Rp)
        return fail(WCSIM_E_INVALID, "fft_pitch must be >= resp_npitch");
    if (!make_plan(L, &pl->planL))
        return fail(WCSIM_E_INVALID, "fft_pitch must factor into 2, 3 and 5");
    // columns per pitch workgroup: the whole chunk while an L x F block fits
    // 64 KB (two workgroups per CU), else halves of it
    pl->Fb = pl->F;
    while (pl->Fb > 4 && sizeof(float2) * (size_t)L * pl->Fb > 64 * 1024)
        pl->Fb /= 2;
    // folded wire-output inverse when nimpact divides L
    const int D = pl->desc.nimpact;
    pl->fold = D > 1 && L % D == 0 && make_plan(L / D, &pl->planF) &&
               twiddle_table_len(L / D) <= 256;
    pl->L10 = pl->fold ? L / D : 0;
    if (sizeof(float2) * ((size_t)L * pl->Fb + (size_t)pl->L10 * pl->Fb + twiddle_table_len(L) +
                          (pl->fold ? twiddle_table_len(pl->L10) + D : 0)) > kLdsBytes ||
        twiddle_table_len(L) > 256)
        return fail(WCSIM_E_INVALID, "pitch block too large for LDS");
    {
        // every pass must stage at most 32 complex values per thread of 1024
        for (int q = 0; q < pl->planL.npass; ++q) {
            const int R = pl->planL.radix[q];
            if ((int64_t)L / R * pl->Fb > 1024LL * (32 / R))
                return fail(WCSIM_E_INVALID, "pitch block too large for one workgroup");
        }
        for (int q = 0; q < pl->planT.npass; ++q) {
            const int R = pl->planT.radix[q];
            if ((int64_t)pl->N2 / R * 2 > 1024LL * (32 / R))
                return fail(WCSIM_E_INVALID, "tick transform too large for one workgroup");
        }
    }
    pl->L = L;
    pl->V = L - pl->Rp + 1;
    pl->nblocks = (int)((pl->Np + pl->V - 1) / pl->V);
    // Wire output: the polyphase pitch pass when each of the nimpact phase
    // filters has at most poly_max_taps() taps (wire_mode 0 or 1), else the
    // overlap-save blocks of L rows (wire_mode 2, or 0 when it does not apply).
    const int wm = sc ? sc->wire_mode : 0;
    if (wm < 0 || wm > 2)
        return fail(WCSIM_E_INVALID, "wire_mode must be 0, 1 or 2");
    const int taps = (int)((pl->Rp + D - 1) / D);
    const bool poly_ok = D > 1 && taps <= poly_max_taps();
    if (wm == 1 && !poly_ok)
        return fail(WCSIM_E_INVALID,
                    "polyphase wire output needs nimpact > 1 and ceil(resp_npitch / nimpact) <= 64");
    pl->poly = poly_ok && wm != 2;
    pl->polyA = taps;
    pl->polyV = poly_block_rows() - taps + 1;
    pl->polyBlocks = (int)((pl->Nw + pl->polyV - 1) / pl->polyV);
    pl->polyCw = D / 2 + pl->r0;
    pl->H = pl->N2 + 1;
    pl->C = (pl->H + pl->F - 1) / pl->F;
    const int det = sc ? sc->deterministic : 0;
    if (det < 0 || det > 1)
        return fail(WCSIM_E_INVALID, "deterministic must be 0 or 1");
    pl->det = det == 1;
    pl->tile = (sc && sc->tile) ? sc->tile : 0;
    if (pl->tile < 0 || pl->tile >= kNumTileShapes)
        return fail(WCSIM_E_INVALID, "unknown tile shape");
    pl->ts = tile_shape(pl->tile);
    pl->ntp = (int)((pl->Np + pl->ts.tp - 1) / pl->ts.tp);
    pl->ntt = (int)((pl->Nt + pl->ts.tt - 1) / pl->ts.tt);
    pl->ntiles = (int64_t)pl->ntp * pl->ntt;
    return WCSIM_OK;
}

template <typename T>
wcsim_status upload(T **dst, const std::vector<T> &src, hipStream_t s)
{
    WCS_HIP(hipMalloc((void **)dst, sizeof(T) * src.size()));
    WCS_HIP(hipMemcpyAsync(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s));
    return WCSIM_OK;
}

wcsim_status plane_create(const wcsim_plane_desc *desc, const wcsim_physics *phys,
                          const wcsim_schedule *sched, const wcsim_plane *donor, void *stream,
                          wcsim_plane **out)
{
    if (!out)
        return fail(WCSIM_E_INVALID, "NULL output handle");
    *out = nullptr;
    wcsim_status st = validate_plane(desc, phys);
    if (st != WCSIM_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    wcsim_plane *pl = new (std::nothrow) wcsim_plane();
    if (!pl)
        return fail(WCSIM_E_NOMEM, "host allocation failed");
    pl->desc = *desc;
    pl->desc.response = nullptr;
    pl->phys = *phys;
    (void)hipGetDevice(&pl->device);
    pl->Np = (int64_t)desc->nwires * desc->nimpact;
    pl->Nt = desc->nticks;
    pl->Nw = desc->nwires;
    pl->Rp = desc->resp_npitch;
    pl->Rt = effective_resp_nticks(desc);
    pl->r0 = desc->resp_origin;
    PlaneParams &k = pl->kp;
    k.v = phys->drift_speed;
    k.DL = phys->DL;
    k.DT = phys->DT;
    k.nsigma = phys->nsigma;
    k.dp = desc->pitch / (double)desc->nimpact;
    k.tick = desc->tick;
    k.t0 = desc->t0;
    k.plane_x = desc->plane_x;
    k.dir_y = desc->dir_y;
    k.dir_z = desc->dir_z;
    k.pitch_origin = desc->pitch_origin;
    k.Np = (int32_t)pl->Np;
    k.Nt = (int32_t)pl->Nt;
    k.nimpact = desc->nimpact;
    k.plane_id = desc->plane_id;
    k.key0 = (uint32_t)phys->seed;
    k.key1 = (uint32_t)(phys->seed >> 32) ^ (uint32_t)desc->plane_id;
    k.lkey0 = (uint32_t)phys->seed ^ 0x6c696665u;
    k.lkey1 = (uint32_t)(phys->seed >> 32);
    k.fluct = phys->fluctuate;
    k.pad_ = 0;
    k.tau = phys->lifetime;
    k.accel = phys->drift_accel;
    if ((st = choose_schedule(pl, sched)) != WCSIM_OK) {
        free_plane(pl);
        return st;
    }
    // the caller's response and electronics response; the plane convolves
    // with their combination, Rp x Rt (effective) built on the device
    const size_t nresp0 = (size_t)pl->Rp * desc->resp_nticks;
    const size_t nelec = (size_t)desc->elec_nticks;
    const size_t nresp = (size_t)pl->Rp * pl->Rt;
    if (donor && donor->spectrum) {
        const wcs_spectrum &d = *donor->spectrum;
        if (d.Rp == pl->Rp && d.Rt == pl->Rt && d.r0 == pl->r0 && d.Nfft == pl->Nfft &&
            d.L == pl->L && d.F == pl->F && d.device == pl->device && (d.twF != nullptr) == pl->fold &&
            d.poly == pl->poly && (!pl->poly || pl->kp.nimpact == donor->kp.nimpact) &&
            d.response.size() == nresp0 && d.elec.size() == nelec &&
            memcmp(d.response.data(), desc->response, sizeof(float) * nresp0) == 0 &&
            (nelec == 0 || memcmp(d.elec.data(), desc->elec_response, sizeof(float) * nelec) == 0)) {
            pl->spectrum = donor->spectrum;
            pl->K = d.K;
            pl->twT = d.twT;
            pl->twHalf = d.twHalf;
            pl->twL = d.twL;
            pl->twF = d.twF;
            pl->KP = d.H;
            pl->twP = d.twP;
            *out = pl;
            return WCSIM_OK;
        }
    }
    float *resp = nullptr;
    void *work = nullptr;
    auto cleanup = [&](wcsim_status r) {
        (void)hipFree(resp);
        (void)hipFree(work);
        if (r != WCSIM_OK)
            free_plane(pl);
        return r;
    };
    auto spec = std::make_shared<wcs_spectrum>();
    pl->spectrum = spec;
    spec->response.assign(desc->response, desc->response + nresp0);
    if (nelec)
        spec->elec.assign(desc->elec_response, desc->elec_response + nelec);
    spec->Rp = pl->Rp;
    spec->Rt = pl->Rt;
    spec->r0 = pl->r0;
    spec->Nfft = pl->Nfft;
    spec->L = pl->L;
    spec->F = pl->F;
    spec->device = pl->device;
    spec->poly = pl->poly;
    if ((st = upload(&spec->twT, twiddles(pl->N2, pl->N2), s)) != WCSIM_OK ||
        (st = upload(&spec->twHalf, twiddles(pl->Nfft, pl->N2 + 1), s)) != WCSIM_OK ||
        (st = upload(&spec->twL, twiddles(pl->L, pl->L), s)) != WCSIM_OK ||
        (pl->fold && (st = upload(&spec->twF, twiddles(pl->L10, pl->L10), s)) != WCSIM_OK) ||
        (pl->poly && (st = upload(&spec->twP, twiddles(poly_block_rows(), poly_block_rows()), s)) !=
                         WCSIM_OK))
        return cleanup(st);
    pl->twT = spec->twT;
    pl->twHalf = spec->twHalf;
    pl->twL = spec->twL;
    pl->twF = spec->twF;
    pl->twP = spec->twP;
    hipError_t e;
    const size_t kbytes = sizeof(float2) * (size_t)pl->C * pl->L * pl->F;
    if ((e = hipMalloc((void **)&spec->K, kbytes)) != hipSuccess)
        return cleanup(check_hip(e, "hipMalloc(response spectrum)"));
    pl->K = spec->K;
    if (pl->poly) {
        const size_t hbytes =
            sizeof(float2) * (size_t)pl->C * pl->kp.nimpact * poly_block_rows() * pl->F;
        if ((e = hipMalloc((void **)&spec->H, hbytes)) != hipSuccess)
            return cleanup(check_hip(e, "hipMalloc(polyphase response spectra)"));
        pl->KP = spec->H;
    }
    // device copies: [combined Rp x Rt | caller's Rp x Rt0 | electronics]
    const size_t rbytes = sizeof(float) * (nresp + nresp0 + nelec);
    if ((e = hipMalloc((void **)&resp, rbytes)) != hipSuccess)
        return cleanup(check_hip(e, "hipMalloc(response)"));
    if ((e = hipMalloc(&work, response_work_bytes(pl))) != hipSuccess)
        return cleanup(check_hip(e, "hipMalloc(response work)"));
    if (nelec == 0) {
        if ((e = hipMemcpyAsync(resp, desc->response, sizeof(float) * nresp,
                                hipMemcpyHostToDevice, s)) != hipSuccess)
            return cleanup(check_hip(e, "hipMemcpyAsync(response)"));
    } else {
        float *r0d = resp + nresp, *ed = r0d + nresp0;
        if ((e = hipMemcpyAsync(r0d, desc->response, sizeof(float) * nresp0,
                                hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(ed, desc->elec_response, sizeof(float) * nelec,
                                hipMemcpyHostToDevice, s)) != hipSuccess)
            return cleanup(check_hip(e, "hipMemcpyAsync(response)"));
        if ((e = launch_combine_response(r0d, pl->Rp, desc->resp_nticks, ed, (int)nelec, resp,
                                         s)) != hipSuccess)
            return cleanup(check_hip(e, "combined response"));
    }
    if ((e = build_response_spectrum(pl, resp, work, s)) != hipSuccess)
        return cleanup(check_hip(e, "response spectrum"));
    if ((e = hipStreamSynchronize(s)) != hipSuccess)
        return cleanup(check_hip(e, "hipStreamSynchronize"));
    *out = pl;
    return cleanup(WCSIM_OK);
}

// Host-side checks of host depos: finite fields, q >= 0, x >= plane_x, a depo
// that can reach the plane, and a window no longer than kMaxWindow bins at the
// longest drift time.
wcsim_status validate_host_depos(const wcsim_plane *pl, const wcsim_depo *d, int64_t n)
{
    const PlaneParams &k = pl->kp;
    double T = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const wcsim_depo &q = d[i];
        if (!finite_all({q.x, q.y, q.z, q.t, q.q}))
            return fail(WCSIM_E_INVALID, "depo " + std::to_string(i) + " has a non-finite field");
        if (q.q < 0.0)
            return fail(WCSIM_E_INVALID, "depo " + std::to_string(i) + " has negative charge");
        if (q.x < k.plane_x)
            return fail(WCSIM_E_INVALID,
                        "depo " + std::to_string(i) + " lies behind the response plane");
        const double L = q.x - k.plane_x;
        const double disc = k.v * k.v - 2.0 * k.accel * L;
        if (disc < 0.0)
            return fail(WCSIM_E_INVALID,
                        "depo " + std::to_string(i) + " cannot reach the response plane");
        T = std::max(T, (2.0 * L) / (k.v + sqrt(disc)));
    }
    const double sp = sqrt(2.0 * pl->kp.DT * T) / pl->kp.dp;
    const double stt = sqrt(2.0 * pl->kp.DL * T) / pl->kp.v / pl->kp.tick;
    if (2.0 * pl->kp.nsigma * std::max(sp, stt) + 2.0 > (double)kMaxWindow)
        return fail(WCSIM_E_INVALID, "patch window longer than 1024 bins");
    return WCSIM_OK;
}

}  // namespace
}  // namespace wcs

using namespace wcs;

extern "C" {

int32_t wcsim_version(void) { return 10400; }

const char *wcsim_last_error(void) { return g_last_error.c_str(); }

wcsim_status wcsim_plane_create(const wcsim_plane_desc *desc, const wcsim_physics *phys,
                                void *stream, wcsim_plane **out)
{
    return plane_create(desc, phys, nullptr, nullptr, stream, out);
}

wcsim_status wcsim_plane_create_with_schedule(const wcsim_plane_desc *desc,
                                              const wcsim_physics *phys,
                                              const wcsim_schedule *sched, void *stream,
                                              wcsim_plane **out)
{
    return plane_create(desc, phys, sched, nullptr, stream, out);
}

wcsim_status wcsim_plane_create_sharing(const wcsim_plane_desc *desc, const wcsim_physics *phys,
                                        const wcsim_plane *donor, void *stream, wcsim_plane **out)
{
    if (!donor)
        return fail(WCSIM_E_INVALID, "NULL spectrum donor");
    wcsim_schedule sc{};
    sc.fft_ticks = donor->Nfft;
    sc.fft_pitch = donor->L;
    sc.freq_chunk = donor->F;
    sc.tile = donor->tile;
    sc.wire_mode = donor->poly ? 0 : 2;
    sc.deterministic = donor->det ? 1 : 0;
    // the donor's transform may be too short for a longer readout
    if (desc && donor->Nfft < desc->nticks + effective_resp_nticks(desc) - 1)
        return plane_create(desc, phys, nullptr, nullptr, stream, out);
    return plane_create(desc, phys, &sc, donor, stream, out);
}

void wcsim_plane_destroy(wcsim_plane *plane)
{
    if (!plane)
        return;
    (void)hipDeviceSynchronize();
    free_plane(plane);
}

wcsim_status wcsim_plane_get_info(const wcsim_plane *pl, wcsim_plane_info *info)
{
    if (!pl || !info)
        return fail(WCSIM_E_INVALID, "NULL argument");
    info->npitch = pl->Np;
    info->nticks = pl->Nt;
    info->nwires = pl->Nw;
    info->nimpact = pl->kp.nimpact;
    info->fft_ticks = pl->Nfft;
    info->fft_pitch = pl->L;
    info->freq_chunk = pl->F;
    info->tile = pl->tile;
    info->nchunks = pl->C;
    info->pitch_blocks = pl->nblocks;
    info->tile_pitch = pl->ts.tp;
    info->tile_ticks = pl->ts.tt;
    info->ntiles = pl->ntiles;
    info->spectrum_bytes = (int64_t)sizeof(float2) * pl->C * pl->L * pl->F +
                           (pl->poly ? (int64_t)sizeof(float2) * pl->C * pl->kp.nimpact *
                                           poly_block_rows() * pl->F
                                     : 0);
    info->pitch_cols = pl->Fb;
    info->wire_fold = pl->fold ? 1 : 0;
    info->wire_polyphase = pl->poly ? 1 : 0;
    info->wire_blocks = pl->poly ? pl->polyBlocks : 0;
    info->deterministic = pl->det ? 1 : 0;
    return WCSIM_OK;
}

wcsim_status wcsim_philox4x32_10(const uint32_t *ctr, const uint32_t *key, int64_t n,
                                 uint32_t *out, void *stream)
{
    if (n < 0 || (n > 0 && (!ctr || !key || !out)))
        return fail(WCSIM_E_INVALID, "bad Philox arguments");
    WCS_HIP(launch_philox(ctr, key, n, out, (hipStream_t)stream));
    return WCSIM_OK;
}

wcsim_status wcsim_digitize(const float *wave, int64_t nrows, int64_t ncols, float gain,
                            float pedestal, float sigma, int32_t bits, uint64_t seed,
                            uint64_t event_id, uint16_t *adc, void *stream)
{
    if (nrows < 0 || ncols < 0 || (nrows > 0 && ncols > 0 && (!wave || !adc)))
        return fail(WCSIM_E_INVALID, "bad digitize sizes or pointers");
    if (ncols > 0 && nrows > INT64_MAX / 4 / ncols)
        return fail(WCSIM_E_INVALID, "waveform too large");
    if (bits < 1 || bits > 16 || !finite_all({gain, pedestal, sigma}) || sigma < 0.0f)
        return fail(WCSIM_E_INVALID, "bad digitize parameters");
    WCS_HIP(launch_digitize(wave, nrows, ncols, gain, pedestal, sigma, bits, seed,
                            (uint32_t)event_id, adc, (hipStream_t)stream));
    return WCSIM_OK;
}

wcsim_status wcsim_digitize_coloured(const float *wave, int64_t nrows, int64_t ncols, float gain,
                                     float pedestal, float sigma, const float *fir, int32_t nfir,
                                     int32_t bits, uint64_t seed, uint64_t event_id, uint16_t *adc,
                                     void *stream)
{
    if (nrows < 0 || ncols < 0 || (nrows > 0 && ncols > 0 && (!wave || !adc)))
        return fail(WCSIM_E_INVALID, "bad digitize sizes or pointers");
    if (ncols > 0 && nrows > INT64_MAX / 4 / ncols)
        return fail(WCSIM_E_INVALID, "waveform too large");
    if (nfir < 1 || nfir > kMaxFir || !fir)
        return fail(WCSIM_E_INVALID, "noise filter: 1..1024 taps");
    if (ncols > 0 && nrows * ((ncols + 1023) / 1024) > (int64_t)UINT32_MAX)
        return fail(WCSIM_E_INVALID, "waveform too large");
    if (bits < 1 || bits > 16 || !finite_all({gain, pedestal, sigma}) || sigma < 0.0f)
        return fail(WCSIM_E_INVALID, "bad digitize parameters");
    WCS_HIP(launch_digitize_fir(wave, nrows, ncols, gain, pedestal, sigma, fir, nfir, bits, seed,
                                (uint32_t)event_id, adc, (hipStream_t)stream));
    return WCSIM_OK;
}

wcsim_status wcsim_rasterize(const wcsim_plane *pl, const wcsim_depo *depos, int64_t n,
                             wcsim_mem mem, uint64_t event_id, void *stream, wcsim_patches **out)
{
    if (!pl)
        return fail(WCSIM_E_STATE, "NULL plane");
    if (!out || n < 0 || (n > 0 && !depos) || (mem != WCSIM_MEM_HOST && mem != WCSIM_MEM_DEVICE))
        return fail(WCSIM_E_INVALID, "bad rasterize arguments");
    if (n > (1LL << 31) - 1)
        return fail(WCSIM_E_INVALID, "too many depos");
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    if (mem == WCSIM_MEM_HOST) {
        wcsim_status st = validate_host_depos(pl, depos, n);
        if (st != WCSIM_OK)
            return st;
    }
    wcsim_patches *P = new (std::nothrow) wcsim_patches();
    if (!P)
        return fail(WCSIM_E_NOMEM, "host allocation failed");
    P->n = n;
    P->device = pl->device;
    void *scratch = nullptr;
    auto bail = [&](wcsim_status r) {
        (void)hipFree(scratch);
        if (r != WCSIM_OK) {
            (void)hipFree(P->meta);
            (void)hipFree(P->offsets);
            (void)hipFree(P->values);
            (void)hipFree(P->staged);
            delete P;
        } else {
            (void)hipFree(P->staged);
            P->staged = nullptr;
            *out = P;
        }
        return r;
    };
    hipError_t e;
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    if ((e = hipMalloc((void **)&P->meta, sizeof(int32_t) * 4 * nn)) != hipSuccess ||
        (e = hipMalloc((void **)&P->offsets, sizeof(int64_t) * (nn + 1))) != hipSuccess ||
        (e = hipMalloc(&scratch, scan_scratch_bytes(n + 1))) != hipSuccess)
        return bail(check_hip(e, "hipMalloc(patch set)"));
    const wcsim_depo *dd = depos;
    if (mem == WCSIM_MEM_HOST && n > 0) {
        if ((e = hipMalloc((void **)&P->staged, sizeof(wcsim_depo) * nn)) != hipSuccess)
            return bail(check_hip(e, "hipMalloc(depos)"));
        if ((e = hipMemcpyAsync(P->staged, depos, sizeof(wcsim_depo) * (size_t)n,
                                hipMemcpyHostToDevice, s)) != hipSuccess)
            return bail(check_hip(e, "hipMemcpyAsync(depos)"));
        dd = P->staged;
    }
    if ((e = launch_patch_sizes(pl, dd, n, P->meta, P->offsets, s)) != hipSuccess ||
        (e = launch_exclusive_scan_i64(P->offsets, n + 1, scratch, s)) != hipSuccess)
        return bail(check_hip(e, "patch sizes"));
    int64_t total = 0;
    if ((e = hipMemcpyAsync(&total, P->offsets + n, sizeof(int64_t), hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return bail(check_hip(e, "patch total"));
    P->nvalues = total;
    if ((e = hipMalloc((void **)&P->values, sizeof(float) * (size_t)std::max<int64_t>(total, 1))) !=
        hipSuccess)
        return bail(check_hip(e, "hipMalloc(patch values)"));
    if ((e = launch_patch_values(pl, dd, n, event_id, P->meta, P->offsets, P->values, s)) !=
        hipSuccess)
        return bail(check_hip(e, "patch values"));
    if ((e = hipStreamSynchronize(s)) != hipSuccess)
        return bail(check_hip(e, "hipStreamSynchronize"));
    return bail(WCSIM_OK);
}

wcsim_status wcsim_patches_count(const wcsim_patches *P, int64_t *ndepos, int64_t *nvalues)
{
    if (!P)
        return fail(WCSIM_E_STATE, "NULL patch set");
    if (ndepos)
        *ndepos = P->n;
    if (nvalues)
        *nvalues = P->nvalues;
    return WCSIM_OK;
}

wcsim_status wcsim_patches_device(const wcsim_patches *P, const int32_t **meta,
                                  const int64_t **offsets, const float **values)
{
    if (!P)
        return fail(WCSIM_E_STATE, "NULL patch set");
    if (meta)
        *meta = P->meta;
    if (offsets)
        *offsets = P->offsets;
    if (values)
        *values = P->values;
    return WCSIM_OK;
}

wcsim_status wcsim_patches_copy_to_host(const wcsim_patches *P, int32_t *meta, int64_t *offsets,
                                        float *values)
{
    if (!P)
        return fail(WCSIM_E_STATE, "NULL patch set");
    if (meta)
        WCS_HIP(hipMemcpy(meta, P->meta, sizeof(int32_t) * 4 * (size_t)P->n, hipMemcpyDeviceToHost));
    if (offsets)
        WCS_HIP(hipMemcpy(offsets, P->offsets, sizeof(int64_t) * (size_t)(P->n + 1),
                          hipMemcpyDeviceToHost));
    if (values && P->nvalues > 0)
        WCS_HIP(hipMemcpy(values, P->values, sizeof(float) * (size_t)P->nvalues,
                          hipMemcpyDeviceToHost));
    return WCSIM_OK;
}

void wcsim_patches_destroy(wcsim_patches *P)
{
    if (!P)
        return;
    (void)hipDeviceSynchronize();
    (void)hipFree(P->meta);
    (void)hipFree(P->offsets);
    (void)hipFree(P->values);
    (void)hipFree(P->staged);
    delete P;
}

wcsim_status wcsim_scatter_add(const wcsim_plane *pl, const wcsim_patches *P, float *grid,
                               int32_t zero_first, void *stream)
{
    if (!pl || !P)
        return fail(WCSIM_E_STATE, "NULL plane or patch set");
    if (!grid)
        return fail(WCSIM_E_INVALID, "NULL grid");
    hipStream_t s = (hipStream_t)stream;
    if (zero_first)
        WCS_HIP(launch_fill_zero(grid, sizeof(float) * (size_t)pl->Np * pl->Nt, s));
    WCS_HIP(launch_scatter_flat(pl, P->n, P->meta, P->offsets, P->values, grid, s));
    return WCSIM_OK;
}

size_t wcsim_convolve_workspace_bytes(const wcsim_plane *pl, wcsim_out out_kind)
{
    if (!pl)
        return 0;
    return conv_work_bytes(pl, out_kind);
}

wcsim_status wcsim_convolve(const wcsim_plane *pl, const float *grid, float *out,
                            wcsim_out out_kind, void *workspace, void *stream)
{
    if (!pl)
        return fail(WCSIM_E_STATE, "NULL plane");
    if (!grid || !out || !workspace)
        return fail(WCSIM_E_INVALID, "NULL grid, output or workspace");
    if (out_kind != WCSIM_OUT_WIRE && out_kind != WCSIM_OUT_PITCH)
        return fail(WCSIM_E_INVALID, "bad output kind");
    if (((uintptr_t)workspace & 255) != 0)
        return fail(WCSIM_E_INVALID, "workspace must be 256-byte aligned");
    WCS_HIP(launch_convolve(pl, grid, out, out_kind, workspace, (hipStream_t)stream));
    return WCSIM_OK;
}

static size_t sim_grid_offset(const wcsim_plane *pl, int64_t n) { return raster_work_bytes(pl, n); }

static size_t sim_conv_offset(const wcsim_plane *pl, int64_t n)
{
    return sim_grid_offset(pl, n) + align_up(sizeof(float) * (size_t)pl->Np * pl->Nt);
}

size_t wcsim_simulate_workspace_bytes(const wcsim_plane *pl, int64_t n, wcsim_out out_kind)
{
    if (!pl || n < 0)
        return 0;
    return sim_conv_offset(pl, n) + conv_work_bytes(pl, out_kind) +
           align_up(sizeof(wcsim_depo) * (size_t)std::max<int64_t>(n, 1));
}

float *wcsim_workspace_grid(const wcsim_plane *pl, void *workspace, int64_t n)
{
    if (!pl || !workspace)
        return nullptr;
    return (float *)((char *)workspace + sim_grid_offset(pl, n));
}

wcsim_status wcsim_workspace_grid_complete(const wcsim_plane *pl, void *workspace, int64_t n,
                                           void *stream)
{
    if (!pl)
        return fail(WCSIM_E_STATE, "NULL plane");
    if (!workspace || n < 0)
        return fail(WCSIM_E_INVALID, "bad workspace arguments");
    if (((uintptr_t)workspace & 255) != 0)
        return fail(WCSIM_E_INVALID, "workspace must be 256-byte aligned");
    const RasterWork rw = raster_work_carve(pl, n, workspace);
    WCS_HIP(launch_clear_unoccupied((float *)((char *)workspace + sim_grid_offset(pl, n)),
                                    (int)pl->Np, (int)pl->Nt, rw.occ, occ_shift_of(pl->Nt),
                                    (hipStream_t)stream));
    return WCSIM_OK;
}

wcsim_status wcsim_workspace_invalid_count(const void *workspace, void *stream, int64_t *count)
{
    if (!workspace || !count)
        return fail(WCSIM_E_INVALID, "NULL argument");
    int32_t c = 0;
    WCS_HIP(hipMemcpyAsync(&c, workspace, sizeof(int32_t), hipMemcpyDeviceToHost,
                           (hipStream_t)stream));
    WCS_HIP(hipStreamSynchronize((hipStream_t)stream));
    *count = c;
    return WCSIM_OK;
}

static wcsim_status simulate_event(const wcsim_plane *pl, const wcsim_depo *depos, int64_t n,
                                   wcsim_mem depo_mem, uint64_t event_id, float *out,
                                   wcsim_out out_kind, wcsim_mem out_mem, void *workspace,
                                   void *stream, const hipEvent_t *ev)
{
    if (!pl)
        return fail(WCSIM_E_STATE, "NULL plane");
    if (n < 0 || (n > 0 && !depos) || !out || !workspace)
        return fail(WCSIM_E_INVALID, "bad simulate arguments");
    if (n > (1LL << 31) - 1)
        return fail(WCSIM_E_INVALID, "too many depos");
    if ((depo_mem != WCSIM_MEM_HOST && depo_mem != WCSIM_MEM_DEVICE) ||
        (out_mem != WCSIM_MEM_HOST && out_mem != WCSIM_MEM_DEVICE))
        return fail(WCSIM_E_INVALID, "bad memory kind");
    if (out_kind != WCSIM_OUT_WIRE && out_kind != WCSIM_OUT_PITCH)
        return fail(WCSIM_E_INVALID, "bad output kind");
    if (((uintptr_t)workspace & 255) != 0)
        return fail(WCSIM_E_INVALID, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    const RasterWork rw = raster_work_carve(pl, n, ws);
    float *grid = (float *)(ws + sim_grid_offset(pl, n));
    char *conv = ws + sim_conv_offset(pl, n);
    wcsim_depo *staged = (wcsim_depo *)(conv + conv_work_bytes(pl, out_kind));
    const wcsim_depo *dd = depos;
    if (depo_mem == WCSIM_MEM_HOST) {
        wcsim_status st = validate_host_depos(pl, depos, n);
        if (st != WCSIM_OK)
            return st;
        if (n > 0)
            WCS_HIP(hipMemcpyAsync(staged, depos, sizeof(wcsim_depo) * (size_t)n,
                                   hipMemcpyHostToDevice, s));
        dd = staged;
    }
    if (ev)
        WCS_HIP(hipEventRecord(ev[0], s));
    // the grid is cleared inside the raster sequence (beside the record
    // building), so stage [0, 1] is empty
    if (ev)
        WCS_HIP(hipEventRecord(ev[1], s));
    WCS_HIP(launch_raster_fused(pl, dd, n, event_id, rw, grid, s, ev ? ev + 2 : nullptr));
    const int64_t nout = (out_kind == WCSIM_OUT_WIRE) ? pl->Nw : pl->Np;
    const size_t out_bytes = sizeof(float) * (size_t)nout * pl->Nt;
    // Host output: the spectrum buffer of pass A is free once pass B has run
    // and is at least as large as the output.
    float *dst = (out_mem == WCSIM_MEM_HOST) ? (float *)conv : out;
    WCS_HIP(launch_convolve(pl, grid, dst, out_kind, conv, s, ev ? ev + 5 : nullptr, rw.occ));
    if (out_mem == WCSIM_MEM_HOST) {
        WCS_HIP(hipMemcpyAsync(out, dst, out_bytes, hipMemcpyDeviceToHost, s));
        WCS_HIP(hipStreamSynchronize(s));
    }
    return WCSIM_OK;
}

wcsim_status wcsim_simulate_event(const wcsim_plane *pl, const wcsim_depo *depos, int64_t n,
                                  wcsim_mem depo_mem, uint64_t event_id, float *out,
                                  wcsim_out out_kind, wcsim_mem out_mem, void *workspace,
                                  void *stream)
{
    return simulate_event(pl, depos, n, depo_mem, event_id, out, out_kind, out_mem, workspace,
                          stream, nullptr);
}

wcsim_status wcsim_simulate_event_profiled(const wcsim_plane *pl, const wcsim_depo *depos,
                                           int64_t n, wcsim_mem depo_mem, uint64_t event_id,
                                           float *out, wcsim_out out_kind, wcsim_mem out_mem,
                                           void *workspace, void *stream, void *const *events)
{
    if (!events)
        return fail(WCSIM_E_INVALID, "NULL event array");
    for (int i = 0; i < WCSIM_NUM_STAGE_EVENTS; ++i)
        if (!events[i])
            return fail(WCSIM_E_INVALID, "NULL event in the event array");
    return simulate_event(pl, depos, n, depo_mem, event_id, out, out_kind, out_mem, workspace,
                          stream, (const hipEvent_t *)events);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free simulate: the workspace lives in a fixed device array that
// every GPU holds from the library's load until the process ends.  In host
// code `scratch` only names the symbol; its device address on each GPU comes
// from hipGetSymbolAddress, taken once per device and cached.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[WCSIM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device (nullptr: not yet)

wcsim_status scratch_of_current_device(int dev, void **ptr)
{
    if (dev < 0 || dev >= kMaxDevices)
        return fail(WCSIM_E_DEVICE, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return check_hip(e != hipSuccess ? e : hipErrorInvalidSymbol,
                             "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return WCSIM_OK;
}
}  // namespace

extern "C" {

wcsim_status wcsim_simulate_event_noalloc(const wcsim_plane *pl, const wcsim_depo *depos,
                                          int64_t n, uint64_t event_id, float *out,
                                          wcsim_out out_kind, void *stream)
{
    if (!pl)
        return fail(WCSIM_E_STATE, "NULL plane");
    if (n < 0 || (n > 0 && !depos) || !out)
        return fail(WCSIM_E_INVALID, "bad simulate arguments");
    if (out_kind != WCSIM_OUT_WIRE && out_kind != WCSIM_OUT_PITCH)
        return fail(WCSIM_E_INVALID, "bad output kind");
    const size_t need = wcsim_simulate_workspace_bytes(pl, n, out_kind);
    if (need > (size_t)WCSIM_NOALLOC_SCRATCH_BYTES)
        return fail(WCSIM_E_INVALID,
                    "event needs " + std::to_string(need) +
                        " bytes of workspace; the allocation-free entry point holds " +
                        std::to_string((size_t)WCSIM_NOALLOC_SCRATCH_BYTES));
    int dev = -1;
    WCS_HIP(hipGetDevice(&dev));
    if (dev != pl->device)
        return fail(WCSIM_E_INVALID, "the current device is not the plane's device");
    void *ws = nullptr;
    wcsim_status st = scratch_of_current_device(dev, &ws);
    if (st != WCSIM_OK)
        return st;
    return simulate_event(pl, depos, n, WCSIM_MEM_DEVICE, event_id, out, out_kind,
                          WCSIM_MEM_DEVICE, ws, stream, nullptr);
}

wcsim_status wcsim_tune_schedules(const wcsim_plane_desc *desc, const wcsim_physics *phys,
                                  const wcsim_schedule *cands, int32_t ncand,
                                  const wcsim_depo *depos, int64_t n, wcsim_out out_kind,
                                  int32_t reps, void *stream, float *ms)
{
    if (!desc || !phys || !cands || !ms || ncand < 1 || reps < 1 || n < 0 || (n > 0 && !depos))
        return fail(WCSIM_E_INVALID, "bad tuning arguments");
    if (out_kind != WCSIM_OUT_WIRE && out_kind != WCSIM_OUT_PITCH)
        return fail(WCSIM_E_INVALID, "bad output kind");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    WCS_HIP(hipEventCreate(&t0));
    if (hipEventCreate(&t1) != hipSuccess) {
        (void)hipEventDestroy(t0);
        return fail(WCSIM_E_DEVICE, "hipEventCreate failed");
    }
    wcsim_status result = WCSIM_OK;
    int timed = 0;
    for (int32_t i = 0; i < ncand && result == WCSIM_OK; ++i) {
        ms[i] = -1.0f;
        wcsim_plane *pl = nullptr;
        if (plane_create(desc, phys, &cands[i], nullptr, stream, &pl) != WCSIM_OK)
            continue;  // not a valid schedule for this plane
        const int64_t nout = (out_kind == WCSIM_OUT_WIRE) ? pl->Nw : pl->Np;
        void *ws = nullptr, *out = nullptr;
        if (hipMalloc(&ws, wcsim_simulate_workspace_bytes(pl, n, out_kind)) != hipSuccess ||
            hipMalloc(&out, sizeof(float) * (size_t)nout * pl->Nt) != hipSuccess) {
            result = fail(WCSIM_E_NOMEM, "device allocation failed while tuning");
        } else {
            std::vector<float> t;
            for (int r = -2; r < reps && result == WCSIM_OK; ++r) {  // r < 0 warm up
                float e = 0.0f;
                if (hipEventRecord(t0, s) != hipSuccess ||
                    (result = simulate_event(pl, depos, n, WCSIM_MEM_DEVICE, 0, (float *)out,
                                             out_kind, WCSIM_MEM_DEVICE, ws, stream,
                                             nullptr)) != WCSIM_OK ||
                    hipEventRecord(t1, s) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
                    hipEventElapsedTime(&e, t0, t1) != hipSuccess) {
                    if (result == WCSIM_OK)
                        result = fail(WCSIM_E_DEVICE, "timing a candidate schedule failed");
                    break;
                }
                if (r >= 0)
                    t.push_back(e);
            }
            if (result == WCSIM_OK) {
                std::sort(t.begin(), t.end());
                ms[i] = t[t.size() / 2];
                ++timed;
            }
        }
        if (out)
            (void)hipFree(out);
        if (ws)
            (void)hipFree(ws);
        wcsim_plane_destroy(pl);
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (result == WCSIM_OK && timed == 0)
        return fail(WCSIM_E_INVALID, "no candidate schedule is valid for this plane");
    return result;
}

}  // extern "C"

namespace wcs {
namespace {

// ---------------------------------------------------------------------------
// Batched form.  The events of a call are grouped by schedule class (planes
// whose kernels can share one launch) and each class is cut into chunks of a
// few events.  A chunk runs as two launch sequences whose kernels each cover
// all of its events: the raster sequence (binning, records, LDS-tiled
// raster) and the convolution sequence (the three FFT passes).  Chunks are
// pipelined over two streams, rasters on one and convolutions on the other,
// so that one chunk's rasterization (bound by vector ALU work) overlaps the
// previous chunk's FFT passes (bound by memory and LDS traffic).  Chunk data
// (raster work, grids, spectra) alternate between two workspace slots: the
// raster of chunk c waits until the convolution of chunk c - 2 has finished
// with the slot.  The descriptor tables of all chunks sit in front of the
// slots and are uploaded once per call.
// ---------------------------------------------------------------------------
constexpr int kChunkEvents = 16;  // events per chunk at most

// Layout of one chunk: its tables (relative to the chunk's table offset) and
// its data (relative to the base of the slot it runs in).
struct ChunkLayout {
    int64_t n_total = 0, ntiles_total = 0, nbands_total = 0;
    bool poly = false;  // wire output through the polyphase pitch pass
    int nblk_r = 0, nblk_p = 0, nblk_c = 0;
    size_t off_bases = 0, tables_bytes = 0;
    size_t off_grid = 0, off_X = 0, off_Y = 0, grid_bytes = 0, data_bytes = 0;
    std::vector<EventCtx> ev;
    std::vector<int32_t> bases;  // 6 arrays of nev + 1
};

struct BatchPlan {
    std::vector<std::vector<int>> chunks;  // event indices of each chunk
    std::vector<ChunkLayout> layouts;
    std::vector<size_t> table_off;         // offset of each chunk's tables
    size_t tables_total = 0, slot_bytes = 0, total = 0;
    int nslots = 1;
    size_t slot_base(int c) const { return tables_total + (size_t)(c % nslots) * slot_bytes; }
};

ChunkLayout plan_chunk(const wcsim_plane *const *planes, const int64_t *n,
                       const std::vector<int> &idx, wcsim_out kind)
{
    ChunkLayout L;
    const int nev = (int)idx.size();
    L.ev.resize((size_t)nev);
    L.poly = kind == WCSIM_OUT_WIRE && planes[idx[0]]->poly;
    L.bases.assign(6 * (size_t)(nev + 1), 0);
    int32_t *bd = &L.bases[0], *bt = bd + (nev + 1), *br = bt + (nev + 1), *bp = br + (nev + 1),
            *bc = bp + (nev + 1), *bb = bc + (nev + 1);
    size_t grid_off = 0, x_off = 0, y_off = 0;
    for (int k = 0; k < nev; ++k) {
        const wcsim_plane *pl = planes[idx[(size_t)k]];
        const int64_t nout = (kind == WCSIM_OUT_WIRE) ? pl->Nw : pl->Np;
        EventCtx &e = L.ev[(size_t)k];
        e = EventCtx{};
        e.kp = pl->kp;
        e.K = L.poly ? pl->KP : pl->K;
        e.depo_base = L.n_total;
        e.n = (int32_t)n[idx[(size_t)k]];
        e.tile_base = (int32_t)L.ntiles_total;
        e.ntt = pl->ntt;
        e.nout = (int32_t)nout;
        e.nblocks = L.poly ? pl->polyBlocks : pl->nblocks;
        e.mode = (kind == WCSIM_OUT_WIRE) ? 1 : 0;
        e.occ_shift = occ_shift_of(pl->Nt);
        // offsets within the chunk's data (the map: within the chunk's maps),
        // turned into pointers per run
        e.occ = (uint8_t *)(uintptr_t)((size_t)kOccCols * (size_t)L.nbands_total);
        e.grid = (float *)(uintptr_t)grid_off;
        e.X = (float2 *)(uintptr_t)x_off;
        e.Y = (float2 *)(uintptr_t)y_off;
        grid_off += align_up(sizeof(float) * (size_t)pl->Np * pl->Nt);
        x_off += align_up(sizeof(float2) * (size_t)pl->C * pl->F * (size_t)pl->Np);
        y_off += align_up(sizeof(float2) * (size_t)pl->C * pl->F * (size_t)nout);
        bd[k] = (int32_t)L.n_total;
        bt[k] = (int32_t)L.ntiles_total;
        br[k] = L.nblk_r;
        bp[k] = L.nblk_p;
        bc[k] = L.nblk_c;
        bb[k] = (int32_t)L.nbands_total;
        L.n_total += n[idx[(size_t)k]];
        L.ntiles_total += pl->ntiles;
        L.nbands_total += occ_bands(pl->Np);
        L.nblk_r += rows_blocks((int)pl->Np);
        L.nblk_p += L.poly ? poly_blocks_total(pl) : pitch_blocks_total(pl);
        L.nblk_c += rows_blocks((int)nout);
    }
    bd[nev] = (int32_t)L.n_total;
    bt[nev] = (int32_t)L.ntiles_total;
    br[nev] = L.nblk_r;
    bp[nev] = L.nblk_p;
    bc[nev] = L.nblk_c;
    bb[nev] = (int32_t)L.nbands_total;
    L.off_bases = align_up(sizeof(EventCtx) * (size_t)nev);
    L.tables_bytes = L.off_bases + align_up(sizeof(int32_t) * L.bases.size());
    const wcsim_plane *pl0 = planes[idx[0]];
    L.off_grid = raster_work_bytes_batch(pl0, L.n_total, L.ntiles_total, L.nbands_total);
    L.grid_bytes = grid_off;
    L.off_X = L.off_grid + grid_off;
    L.off_Y = L.off_X + x_off;
    L.data_bytes = L.off_Y + y_off;
    return L;
}

std::vector<std::vector<int>> schedule_groups(const wcsim_plane *const *planes, int nevents)
{
    std::vector<std::vector<int>> groups;
    for (int e = 0; e < nevents; ++e) {
        bool placed = false;
        for (auto &g : groups)
            if (same_schedule_class(planes[g[0]], planes[e])) {
                g.push_back(e);
                placed = true;
                break;
            }
        if (!placed)
            groups.push_back({e});
    }
    return groups;
}

// Chunks of each schedule class: as many as kChunkEvents requires, with event
// counts differing by at most one, in the callers' order.
BatchPlan plan_batch(const wcsim_plane *const *planes, const int64_t *n, int nevents,
                     wcsim_out kind)
{
    BatchPlan bp;
    for (const auto &g : schedule_groups(planes, nevents)) {
        const int nch = ((int)g.size() + kChunkEvents - 1) / kChunkEvents;
        size_t pos = 0;
        for (int c = 0; c < nch; ++c) {
            const size_t take = g.size() / nch + ((size_t)c < g.size() % nch ? 1 : 0);
            bp.chunks.emplace_back(g.begin() + pos, g.begin() + pos + take);
            pos += take;
        }
    }
    for (const auto &c : bp.chunks) {
        bp.layouts.push_back(plan_chunk(planes, n, c, kind));
        bp.table_off.push_back(bp.tables_total);
        bp.tables_total += align_up(bp.layouts.back().tables_bytes);
        bp.slot_bytes = std::max(bp.slot_bytes, align_up(bp.layouts.back().data_bytes));
    }
    bp.nslots = bp.chunks.size() > 1 ? 2 : 1;
    bp.total = bp.tables_total + (size_t)bp.nslots * bp.slot_bytes;
    return bp;
}

// Per-run fields of the descriptors and their device pointers.
void fill_descriptors(BatchPlan &bp, char *ws, const wcsim_depo *const *depos, const int64_t *n,
                      const uint64_t *event_ids, float *const *outs)
{
    for (size_t c = 0; c < bp.chunks.size(); ++c) {
        ChunkLayout &L = bp.layouts[c];
        const std::vector<int> &g = bp.chunks[c];
        char *data = ws + bp.slot_base((int)c);
        const wcsim_plane *pl0 = nullptr;  // the carve does not depend on the plane
        uint8_t *occ =
            raster_work_carve_batch(pl0, L.n_total, L.ntiles_total, L.nbands_total, data).occ;
        for (size_t k = 0; k < g.size(); ++k) {
            EventCtx &e = L.ev[k];
            e.depos = depos[g[k]];
            e.n = (int32_t)n[g[k]];
            e.event = (uint32_t)event_ids[g[k]];
            e.out = outs[g[k]];
            e.occ = occ + (uintptr_t)e.occ;
            e.grid = (float *)(data + L.off_grid + (uintptr_t)e.grid);
            e.X = (float2 *)(data + L.off_X + (uintptr_t)e.X);
            e.Y = (float2 *)(data + L.off_Y + (uintptr_t)e.Y);
        }
    }
}

void pack_tables(const BatchPlan &bp, char *host)
{
    for (size_t c = 0; c < bp.chunks.size(); ++c) {
        const ChunkLayout &L = bp.layouts[c];
        char *h = host + bp.table_off[c];
        memcpy(h, L.ev.data(), sizeof(EventCtx) * L.ev.size());
        memcpy(h + L.off_bases, L.bases.data(), sizeof(int32_t) * L.bases.size());
    }
}

BatchTables tables_of(const BatchPlan &bp, int c, char *ws)
{
    const ChunkLayout &L = bp.layouts[(size_t)c];
    const int nev = (int)L.ev.size();
    char *t = ws + bp.table_off[(size_t)c];
    BatchTables bt;
    bt.ev = (const EventCtx *)t;
    const int32_t *b0 = (const int32_t *)(t + L.off_bases);
    bt.depo_base = b0;
    bt.tile_base = b0 + (nev + 1);
    bt.rblk_base = b0 + 2 * (nev + 1);
    bt.pblk_base = b0 + 3 * (nev + 1);
    bt.cblk_base = b0 + 4 * (nev + 1);
    bt.band_base = b0 + 5 * (nev + 1);
    bt.nev = nev;
    return bt;
}

// Launches of a whole batch whose tables are already in the workspace.  The
// stream sR runs each chunk's rasterization and then the inverse tick-axis
// pass (pass C) of the chunk before it; sF runs each chunk's passes A and B.
// The raster side has the shorter work, so it takes pass C.  Per workspace
// slot, `ev` holds kPipeEvents / 2 events: raster done (pass A may read the
// grid), pass A done (the next raster of the slot may overwrite grid and
// records), pass B done (pass C may read Y) and pass C done (the next pass B
// of the slot may overwrite Y).  The batch is complete in sR's order (its
// last pass C waits for the last pass B).  `marks` (nullable):
// WCSIM_BATCH_STAGE_EVENTS timing events per chunk (see
// wcsim_simulate_batch_profiled).
constexpr int kPipeEvents = 8;

hipError_t launch_pipeline(const BatchPlan &bp, const wcsim_plane *const *planes, char *ws,
                           hipStream_t sR, hipStream_t sF, const hipEvent_t *ev,
                           const hipEvent_t *marks = nullptr)
{
    hipError_t e;
    const hipEvent_t *evR = ev, *evA = ev + 2, *evB = ev + 4, *evC = ev + 6;
    const int nch = (int)bp.chunks.size();
    auto pass_c = [&](int c) -> hipError_t {
        const ChunkLayout &L = bp.layouts[(size_t)c];
        const wcsim_plane *pl0 = planes[bp.chunks[(size_t)c][0]];
        const int slot = c % bp.nslots;
        const hipEvent_t *mk = marks ? marks + (size_t)c * WCSIM_BATCH_STAGE_EVENTS : nullptr;
        hipError_t r;
        if ((r = hipStreamWaitEvent(sR, evB[slot], 0)) != hipSuccess ||
            (mk && (r = hipEventRecord(mk[8], sR)) != hipSuccess) ||
            (r = launch_convolve_batch_c(pl0, tables_of(bp, c, ws), L.nblk_c, sR)) !=
                hipSuccess ||
            (mk && (r = hipEventRecord(mk[7], sR)) != hipSuccess))
            return r;
        return hipEventRecord(evC[slot], sR);
    };
    for (int c = 0; c < nch; ++c) {
        const ChunkLayout &L = bp.layouts[(size_t)c];
        const wcsim_plane *pl0 = planes[bp.chunks[(size_t)c][0]];
        const BatchTables bt = tables_of(bp, c, ws);
        const int slot = c % bp.nslots;
        char *data = ws + bp.slot_base(c);
        const bool reuse = c >= bp.nslots;  // the slot held chunk c - nslots
        if (reuse && (e = hipStreamWaitEvent(sR, evA[slot], 0)) != hipSuccess)
            return e;
        const hipEvent_t *mk = marks ? marks + (size_t)c * WCSIM_BATCH_STAGE_EVENTS : nullptr;
        const RasterWork rw =
            raster_work_carve_batch(pl0, L.n_total, L.ntiles_total, L.nbands_total, data);
        if ((mk && (e = hipEventRecord(mk[0], sR)) != hipSuccess) ||
            (e = launch_raster_batch(pl0, bt, L.n_total, L.ntiles_total, L.nbands_total, rw, sR,
                                     mk ? mk + 1 : nullptr)) != hipSuccess ||
            (e = hipEventRecord(evR[slot], sR)) != hipSuccess)
            return e;
        if (c > 0 && (e = pass_c(c - 1)) != hipSuccess)
            return e;
        if ((e = hipStreamWaitEvent(sF, evR[slot], 0)) != hipSuccess ||
            (mk && (e = hipEventRecord(mk[4], sF)) != hipSuccess) ||
            (e = launch_convolve_batch_ab(pl0, bt, L.nblk_r, L.nblk_p, L.poly, sF,
                                          mk ? mk + 5 : nullptr, evA[slot],
                                          reuse ? evC[slot] : nullptr)) != hipSuccess ||
            (e = hipEventRecord(evB[slot], sF)) != hipSuccess)
            return e;
    }
    if (nch > 0)
        return pass_c(nch - 1);
    return hipSuccess;
}

wcsim_status check_batch_args(const wcsim_plane *const *planes, const wcsim_depo *const *depos,
                              const int64_t *n, const uint64_t *event_ids, int32_t nevents,
                              float *const *outs, wcsim_out out_kind, void *workspace)
{
    if (!planes || !depos || !n || !event_ids || !outs || !workspace || nevents < 0)
        return fail(WCSIM_E_INVALID, "bad batch arguments");
    if (out_kind != WCSIM_OUT_WIRE && out_kind != WCSIM_OUT_PITCH)
        return fail(WCSIM_E_INVALID, "bad output kind");
    if (((uintptr_t)workspace & 255) != 0)
        return fail(WCSIM_E_INVALID, "workspace must be 256-byte aligned");
    int64_t n_all = 0;
    for (int32_t e = 0; e < nevents; ++e) {
        if (!planes[e])
            return fail(WCSIM_E_STATE, "NULL plane in batch");
        if (n[e] < 0 || (n[e] > 0 && !depos[e]) || !outs[e])
            return fail(WCSIM_E_INVALID, "bad depos or output of batch event " + std::to_string(e));
        n_all += n[e];
    }
    if (n_all > (1LL << 31) - 1)
        return fail(WCSIM_E_INVALID, "too many depos in one batch");
    return WCSIM_OK;
}

// Pinned host staging of the descriptor tables of this thread's direct batch
// calls; the event marks when the last upload from it has completed.
struct HostStaging {
    void *buf = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    ~HostStaging()
    {
        if (done)
            (void)hipEventSynchronize(done);
        if (buf)
            (void)hipHostFree(buf);
        if (done)
            (void)hipEventDestroy(done);
    }
};
thread_local HostStaging g_staging;

wcsim_status stage_upload(const void *src, size_t bytes, void *dst, hipStream_t s)
{
    HostStaging &h = g_staging;
    if (!h.done)
        WCS_HIP(hipEventCreateWithFlags(&h.done, hipEventDisableTiming));
    WCS_HIP(hipEventSynchronize(h.done));  // the previous upload has left the buffer
    if (h.cap < bytes) {
        if (h.buf)
            WCS_HIP(hipHostFree(h.buf));
        h.buf = nullptr;
        h.cap = 0;
        WCS_HIP(hipHostMalloc(&h.buf, bytes, hipHostMallocDefault));
        h.cap = bytes;
    }
    memcpy(h.buf, src, bytes);
    WCS_HIP(hipMemcpyAsync(dst, h.buf, bytes, hipMemcpyHostToDevice, s));
    WCS_HIP(hipEventRecord(h.done, s));
    return WCSIM_OK;
}

// The second stream and the ordering events of this thread's direct batch
// calls, one set per device (default priority, non-blocking).
struct PipeStreams {
    int device = -1;
    hipStream_t sF = nullptr;
    hipEvent_t ev[kPipeEvents] = {};
    ~PipeStreams()
    {
        if (sF) {
            (void)hipStreamSynchronize(sF);
            (void)hipStreamDestroy(sF);
        }
        for (hipEvent_t e : ev)
            if (e)
                (void)hipEventDestroy(e);
    }
};
thread_local std::vector<std::unique_ptr<PipeStreams>> g_pipes;

wcsim_status pipe_streams(PipeStreams **out)
{
    int dev = -1;
    WCS_HIP(hipGetDevice(&dev));
    for (auto &p : g_pipes)
        if (p->device == dev) {
            *out = p.get();
            return WCSIM_OK;
        }
    std::unique_ptr<PipeStreams> p(new (std::nothrow) PipeStreams());
    if (!p)
        return fail(WCSIM_E_NOMEM, "host allocation failed");
    p->device = dev;
    WCS_HIP(hipStreamCreateWithFlags(&p->sF, hipStreamNonBlocking));
    for (hipEvent_t &e : p->ev)
        WCS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    *out = p.get();
    g_pipes.push_back(std::move(p));
    return WCSIM_OK;
}

}  // namespace
}  // namespace wcs

struct wcsim_batch {
    std::vector<const wcsim_plane *> planes;
    std::vector<int64_t> capacity;
    wcsim_out kind;
    char *ws = nullptr;
    wcs::BatchPlan plan;
    void *pinned = nullptr;
    hipEvent_t done = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace wcs {
namespace {

void destroy_batch(wcsim_batch *b)
{
    if (b->done)
        (void)hipEventSynchronize(b->done);
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->pinned)
        (void)hipHostFree(b->pinned);
    if (b->done)
        (void)hipEventDestroy(b->done);
    delete b;
}

}  // namespace
}  // namespace wcs

extern "C" {

size_t wcsim_batch_workspace_bytes(const wcsim_plane *const *planes, const int64_t *n,
                                   int32_t nevents, wcsim_out out_kind)
{
    if (!planes || !n || nevents <= 0)
        return 0;
    for (int32_t e = 0; e < nevents; ++e)
        if (!planes[e] || n[e] < 0)
            return 0;
    return plan_batch(planes, n, nevents, out_kind).total;
}

int32_t wcsim_batch_chunk_count(const wcsim_plane *const *planes, const int64_t *n,
                                int32_t nevents, wcsim_out out_kind)
{
    if (!planes || !n || nevents <= 0)
        return 0;
    for (int32_t e = 0; e < nevents; ++e)
        if (!planes[e] || n[e] < 0)
            return 0;
    return (int32_t)plan_batch(planes, n, nevents, out_kind).chunks.size();
}

static wcsim_status simulate_batch(const wcsim_plane *const *planes,
                                   const wcsim_depo *const *depos, const int64_t *n,
                                   const uint64_t *event_ids, int32_t nevents,
                                   float *const *outs, wcsim_out out_kind, void *workspace,
                                   void *stream, const hipEvent_t *marks)
{
    wcsim_status st = check_batch_args(planes, depos, n, event_ids, nevents, outs, out_kind,
                                       workspace);
    if (st != WCSIM_OK || nevents == 0)
        return st;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    PipeStreams *ps = nullptr;
    if ((st = pipe_streams(&ps)) != WCSIM_OK)
        return st;
    BatchPlan bp = plan_batch(planes, n, nevents, out_kind);
    fill_descriptors(bp, ws, depos, n, event_ids, outs);
    std::vector<char> host(bp.tables_total);
    pack_tables(bp, host.data());
    if ((st = stage_upload(host.data(), host.size(), ws, s)) != WCSIM_OK)
        return st;
    WCS_HIP(launch_pipeline(bp, planes, ws, s, ps->sF, ps->ev, marks));
    return WCSIM_OK;
}

wcsim_status wcsim_simulate_batch(const wcsim_plane *const *planes,
                                  const wcsim_depo *const *depos, const int64_t *n,
                                  const uint64_t *event_ids, int32_t nevents, float *const *outs,
                                  wcsim_out out_kind, void *workspace, void *stream)
{
    return simulate_batch(planes, depos, n, event_ids, nevents, outs, out_kind, workspace, stream,
                          nullptr);
}

wcsim_status wcsim_simulate_batch_profiled(const wcsim_plane *const *planes,
                                           const wcsim_depo *const *depos, const int64_t *n,
                                           const uint64_t *event_ids, int32_t nevents,
                                           float *const *outs, wcsim_out out_kind,
                                           void *workspace, void *stream, void *const *events,
                                           int32_t nevents_events)
{
    if (!planes || !n || nevents <= 0)
        return fail(WCSIM_E_INVALID, "bad batch arguments");
    const int32_t nch = wcsim_batch_chunk_count(planes, n, nevents, out_kind);
    if (!events || nevents_events != nch * WCSIM_BATCH_STAGE_EVENTS)
        return fail(WCSIM_E_INVALID, "need WCSIM_BATCH_STAGE_EVENTS events per chunk");
    for (int32_t i = 0; i < nevents_events; ++i)
        if (!events[i])
            return fail(WCSIM_E_INVALID, "NULL event in the event array");
    return simulate_batch(planes, depos, n, event_ids, nevents, outs, out_kind, workspace, stream,
                          (const hipEvent_t *)events);
}

wcsim_status wcsim_batch_create(const wcsim_plane *const *planes, const int64_t *capacity,
                                int32_t nevents, wcsim_out out_kind, void *workspace,
                                wcsim_batch **out)
{
    if (!out || !planes || !capacity || nevents <= 0 || !workspace)
        return fail(WCSIM_E_INVALID, "bad batch arguments");
    *out = nullptr;
    if (out_kind != WCSIM_OUT_WIRE && out_kind != WCSIM_OUT_PITCH)
        return fail(WCSIM_E_INVALID, "bad output kind");
    if (((uintptr_t)workspace & 255) != 0)
        return fail(WCSIM_E_INVALID, "workspace must be 256-byte aligned");
    int64_t n_all = 0;
    for (int32_t e = 0; e < nevents; ++e) {
        if (!planes[e])
            return fail(WCSIM_E_STATE, "NULL plane in batch");
        if (capacity[e] < 0)
            return fail(WCSIM_E_INVALID, "negative capacity");
        n_all += capacity[e];
    }
    if (n_all > (1LL << 31) - 1)
        return fail(WCSIM_E_INVALID, "too many depos in one batch");
    wcsim_batch *b = new (std::nothrow) wcsim_batch();
    if (!b)
        return fail(WCSIM_E_NOMEM, "host allocation failed");
    b->planes.assign(planes, planes + nevents);
    b->capacity.assign(capacity, capacity + nevents);
    b->kind = out_kind;
    b->ws = (char *)workspace;
    b->plan = plan_batch(planes, capacity, nevents, out_kind);
    auto bail = [&](wcsim_status st) {
        destroy_batch(b);
        return st;
    };
    hipError_t e;
    if ((e = hipHostMalloc(&b->pinned, std::max<size_t>(b->plan.tables_total, 256),
                           hipHostMallocDefault)) != hipSuccess)
        return bail(check_hip(e, "hipHostMalloc(batch tables)"));
    if ((e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming)) != hipSuccess)
        return bail(check_hip(e, "hipEventCreate"));
    // capture on two private streams (default priority), joined at the end
    hipStream_t cs = nullptr, fs = nullptr;
    hipEvent_t ev[kPipeEvents] = {};
    auto release = [&]() {
        for (hipEvent_t x : ev)
            if (x)
                (void)hipEventDestroy(x);
        if (fs)
            (void)hipStreamDestroy(fs);
        if (cs)
            (void)hipStreamDestroy(cs);
    };
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&fs, hipStreamNonBlocking);
    for (int k = 0; k < kPipeEvents && e == hipSuccess; ++k)
        e = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
    if (e != hipSuccess) {
        release();
        return bail(check_hip(e, "batch capture streams"));
    }
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws, b->pinned, b->plan.tables_total, hipMemcpyHostToDevice, cs);
    if (e == hipSuccess)
        e = launch_pipeline(b->plan, planes, b->ws, cs, fs, ev);
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess)
        e = e2;
    if (e == hipSuccess)
        e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    if (graph)
        (void)hipGraphDestroy(graph);
    release();
    if (e != hipSuccess)
        return bail(check_hip(e, "batch graph capture"));
    *out = b;
    return WCSIM_OK;
}

wcsim_status wcsim_batch_run(wcsim_batch *b, const wcsim_depo *const *depos, const int64_t *n,
                             const uint64_t *event_ids, float *const *outs, void *stream)
{
    if (!b)
        return fail(WCSIM_E_STATE, "NULL batch");
    const int32_t nev = (int32_t)b->planes.size();
    wcsim_status st = check_batch_args(b->planes.data(), depos, n, event_ids, nev, outs, b->kind,
                                       b->ws);
    if (st != WCSIM_OK)
        return st;
    for (int32_t e = 0; e < nev; ++e)
        if (n[e] > b->capacity[(size_t)e])
            return fail(WCSIM_E_INVALID, "event " + std::to_string(e) + " exceeds its capacity");
    WCS_HIP(hipEventSynchronize(b->done));  // the previous run has read the tables
    BatchPlan bp = b->plan;
    fill_descriptors(bp, b->ws, depos, n, event_ids, outs);
    pack_tables(bp, (char *)b->pinned);
    WCS_HIP(hipGraphLaunch(b->exec, (hipStream_t)stream));
    WCS_HIP(hipEventRecord(b->done, (hipStream_t)stream));
    return WCSIM_OK;
}

void wcsim_batch_destroy(wcsim_batch *b)
{
    if (b)
        destroy_batch(b);
}

}  // extern "C"
