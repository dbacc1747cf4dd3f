// Driver for the sanitizer build of libwcsim's host code (AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side only): calls the C ABI on
// malformed arguments, which the library must reject on the host before
// touching a device.  Any out-of-bounds access or undefined operation in the
// validation aborts the run.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "wcsim.h"

static int check(wcsim_status got, wcsim_status want, const char *what)
{
    if (got != want) {
        printf("%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, wcsim_last_error());
        return 1;
    }
    return 0;
}

int main()
{
    int bad = 0;
    std::vector<float> resp(21 * 20, 0.01f);
    wcsim_plane_desc d;
    memset(&d, 0, sizeof d);
    d.plane_id = 0;
    d.nwires = 10;
    d.nimpact = 10;
    d.nticks = 100;
    d.pitch = 5.0;
    d.tick = 0.5;
    d.dir_z = 1.0;
    d.resp_npitch = 21;
    d.resp_nticks = 20;
    d.resp_origin = 10;
    d.response = resp.data();
    wcsim_physics ph;
    memset(&ph, 0, sizeof ph);
    ph.drift_speed = 1.6;
    ph.DL = 4e-4;
    ph.DT = 8.8e-4;
    ph.nsigma = 3.0;
    wcsim_plane *pl = nullptr;
    // each field broken in turn
    auto try_desc = [&](wcsim_plane_desc dd, wcsim_physics pp, const char *what) {
        return check(wcsim_plane_create(&dd, &pp, nullptr, &pl), WCSIM_E_INVALID, what);
    };
    wcsim_plane_desc x = d;
    x.nwires = 0;
    bad += try_desc(x, ph, "nwires");
    x = d;
    x.resp_origin = 21;
    bad += try_desc(x, ph, "resp_origin");
    x = d;
    x.dir_z = 0.5;
    bad += try_desc(x, ph, "dir");
    x = d;
    resp[7] = NAN;
    bad += try_desc(x, ph, "response value");
    resp[7] = 0.01f;
    x = d;
    std::vector<float> el(5, 1.0f);
    el[4] = INFINITY;
    x.elec_nticks = 5;
    x.elec_response = el.data();
    bad += try_desc(x, ph, "electronics value");
    wcsim_physics q = ph;
    q.drift_accel = NAN;
    bad += try_desc(d, q, "drift_accel");
    q = ph;
    q.lifetime = -1.0;
    bad += try_desc(d, q, "lifetime");
    bad += check(wcsim_plane_create(nullptr, &ph, nullptr, &pl), WCSIM_E_INVALID, "NULL desc");
    // entry points on a NULL plane or bad arguments
    float out[4];
    bad += check(wcsim_simulate_event(nullptr, nullptr, 0, WCSIM_MEM_DEVICE, 0, out, WCSIM_OUT_WIRE,
                                      WCSIM_MEM_DEVICE, out, nullptr),
                 WCSIM_E_STATE, "simulate NULL plane");
    bad += check(wcsim_simulate_event_noalloc(nullptr, nullptr, 0, 0, out, WCSIM_OUT_WIRE, nullptr),
                 WCSIM_E_STATE, "noalloc NULL plane");
    bad += check(wcsim_rasterize(nullptr, nullptr, 0, WCSIM_MEM_HOST, 0, nullptr, nullptr),
                 WCSIM_E_STATE, "rasterize NULL plane");
    bad += check(wcsim_digitize(out, 1, 4, 1.0f, 0.0f, -1.0f, 12, 0, 0, nullptr, nullptr),
                 WCSIM_E_INVALID, "digitize sigma");
    bad += check(wcsim_digitize(out, 1, 4, 1.0f, 0.0f, 1.0f, 17, 0, 0, (uint16_t *)out, nullptr),
                 WCSIM_E_INVALID, "digitize bits");
    bad += check(wcsim_digitize_coloured(out, 1, 4, 1.0f, 0.0f, 1.0f, out, 1025, 12, 0, 0,
                                         (uint16_t *)out, nullptr),
                 WCSIM_E_INVALID, "fir length");
    const wcsim_plane *planes[2] = {nullptr, nullptr};
    int64_t n[2] = {1, 1};
    bad += (wcsim_batch_workspace_bytes(planes, n, 2, WCSIM_OUT_WIRE) != 0);
    bad += (wcsim_batch_chunk_count(planes, n, 2, WCSIM_OUT_WIRE) != 0);
    bad += check(wcsim_simulate_batch(planes, nullptr, n, nullptr, 2, nullptr, WCSIM_OUT_WIRE,
                                      nullptr, nullptr),
                 WCSIM_E_INVALID, "batch NULL arrays");
    bad += check(wcsim_philox4x32_10(nullptr, nullptr, 4, nullptr, nullptr), WCSIM_E_INVALID,
                 "philox NULL");
    printf("sanitized library run %s, version %d\n", bad ? "FAILED" : "ok", wcsim_version());
    return bad ? 1 : 0;
}
