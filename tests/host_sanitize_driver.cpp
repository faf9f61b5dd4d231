// Host-side sanitizer run of the library (test infrastructure): linked with
// the library's sources built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side only, it exercises the calls
// that validate arguments and manage state without touching a device:
// options, size estimates, argument rejection, the allocator switch.
#include <cstdio>
#include <cstring>

#include "bcmg.h"

int main() {
    int bad = 0;
    bcmg_options o;
    bad |= bcmg_default_options(&o) != BCMG_OK;
    int64_t b = 0;
    for (int d = 1; d <= 3; d++)
        for (int N = 8; N <= (d == 3 ? 1024 : 4096); N *= 2)
            for (int prec = 0; prec < 2; prec++) bad |= bcmg_estimate_bytes(d, N, prec, &b) != BCMG_OK || b <= 0;
    bcmg_problem *P = nullptr;
    const double *fake = (const double *)16;  // never dereferenced: every case fails validation
    struct Case {
        int d, N;
        int field, value;
    } cases[] = {{4, 64, -1, 0}, {2, 63, -1, 0}, {2, 4, -1, 0}, {3, 2048, -1, 0}, {2, 64, 0, 0},
                 {2, 64, 1, 2},  {2, 64, 2, 0},  {2, 64, 3, 7},  {2, 64, 4, 9},    {2, 64, 5, 3}};
    for (const Case &c : cases) {
        bcmg_default_options(&o);
        if (c.field == 0) o.ext_iters = c.value;
        if (c.field == 1) o.coarsest_N = c.value;
        if (c.field == 2) o.max_cycles = c.value;
        if (c.field == 3) o.precision = c.value;
        if (c.field == 4) o.layout = c.value;
        if (c.field == 5) o.seg_len = c.value;
        bad |= bcmg_setup(c.d, c.N, fake, &o, nullptr, &P) != BCMG_ERR_INVALID || P != nullptr;
        bad |= strlen(bcmg_last_error()) == 0;
    }
    bad |= bcmg_setup(2, 64, nullptr, nullptr, nullptr, &P) != BCMG_ERR_INVALID;
    bad |= bcmg_set_allocator(nullptr, nullptr, nullptr) != BCMG_OK;
    bad |= bcmg_destroy(nullptr) != BCMG_OK;
    bad |= bcmg_batch_destroy(nullptr) != BCMG_OK;
    bad |= bcmg_timing_enable(1) != BCMG_OK || bcmg_timing_enable(0) != BCMG_OK;
    std::printf("host calls: %s\n", bad ? "bad" : "ok");
    return bad;
}
