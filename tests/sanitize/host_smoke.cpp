// Runs the host side of libtdse (argument validation, status strings, the
// band and resampling checks) in a build with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code.  Every call here is refused
// before it reaches a device, so the run needs no GPU; any memory error or
// undefined operation in the host code aborts it.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "libtdse.h"

#define CHECK(cond)                                                             \
    do {                                                                        \
        if (!(cond)) {                                                          \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            return 1;                                                           \
        }                                                                       \
    } while (0)

static tdse_params good()
{
    tdse_params p{};
    p.dx = 0.2;
    p.dt = 0.05;
    p.a = 1.2;
    p.charge_z = 1.0;
    p.mask_fraction = 0.1;
    p.mask_power = 0.125;
    p.nt = 100;
    p.flags = 0;
    return p;
}

int main()
{
    CHECK(std::strstr(tdse_version(), "gfx950") != nullptr);
    for (int s = 0; s >= -7; --s) CHECK(tdse_status_string(s) != nullptr);
    CHECK(std::strcmp(tdse_status_string(-99), "unknown status") == 0);

    // plan creation: every bad parameter is refused before the device
    tdse_plan plan = nullptr;
    int32_t ns[3] = {256, 300, 4096};
    std::vector<tdse_params> bad;
    for (int f = 0; f < 8; ++f) {
        tdse_params p = good();
        switch (f) {
            case 0: p.dx = 0.0; break;
            case 1: p.dt = -1.0; break;
            case 2: p.a = -1.0; break;
            case 3: p.mask_fraction = 0.5; break;
            case 4: p.mask_fraction = -0.1; break;
            case 5: p.nt = -3; break;
            case 6: p.flags = 1; break;
            default: p.mask_power = 0.0; break;
        }
        bad.push_back(p);
    }
    for (const tdse_params& p : bad) {
        CHECK(tdse_plan_create(&p, 3, ns, 0, 0, &plan) == TDSE_E_INVALID);
        CHECK(std::strlen(tdse_last_error()) > 0);
        CHECK(plan == nullptr);
    }
    tdse_params p = good();
    int32_t tiny[1] = {8};
    int32_t huge[1] = {20000};
    CHECK(tdse_plan_create(&p, 1, tiny, 0, 0, &plan) == TDSE_E_INVALID);
    CHECK(tdse_plan_create(&p, 1, huge, 0, 0, &plan) == TDSE_E_UNSUPPORTED);
    CHECK(tdse_plan_create(&p, 0, ns, 0, 0, &plan) == TDSE_E_INVALID);
    CHECK(tdse_plan_create(&p, 3, nullptr, 0, 0, &plan) == TDSE_E_INVALID);
    CHECK(tdse_plan_create(&p, 3, ns, 0, 0, nullptr) == TDSE_E_INVALID);
    CHECK(tdse_plan_create(nullptr, 3, ns, 0, 0, &plan) == TDSE_E_INVALID);
    CHECK(tdse_plan_create(&p, 3, ns, 1u << 20, 0, &plan) == TDSE_E_INVALID);
    CHECK(tdse_plan_create(&p, 3, ns, TDSE_OPT_STORE_CHECKPOINTS, 0, &plan) == TDSE_E_INVALID);
    CHECK(tdse_plan_create(&p, 3, ns, 0, -1, &plan) == TDSE_E_INVALID);

    // calls on a NULL plan
    double* fake = reinterpret_cast<double*>(16);
    CHECK(tdse_propagate_batch(nullptr, fake, nullptr, fake, nullptr, nullptr, nullptr, nullptr,
                               nullptr) == TDSE_E_INVALID);
    CHECK(tdse_adjoint_batch(nullptr, fake, nullptr, fake, fake, nullptr, nullptr, nullptr) ==
          TDSE_E_INVALID);
    CHECK(tdse_plan_destroy(nullptr) == TDSE_OK || std::strlen(tdse_last_error()) > 0);
    int64_t off[4];
    CHECK(tdse_plan_psi_offsets(nullptr, off) == TDSE_E_INVALID);

    // ground state and fit validation
    CHECK(tdse_ground_state(&p, 8, 1.0, 10, 1e-12, fake, nullptr, nullptr) == TDSE_E_INVALID);
    CHECK(tdse_ground_state(&p, 256, 0.0, 10, 1e-12, fake, nullptr, nullptr) == TDSE_E_INVALID);
    double a_out = 0.0;
    CHECK(tdse_soft_core_for_ip(-1.0, 256, 0.2, 1.0, 1e-12, 0.5, 3.0, &a_out, nullptr) ==
          TDSE_E_INVALID);
    CHECK(tdse_soft_core_for_ip(0.5, 256, 0.2, 1.0, 1e-12, 3.0, 0.5, &a_out, nullptr) ==
          TDSE_E_INVALID);

    // harmonic band: the bins of the definition
    int32_t k_lo = 0, nk = 0;
    CHECK(tdse_harmonic_band(22047, 0.05, 0.057, 21, 31, &k_lo, &nk) == TDSE_OK);
    const double dw = 2.0 * M_PI / (22048 * 0.05);
    CHECK(k_lo * dw >= 21 * 0.057 && (k_lo - 1) * dw < 21 * 0.057);
    CHECK((k_lo + nk - 1) * dw <= 31 * 0.057 && (k_lo + nk) * dw > 31 * 0.057);
    CHECK(tdse_harmonic_band(100, 0.05, 0.057, 31, 21, &k_lo, &nk) == TDSE_E_INVALID);

    // resampling validation (host checks only)
    CHECK(tdse_resample_field(4, 64, 0.3, 0.07, 100, fake, fake, 16 * 4 * 33, fake, nullptr) ==
          TDSE_E_INVALID);
    CHECK(tdse_resample_field(4, 64, 0.3, 0.1, 192, fake, fake, 16 * 4 * 33, fake, nullptr) ==
          TDSE_E_INVALID);
    CHECK(tdse_resample_field(4, 64, 0.3, 0.1, 100, fake, fake, 16 * 4 * 33 - 1, fake, nullptr) ==
          TDSE_E_INVALID);
    CHECK(tdse_resample_field(0, 64, 0.3, 0.1, 100, fake, fake, 16 * 4 * 33, fake, nullptr) ==
          TDSE_E_INVALID);
    std::printf("host smoke: ok\n");
    return 0;
}
