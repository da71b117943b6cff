// Calls every C-ABI entry point of the library on its host-only paths --
// size queries, parameter and argument validation, refusal of non-finite or
// inconsistent inputs, the static-scratch limit, NULL handles -- with the
// library's host code built with AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_host_sanitized.py; no GPU, no
// device work: every call here returns before reaching the device).  Exit
// 0 when every call returns the documented code.
#include "swe.h"

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

static int g_bad = 0;
#define EXPECT(expr, code)                                                                        \
    do {                                                                                          \
        const int rc_ = (expr);                                                                   \
        if (rc_ != (code)) {                                                                      \
            printf("FAIL %s -> %d (want %d): %s\n", #expr, rc_, (int)(code), swe_last_error()); \
            ++g_bad;                                                                              \
        }                                                                                         \
    } while (0)

static swe_params base(int nx, int ny)
{
    swe_params p;
    std::memset(&p, 0, sizeof p);
    p.nx = nx; p.ny = ny; p.dx = 500.0; p.dy = 400.0; p.g = 9.81; p.courant = 0.45; p.theta = 1.3;
    p.kappa = 1e-3; p.friction = SWE_FRICTION_LINEAR; p.friction_coeff = 3e-3; p.rho_w = 1025.0;
    p.frs_width = 10; p.frs_d0 = 2.0; p.compensated_state = 1;
    return p;
}

int main()
{
    size_t bytes = 0, prev = 0;
    // workspace sizes grow with the domain and with the compensated state
    for (int n : {2, 3, 61, 640, 2600}) {
        swe_params p = base(n, n / 2 + 2);
        EXPECT(swe_workspace_bytes(&p, 2, 4, &bytes), SWE_OK);
        if (bytes <= prev) { printf("FAIL workspace does not grow at %d\n", n); ++g_bad; }
        prev = bytes;
        p.compensated_state = 0;
        size_t b0 = 0;
        EXPECT(swe_workspace_bytes(&p, 2, 4, &b0), SWE_OK);
        if (b0 >= bytes) { printf("FAIL float32 state not smaller at %d\n", n); ++g_bad; }
    }
    // invalid parameters
    {
        swe_params p = base(10, 10);
        swe_params q;
        q = p; q.nx = 1; EXPECT(swe_workspace_bytes(&q, 1, 0, &bytes), SWE_E_ARG);
        q = p; q.courant = 0.0; EXPECT(swe_workspace_bytes(&q, 1, 0, &bytes), SWE_E_ARG);
        q = p; q.courant = NAN; EXPECT(swe_workspace_bytes(&q, 1, 0, &bytes), SWE_E_ARG);
        q = p; q.theta = 2.5; EXPECT(swe_workspace_bytes(&q, 1, 0, &bytes), SWE_E_ARG);
        q = p; q.kappa = -1.0; EXPECT(swe_workspace_bytes(&q, 1, 0, &bytes), SWE_E_ARG);
        q = p; q.bc[0] = SWE_BC_PERIODIC; EXPECT(swe_workspace_bytes(&q, 1, 0, &bytes), SWE_E_ARG);
        q = p; q.bc[2] = 7; EXPECT(swe_workspace_bytes(&q, 1, 0, &bytes), SWE_E_ARG);
        q = p; q.friction = 9; EXPECT(swe_workspace_bytes(&q, 1, 0, &bytes), SWE_E_ARG);
        q = p; q.frs_width = 33; EXPECT(swe_workspace_bytes(&q, 1, 0, &bytes), SWE_E_ARG);
        q = p; q.frs_d0 = 0.0; EXPECT(swe_workspace_bytes(&q, 1, 0, &bytes), SWE_E_ARG);
        q = p; q.north_projection = 2; EXPECT(swe_workspace_bytes(&q, 1, 0, &bytes), SWE_E_ARG);
        q = p; q.compensated_state = -1; EXPECT(swe_workspace_bytes(&q, 1, 0, &bytes), SWE_E_ARG);
        q = p; q.nx = 70000; q.ny = 70000; EXPECT(swe_workspace_bytes(&q, 1, 0, &bytes), SWE_E_ARG);
        EXPECT(swe_workspace_bytes(nullptr, 1, 0, &bytes), SWE_E_ARG);
        EXPECT(swe_workspace_bytes(&p, 0, 0, &bytes), SWE_E_ARG);
        EXPECT(swe_workspace_bytes(&p, 1, 0, nullptr), SWE_E_ARG);
    }
    // init: refusals before any device work
    {
        const int nx = 12, ny = 9;
        swe_params p = base(nx, ny);
        std::vector<float> Hc((nx + 1) * (ny + 1), 20.f), f(nx * ny, 1e-4f), z(nx * ny, 0.f);
        std::vector<uint8_t> land(nx * ny, 0);
        size_t need = 0;
        EXPECT(swe_workspace_bytes(&p, 1, 0, &need), SWE_OK);
        // never dereferenced: every call below returns before device work
        void *fake = reinterpret_cast<void *>((uintptr_t)1 << 40);
        swe_domain *d = nullptr;
        EXPECT(swe_init_domain(&p, fake, need, nullptr, 1, 0, Hc.data(), land.data(), f.data(), nullptr, z.data(),
                               z.data(), z.data(), nullptr), SWE_E_ARG);
        EXPECT(swe_init_domain(&p, fake, need, nullptr, 1, 0, nullptr, land.data(), f.data(), nullptr, z.data(),
                               z.data(), z.data(), &d), SWE_E_ARG);
        EXPECT(swe_init_domain(&p, reinterpret_cast<char *>(fake) + 4, need, nullptr, 1, 0, Hc.data(), land.data(),
                               f.data(), nullptr, z.data(), z.data(), z.data(), &d), SWE_E_ARG);
        std::vector<float> bad = z;
        bad[17] = NAN;
        EXPECT(swe_init_domain(&p, fake, need, nullptr, 1, 0, Hc.data(), land.data(), f.data(), nullptr, bad.data(),
                               z.data(), z.data(), &d), SWE_E_ARG);
        std::vector<float> Hb = Hc;
        Hb[5] = INFINITY;
        EXPECT(swe_init_domain(&p, fake, need, nullptr, 1, 0, Hb.data(), land.data(), f.data(), nullptr, z.data(),
                               z.data(), z.data(), &d), SWE_E_ARG);
        EXPECT(swe_init_domain(&p, fake, need - 256, nullptr, 1, 0, Hc.data(), land.data(), f.data(), nullptr,
                               z.data(), z.data(), z.data(), &d), SWE_E_NOMEM);
        swe_params q = p;
        q.bc[0] = q.bc[1] = SWE_BC_PERIODIC;
        Hb = Hc;
        Hb[(size_t)3 * (nx + 1) + nx] = 21.f;  // periodic seam depths differ
        EXPECT(swe_workspace_bytes(&q, 1, 0, &need), SWE_OK);
        EXPECT(swe_init_domain(&q, fake, need, nullptr, 1, 0, Hb.data(), land.data(), f.data(), nullptr, z.data(),
                               z.data(), z.data(), &d), SWE_E_ARG);
        q = p;
        q.bc[3] = SWE_BC_NESTED;  // nested side needs boundary snapshots
        EXPECT(swe_workspace_bytes(&q, 1, 2, &need), SWE_OK);
        EXPECT(swe_init_domain(&q, fake, need, nullptr, 1, 0, Hc.data(), land.data(), f.data(), nullptr, z.data(),
                               z.data(), z.data(), &d), SWE_E_ARG);
    }
    // NULL handles
    EXPECT(swe_step(nullptr, 1), SWE_E_ARG);
    EXPECT(swe_step_dt(nullptr, 1, nullptr), SWE_E_ARG);
    EXPECT(swe_run_until(nullptr, 1.0, nullptr), SWE_E_ARG);
    EXPECT(swe_read_state(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr), SWE_E_ARG);
    EXPECT(swe_set_state(nullptr, nullptr, nullptr, nullptr, 0.0), SWE_E_ARG);
    EXPECT(swe_diagnostics(nullptr, nullptr, nullptr), SWE_E_ARG);
    EXPECT(swe_status(nullptr), SWE_E_ARG);
    EXPECT(swe_set_dt_policy(nullptr, 1.0), SWE_E_ARG);
    EXPECT(swe_set_forcing(nullptr, SWE_FORCING_WIND_STRESS, 1, nullptr, nullptr), SWE_E_ARG);
    EXPECT(swe_set_tiling(nullptr, 4, 0), SWE_E_ARG);
    EXPECT(swe_list_tilings(nullptr, 1, nullptr, 0, nullptr), SWE_E_ARG);
    EXPECT(swe_autotune_tiling(nullptr, nullptr), SWE_E_ARG);
    EXPECT(swe_enable_timing(nullptr, 1), SWE_E_ARG);
    swe_destroy(nullptr);
    // ensembles and the server
    EXPECT(swe_ensemble_workspace_bytes(nullptr, 0, 0, &bytes), SWE_E_ARG);
    EXPECT(swe_ensemble_create(nullptr, 0, nullptr, 0, nullptr, 0, 0, nullptr), SWE_E_ARG);
    EXPECT(swe_ensemble_step(nullptr, 1), SWE_E_ARG);
    swe_ensemble_destroy(nullptr);
    swe_server *srv = nullptr;
    EXPECT(swe_server_create(nullptr, 1 << 20, nullptr, nullptr, 4, 8, 0, 0, &srv), SWE_E_ARG);
    EXPECT(swe_server_create(reinterpret_cast<void *>((uintptr_t)1 << 40), 1 << 20, nullptr, nullptr, 0, 8, 0, 0,
                             &srv), SWE_E_ARG);
    EXPECT(swe_server_create(reinterpret_cast<void *>(((uintptr_t)1 << 40) + 8), 1 << 20, nullptr, nullptr, 4, 8, 0,
                             0, &srv), SWE_E_ARG);
    EXPECT(swe_server_submit(nullptr, nullptr), SWE_E_ARG);
    EXPECT(swe_server_tick(nullptr, nullptr, nullptr), SWE_E_ARG);
    swe_server_destroy(nullptr);
    // preprocessing
    EXPECT(swe_reconstruct_bathymetry(0, 5, nullptr, nullptr, 1, 0.5f, nullptr, nullptr, nullptr), SWE_E_ARG);
    EXPECT(swe_reconstruct_bathymetry(5, 5, nullptr, nullptr, 1, 0.5f, nullptr, nullptr, nullptr), SWE_E_ARG);
    EXPECT(swe_reconstruct_bathymetry_noalloc(4095, 4095, nullptr, nullptr, 3, 0.5f, nullptr, nullptr), SWE_E_ARG);
    EXPECT(swe_reconstruct_bathymetry_noalloc(0, 3, nullptr, nullptr, 3, 0.5f, nullptr, nullptr), SWE_E_ARG);
    EXPECT(swe_erode_land(5, 5, nullptr, nullptr, nullptr, nullptr, nullptr, 5.f, nullptr, nullptr, nullptr, nullptr,
                          nullptr, nullptr), SWE_E_ARG);
    EXPECT(swe_refine2(5, 5, 1, nullptr, nullptr, 1.f, nullptr, nullptr, nullptr, nullptr, nullptr), SWE_E_ARG);
    EXPECT(swe_coarsen2(5, 5, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr), SWE_E_ARG);
    EXPECT(swe_wind_field_bytes(0, 4, 4, &bytes), SWE_E_ARG);
    EXPECT(swe_wind_field_bytes(2, 4, 4, &bytes), SWE_OK);
    if (!swe_last_error()) { printf("FAIL swe_last_error returned NULL\n"); ++g_bad; }
    printf("abi host paths bad %d\n", g_bad);
    return g_bad != 0;
}
