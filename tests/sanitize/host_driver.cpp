// Exercises the host-only paths of the library's C ABI (argument checks,
// handle creation, replica building with cores and groups, workspace sizing
// and attachment, the closed-form helpers, teardown) for a build whose host
// code carries AddressSanitizer and UndefinedBehaviorSanitizer.  None of these
// calls needs a GPU.  Exit status 0 when every call returned as expected.
#include "crmc.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#define EXPECT(c)                                                        \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::fprintf(stderr, "failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                    \
        }                                                                \
    } while (0)

int main()
{
    crmc_params p;
    std::memset(&p, 0, sizeof p);
    p.n_replicas = 2; p.precision = 32; p.trials_per_cell = 2; p.pairing = 1; p.ion_coupling = 1;
    p.lB = 2.0; p.rc = 6.0; p.eps_wca = 1.0; p.rho0NA = 0.0269424; p.pKw = 14.0; p.kappa = 0.5; p.pKb = 5.0;
    p.learned_eps = 0.1; p.seed = 42;
    crmc_t h = nullptr;
    crmc_params bad = p;
    bad.rc = 1.0;
    EXPECT(crmc_create(&bad, &h) == CRMC_E_ARG && h == nullptr);
    bad = p;
    bad.workspace = &bad;
    bad.workspace_bytes = 8;
    EXPECT(crmc_create(&bad, &h) == CRMC_E_ARG);
    EXPECT(crmc_create(&p, &h) == CRMC_OK && h);
    int64_t ws = -1;
    EXPECT(crmc_workspace_size(h, &ws) == CRMC_E_STATE);
    // a cloud of sites and ions around two cores, groups by index
    const int n = 300;
    std::vector<double> xyz(3 * n);
    std::vector<int32_t> kind(n), group(n);
    unsigned s = 12345u;
    for (int i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) {
            s = s * 1664525u + 1013904223u;
            xyz[3 * i + d] = 40.0 * (s >> 8) / 16777216.0 - 3.0;
        }
        kind[i] = i < 100 ? CRMC_ACID : (i < 180 ? CRMC_BASE : (i < 240 ? CRMC_XPOS : CRMC_XNEG));
        group[i] = (i * 7) % 5 - 2;
    }
    const double core_xyz[6] = {10.0, 10.0, 10.0, 30.0, 30.0, 30.0};
    const double core_R[2] = {2.0, 3.0};
    EXPECT(crmc_build_cells(h, 2, 40.0, 0, 0, n, xyz.data(), kind.data(), nullptr, group.data(), 2, core_xyz,
                            core_R) == CRMC_E_ARG);
    EXPECT(crmc_build_cells(h, 0, 20.0, 0, 0, n, xyz.data(), kind.data(), nullptr, group.data(), 2, core_xyz,
                            core_R) == CRMC_E_ARG); // L < 4 rc
    EXPECT(crmc_build_cells(h, 0, 40.0, 5, 0, n, xyz.data(), kind.data(), nullptr, group.data(), 2, core_xyz,
                            core_R) == CRMC_E_ARG); // odd grid
    EXPECT(crmc_build_cells(h, 0, 40.0, 0, 0, n, xyz.data(), kind.data(), nullptr, group.data(), 2, core_xyz,
                            core_R) == CRMC_OK);
    EXPECT(crmc_build_cells(h, 0, 40.0, 0, 0, n, xyz.data(), kind.data(), nullptr, group.data(), 2, core_xyz,
                            core_R) == CRMC_OK); // rebuilt
    EXPECT(crmc_build_cells(h, 1, 48.0, 6, 0, 180, xyz.data(), kind.data(), nullptr, nullptr, 0, nullptr,
                            nullptr) == CRMC_OK);
    EXPECT(crmc_workspace_size(h, &ws) == CRMC_OK && ws > 0);
    int64_t own = -1, used = -1, lf = -1;
    EXPECT(crmc_memory(h, &own, &used, &lf) == CRMC_OK && own == 0 && used == 0 && lf == 0);
    std::vector<unsigned char> fake(256);
    EXPECT(crmc_set_workspace(h, fake.data(), 16) == CRMC_E_ARG);
    EXPECT(crmc_set_workspace(h, (void*)((uintptr_t)1 << 40), ws) == CRMC_OK); // never dereferenced here
    EXPECT(crmc_memory(h, &own, &used, &lf) == CRMC_OK && lf >= ws - 256);
    EXPECT(crmc_set_workspace(h, (void*)((uintptr_t)1 << 40), ws) == CRMC_E_STATE);
    EXPECT(crmc_set_proposal(h, 1, 0.5) == CRMC_OK && crmc_set_proposal(h, 1, 2.0) == CRMC_E_ARG);
    EXPECT(crmc_set_proposal_offsets(h, 1, -0.5, 0.5) == CRMC_OK);
    EXPECT(std::strlen(crmc_last_error(h)) > 0);
    const double pIX = crmc_pIX_from_salt(2.0, 4.5, 14.0);
    EXPECT(std::isfinite(pIX) && pIX < 2.0);
    double fr[4];
    EXPECT(crmc_ungroup_fractions(4.5, 14.0, 2.0, 2.0, pIX, pIX, fr) == CRMC_OK);
    EXPECT(std::fabs(fr[0] + fr[1] - 1.0) < 1e-12);
    EXPECT(crmc_ungroup_fractions(4.5, 14.0, NAN, 2.0, pIX, pIX, fr) == CRMC_E_ARG);
    crmc_destroy(h);
    std::printf("host driver ok\n");
    return 0;
}
