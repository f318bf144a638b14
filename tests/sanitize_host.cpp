// Host-side driver of the library's host code (geometry checks, buffer
// layout, rate tables and quantisation, domain sizes, argument errors) for a
// build instrumented with AddressSanitizer and UndefinedBehaviorSanitizer on
// the host.  None of these calls touches the GPU.
#include <cstdio>
#include <cstdint>
#include <cstring>

#include "../include/fkmc.h"

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static uint32_t next_u32()
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (uint32_t)(rng >> 11);
}

int main()
{
    int bad = 0;
    for (int it = 0; it < 3000; it++) {
        fkmc_geometry g[3];
        const uint32_t n = 1 + next_u32() % 3;
        for (uint32_t i = 0; i < n; i++) {
            std::memset(&g[i], 0, sizeof g[i]);
            for (int a = 0; a < 3; a++) {
                g[i].L[a] = (int32_t)(next_u32() % 70) - 2;       // includes invalid sizes
                g[i].frag[a] = (int32_t)(next_u32() % 30) - 1;
            }
            if (next_u32() % 3 == 0) g[i].frag[0] = g[i].frag[1] = g[i].frag[2] = 0;
            g[i].a_angstrom = 3.905;
            g[i].seed = next_u32();
            g[i].lattice_id = i;
        }
        size_t sz[3];
        fkmc_status s = fkmc_query_sizes(g, n, sz);
        if (s == FKMC_OK && (sz[0] == 0 || sz[2] == 0)) bad++;
        uint64_t dom = 0;
        (void)fkmc_max_domain_sites(&g[0], &dom);
        fkmc_rate_params p;
        std::memset(&p, 0, sizeof p);
        p.nu = 1e13;
        p.T = 200.0 + next_u32() % 900;
        p.Ea_O = 0.3 + (next_u32() % 100) * 0.01;
        p.Ea_H = 0.1 + (next_u32() % 100) * 0.01;
        p.E_z = (double)(next_u32() % 1000) * 1e6 - 5e8;
        p.q = 2.0;
        p.gb_period_cells = (int32_t)(next_u32() % 6);
        p.gb_axes_mask = (int32_t)(next_u32() % 8);
        p.gb_dE = (next_u32() % 50) * 0.01;
        double raw[12], qt[12], q = 0, rel = 0;
        (void)fkmc_rate_table_host(&p, 3.905, 1 + next_u32() % 100000, raw, qt, &q, &rel);
        (void)fkmc_rate_table_host(&p, 3.905, 0, raw, qt, nullptr, nullptr);
    }
    // argument errors
    if (fkmc_query_sizes(nullptr, 1, nullptr) == FKMC_OK) bad++;
    if (fkmc_rate_table_host(nullptr, 3.905, 8, nullptr, nullptr, nullptr, nullptr) == FKMC_OK) bad++;
    if (fkmc_max_domain_sites(nullptr, nullptr) == FKMC_OK) bad++;
    std::printf("host driver done, %d unexpected results\n", bad);
    return bad ? 1 : 0;
}
