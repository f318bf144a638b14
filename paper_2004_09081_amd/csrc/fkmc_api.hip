// C ABI of the fragment kMC library (declared in include/fkmc.h): argument
// checks, the brick plan of each lattice, rate tables, and the host loop
// that enqueues cycles of 8 phase launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fkmc.h"
#include "fkmc_internal.h"

using namespace fkmc;

namespace {

thread_local std::string g_err;

fkmc_status fail(fkmc_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_OK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(FKMC_E_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),   \
                        __FILE__, __LINE__);                                             \
    } while (0)

#define LAUNCH_OK(expr)                                                                  \
    do {                                                                                 \
        int e_ = (expr);                                                                 \
        if (e_ != 0)                                                                     \
            return fail(FKMC_E_DEVICE, "%s: %s", #expr, hipGetErrorString((hipError_t)e_)); \
    } while (0)

// Boltzmann constant in eV/K: k_B/e of the exact SI values (1.380649e-23 J/K,
// 1.602176634e-19 C), nearest binary64.
constexpr double kKB = 0x1.696fe94e2cf9ep-14;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Sub-block boundaries along one axis: fragments of F cells (remainder of
// >= 2 cells its own fragment, 1 cell merged into the last), each halved
// (lower half ceil, upper floor).  Plain mode: one block [0, L).
std::vector<int32_t> axis_bounds(int L, int F, bool plain)
{
    std::vector<int32_t> b;
    if (plain) return {0, L};
    std::vector<int> sizes;
    if (F >= L) {
        sizes.push_back(L);
    } else {
        const int nf = L / F, r = L - nf * F;
        sizes.assign(nf, F);
        if (r >= 2) sizes.push_back(r);
        else if (r == 1) sizes.back() += 1;
    }
    int x = 0;
    b.push_back(0);
    for (int s : sizes) {
        b.push_back(x + (s + 1) / 2);
        x += s;
        b.push_back(x);
    }
    return b;
}

bool is_plain(const fkmc_geometry& g) { return g.frag[0] == 0 && g.frag[1] == 0 && g.frag[2] == 0; }

fkmc_status check_geometry(const fkmc_geometry& g, uint32_t idx)
{
    for (int a = 0; a < 3; a++)
        if (g.L[a] < 2 || g.L[a] > 65535)
            return fail(FKMC_E_INVALID, "lattice %u: L[%d]=%d outside [2, 65535]", idx, a, g.L[a]);
    const bool plain = is_plain(g);
    if (!plain)
        for (int a = 0; a < 3; a++)
            if (g.frag[a] <= 0)
                return fail(FKMC_E_INVALID, "lattice %u: frag must be all 0 (plain) or all > 0", idx);
    if (!(g.a_angstrom > 0.0) || !std::isfinite(g.a_angstrom))
        return fail(FKMC_E_INVALID, "lattice %u: a_angstrom must be positive", idx);
    const double n = 3.0 * g.L[0] * (double)g.L[1] * g.L[2];
    if (n > 9.0e15) return fail(FKMC_E_UNSUPPORTED, "lattice %u too large", idx);
    return FKMC_OK;
}

// Largest sub-block footprint (sites) of a fragment geometry.
uint64_t max_footprint(const fkmc_geometry& g, int* wmax = nullptr)
{
    std::vector<int> w[3];
    for (int a = 0; a < 3; a++) {
        auto b = axis_bounds(g.L[a], g.frag[a], false);
        for (size_t i = 0; i + 1 < b.size(); i++) w[a].push_back(b[i + 1] - b[i]);
    }
    uint64_t best = 0;
    int wm = 0;
    for (int x : w[0])
        for (int y : w[1])
            for (int z : w[2]) {
                const uint64_t s = 3ull * x * y * z + (uint64_t)y * z + (uint64_t)z * x + (uint64_t)x * y;
                best = std::max(best, s);
                wm = std::max(wm, std::max(x, std::max(y, z)));
            }
    if (wmax) *wmax = wm;
    return best;
}

uint64_t domain_sites(const fkmc_geometry& g)
{
    if (is_plain(g)) return 3ull * g.L[0] * g.L[1] * g.L[2];
    return max_footprint(g);
}

void raw_rates(const fkmc_rate_params& p, double a, double out[12])
{
    for (int X = 0; X < 2; X++)
        for (int dzi = 0; dzi < 3; dzi++)
            for (int g = 0; g < 2; g++) {
                const double Ea = X == 0 ? p.Ea_O : p.Ea_H;
                const double dz = (double)(dzi - 1);
                const double hs = a * 1e-10 / 2.0;
                const double dEf = -(p.q * p.E_z * dz * hs);
                const double b = Ea + dEf / 2.0 + (double)g * p.gb_dE;
                out[(X * 3 + dzi) * 2 + g] = p.nu * std::exp(-b / (kKB * p.T));
            }
}

// Round to multiples of q = 2^e, e = ceil(log2 kmax) - 53 + ceil(log2 n_ev).
fkmc_status quantise(const double raw[12], uint64_t n_ev, double out[12], double* q_out,
                     double* rel_out)
{
    double kmax = 0.0;
    for (int i = 0; i < 12; i++) {
        if (!(raw[i] >= 0.0) || std::isinf(raw[i]))
            return fail(FKMC_E_INVALID, "rate %d is negative or not finite", i);
        kmax = std::max(kmax, raw[i]);
    }
    if (n_ev < 1) n_ev = 1;
    double rel = 0.0, q = 0.0;
    if (kmax == 0.0) {
        for (int i = 0; i < 12; i++) out[i] = 0.0;
    } else {
        int ex;
        std::frexp(kmax, &ex);
        if (std::ldexp(1.0, ex - 1) == kmax) ex -= 1;
        int lg = 0;
        while ((1ull << lg) < n_ev) lg++;
        q = std::ldexp(1.0, ex - 53 + lg);
        for (int i = 0; i < 12; i++) {
            const double m = std::rint(raw[i] / q);
            out[i] = m * q;
            if (raw[i] > 0.0) {
                if (m < 1024.0)
                    return fail(FKMC_E_RANGE,
                                "rate %d = %g keeps fewer than 10 bits at quantum %g (rate ratio "
                                "too large for exact sums over %llu events)",
                                i, raw[i], q, (unsigned long long)n_ev);
                rel = std::max(rel, std::fabs(out[i] - raw[i]) / raw[i]);
            }
        }
    }
    if (q_out) *q_out = q;
    if (rel_out) *rel_out = rel;
    return FKMC_OK;
}

struct Layout {
    size_t occ_bytes, disp_bytes, work_bytes;
    std::vector<int64_t> occ_off, disp_off;
    size_t o_desc, o_call, o_state, o_buckets, o_stat, o_counts, o_plain, o_batch, o_tile2lat, o_tiles, o_bounds, o_c2s, o_groups;
    size_t o_stage;          // canonical-order transfers: stage_sites bytes, then stage_sites int32x3
    size_t o_site;           // ids of the plain lattices with site energies
    int64_t stage_sites;
    int32_t n_tiles;
    std::vector<std::vector<int32_t>> bounds[3];
};

Layout plan(const fkmc_geometry* g, uint32_t n)
{
    Layout Y;
    size_t occ = 0, disp = 0;
    int32_t tiles = 0, nb = 0, nc = 0;
    uint64_t maxN = 1;
    for (int a = 0; a < 3; a++) Y.bounds[a].resize(n);
    for (uint32_t i = 0; i < n; i++) {
        const uint64_t N = 3ull * g[i].L[0] * g[i].L[1] * g[i].L[2];
        maxN = std::max(maxN, N);
        Y.occ_off.push_back((int64_t)occ);
        occ = align_up(occ + N, 256);
        Y.disp_off.push_back((int64_t)disp);
        disp = align_up(disp + N, 16);
        const bool pl = is_plain(g[i]);
        int nf = 1;
        for (int a = 0; a < 3; a++) {
            Y.bounds[a][i] = axis_bounds(g[i].L[a], g[i].frag[a], pl);
            nf *= (int)(Y.bounds[a][i].size() - 1) / (pl ? 1 : 2);
            nb += (int)Y.bounds[a][i].size();
            nc += g[i].L[a];
        }
        if (!pl) tiles += nf;
    }
    Y.n_tiles = tiles;
    Y.occ_bytes = occ + 64;             // tail slack for 16-byte chunk reads
    Y.disp_bytes = (disp + 1) * sizeof(int4);
    size_t w = 0;
    auto take = [&](size_t bytes) { size_t o = w; w = align_up(w + bytes, 256); return o; };
    Y.o_desc = take(n * sizeof(LatDesc));
    Y.o_call = take(n * sizeof(LatCall));
    Y.o_state = take(n * sizeof(LatState));
    Y.o_buckets = take((size_t)n * kHopBuckets * 2 * sizeof(unsigned long long));
    Y.o_stat = take((size_t)n * 3 * kStatFields * sizeof(long long));
    Y.o_counts = take((size_t)n * 2 * sizeof(uint64_t));
    Y.o_plain = take((size_t)n * sizeof(int32_t));
    Y.o_batch = take((size_t)n * sizeof(int32_t));
    Y.o_tile2lat = take((size_t)std::max(tiles, 1) * sizeof(int32_t));
    Y.o_tiles = take((size_t)8 * std::max(tiles, 1) * sizeof(TileRec));
    Y.o_bounds = take((size_t)nb * sizeof(int32_t));
    Y.o_c2s = take((size_t)nc * sizeof(int32_t));
    Y.o_groups = take((size_t)std::max(tiles, 1) * sizeof(int2));
    Y.o_site = take((size_t)n * sizeof(int32_t));
    Y.stage_sites = (int64_t)std::min<uint64_t>(maxN, (uint64_t)kStageSites);
    Y.o_stage = take(align_up((size_t)Y.stage_sites, 16) + (size_t)Y.stage_sites * 12);
    Y.work_bytes = w;
    return Y;
}

// Host-built geometry of every tile of every colour, [colour][tile]: the
// sub-block of colour c of fragment f (lower half ceil, upper half floor of
// the fragment along each axis) and its footprint segments in the brick
// layout.
std::vector<TileRec> tile_records(const std::vector<LatDesc>& desc, const Layout& Y,
                                  const std::vector<int32_t>& tile2lat)
{
    const size_t nt = tile2lat.size();
    std::vector<TileRec> out(8 * nt);
    for (size_t t = 0; t < nt; t++) {
        const int lat = tile2lat[t];
        const LatDesc& D = desc[lat];
        const int f = (int)t - D.tile0;
        const int nf0 = D.nsb[0] / 2, nf1 = D.nsb[1] / 2;
        const int fi[3] = {f % nf0, (f / nf0) % nf1, f / (nf0 * nf1)};
        const std::vector<int32_t>* b[3] = {&Y.bounds[0][lat], &Y.bounds[1][lat], &Y.bounds[2][lat]};
        auto base = [&](int x0, int y0, int z0, int wy, int wz) {
            return 3 * ((int64_t)z0 * D.L[1] * D.L[0] + (int64_t)wz * ((int64_t)y0 * D.L[0] + (int64_t)wy * x0));
        };
        for (int c = 0; c < 8; c++) {
            int lo[3], w[3], lo1[3], w1[3];
            for (int a = 0; a < 3; a++) {
                const int sb = 2 * fi[a] + ((c >> a) & 1);
                const int nx = sb + 1 == D.nsb[a] ? 0 : sb + 1;
                lo[a] = (*b[a])[sb];
                w[a] = (*b[a])[sb + 1] - lo[a];
                lo1[a] = (*b[a])[nx];
                w1[a] = (*b[a])[nx + 1] - lo1[a];
            }
            TileRec& R = out[(size_t)c * nt + t];
            std::memset(&R, 0, sizeof R);
            R.ox = (uint16_t)lo[0];
            R.oy = (uint16_t)lo[1];
            R.oz = (uint16_t)lo[2];
            R.wx = (uint8_t)w[0];
            R.wy = (uint8_t)w[1];
            R.wz = (uint8_t)w[2];
            R.st[0] = base(lo[0], lo[1], lo[2], w[1], w[2]);
            R.st[1] = base(lo1[0], lo[1], lo[2], w[1], w[2]);
            R.st[2] = base(lo[0], lo1[1], lo[2], w1[1], w[2]) + (int64_t)w[0] * w1[1] * w[2];
            R.st[3] = base(lo[0], lo[1], lo1[2], w[1], w1[2]) + 2 * (int64_t)w[0] * w[1] * w1[2];
        }
    }
    return out;
}

}  // namespace

struct fkmc_lattice {
    uint32_t n = 0;
    std::vector<fkmc_geometry> geo;
    hipStream_t stream = nullptr;
    fkmc_buffers buf{};
    Layout Y;
    DevPtrs P{};
    std::vector<LatDesc> desc;
    std::vector<int32_t> plain_ids;
    int32_t* d_plain_ids = nullptr;
    int32_t* d_batch_ids = nullptr;
    std::vector<int32_t> batch_ids;       // fragment lattices
    uint64_t* d_counts = nullptr;
    int fp_stride = 0;                    // LDS bytes of the largest staged footprint
    int phase_group = 0;                  // lockstep kernel: tiles per wave (0: not chosen yet)
    int group_override = 0;               // fkmc_set_group (0: automatic)
    int2* d_groups = nullptr;
    int schedule = FKMC_SCHEDULE_AUTO;
    int batch_waves = 0;                  // fkmc_set_schedule (0: automatic, auto_waves)
    int call_waves = 4;                   // wavefronts per workgroup of this call's persistent launch
    int cu_lds = 131072;                  // LDS of a compute unit
    int n_cu = 256;                       // compute units
    int batch_region_bytes = 0;
    std::vector<uint64_t> n_vac;
    std::vector<uint64_t> n_o, n_h;       // ion counts (conserved by hops)
    std::vector<char> rates_ok;
    std::vector<double> t_frag;           // fragment-mode clock
    std::vector<uint64_t> cycles_host;    // cycles at the end of the last call
    std::vector<LatCall> call;
    std::vector<double> qstep, qrel;
    LatState* h_state = nullptr;          // pinned mirror
    bool timing = false;
    std::vector<hipEvent_t> ev;
    double last_avg_ms = 0.0;
    uint64_t last_launches = 0;
    hipGraphExec_t graph = nullptr;       // kGraphCycles lockstep cycles
    bool use_graph = true;
    bool last_persistent = false;  // the last fkmc_advance ran the persistent kernel
    bool plain_lds = true;         // plain lattices that fit run in LDS in the persistent kernel
    std::vector<int32_t> launch_ids;       // this call's persistent-kernel lattices
    std::vector<int32_t> slow_plain_ids;   // this call's plain lattices kept in HBM
    // launch-order cost of each lattice: the least device time over the
    // persistent calls of one shape (0: not measured); the least is the
    // run with the least interference from the workgroup sharing its CU
    std::vector<uint64_t> cost_ticks;
    uint64_t cost_shape[2] = {0, 0};       // (max_cycles, min_hops) of those calls
    int static_dev = -1;                   // fkmc_create_static: device whose scratch it holds
    std::vector<fkmc_rate_params> params;  // last fkmc_set_rates parameters
    std::vector<char> have_params;         // 0 after fkmc_set_rate_table
    int32_t* d_site_ids = nullptr;
};

// Work space of fkmc_create_static: one array per device, for callers that
// cannot allocate device memory.  Host code never passes `scratch` itself to
// a kernel or copy: its device address comes from hipGetSymbolAddress, once
// per device (with that device current), and is kept in g_scratch.
static constexpr size_t kStaticWorkBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWorkBytes];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[kMaxDevices] = {};
static bool g_scratch_held[kMaxDevices] = {};

static constexpr int kGraphCycles = 8;

namespace {

fkmc_status upload_desc(fkmc_lattice* L)
{
    HIP_OK(hipMemcpyAsync((char*)L->buf.work + L->Y.o_desc, L->desc.data(),
                          L->n * sizeof(LatDesc), hipMemcpyHostToDevice, L->stream));
    HIP_OK(hipStreamSynchronize(L->stream));
    return FKMC_OK;
}

fkmc_status reset_counters(fkmc_lattice* L, int64_t only = -1)
{
    char* w = (char*)L->buf.work;
    for (uint32_t i = 0; i < L->n; i++) {
        if (only >= 0 && (int64_t)i != only) continue;
        HIP_OK(hipMemsetAsync(w + L->Y.o_state + i * sizeof(LatState), 0, sizeof(LatState), L->stream));
        HIP_OK(hipMemsetAsync(w + L->Y.o_buckets + (size_t)i * kHopBuckets * 2 * 8, 0,
                              (size_t)kHopBuckets * 2 * 8, L->stream));
        L->t_frag[i] = 0.0;
        L->cycles_host[i] = 0;
    }
    return FKMC_OK;
}

fkmc_status read_states(fkmc_lattice* L)
{
    HIP_OK(hipMemcpyAsync(L->h_state, (char*)L->buf.work + L->Y.o_state, L->n * sizeof(LatState),
                          hipMemcpyDeviceToHost, L->stream));
    HIP_OK(hipStreamSynchronize(L->stream));
    for (uint32_t i = 0; i < L->n; i++)
        if (L->h_state[i].err & 1u)
            return fail(FKMC_E_RANGE, "lattice %u: too many vacancies in one BKL domain", i);
        else if (L->h_state[i].err & 4u)
            return fail(FKMC_E_RANGE, "lattice %u: a hop's site-energy difference exceeds the window", i);
    return FKMC_OK;
}

}  // namespace

extern "C" {

const char* fkmc_last_error(void) { return g_err.c_str(); }

fkmc_status fkmc_query_sizes(const fkmc_geometry* geoms, uint32_t n, size_t bytes_out[3])
{
    if (!geoms || !bytes_out || n == 0) return fail(FKMC_E_INVALID, "null argument or n = 0");
    for (uint32_t i = 0; i < n; i++) {
        fkmc_status s = check_geometry(geoms[i], i);
        if (s) return s;
    }
    Layout Y = plan(geoms, n);
    bytes_out[0] = Y.occ_bytes;
    bytes_out[1] = Y.disp_bytes;
    bytes_out[2] = Y.work_bytes;
    return FKMC_OK;
}

fkmc_status fkmc_max_domain_sites(const fkmc_geometry* g, uint64_t* out)
{
    if (!g || !out) return fail(FKMC_E_INVALID, "null argument");
    fkmc_status s = check_geometry(*g, 0);
    if (s) return s;
    *out = domain_sites(*g);
    return FKMC_OK;
}

fkmc_status fkmc_rate_table_host(const fkmc_rate_params* p, double a_angstrom, uint64_t n_ev,
                                 double raw_out[12], double quant_out[12], double* q_out,
                                 double* max_rel_out)
{
    if (!p || !raw_out || !quant_out) return fail(FKMC_E_INVALID, "null argument");
    if (!(p->T > 0.0) || !(p->nu >= 0.0)) return fail(FKMC_E_INVALID, "T must be > 0, nu >= 0");
    raw_rates(*p, a_angstrom, raw_out);
    return quantise(raw_out, n_ev, quant_out, q_out, max_rel_out);
}

// Handle over n lattices in the given buffers.  static_dev >= 0: the work
// buffer is that device's static scratch (no pinned host mirror; cleared by
// a fill kernel).
static fkmc_status create_impl(const fkmc_geometry* geoms, uint32_t n, const fkmc_buffers* buf,
                               void* hip_stream, fkmc_lattice** out, const Layout& Y, int static_dev)
{
    if (!buf->occ || !buf->disp || !buf->work) return fail(FKMC_E_INVALID, "null device buffer");
    if (buf->bytes[0] < Y.occ_bytes || buf->bytes[1] < Y.disp_bytes || buf->bytes[2] < Y.work_bytes)
        return fail(FKMC_E_NOMEM, "buffers too small: need %zu/%zu/%zu bytes", Y.occ_bytes,
                    Y.disp_bytes, Y.work_bytes);
    if (((uintptr_t)buf->occ & 255) || ((uintptr_t)buf->work & 255) || ((uintptr_t)buf->disp & 15))
        return fail(FKMC_E_NOMEM, "misaligned device buffer");
    int maxfp = 0;
    for (uint32_t i = 0; i < n; i++) {
        if (is_plain(geoms[i])) continue;
        int wm = 0;
        const uint64_t fp = max_footprint(geoms[i], &wm);
        if (wm > kMaxWidth) return fail(FKMC_E_UNSUPPORTED, "lattice %u: sub-block edge %d > %d", i, wm, kMaxWidth);
        maxfp = std::max<int>(maxfp, (int)fp);
    }
    const int fps = maxfp ? footprint_stride(maxfp) : 0;
    if (kWaveScratch + fps > kMaxLdsPerBlock)
        return fail(FKMC_E_UNSUPPORTED, "sub-block footprint of %d sites exceeds the LDS budget", maxfp);

    fkmc_lattice* L = new fkmc_lattice();
    L->n = n;
    L->geo.assign(geoms, geoms + n);
    L->stream = (hipStream_t)hip_stream;
    L->buf = *buf;
    L->Y = Y;
    L->fp_stride = fps;
    L->n_vac.assign(n, 0);
    L->n_o.assign(n, 0);
    L->n_h.assign(n, 0);
    for (uint32_t i = 0; i < n; i++) L->n_o[i] = 3ull * geoms[i].L[0] * geoms[i].L[1] * geoms[i].L[2];
    L->rates_ok.assign(n, 0);
    L->t_frag.assign(n, 0.0);
    L->cycles_host.assign(n, 0);
    L->call.resize(n);
    L->qstep.assign(n, 0.0);
    L->qrel.assign(n, 0.0);
    L->params.assign(n, fkmc_rate_params{});
    L->have_params.assign(n, 0);
    L->static_dev = static_dev;
    if (static_dev >= 0) {
        L->h_state = new LatState[n];
    } else if (hipHostMalloc((void**)&L->h_state, n * sizeof(LatState), hipHostMallocDefault) != hipSuccess) {
        delete L;
        return fail(FKMC_E_DEVICE, "pinned host allocation failed");
    }
    char* w = (char*)buf->work;
    // host tables
    std::vector<int32_t> bounds, c2s, tile2lat;
    L->desc.resize(n);
    for (uint32_t i = 0; i < n; i++) {
        LatDesc& D = L->desc[i];
        std::memset(&D, 0, sizeof D);
        const fkmc_geometry& g = geoms[i];
        for (int a = 0; a < 3; a++) {
            D.L[a] = g.L[a];
            D.nsb[a] = (int32_t)Y.bounds[a][i].size() - 1;
        }
        D.plain = is_plain(g) ? 1 : 0;
        D.site_window = -1;
        for (int a = 0; a < 3; a++) {
            D.nf[a] = D.plain ? 1 : D.nsb[a] / 2;
            D.F[a] = (D.plain || g.frag[a] >= g.L[a]) ? g.L[a] : g.frag[a];
        }
        D.seed = g.seed;
        D.lattice_id = g.lattice_id;
        D.bounds_off = (int32_t)bounds.size();
        for (int a = 0; a < 3; a++)
            bounds.insert(bounds.end(), Y.bounds[a][i].begin(), Y.bounds[a][i].end());
        D.c2s_off = (int32_t)c2s.size();
        for (int a = 0; a < 3; a++) {
            const auto& b = Y.bounds[a][i];
            for (int x = 0, s = 0; x < g.L[a]; x++) {
                while (b[s + 1] <= x) s++;
                c2s.push_back(s);
            }
        }
        D.occ_off = Y.occ_off[i];
        D.disp_off = Y.disp_off[i];
        D.n_sites = 3ll * g.L[0] * g.L[1] * g.L[2];
        if (D.plain) {
            L->plain_ids.push_back((int32_t)i);
        } else {
            L->batch_ids.push_back((int32_t)i);
            D.tile0 = (int32_t)tile2lat.size();
            const int nf = (D.nsb[0] / 2) * (D.nsb[1] / 2) * (D.nsb[2] / 2);
            for (int f = 0; f < nf; f++) tile2lat.push_back((int32_t)i);
        }
    }
    L->P.occ = (int8_t*)buf->occ;
    L->P.disp = (int4*)buf->disp;
    L->P.desc = (const LatDesc*)(w + Y.o_desc);
    L->P.call = (LatCall*)(w + Y.o_call);
    L->P.state = (LatState*)(w + Y.o_state);
    L->P.buckets = (unsigned long long*)(w + Y.o_buckets);
    L->P.tile2lat = (const int32_t*)(w + Y.o_tile2lat);
    L->P.tiles = (const TileRec*)(w + Y.o_tiles);
    L->P.bounds = (const int32_t*)(w + Y.o_bounds);
    L->P.c2s = (const int32_t*)(w + Y.o_c2s);
    L->P.stat_acc = (long long*)(w + Y.o_stat);
    L->P.n_lat = (int32_t)n;
    L->P.n_tiles = Y.n_tiles;
    L->d_plain_ids = (int32_t*)(w + Y.o_plain);
    L->d_batch_ids = (int32_t*)(w + Y.o_batch);
    L->d_site_ids = (int32_t*)(w + Y.o_site);
    L->P.batch_ids = L->d_batch_ids;
    L->P.fp_stride = fps;
    L->d_groups = (int2*)(w + Y.o_groups);
    L->P.groups = L->d_groups;
    {
        int dev = 0, smem = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            if (hipDeviceGetAttribute(&smem, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
                smem > 0)
                L->cu_lds = std::min(smem, 163840);
            if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
                L->n_cu = ncu;
        }
    }
    L->d_counts = (uint64_t*)(w + Y.o_counts);

    auto cleanup = [&](fkmc_status s) {
        if (static_dev >= 0) delete[] L->h_state;
        else (void)hipHostFree(L->h_state);
        delete L;
        return s;
    };
#define CREATE_OK(expr)                                                             \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess)                                                       \
            return cleanup(fail(FKMC_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_))); \
    } while (0)
    if (static_dev >= 0) {
        // the scratch keeps the previous handle's contents: clear all this
        // handle uses
        CREATE_OK((hipError_t)launch_fill_zero(buf->work, Y.work_bytes, L->stream));
        CREATE_OK((hipError_t)launch_fill_zero(buf->occ, Y.occ_bytes, L->stream));
        CREATE_OK((hipError_t)launch_fill_zero(buf->disp, Y.disp_bytes, L->stream));
    } else {
        CREATE_OK(hipMemsetAsync(buf->work, 0, Y.work_bytes, L->stream));
        CREATE_OK(hipMemsetAsync(buf->occ, 0, Y.occ_bytes, L->stream));
        CREATE_OK(hipMemsetAsync(buf->disp, 0, Y.disp_bytes, L->stream));
    }
    CREATE_OK(hipMemcpyAsync(w + Y.o_desc, L->desc.data(), n * sizeof(LatDesc), hipMemcpyHostToDevice, L->stream));
    if (!bounds.empty())
        CREATE_OK(hipMemcpyAsync(w + Y.o_bounds, bounds.data(), bounds.size() * 4, hipMemcpyHostToDevice, L->stream));
    CREATE_OK(hipMemcpyAsync(w + Y.o_c2s, c2s.data(), c2s.size() * 4, hipMemcpyHostToDevice, L->stream));
    std::vector<TileRec> recs;
    if (!tile2lat.empty()) {
        CREATE_OK(hipMemcpyAsync(w + Y.o_tile2lat, tile2lat.data(), tile2lat.size() * 4, hipMemcpyHostToDevice, L->stream));
        recs = tile_records(L->desc, Y, tile2lat);
        CREATE_OK(hipMemcpyAsync(w + Y.o_tiles, recs.data(), recs.size() * sizeof(TileRec), hipMemcpyHostToDevice, L->stream));
    }
    L->slow_plain_ids = L->plain_ids;
    L->launch_ids = L->batch_ids;
    if (!L->plain_ids.empty())
        CREATE_OK(hipMemcpyAsync(L->d_plain_ids, L->plain_ids.data(), L->plain_ids.size() * 4, hipMemcpyHostToDevice, L->stream));
    if (!L->batch_ids.empty())
        CREATE_OK(hipMemcpyAsync(L->d_batch_ids, L->batch_ids.data(), L->batch_ids.size() * 4, hipMemcpyHostToDevice, L->stream));
    CREATE_OK(hipStreamSynchronize(L->stream));
#undef CREATE_OK
    *out = L;
    return FKMC_OK;
}

fkmc_status fkmc_create(const fkmc_geometry* geoms, uint32_t n, const fkmc_buffers* buf,
                        void* hip_stream, fkmc_lattice** out)
{
    if (!geoms || !buf || !out || n == 0) return fail(FKMC_E_INVALID, "null argument or n = 0");
    *out = nullptr;
    for (uint32_t i = 0; i < n; i++) {
        fkmc_status s = check_geometry(geoms[i], i);
        if (s) return s;
    }
    return create_impl(geoms, n, buf, hip_stream, out, plan(geoms, n), -1);
}

fkmc_status fkmc_create_static(const fkmc_geometry* geoms, uint32_t n, void* occ, size_t occ_bytes,
                               void* disp, size_t disp_bytes, void* hip_stream, fkmc_lattice** out)
{
    if (!geoms || !out || n == 0) return fail(FKMC_E_INVALID, "null argument or n = 0");
    *out = nullptr;
    for (uint32_t i = 0; i < n; i++) {
        fkmc_status s = check_geometry(geoms[i], i);
        if (s) return s;
    }
    Layout Y = plan(geoms, n);
    if (Y.work_bytes > kStaticWorkBytes)
        return fail(FKMC_E_NOMEM, "work space of %zu bytes exceeds the static scratch of %zu bytes",
                    Y.work_bytes, kStaticWorkBytes);
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FKMC_E_UNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FKMC_E_DEVICE, "address of the static scratch on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    if (g_scratch_held[dev])
        return fail(FKMC_E_STATE, "the static scratch of device %d is held by another handle", dev);
    fkmc_buffers buf{};
    buf.occ = occ;
    buf.disp = disp;
    buf.work = g_scratch[dev];
    buf.bytes[0] = occ_bytes;
    buf.bytes[1] = disp_bytes;
    buf.bytes[2] = kStaticWorkBytes;
    fkmc_status s = create_impl(geoms, n, &buf, hip_stream, out, Y, dev);
    if (s == FKMC_OK) g_scratch_held[dev] = true;
    return s;
}

fkmc_status fkmc_destroy(fkmc_lattice* L)
{
    if (!L) return FKMC_OK;
    (void)hipStreamSynchronize(L->stream);
    for (auto e : L->ev) (void)hipEventDestroy(e);
    if (L->graph) (void)hipGraphExecDestroy(L->graph);
    if (L->static_dev >= 0) {
        delete[] L->h_state;
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        g_scratch_held[L->static_dev] = false;
    } else if (L->h_state) {
        (void)hipHostFree(L->h_state);
    }
    delete L;
    return FKMC_OK;
}

uint32_t fkmc_count(const fkmc_lattice* L) { return L ? L->n : 0; }

fkmc_status fkmc_init_random(fkmc_lattice* L, const uint64_t* n_vac, const uint64_t* n_h)
{
    if (!L || !n_vac || !n_h) return fail(FKMC_E_INVALID, "null argument");
    std::vector<uint64_t> cnt(2 * L->n);
    for (uint32_t i = 0; i < L->n; i++) {
        const uint64_t N = (uint64_t)L->desc[i].n_sites;
        if (n_vac[i] > N || n_h[i] > N - n_vac[i])
            return fail(FKMC_E_INVALID, "lattice %u: %llu + %llu particles exceed %llu sites", i,
                        (unsigned long long)n_vac[i], (unsigned long long)n_h[i], (unsigned long long)N);
        cnt[2 * i] = n_vac[i];
        cnt[2 * i + 1] = n_h[i];
    }
    HIP_OK(hipMemsetAsync(L->buf.occ, 0, L->Y.occ_bytes, L->stream));
    HIP_OK(hipMemsetAsync(L->buf.disp, 0, L->Y.disp_bytes, L->stream));
    fkmc_status s = reset_counters(L);
    if (s) return s;
    HIP_OK(hipMemcpyAsync(L->d_counts, cnt.data(), cnt.size() * 8, hipMemcpyHostToDevice, L->stream));
    LAUNCH_OK(launch_init(L->P, L->d_counts, (int)L->n, L->stream));
    HIP_OK(hipStreamSynchronize(L->stream));
    for (uint32_t i = 0; i < L->n; i++) {
        L->n_vac[i] = n_vac[i];
        L->n_h[i] = n_h[i];
        L->phase_group = 0;
        L->n_o[i] = (uint64_t)L->desc[i].n_sites - n_vac[i] - n_h[i];
        L->rates_ok[i] = 0;
        L->desc[i].site_window = -1;
    }
    return FKMC_OK;
}

fkmc_status fkmc_set_occupancy(fkmc_lattice* L, uint32_t i, const int8_t* host, size_t n)
{
    if (!L || !host) return fail(FKMC_E_INVALID, "null argument");
    if (i >= L->n) return fail(FKMC_E_INVALID, "lattice index %u out of range", i);
    const size_t N = (size_t)L->desc[i].n_sites;
    if (n != N) return fail(FKMC_E_INVALID, "occupancy has %zu entries, lattice has %zu sites", n, N);
    uint64_t nv = 0, nh = 0;
    for (size_t k = 0; k < N; k++) {
        if (host[k] < 0 || host[k] > 2) return fail(FKMC_E_INVALID, "species code %d at %zu", host[k], k);
        nv += host[k] == kSpV;
        nh += host[k] == kSpH;
    }
    // chunks through the work buffer's stage slice; stream order keeps a
    // chunk's copy behind the previous chunk's kernel
    int8_t* stage = (int8_t*)((char*)L->buf.work + L->Y.o_stage);
    hipError_t e = hipSuccess;
    int le = 0;
    for (int64_t b = 0; b < (int64_t)N && e == hipSuccess && le == 0; b += L->Y.stage_sites) {
        const int64_t c = std::min<int64_t>(L->Y.stage_sites, (int64_t)N - b);
        e = hipMemcpyAsync(stage, host + b, (size_t)c, hipMemcpyHostToDevice, L->stream);
        if (e == hipSuccess) le = launch_scatter(L->P, (int)i, b, c, stage, L->stream);
    }
    hipError_t e2 = hipStreamSynchronize(L->stream);
    if (e != hipSuccess || le != 0 || e2 != hipSuccess)
        return fail(FKMC_E_DEVICE, "set_occupancy copy failed");
    fkmc_status s = reset_counters(L, i);
    if (s) return s;
    HIP_OK(hipStreamSynchronize(L->stream));
    L->n_vac[i] = nv;
    L->n_h[i] = nh;
    L->phase_group = 0;
    L->n_o[i] = N - nv - nh;
    L->rates_ok[i] = 0;
    L->desc[i].site_window = -1;
    return FKMC_OK;
}

// Rates of ion species absent from the lattice are zeroed (hops conserve
// the species counts), so they never set the quantum.
static fkmc_status set_table(fkmc_lattice* L, uint32_t i, const double raw_in[12])
{
    double raw[12];
    for (int e = 0; e < 12; e++) raw[e] = raw_in[e];
    if (L->n_o[i] == 0)
        for (int e = 0; e < 6; e++) raw[e] = 0.0;
    if (L->n_h[i] == 0)
        for (int e = 6; e < 12; e++) raw[e] = 0.0;
    const uint64_t nev = 8ull * std::min<uint64_t>(std::max<uint64_t>(L->n_vac[i], 1), domain_sites(L->geo[i]));
    double k[12], q, rel;
    fkmc_status s = quantise(raw, nev, k, &q, &rel);
    if (s) return fail(s, "lattice %u: %s", i, g_err.c_str());
    std::memcpy(L->desc[i].k12, k, sizeof k);
    L->qstep[i] = q;
    L->qrel[i] = rel;
    return FKMC_OK;
}

fkmc_status fkmc_set_rates(fkmc_lattice* L, const fkmc_rate_params* params)
{
    if (!L || !params) return fail(FKMC_E_INVALID, "null argument");
    std::vector<LatDesc> backup = L->desc;
    for (uint32_t i = 0; i < L->n; i++) {
        const fkmc_rate_params& p = params[i];
        if (!(p.T > 0.0) || !(p.nu >= 0.0) || !std::isfinite(p.E_z) || !std::isfinite(p.q) ||
            p.gb_period_cells < 0)
            return fail(FKMC_E_INVALID, "lattice %u: invalid rate parameters", i);
        double raw[12];
        raw_rates(p, L->geo[i].a_angstrom, raw);
        fkmc_status s = set_table(L, i, raw);
        if (s) {
            L->desc = backup;
            return s;
        }
        L->desc[i].gb_period = p.gb_period_cells;
        L->desc[i].gb_mask = p.gb_axes_mask;
        L->desc[i].site_window = -1;
    }
    fkmc_status s = upload_desc(L);
    if (s) {
        L->desc = backup;
        return s;
    }
    for (uint32_t i = 0; i < L->n; i++) {
        L->rates_ok[i] = 1;
        L->params[i] = params[i];
        L->have_params[i] = 1;
    }
    return FKMC_OK;
}

// Site-energy model buffer of lattice i: Fe bitmap (one bit per cell, 32-bit
// words), padded to 256 bytes, then 12 (2 window + 1) quantised rates.
static size_t site_fe_bytes(const fkmc_geometry& g)
{
    const uint64_t cells = (uint64_t)g.L[0] * g.L[1] * g.L[2];
    return align_up((size_t)((cells + 31) / 32) * 4, 256);
}

fkmc_status fkmc_site_model_bytes(const fkmc_lattice* L, uint32_t i, int32_t window_meV, size_t* bytes)
{
    if (!L || !bytes) return fail(FKMC_E_INVALID, "null argument");
    if (i >= L->n) return fail(FKMC_E_INVALID, "lattice index %u out of range", i);
    if (window_meV < 0 || window_meV > kMaxSiteWindow)
        return fail(FKMC_E_INVALID, "window %d meV outside 0..%d", window_meV, kMaxSiteWindow);
    *bytes = site_fe_bytes(L->geo[i]) + (size_t)12 * (2 * window_meV + 1) * sizeof(double);
    return FKMC_OK;
}

fkmc_status fkmc_set_site_model(fkmc_lattice* L, uint32_t i, const uint8_t* fe, const int32_t e_fe[4],
                                const int32_t e_vv[6], int32_t window_meV, void* dev, size_t bytes)
{
    if (!L || !fe || !e_fe || !e_vv || !dev) return fail(FKMC_E_INVALID, "null argument");
    size_t need = 0;
    fkmc_status st = fkmc_site_model_bytes(L, i, window_meV, &need);
    if (st) return st;
    const fkmc_geometry& g = L->geo[i];
    for (int a = 0; a < 3; a++)
        if (g.L[a] < 5) return fail(FKMC_E_UNSUPPORTED, "lattice %u: site energies need L >= 5 cells", i);
    if (L->desc[i].plain) {
        if (L->n_vac[i] > (uint64_t)kMaxSiteSlots)
            return fail(FKMC_E_UNSUPPORTED, "lattice %u: %llu vacancies, site energies hold %d", i,
                        (unsigned long long)L->n_vac[i], kMaxSiteSlots);
    } else {
        // every sub-block wider than the vacancy-vacancy reach (the squared
        // doubled distance of the farthest shell with a nonzero energy), so
        // that the sub-blocks of a phase never read each other's sites
        static const int kShellN2[6] = {2, 4, 6, 8, 10, 16};
        int reach = 0;
        for (int k = 0; k < 6; k++)
            if (e_vv[k] != 0) reach = kShellN2[k];
        for (int a = 0; a < 3; a++) {
            const std::vector<int32_t>& b = L->Y.bounds[a][i];
            for (size_t k = 0; k + 1 < b.size(); k++) {
                const int w = b[k + 1] - b[k];
                if (4 * w * w <= reach)
                    return fail(FKMC_E_UNSUPPORTED,
                                "lattice %u: a %d-cell sub-block lies within the vacancy-vacancy reach "
                                "(squared doubled distance %d): site energies on fragments need 4 w^2 > reach",
                                i, w, reach);
            }
        }
    }
    if (!L->rates_ok[i] || !L->have_params[i])
        return fail(FKMC_E_STATE, "lattice %u: set the rates with fkmc_set_rates first", i);
    if (bytes < need || ((uintptr_t)dev & 255)) return fail(FKMC_E_NOMEM, "site buffer: need %zu bytes, 256-aligned", need);
    const uint64_t cells = (uint64_t)g.L[0] * g.L[1] * g.L[2];
    std::vector<uint32_t> bits((size_t)((cells + 31) / 32), 0u);
    for (uint64_t c = 0; c < cells; c++) {
        if (fe[c] > 1) return fail(FKMC_E_INVALID, "Fe map value %d at cell %llu", fe[c], (unsigned long long)c);
        if (fe[c]) bits[c >> 5] |= 1u << (c & 31);
    }
    // rates: quantised products of the Arrhenius rates (absent species
    // zeroed) and exp(-dE/(2 k_B T)), quantum from the largest product
    const fkmc_rate_params& p = L->params[i];
    double raw[12];
    raw_rates(p, g.a_angstrom, raw);
    if (L->n_o[i] == 0)
        for (int e = 0; e < 6; e++) raw[e] = 0.0;
    if (L->n_h[i] == 0)
        for (int e = 6; e < 12; e++) raw[e] = 0.0;
    const int W = window_meV, WW = 2 * window_meV + 1;
    std::vector<double> f((size_t)WW), table((size_t)12 * WW, 0.0);
    for (int j = 0; j < WW; j++) f[j] = std::exp(-((double)(j - W) * 1e-3) / (2.0 * kKB * p.T));
    double rmax = 0.0;
    for (int e = 0; e < 12; e++) rmax = std::max(rmax, raw[e]);
    if (rmax > 0.0) {
        const double kmax = rmax * f[0];
        uint64_t n_ev = 8ull * std::min<uint64_t>(std::max<uint64_t>(L->n_vac[i], 1), (uint64_t)L->desc[i].n_sites);
        int ex;
        std::frexp(kmax, &ex);
        if (std::ldexp(1.0, ex - 1) == kmax) ex -= 1;
        int lg = 0;
        while ((1ull << lg) < n_ev) lg++;
        const double q = std::ldexp(1.0, ex - 53 + lg);
        for (int e = 0; e < 12; e++) {
            if (raw[e] == 0.0) continue;
            for (int j = 0; j < WW; j++) {
                const double k = raw[e] * f[j];
                const double m = std::rint(k / q);
                if (m < 1024.0)
                    return fail(FKMC_E_RANGE, "lattice %u: rate %g at dE %d meV keeps fewer than 10 bits at "
                                "quantum %g (narrow the window)", i, k, j - W, q);
                table[(size_t)e * WW + j] = m * q;
            }
        }
    }
    char* d = (char*)dev;
    HIP_OK(hipMemcpyAsync(d, bits.data(), bits.size() * 4, hipMemcpyHostToDevice, L->stream));
    HIP_OK(hipMemcpyAsync(d + site_fe_bytes(g), table.data(), table.size() * sizeof(double), hipMemcpyHostToDevice,
                          L->stream));
    LatDesc backup = L->desc[i];
    LatDesc& D = L->desc[i];
    D.site_window = W;
    for (int k = 0; k < 4; k++) D.site_e_fe[k] = e_fe[k];
    for (int k = 0; k < 6; k++) D.site_e_vv[k] = e_vv[k];
    D.site_fe = (const uint32_t*)d;
    D.site_table = (const double*)(d + site_fe_bytes(g));
    st = upload_desc(L);
    if (st) {
        L->desc[i] = backup;
        return st;
    }
    // a fragment lattice moves from the tile groups to the site-model list
    L->phase_group = 0;
    if (L->graph) {
        (void)hipGraphExecDestroy(L->graph);
        L->graph = nullptr;
    }
    return FKMC_OK;
}

fkmc_status fkmc_gb_map_bytes(const fkmc_lattice* L, uint32_t i, size_t* bytes)
{
    if (!L || !bytes) return fail(FKMC_E_INVALID, "null argument");
    if (i >= L->n) return fail(FKMC_E_INVALID, "lattice index %u out of range", i);
    *bytes = align_up((size_t)((L->desc[i].n_sites + 31) / 32) * 4, 256);
    return FKMC_OK;
}

fkmc_status fkmc_set_gb_map(fkmc_lattice* L, uint32_t i, const uint8_t* map, void* dev, size_t bytes)
{
    if (!L) return fail(FKMC_E_INVALID, "null handle");
    if (i >= L->n) return fail(FKMC_E_INVALID, "lattice index %u out of range", i);
    LatDesc backup = L->desc[i];
    if (!map) {
        L->desc[i].gb_map = nullptr;
    } else {
        size_t need = 0;
        fkmc_status st = fkmc_gb_map_bytes(L, i, &need);
        if (st) return st;
        if (!dev || bytes < need || ((uintptr_t)dev & 255))
            return fail(FKMC_E_NOMEM, "boundary map buffer: need %zu bytes, 256-aligned", need);
        const int64_t N = L->desc[i].n_sites;
        std::vector<uint32_t> bits((size_t)((N + 31) / 32), 0u);
        for (int64_t n = 0; n < N; n++) {
            if (map[n] > 1) return fail(FKMC_E_INVALID, "boundary map value %d at site %lld", map[n], (long long)n);
            if (map[n]) bits[(size_t)(n >> 5)] |= 1u << (n & 31);
        }
        HIP_OK(hipMemcpyAsync(dev, bits.data(), bits.size() * 4, hipMemcpyHostToDevice, L->stream));
        L->desc[i].gb_map = (const uint32_t*)dev;
    }
    fkmc_status st = upload_desc(L);
    if (st) {
        L->desc[i] = backup;
        return st;
    }
    // the lockstep kernel with the map branch only while some lattice has a map
    int32_t any = 0;
    for (uint32_t k = 0; k < L->n; k++) any |= L->desc[k].gb_map ? 1 : 0;
    if (any != L->P.gb_maps && L->graph) {
        (void)hipGraphExecDestroy(L->graph);
        L->graph = nullptr;
    }
    L->P.gb_maps = any;
    return FKMC_OK;
}

fkmc_status fkmc_set_rate_table(fkmc_lattice* L, uint32_t i, const double* k12, size_t n)
{
    if (!L || !k12) return fail(FKMC_E_INVALID, "null argument");
    if (i >= L->n || n != 12) return fail(FKMC_E_INVALID, "bad index or table size");
    LatDesc backup = L->desc[i];
    fkmc_status s = set_table(L, i, k12);
    if (s) return s;
    L->desc[i].site_window = -1;
    s = upload_desc(L);
    if (s) {
        L->desc[i] = backup;
        return s;
    }
    L->rates_ok[i] = 1;
    L->have_params[i] = 0;
    return FKMC_OK;
}

fkmc_status fkmc_get_rate_table(const fkmc_lattice* L, uint32_t i, double* k12, size_t n)
{
    if (!L || !k12) return fail(FKMC_E_INVALID, "null argument");
    if (i >= L->n || n < 12) return fail(FKMC_E_INVALID, "bad index or table size");
    std::memcpy(k12, L->desc[i].k12, 12 * sizeof(double));
    return FKMC_OK;
}

// Tiles one wave runs at once for a lattice whose footprints hold lam
// vacancies on average: the largest group (each tile then has 64/group
// lanes and slots) for which at most 2 % of the tiles overflow their slots
// (Poisson tail), within `lds` bytes of staged footprints per wave; groups
// of 8, 4 or 1 only unless `all` (the lockstep kernel also runs 2).
static int pick_group(double lam, int fp_stride, int lds, bool all)
{
    auto fits = [&](int slots) {
        double p = std::exp(-lam), c = p;
        for (int k = 1; k <= slots; k++) {
            p *= lam / k;
            c += p;
        }
        return 1.0 - c <= 0.02;
    };
    for (int g = 8; g > 1; g /= 2) {
        if (g == 2 && !all) continue;
        if (fits(64 / g) && (int64_t)g * fp_stride <= lds) return g;
    }
    return 1;
}

// Vacancy slots a launch of the HBM plain kernels holds in LDS: the largest
// vacancy count among its lattices, rounded up to 256 (at most
// kMaxPlainSlots; a lattice past that reports FKMC_E_RANGE from the kernel).
static int plain_slot_cap(const fkmc_lattice* L, const int32_t* ids, size_t n)
{
    uint64_t mx = 1;
    for (size_t k = 0; k < n; k++) mx = std::max<uint64_t>(mx, L->n_vac[ids[k]]);
    return (int)std::min<uint64_t>((uint64_t)kMaxPlainSlots, (mx + 255) & ~(uint64_t)255);
}

static double mean_footprint_vacancies(const fkmc_lattice* L, uint32_t i)
{
    return (double)L->n_vac[i] * (double)max_footprint(L->geo[i]) / (double)L->desc[i].n_sites;
}

// Lockstep schedule: choose the group size for the set (the smallest over
// its fragment lattices) and lay out one (lattice, first fragment) entry
// per wave; groups never span two lattices.
static fkmc_status prepare_lockstep(fkmc_lattice* L)
{
    if (L->phase_group) return FKMC_OK;
    // at most 4: more staged footprints per wave cost more occupancy than
    // the shared steps save (measured on the 600^3 sweep)
    int g = 4;
    for (int32_t i : L->batch_ids)
        g = std::min(g, pick_group(mean_footprint_vacancies(L, i), L->fp_stride, 32768 - kWaveScratchStaged, true));
    if (L->group_override) {
        g = L->group_override;
    } else {
        // few tiles: fewer per wavefront, until a launch has two wavefronts
        // per SIMD or one tile each (80 wavefronts of 4 tiles leave most of
        // the GPU idle: the five-lattice 48^3 set takes 1.34 s per 2e6 hops
        // each that way, 0.81 s with one tile per wavefront)
        int64_t tiles = 0;
        for (int32_t i : L->batch_ids)
            if (L->desc[i].site_window < 0) tiles += (int64_t)L->desc[i].nf[0] * L->desc[i].nf[1] * L->desc[i].nf[2];
        while (g > 1 && tiles / g < 8 * (int64_t)L->n_cu) g /= 2;
    }
    while (g > 1 && kWaveScratchStaged + g * L->fp_stride > 65536) g /= 2;
    // lattices with a site model: one entry per sub-block, after the groups
    std::vector<int2> groups, site_groups;
    for (int32_t i : L->batch_ids) {
        const LatDesc& D = L->desc[i];
        const int nt = D.nf[0] * D.nf[1] * D.nf[2];
        if (D.site_window >= 0) {
            for (int f = 0; f < nt; f++) site_groups.push_back(make_int2(i, f));
            continue;
        }
        for (int f0 = 0; f0 < nt; f0 += g) groups.push_back(make_int2(i, f0));
    }
    const size_t ng = groups.size();
    groups.insert(groups.end(), site_groups.begin(), site_groups.end());
    if (!groups.empty())
        HIP_OK(hipMemcpyAsync(L->d_groups, groups.data(), groups.size() * sizeof(int2),
                              hipMemcpyHostToDevice, L->stream));
    HIP_OK(hipStreamSynchronize(L->stream));
    L->P.n_groups = (int32_t)ng;
    L->P.site_groups = L->d_groups + ng;
    L->P.n_site_groups = (int32_t)site_groups.size();
    L->P.lds_wave_bytes = kWaveScratchStaged + g * L->fp_stride;
    if (L->graph) {
        (void)hipGraphExecDestroy(L->graph);
        L->graph = nullptr;
    }
    L->phase_group = g;
    return FKMC_OK;
}

static fkmc_status record_phase(fkmc_lattice* L, int colour, size_t& ev_used)
{
    if (L->timing && ev_used + 2 <= L->ev.size()) {
        HIP_OK(hipEventRecord(L->ev[ev_used], L->stream));
        LAUNCH_OK(launch_phase(L->P, colour, L->phase_group, L->stream));
        LAUNCH_OK(launch_phase_site(L->P, colour, L->stream));
        HIP_OK(hipEventRecord(L->ev[ev_used + 1], L->stream));
        ev_used += 2;
    } else {
        LAUNCH_OK(launch_phase(L->P, colour, L->phase_group, L->stream));
        LAUNCH_OK(launch_phase_site(L->P, colour, L->stream));
    }
    return FKMC_OK;
}

static fkmc_status prepare_call(fkmc_lattice* L, const double* t_sync, uint64_t max_cycles,
                                uint64_t min_hops, bool need_tsync_frag)
{
    for (uint32_t i = 0; i < L->n; i++) {
        if (!L->rates_ok[i]) return fail(FKMC_E_STATE, "lattice %u: rates not set", i);
        const bool pl = L->desc[i].plain;
        const double ts = t_sync ? t_sync[i] : 0.0;
        if (!pl && need_tsync_frag && !(ts > 0.0 && std::isfinite(ts)))
            return fail(FKMC_E_INVALID, "lattice %u: t_sync must be positive and finite", i);
        if (pl && !(ts >= 0.0)) return fail(FKMC_E_INVALID, "lattice %u: negative horizon", i);
        L->call[i] = LatCall{ts, min_hops, max_cycles, 0, 0};
    }
    HIP_OK(hipMemcpyAsync(L->P.call, L->call.data(), L->n * sizeof(LatCall), hipMemcpyHostToDevice,
                          L->stream));
    HIP_OK(hipStreamSynchronize(L->stream));
    return FKMC_OK;
}

// Persistent-kernel plan.  A workgroup's dynamic LDS is one region plus
// the waves' scratch; the region holds either the whole lattice (occupancy,
// vacancy list, cell -> sub-block maps) or every wave's staged footprints,
// so a lattice stays in LDS whenever its slab fits the region's bound (two
// workgroups per CU).  Each lattice also gets its group size (8, 4 or 1).
// Plain lattices in the list are held in LDS (plain_lds_fits).
static int batch_lds_bound(const fkmc_lattice* L)
{
    // the kernel needs more than 128 VGPRs, so a compute unit holds 8 of its
    // wavefronts: two workgroups of up to 4, or one of more
    const int per_cu = L->call_waves <= 4 ? 2 : 1;
    return L->cu_lds / per_cu - L->call_waves * kWaveScratch - kRecCache - 64;
}

// LDS of a plain lattice run by the persistent kernel: canonical occupancy
// at 2 bits per site, vacancy list, and the 8 rates (8 bytes each) and
// target species (1 byte each) of every slot (64, 128, 256 or 512 slots).
static int64_t plain_lds_bytes(const fkmc_lattice* L, uint32_t i)
{
    const uint64_t nv = L->n_vac[i];
    const int64_t slots = nv <= 64 ? 64 : (nv <= 128 ? 128 : (nv <= 256 ? 256 : 512));
    const int64_t words = (L->desc[i].n_sites + 15) >> 4;
    return ((4 * words + 15) & ~(int64_t)15) + 4 * (((int64_t)nv + 3) & ~3) + (8 + 1) * 8 * slots;
}

static bool plain_lds_fits(const fkmc_lattice* L, uint32_t i)
{
    const fkmc_geometry& g = L->geo[i];
    if (!L->plain_lds || !L->desc[i].plain || L->n_vac[i] > (uint64_t)kPlainLdsSlots) return false;
    if (L->desc[i].gb_map) return false;  // boundary-site maps: the HBM kernel
    // packed doubled coordinates: 11 bits for x and y, 10 for z
    if (g.L[0] > 1023 || g.L[1] > 1023 || g.L[2] > 512) return false;
    return plain_lds_bytes(L, i) <= std::min(batch_lds_bound(L), 65536);
}

static fkmc_status plan_batch(fkmc_lattice* L, const std::vector<int32_t>& ids)
{
    const int waves = L->call_waves;
    const int bound = batch_lds_bound(L);
    int region = 0;
    for (int32_t i : ids) {
        LatDesc& D = L->desc[i];
        const fkmc_geometry& g = L->geo[i];
        if (D.plain) {
            D.n_vac = (int32_t)L->n_vac[i];
            D.resident = 1;
            D.fast = 1;
            D.group = 1;
            region = std::max<int>(region, (int)plain_lds_bytes(L, i));
            continue;
        }
        const double lam = mean_footprint_vacancies(L, i);
        const int64_t slab = ((D.n_sites + 15) & ~(int64_t)15) + 4 * (((int64_t)L->n_vac[i] + 3) & ~3) +
                             g.L[0] + g.L[1] + g.L[2];
        bool small = slab <= std::min(bound, 65536);
        for (int a = 0; a < 3; a++) small = small && D.nsb[a] <= 255 && g.L[a] <= 1023;
        D.n_vac = (int32_t)L->n_vac[i];
        D.resident = small ? 1 : 0;
        // one fragment, in LDS, at most 32 vacancies: a block of lanes per vacancy
        // (packed doubled coordinates give z 10 bits)
        D.fast = small && !L->group_override && !D.gb_map && D.nf[0] == 1 && D.nf[1] == 1 && D.nf[2] == 1 &&
                         g.L[2] <= 512 && L->n_vac[i] <= 32
                     ? 1
                     : 0;
        const int fps = footprint_stride((int)max_footprint(g));
        D.fp_stride = fps;
        if (L->group_override) {
            D.group = L->group_override == 8 || L->group_override == 4 ? L->group_override : 1;
            if (!small && (int64_t)waves * D.group * fps > std::min(bound, 65536)) D.group = 1;
            region = std::max<int>(region, small ? (int)slab : waves * D.group * fps);
            if (!small && (int64_t)waves * fps > std::min(bound, 65536))
                return fail(FKMC_E_UNSUPPORTED, "lattice %d: %d waves need %lld bytes of LDS", (int)i,
                            waves, (long long)waves * fps + waves * kWaveScratch);
        } else if (small) {
            // a lattice of fewer than 4 tiles per colour runs them one by one
            D.group = D.nf[0] * D.nf[1] * D.nf[2] < 4 ? 1 : pick_group(lam, 0, 0, false);
            region = std::max<int>(region, (int)slab);
        } else {
            // staged footprints keep LDS addresses below 2^16
            const int area = std::min(bound, 65536);
            D.group = D.nf[0] * D.nf[1] * D.nf[2] < 4 ? 1 : pick_group(lam, fps, area / waves, false);
            if ((int64_t)waves * D.group * fps > area)
                return fail(FKMC_E_UNSUPPORTED, "lattice %d: %d waves need %lld bytes of LDS", (int)i,
                            waves, (long long)waves * fps + waves * kWaveScratch);
            region = std::max<int>(region, waves * D.group * fps);
        }
    }
    L->batch_region_bytes = (region + 15) & ~15;
    return upload_desc(L);
}

// A set that the persistent kernel can give one compute unit per lattice
// (at most as many lattices as compute units), whose fragment lattices have
// at most 128 tiles per colour (16 per wavefront of 8): each workgroup then
// runs 8 wavefronts.  Measured on the 48^3 accuracy set (five lattices in
// 12^3 fragments, 64 tiles per colour): 0.73 s per 2e6 hops each, against
// 1.58 s with 4 wavefronts and 1.34 s on the lockstep schedule.
static bool small_set(const fkmc_lattice* L)
{
    if (L->batch_ids.size() + L->plain_ids.size() > (size_t)L->n_cu) return false;
    for (int32_t i : L->batch_ids) {
        const LatDesc& D = L->desc[i];
        if ((int64_t)D.nf[0] * D.nf[1] * D.nf[2] > 128) return false;
    }
    return true;
}

// Wavefronts per workgroup of the persistent kernel: the caller's choice,
// else 8 for a small set and 4 otherwise.
static int auto_waves(const fkmc_lattice* L)
{
    if (L->batch_waves) return L->batch_waves;
    return small_set(L) ? 8 : 4;
}

// AUTO: the persistent kernel gives every lattice one workgroup, which pays
// off for an ensemble (at least 32 lattices, or lattices small enough to sit
// in LDS); a few large lattices are better served by lockstep launches that
// spread every lattice's tiles over the whole GPU.  A small set (above)
// takes the persistent kernel too.
static bool use_persistent(const fkmc_lattice* L)
{
    if (L->batch_ids.empty()) return false;
    // fragment lattices with a site model run one phase per launch
    for (int32_t i : L->batch_ids)
        if (L->desc[i].site_window >= 0) return false;
    if (L->schedule == FKMC_SCHEDULE_LOCKSTEP) return false;
    if (L->schedule == FKMC_SCHEDULE_PERSISTENT) return true;
    if (L->batch_ids.size() < 2) return false;
    if (L->batch_waves == 0 && small_set(L)) return true;
    if (L->batch_ids.size() >= 32) return true;
    for (int32_t i : L->batch_ids)
        if (L->desc[i].n_sites > 49152) return false;
    return true;
}

fkmc_status fkmc_advance(fkmc_lattice* L, const double* t_sync, uint64_t max_cycles, uint64_t min_hops)
{
    if (!L) return fail(FKMC_E_INVALID, "null handle");
    const bool any_frag = L->Y.n_tiles > 0;
    if (any_frag && !t_sync) return fail(FKMC_E_INVALID, "t_sync required for fragment lattices");
    // Plain lattices that fit run in LDS in the persistent kernel (with the
    // fragment lattices when those use it); the others keep the HBM kernel.
    L->call_waves = auto_waves(L);
    const bool persist = any_frag && max_cycles > 0 && use_persistent(L);
    std::vector<int32_t> ids, slow, site;
    if (persist) ids = L->batch_ids;
    for (int32_t i : L->plain_ids) {
        L->desc[i].resident = 0;
        if (L->desc[i].site_window >= 0) site.push_back(i);
        else if (plain_lds_fits(L, (uint32_t)i)) ids.push_back(i);
        else slow.push_back(i);
    }
    // Order of the persistent launch (results do not depend on it): once
    // every lattice has a cost from earlier calls of this shape, the heaviest
    // half goes first, heaviest first, then the rest lightest first, so that
    // workgroups dispatched half a launch apart (which share a compute unit
    // when every workgroup is resident) pair heavy with light.
    if (L->cost_ticks.size() != L->n || L->cost_shape[0] != max_cycles || L->cost_shape[1] != min_hops) {
        L->cost_ticks.assign(L->n, 0);
        L->cost_shape[0] = max_cycles;
        L->cost_shape[1] = min_hops;
    }
    {
        bool timed = ids.size() >= 2;
        for (int32_t i : ids) timed = timed && L->cost_ticks[i] > 0;
        if (timed) {
            std::stable_sort(ids.begin(), ids.end(), [&](int32_t a, int32_t b) {
                return L->cost_ticks[a] > L->cost_ticks[b];
            });
            std::reverse(ids.begin() + (ids.size() + 1) / 2, ids.end());
        }
    }
    // (both lists are read by the copies before prepare_call synchronises)
    if (slow != L->slow_plain_ids) {
        L->slow_plain_ids = slow;
        if (!slow.empty())
            HIP_OK(hipMemcpyAsync(L->d_plain_ids, L->slow_plain_ids.data(), slow.size() * 4,
                                  hipMemcpyHostToDevice, L->stream));
    }
    if (ids != L->launch_ids) {
        L->launch_ids = ids;
        if (!ids.empty())
            HIP_OK(hipMemcpyAsync(L->d_batch_ids, L->launch_ids.data(), ids.size() * 4, hipMemcpyHostToDevice,
                                  L->stream));
    }
    if (!site.empty())
        HIP_OK(hipMemcpyAsync(L->d_site_ids, site.data(), site.size() * 4, hipMemcpyHostToDevice, L->stream));
    fkmc_status s = prepare_call(L, t_sync, max_cycles, min_hops, true);
    if (s) return s;
    LAUNCH_OK(launch_plain(L->P, L->d_plain_ids, (int)slow.size(), plain_slot_cap(L, slow.data(), slow.size()),
                           L->stream));
    LAUNCH_OK(launch_plain_site(L->P, L->d_site_ids, (int)site.size(), L->stream));
    size_t ev_used = 0;
    if (L->timing && any_frag && L->ev.empty()) {
        L->ev.resize(2 * 2048);
        for (auto& e : L->ev) HIP_OK(hipEventCreate(&e));
    }
    L->last_persistent = persist;
    if (!ids.empty()) {
        s = plan_batch(L, ids);
        if (s) return s;
        DevPtrs P = L->P;
        P.lds_region_bytes = L->batch_region_bytes;
        const bool timed = L->timing && persist;
        if (timed) HIP_OK(hipEventRecord(L->ev[0], L->stream));
        LAUNCH_OK(launch_batch(P, (int)ids.size(), L->call_waves, L->stream));
        if (timed) {
            HIP_OK(hipEventRecord(L->ev[1], L->stream));
            ev_used = 2;
        }
    }
    if (!persist && any_frag && max_cycles > 0) {
        s = prepare_lockstep(L);
        if (s) return s;
        LAUNCH_OK(launch_cycle_begin(L->P, L->stream));
        // Cycles are enqueued in batches; the device marks a lattice done once
        // it reaches its target, after which its kernels return at once, so
        // cycles enqueued beyond the target change nothing.  Without event
        // timing, whole batches of cycles are replayed from a prebuilt graph.
        const bool graph = L->use_graph && !L->timing && L->P.n_site_groups == 0;
        if (graph && !L->graph) {
            LAUNCH_OK(build_cycle_graph(L->P, L->phase_group, kGraphCycles, &L->graph));
        }
        uint64_t batch = min_hops > 0 ? 1 : max_cycles;
        uint64_t cyc = 0;
        while (cyc < max_cycles) {
            uint64_t nb = std::min(batch, max_cycles - cyc);
            if (graph) {
                nb = (nb + kGraphCycles - 1) / kGraphCycles * kGraphCycles;
                for (uint64_t b = 0; b < nb; b += kGraphCycles) HIP_OK(hipGraphLaunch(L->graph, L->stream));
            } else {
                for (uint64_t b = 0; b < nb; b++) {
                    for (int c = 0; c < 8; c++) {
                        s = record_phase(L, c, ev_used);
                        if (s) return s;
                    }
                    LAUNCH_OK(launch_cycle_end(L->P, L->stream));
                }
            }
            cyc += nb;
            if (cyc >= max_cycles) break;
            s = read_states(L);
            if (s) return s;
            bool all = true;
            for (uint32_t i = 0; i < L->n; i++)
                if (!L->desc[i].plain && !L->h_state[i].done) all = false;
            if (all) break;
            batch = std::min<uint64_t>(batch * 2, 64);
        }
    }
    s = read_states(L);
    if (s) return s;
    for (int32_t i : ids) {
        const uint64_t b = L->h_state[i].busy_ticks;
        if (b > 0) L->cost_ticks[i] = L->cost_ticks[i] ? std::min(L->cost_ticks[i], b) : b;
    }
    for (uint32_t i = 0; i < L->n; i++) {
        if (L->desc[i].plain) continue;
        const uint64_t nc = L->h_state[i].cycles - L->cycles_host[i];
        L->t_frag[i] = L->t_frag[i] + (double)nc * L->call[i].t_sync;
        L->cycles_host[i] = L->h_state[i].cycles;
    }
    L->last_launches = 0;
    L->last_avg_ms = 0.0;
    if (L->timing && ev_used) {
        double tot = 0.0;
        for (size_t k = 0; k < ev_used; k += 2) {
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, L->ev[k], L->ev[k + 1]));
            tot += ms;
        }
        L->last_launches = ev_used / 2;
        L->last_avg_ms = tot / (double)(ev_used / 2);
    }
    return FKMC_OK;
}

// Checkpoint layout (all little-endian, host byte order): header, then the
// canonical occupancy (N int8) and displacements (3N int32).
struct CkptHeader {
    char magic[8];       // "FKMCCKP1"
    int32_t L[3], frag[3];
    double a_angstrom;
    uint32_t seed, lattice_id;
    int64_t n_sites;
    uint64_t cycles, draws, hops[2], n_vac, n_h;
    double t;
    double k12[12];
    int32_t gb_period, gb_mask;
    int32_t rates_ok, pad;
};

fkmc_status fkmc_checkpoint_size(const fkmc_lattice* L, uint32_t i, size_t* bytes)
{
    if (!L || !bytes || i >= L->n) return fail(FKMC_E_INVALID, "bad argument");
    *bytes = sizeof(CkptHeader) + (size_t)L->desc[i].n_sites * 13;
    return FKMC_OK;
}

fkmc_status fkmc_checkpoint(fkmc_lattice* L, uint32_t i, void* host, size_t bytes)
{
    size_t need = 0;
    fkmc_status s = fkmc_checkpoint_size(L, i, &need);
    if (s) return s;
    if (!host || bytes < need) return fail(FKMC_E_INVALID, "checkpoint buffer too small (%zu < %zu)", bytes, need);
    std::vector<fkmc_stats> st(L->n);
    s = fkmc_read_stats(L, st.data());
    if (s) return s;
    CkptHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, "FKMCCKP1", 8);
    for (int a = 0; a < 3; a++) {
        h.L[a] = L->geo[i].L[a];
        h.frag[a] = L->geo[i].frag[a];
    }
    h.a_angstrom = L->geo[i].a_angstrom;
    h.seed = L->geo[i].seed;
    h.lattice_id = L->geo[i].lattice_id;
    h.n_sites = L->desc[i].n_sites;
    h.cycles = st[i].cycles;
    h.draws = st[i].draws;
    h.hops[0] = st[i].hops[0];
    h.hops[1] = st[i].hops[1];
    h.n_vac = L->n_vac[i];
    h.n_h = L->n_h[i];
    h.t = st[i].t;
    std::memcpy(h.k12, L->desc[i].k12, sizeof h.k12);
    h.gb_period = L->desc[i].gb_period;
    h.gb_mask = L->desc[i].gb_mask;
    h.rates_ok = L->rates_ok[i];
    char* out = (char*)host;
    std::memcpy(out, &h, sizeof h);
    const size_t N = (size_t)h.n_sites;
    return fkmc_read_state(L, i, (int8_t*)(out + sizeof h), (int32_t*)(out + sizeof h + N), N);
}

// Restore lattice i (same geometry) from a checkpoint: state, clock,
// counters and rate table; the continuation is identical to the original run.
fkmc_status fkmc_restore(fkmc_lattice* L, uint32_t i, const void* host, size_t bytes)
{
    if (!L || !host || i >= L->n) return fail(FKMC_E_INVALID, "bad argument");
    if (bytes < sizeof(CkptHeader)) return fail(FKMC_E_INVALID, "checkpoint too short");
    CkptHeader h;
    std::memcpy(&h, host, sizeof h);
    if (std::memcmp(h.magic, "FKMCCKP1", 8) != 0) return fail(FKMC_E_INVALID, "not a checkpoint");
    const fkmc_geometry& g = L->geo[i];
    for (int a = 0; a < 3; a++)
        if (h.L[a] != g.L[a] || h.frag[a] != g.frag[a]) return fail(FKMC_E_INVALID, "geometry differs");
    if (h.seed != g.seed || h.lattice_id != g.lattice_id || h.a_angstrom != g.a_angstrom)
        return fail(FKMC_E_INVALID, "key or lattice constant differs");
    const size_t N = (size_t)L->desc[i].n_sites;
    if (bytes < sizeof h + N * 13) return fail(FKMC_E_INVALID, "checkpoint too short");
    const char* in = (const char*)host;
    const int8_t* occ = (const int8_t*)(in + sizeof h);
    std::vector<int32_t> disp((size_t)N * 3);
    std::memcpy(disp.data(), in + sizeof h + N, N * 12);
    fkmc_status s = fkmc_set_occupancy(L, i, occ, N);
    if (s) return s;
    // displacements: canonical int32x3 -> storage int4 via a device gather of the copy
    int32_t* stage = (int32_t*)((char*)L->buf.work + L->Y.o_stage);
    hipError_t e1 = hipSuccess;
    int le = 0;
    for (int64_t b = 0; b < (int64_t)N && e1 == hipSuccess && le == 0; b += L->Y.stage_sites) {
        const int64_t c = std::min<int64_t>(L->Y.stage_sites, (int64_t)N - b);
        e1 = hipMemcpyAsync(stage, disp.data() + 3 * b, (size_t)c * 12, hipMemcpyHostToDevice, L->stream);
        if (e1 == hipSuccess) le = launch_scatter_disp(L->P, (int)i, b, c, stage, L->stream);
    }
    hipError_t e2 = hipStreamSynchronize(L->stream);
    if (e1 != hipSuccess || le != 0 || e2 != hipSuccess) return fail(FKMC_E_DEVICE, "restore copy failed");
    // clock and counters
    LatState st;
    std::memset(&st, 0, sizeof st);
    st.cycles = h.cycles;
    st.draws = h.draws;
    st.t = L->desc[i].plain ? h.t : 0.0;
    st.hops[0] = h.hops[0];
    st.hops[1] = h.hops[1];
    HIP_OK(hipMemcpyAsync((char*)L->buf.work + L->Y.o_state + i * sizeof(LatState), &st, sizeof st,
                          hipMemcpyHostToDevice, L->stream));
    unsigned long long b[2] = {h.hops[0], h.hops[1]};
    HIP_OK(hipMemcpyAsync((char*)L->buf.work + L->Y.o_buckets + (size_t)i * kHopBuckets * 2 * 8, b, 16,
                          hipMemcpyHostToDevice, L->stream));
    HIP_OK(hipStreamSynchronize(L->stream));
    L->t_frag[i] = L->desc[i].plain ? 0.0 : h.t;
    L->cycles_host[i] = h.cycles;
    std::memcpy(L->desc[i].k12, h.k12, sizeof h.k12);
    L->desc[i].gb_period = h.gb_period;
    L->desc[i].gb_mask = h.gb_mask;
    s = upload_desc(L);
    if (s) return s;
    L->rates_ok[i] = h.rates_ok;
    L->have_params[i] = 0;
    return FKMC_OK;
}

fkmc_status fkmc_set_graph(fkmc_lattice* L, int32_t enable)
{
    if (!L) return fail(FKMC_E_INVALID, "null handle");
    L->use_graph = enable != 0;
    return FKMC_OK;
}

fkmc_status fkmc_advance_atomic(fkmc_lattice* L, uint32_t n_frg, uint64_t n_stages)
{
    if (!L) return fail(FKMC_E_INVALID, "null handle");
    if (n_frg < 1 || n_frg > 64) return fail(FKMC_E_INVALID, "n_frg = %u: must be 1..64", n_frg);
    int64_t lds = 0;
    std::vector<int32_t> in_lds, in_hbm;
    for (uint32_t i = 0; i < L->n; i++) {
        if (!L->rates_ok[i]) return fail(FKMC_E_STATE, "lattice %u: rates not set", i);
        const fkmc_geometry& g = L->geo[i];
        if (L->desc[i].site_window >= 0)
            return fail(FKMC_E_UNSUPPORTED, "lattice %u: the atom-selection scheme has no site energies", i);
        if (L->desc[i].gb_map)
            return fail(FKMC_E_UNSUPPORTED, "lattice %u: the atom-selection scheme has no boundary-site map", i);
        if (!L->desc[i].plain)
            return fail(FKMC_E_UNSUPPORTED, "lattice %u: the atom-selection scheme runs unfragmented lattices", i);
        const int64_t b = plain_lds_bytes(L, i);
        const bool fits = L->n_vac[i] <= (uint64_t)kPlainLdsSlots && g.L[0] <= 1023 && g.L[1] <= 1023 &&
                          g.L[2] <= 512 && b <= 65536 - 256;
        if (fits && L->plain_lds) {
            // plus the slot totals, two cell-mark bitmaps and the refresh list
            const int64_t nv = (int64_t)L->n_vac[i];
            const int64_t slots = nv <= 64 ? 64 : (nv <= 128 ? 128 : (nv <= 256 ? 256 : 512));
            lds = std::max(lds, b + 8 * slots + 8 * (int64_t)kAtomMarkWords + 2 * slots);
            L->desc[i].n_vac = (int32_t)L->n_vac[i];
            L->desc[i].resident = 1;
            in_lds.push_back((int32_t)i);
        } else if (L->n_vac[i] <= (uint64_t)kMaxPlainSlots) {
            L->desc[i].resident = 0;
            in_hbm.push_back((int32_t)i);
        } else {
            return fail(FKMC_E_UNSUPPORTED,
                        "lattice %u: %llu vacancies; the atom-selection scheme runs at most %d",
                        i, (unsigned long long)L->n_vac[i], kMaxPlainSlots);
        }
    }
    if (L->n == 0 || n_stages == 0) return FKMC_OK;
    fkmc_status s = upload_desc(L);
    if (s) return s;
    // every lattice is plain: the plain-id buffer holds them all, those held
    // in LDS first
    std::vector<int32_t> ord = in_lds;
    ord.insert(ord.end(), in_hbm.begin(), in_hbm.end());
    if (L->slow_plain_ids != ord) {
        L->slow_plain_ids = ord;
        HIP_OK(hipMemcpyAsync(L->d_plain_ids, ord.data(), ord.size() * 4, hipMemcpyHostToDevice,
                              L->stream));
    }
    L->last_persistent = false;
    LAUNCH_OK(launch_atomic(L->P, L->d_plain_ids, (int)in_lds.size(), (size_t)((lds + 15) & ~15), n_frg,
                            n_stages, L->stream));
    LAUNCH_OK(launch_atomic_hbm(L->P, L->d_plain_ids + in_lds.size(), (int)in_hbm.size(),
                                plain_slot_cap(L, in_hbm.data(), in_hbm.size()), n_frg, n_stages, L->stream));
    return read_states(L);
}

fkmc_status fkmc_set_plain_lds(fkmc_lattice* L, int32_t enable)
{
    if (!L) return fail(FKMC_E_INVALID, "null handle");
    if (enable != 0 && enable != 1) return fail(FKMC_E_INVALID, "enable must be 0 or 1");
    L->plain_lds = enable != 0;
    return FKMC_OK;
}

fkmc_status fkmc_set_group(fkmc_lattice* L, int32_t group)
{
    if (!L) return fail(FKMC_E_INVALID, "null handle");
    if (group != 0 && group != 1 && group != 2 && group != 4 && group != 8)
        return fail(FKMC_E_INVALID, "group must be 0, 1, 2, 4 or 8");
    L->group_override = group;
    L->phase_group = 0;
    return FKMC_OK;
}

fkmc_status fkmc_set_schedule(fkmc_lattice* L, int32_t schedule, int32_t waves)
{
    if (!L) return fail(FKMC_E_INVALID, "null handle");
    if (schedule < FKMC_SCHEDULE_AUTO || schedule > FKMC_SCHEDULE_PERSISTENT)
        return fail(FKMC_E_INVALID, "unknown schedule %d", schedule);
    if (waves != 0 && (waves < 1 || waves > 8))
        return fail(FKMC_E_INVALID, "waves per workgroup must be 1..8");
    L->schedule = schedule;
    if (waves) L->batch_waves = waves;
    return FKMC_OK;
}

fkmc_status fkmc_run_phase(fkmc_lattice* L, const double* t_sync, int32_t colour)
{
    if (!L || !t_sync) return fail(FKMC_E_INVALID, "null argument");
    if (colour < 0 || colour > 7) return fail(FKMC_E_INVALID, "colour must be 0..7");
    fkmc_status s = prepare_call(L, t_sync, 1, 0, true);
    if (s) return s;
    LAUNCH_OK(launch_cycle_begin(L->P, L->stream));
    s = prepare_lockstep(L);
    if (s) return s;
    LAUNCH_OK(launch_phase(L->P, colour, L->phase_group, L->stream));
    LAUNCH_OK(launch_phase_site(L->P, colour, L->stream));
    return read_states(L);
}

fkmc_status fkmc_sync(fkmc_lattice* L)
{
    if (!L) return fail(FKMC_E_INVALID, "null handle");
    return read_states(L);
}

fkmc_status fkmc_read_state(fkmc_lattice* L, uint32_t i, int8_t* occ, int32_t* disp, size_t n)
{
    if (!L || !occ) return fail(FKMC_E_INVALID, "null argument");
    if (i >= L->n) return fail(FKMC_E_INVALID, "lattice index out of range");
    const size_t N = (size_t)L->desc[i].n_sites;
    if (n != N) return fail(FKMC_E_INVALID, "buffer has %zu entries, lattice has %zu sites", n, N);
    fkmc_status s = read_states(L);
    if (s) return s;
    // chunks through the work buffer's stage slice: occupancy bytes first,
    // then the chunk's displacements
    int8_t* t_occ = (int8_t*)((char*)L->buf.work + L->Y.o_stage);
    int32_t* t_disp = disp ? (int32_t*)(t_occ + align_up((size_t)L->Y.stage_sites, 16)) : nullptr;
    int le = 0;
    hipError_t e1 = hipSuccess, e2 = hipSuccess;
    for (int64_t b = 0; b < (int64_t)N && !le && e1 == hipSuccess && e2 == hipSuccess; b += L->Y.stage_sites) {
        const int64_t c = std::min<int64_t>(L->Y.stage_sites, (int64_t)N - b);
        le = launch_gather(L->P, (int)i, b, c, t_occ, t_disp, L->stream);
        if (le) break;
        e1 = hipMemcpyAsync(occ + b, t_occ, (size_t)c, hipMemcpyDeviceToHost, L->stream);
        if (disp && e1 == hipSuccess)
            e2 = hipMemcpyAsync(disp + 3 * b, t_disp, (size_t)c * 12, hipMemcpyDeviceToHost, L->stream);
    }
    hipError_t e3 = hipStreamSynchronize(L->stream);
    if (le || e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
        return fail(FKMC_E_DEVICE, "read_state failed");
    return FKMC_OK;
}

fkmc_status fkmc_read_stats(fkmc_lattice* L, fkmc_stats* out)
{
    if (!L || !out) return fail(FKMC_E_INVALID, "null argument");
    HIP_OK(hipMemsetAsync(L->P.stat_acc, 0, (size_t)L->n * 3 * kStatFields * 8, L->stream));
    for (uint32_t i = 0; i < L->n; i++)
        LAUNCH_OK(launch_stats(L->P, (int)i, L->desc[i].n_sites, L->stream));
    std::vector<long long> acc((size_t)L->n * 3 * kStatFields);
    std::vector<unsigned long long> bk((size_t)L->n * kHopBuckets * 2);
    HIP_OK(hipMemcpyAsync(acc.data(), L->P.stat_acc, acc.size() * 8, hipMemcpyDeviceToHost, L->stream));
    HIP_OK(hipMemcpyAsync(bk.data(), L->P.buckets, bk.size() * 8, hipMemcpyDeviceToHost, L->stream));
    fkmc_status s = read_states(L);
    if (s) return s;
    for (uint32_t i = 0; i < L->n; i++) {
        fkmc_stats& o = out[i];
        std::memset(&o, 0, sizeof o);
        const LatState& S = L->h_state[i];
        if (L->desc[i].plain) {
            o.t = S.t;
            o.draws = S.draws;
            o.hops[0] = S.hops[0];
            o.hops[1] = S.hops[1];
            o.busy_ms = (double)S.busy_ticks / 100000.0;
            o.lds_resident = L->desc[i].resident ? 1u : 0u;
        } else {
            o.t = L->t_frag[i];
            o.cycles = S.cycles;
            o.busy_ms = (double)S.busy_ticks / 100000.0;  // 100 MHz real-time counter
            o.lds_resident = L->last_persistent && L->desc[i].resident ? 1u : 0u;
            o.tile_group = L->last_persistent ? (uint32_t)L->desc[i].group : 0u;
            for (int b = 0; b < kHopBuckets; b++) {
                o.hops[0] += bk[((size_t)i * kHopBuckets + b) * 2];
                o.hops[1] += bk[((size_t)i * kHopBuckets + b) * 2 + 1];
            }
        }
        const double h = L->geo[i].a_angstrom / 2.0;
        for (int sp = 0; sp < 3; sp++) {
            const long long* a = &acc[((size_t)i * 3 + sp) * kStatFields];
            o.count[sp] = (uint64_t)a[0];
            for (int c = 0; c < 3; c++) o.sum_r[sp][c] = a[1 + c];
            for (int c = 0; c < 6; c++) o.sum_rr[sp][c] = a[4 + c];
            const double nX = a[0] > 0 ? (double)a[0] : 1.0;
            o.msd[sp] = h * h * (double)(a[4] + a[5] + a[6]) / nX;
            const double t = o.t;
            o.D[sp] = t > 0 ? o.msd[sp] / (6.0 * t) : NAN;
            double mean[3];
            for (int c = 0; c < 3; c++) {
                mean[c] = (double)a[1 + c] / nX;
                o.drift[sp][c] = t > 0 ? h * mean[c] / t : NAN;
            }
            const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
            for (int c = 0; c < 6; c++) {
                const double cov = (double)a[4 + c] / nX - mean[pa[c]] * mean[pb[c]];
                o.Dtensor[sp][c] = t > 0 ? h * h * cov / (2.0 * t) : NAN;
            }
        }
    }
    return FKMC_OK;
}

fkmc_status fkmc_set_timing(fkmc_lattice* L, int32_t enable)
{
    if (!L) return fail(FKMC_E_INVALID, "null handle");
    L->timing = enable != 0;
    return FKMC_OK;
}

fkmc_status fkmc_phase_timing(const fkmc_lattice* L, double* avg_ms, uint64_t* launches)
{
    if (!L || !avg_ms || !launches) return fail(FKMC_E_INVALID, "null argument");
    *avg_ms = L->last_avg_ms;
    *launches = L->last_launches;
    return FKMC_OK;
}

fkmc_status fkmc_quantisation(const fkmc_lattice* L, uint32_t i, double* q, double* max_rel)
{
    if (!L || !q || !max_rel || i >= L->n) return fail(FKMC_E_INVALID, "bad argument");
    *q = L->qstep[i];
    *max_rel = L->qrel[i];
    return FKMC_OK;
}

}  // extern "C"
