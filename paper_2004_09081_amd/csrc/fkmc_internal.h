// Internal layout shared by the library's kernels and host code.
//
// HBM layout of one lattice (occupancy int8, displacement int32x4 with the
// same site numbering): the lattice is cut into the sub-blocks of the
// fragment decomposition (plain mode: one block).  Sub-block (bi, bj, bk)
// with cell ranges [x0,x0+wx) x [y0,y0+wy) x [z0,z0+wz) is one contiguous
// brick at offset 3 (z0 Ly Lx + wz (y0 Lx + wy x0)).  Inside a brick the
// three site types are stored as planes of V = wx wy wz bytes, each with
// its own face axis slowest:
//   type 0: (x wz + z) wy + y        (x = 0 face first)
//   type 1: V + (y wz + z) wx + x    (y = 0 face first)
//   type 2: 2V + (z wy + y) wx + x   (z = 0 face first)
// so the +x, +y and +z faces a phase needs from the neighbouring bricks are
// each one contiguous run of bytes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fkmc {

constexpr int kSpO = 0;
constexpr int kSpH = 1;
constexpr int kSpV = 2;

constexpr int kMaxWidth = 100;      // largest sub-block edge (cells)
constexpr int kMaxLdsPerBlock = 65536;  // dynamic LDS of one phase workgroup
constexpr int kMaxSlots = 128;      // vacancies per fragment-mode footprint
// vacancies per plain-mode lattice in the HBM kernels (their slots and
// totals sit in LDS, 16-18 bytes each, sized per launch for its largest
// lattice: 8192 slots take 128-148 KB of the 160 KB of a compute unit)
constexpr int kMaxPlainSlots = 8192;
constexpr int kPlainLdsSlots = 512;
constexpr int kAtomMarkBits = 13;     // hashed cell bitmap of the LDS atom-selection kernel
constexpr int kAtomMarkWords = 1 << (kAtomMarkBits - 5);   // vacancies per plain lattice held in LDS
constexpr int kHopBuckets = 256;    // spread of the per-lattice hop counters
constexpr int kStatFields = 10;     // count, r(3), rr(6)

// Static description of one lattice (device copy in the work buffer).
struct LatDesc {
    int32_t L[3];
    int32_t nsb[3];       // sub-blocks per axis (2 per fragment; 1 in plain mode)
    int32_t F[3];         // fragment edge (cells); last fragment takes the remainder
    int32_t nf[3];        // fragments per axis
    int32_t plain;
    int32_t resident;     // persistent kernel keeps the whole lattice in LDS
    int32_t n_vac;        // vacancies (conserved), sizes the resident vacancy list
    int32_t group;        // persistent kernel: tiles one wave runs at once (1, 4 or 8)
    int32_t fp_stride;    // persistent kernel: LDS bytes of one staged footprint
    int32_t fast;         // persistent kernel: vacancy-centric path (one fragment with <= 32
                          // vacancies, or plain with <= 512), lattice held in LDS
    uint32_t seed;
    uint32_t lattice_id;
    int32_t gb_period;
    int32_t gb_mask;
    int32_t tile0;        // first global tile index of this lattice (fragment mode)
    int32_t bounds_off;   // sub-block boundaries: [nsb0+1][nsb1+1][nsb2+1]
    int32_t c2s_off;      // cell -> sub-block index: [L0][L1][L2]
    int64_t occ_off;      // byte offset in the occupancy buffer
    int64_t disp_off;     // element (int4) offset in the displacement buffer
    int64_t n_sites;
    double k12[12];       // quantised rates, (X*3 + dz+1)*2 + g
    // site-energy interactions (plain lattices; site_window < 0: none)
    int32_t site_window;  // largest |dE_site| of a hop, meV
    int32_t site_e_fe[4]; // meV, vacancy-Fe over B-site shells |r|^2 = 1, 5, 9, 13 (a/2)^2
    int32_t site_e_vv[6]; // meV, vacancy-vacancy over O-site shells 2, 4, 6, 8, 10, 16
    int32_t site_pad;
    const uint32_t* site_fe;   // Fe bitmap, one bit per cell (canonical cell order)
    const double* site_table;  // quantised rates [(X*3 + dz+1)*2 + g][dE + window]
    // boundary sites as a map (Voronoi grains): one bit per site in canonical
    // order; when set it replaces the planes (nullptr: planes)
    const uint32_t* gb_map;
};

// Per-call parameters.
struct LatCall {
    double t_sync;
    uint64_t min_hops;
    uint64_t max_cycles;
    uint64_t hops_start;
    uint64_t cycles_start;
};

// Dynamic state.
struct LatState {
    uint64_t cycles;
    uint32_t done;
    uint32_t err;         // bit 0: slot overflow, bit 1: displacement overflow
    double t;             // plain-mode clock
    uint64_t draws;       // plain-mode draw counter
    uint64_t hops[2];     // plain-mode hop counters (O, H)
    uint64_t busy_ticks;  // persistent kernel: real-time ticks of the last call
    uint64_t steps;       // persistent kernel: BKL draws of the last call
};

// Geometry of one tile (sub-block of one colour of one fragment), built on
// the host: origin and width per axis, and the storage offsets of the four
// footprint segments (brick, +x face, +y face, +z face).  48 bytes.
struct TileRec {
    int64_t st[4];
    uint16_t ox, oy, oz;
    uint8_t wx, wy, wz, pad;
    uint32_t pad2;
};

struct DevPtrs {
    int8_t* occ;
    int4* disp;
    const LatDesc* desc;
    LatCall* call;
    LatState* state;
    unsigned long long* buckets;   // [n][kHopBuckets][2]
    const int32_t* tile2lat;       // [n_tiles]
    const TileRec* tiles;          // [8][n_tiles]
    const int32_t* bounds;
    const int32_t* c2s;
    long long* stat_acc;           // [n][3][kStatFields]
    int32_t n_lat;
    int32_t n_tiles;               // fragment-mode tiles per colour, all lattices
    const int32_t* batch_ids;      // lattices run by the persistent kernel
    const int2* groups;            // lockstep kernel: (lattice, first fragment) per wave
    int32_t n_groups;
    const int2* site_groups;       // lockstep site-model kernel: (lattice, fragment) per workgroup
    int32_t n_site_groups;
    int32_t gb_maps;               // nonzero when a lattice of the set has a boundary-site map
    int32_t fp_stride;             // LDS bytes of one staged footprint
    int32_t lds_region_bytes;      // persistent kernel: resident slab or staged footprints
    int32_t lds_wave_bytes;        // lockstep kernel: per-wave scratch plus footprints
};

// Per-wave LDS scratch of both fragment kernels (slot lists, tile records,
// rate table); staged footprints come after it.
constexpr int kWaveScratch = 3104;
// lockstep kernel: the same scratch without its last two arrays (the slots'
// vacancy-list indices, which only LDS-resident lattices use)
constexpr int kWaveScratchStaged = 2592;
constexpr int kPhaseWaves = 2;     // waves per lockstep workgroup
constexpr int kRecCache = 8 * 8 * 48;  // persistent kernel: tile records of a one-group lattice
// Sites per chunk of the canonical-order transfers at the ABI (occupancy and
// displacements, 13 bytes per site), staged through a slice of the work
// buffer so that the library allocates no device memory.
constexpr int64_t kStageSites = 1 << 19;

// Kernel launchers (fkmc_device.hip).  All return a hipError_t value.
int launch_init(const DevPtrs& P, const uint64_t* d_counts, int n_lat, void* stream);
int launch_phase(const DevPtrs& P, int colour, int group, void* stream);
// Fragment lattices with a site model: one workgroup per sub-block of the colour.
int launch_phase_site(const DevPtrs& P, int colour, void* stream);
int launch_cycle_begin(const DevPtrs& P, void* stream);
int launch_cycle_end(const DevPtrs& P, void* stream);
int launch_plain(const DevPtrs& P, const int32_t* d_plain_ids, int n_plain, int cap, void* stream);
// Plain BKL with site-energy interactions, one workgroup per listed lattice.
constexpr int kMaxSiteSlots = 2048;
constexpr int kMaxSiteWindow = 2047;  // meV: table indices stay below 2^16
int launch_plain_site(const DevPtrs& P, const int32_t* d_ids, int n, void* stream);
int launch_atomic_hbm(const DevPtrs& P, const int32_t* d_ids, int n, int cap, uint32_t n_frg,
                      uint64_t n_stages, void* stream);
int launch_stats(const DevPtrs& P, int lat, int64_t n_sites, void* stream);
// Canonical <-> storage order over canonical sites [begin, begin + count) of
// one lattice; the canonical arrays hold exactly those sites.
int launch_gather(const DevPtrs& P, int lat, int64_t begin, int64_t count, int8_t* d_occ_canon,
                  int32_t* d_disp_canon, void* stream);
int launch_scatter(const DevPtrs& P, int lat, int64_t begin, int64_t count, const int8_t* d_occ_canon,
                   void* stream);
int launch_batch(const DevPtrs& P, int n_batch, int waves, void* stream);
int launch_atomic(const DevPtrs& P, const int32_t* d_ids, int n, size_t lds, uint32_t n_frg,
                  uint64_t n_stages, void* stream);
int build_cycle_graph(const DevPtrs& P, int group, int cycles, hipGraphExec_t* out);
int launch_scatter_disp(const DevPtrs& P, int lat, int64_t begin, int64_t count,
                        const int32_t* d_disp_canon, void* stream);
// Zero `bytes` bytes at p (a fill kernel: 16-byte stores, byte tail).
int launch_fill_zero(void* p, size_t bytes, void* stream);
// LDS bytes of one staged footprint of at most max_footprint_bytes sites
// (four 16-byte-aligned segments).
int footprint_stride(int max_footprint_bytes);

}  // namespace fkmc
