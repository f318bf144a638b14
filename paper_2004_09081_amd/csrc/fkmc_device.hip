// HIP kernels (gfx950) of the fragment kMC hot path.
//
// Fragment phase: one 64-lane wavefront per sub-block ("tile").  The wave
// copies the tile's footprint (its brick plus the three +faces of the
// neighbouring bricks, all contiguous runs in the brick layout) from HBM into
// LDS with 16-byte loads, collects the vacancies, orders them by canonical
// site index, and runs the BKL loop (Eqs. TransitionProb, eventSelection,
// TimeStep) on LDS: each lane owns a contiguous group of vacancy slots and
// the 8 events of each, the cumulative rates come from a wavefront prefix
// sum of exact binary64 values, Philox4x32-10 supplies the two uniforms,
// and the clock uses a logarithm made only of correctly rounded operations.
// Each hop writes its two occupancy bytes and two displacement entries
// straight back to HBM; sub-blocks of one colour never share a site, so no
// other wave of the launch touches them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fkmc_internal.h"

namespace fkmc {

// ----------------------------------------------------------------------------
// Hop vectors in units of a/2, 8 per site type in ascending lexicographic
// order of (hx, hy, hz); 6 bits per hop: (hx+1) | (hy+1)<<2 | (hz+1)<<4.
//   type 0: (-1,-1,0) (-1,0,-1) (-1,0,1) (-1,1,0) (1,-1,0) (1,0,-1) (1,0,1) (1,1,0)
//   type 1: (-1,-1,0) (-1,1,0) (0,-1,-1) (0,-1,1) (0,1,-1) (0,1,1) (1,-1,0) (1,1,0)
//   type 2: (-1,0,-1) (-1,0,1) (0,-1,-1) (0,-1,1) (0,1,-1) (0,1,1) (1,0,-1) (1,0,1)
__device__ __forceinline__ void hop_vec(int t, int d, int& hx, int& hy, int& hz)
{
    const uint64_t tab = t == 0 ? 0x6a6192624110ull : (t == 1 ? 0x692a49841610ull : 0x986a49841904ull);
    const int v = (int)((tab >> (6 * d)) & 63);
    hx = (v & 3) - 1;
    hy = ((v >> 2) & 3) - 1;
    hz = ((v >> 4) & 3) - 1;
}

// Site type from the parities of doubled coordinates (exactly one is even).
__device__ __forceinline__ int site_type(int X, int Y)
{
    return (X & 1) == 0 ? 0 : ((Y & 1) == 0 ? 1 : 2);
}

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): multipliers 0xD2511F53, 0xCD9E8D57,
// key increments 0x9E3779B9, 0xBB67AE85.
__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1, uint32_t& o0, uint32_t& o1,
                                         uint32_t& o2, uint32_t& o3)
{
#pragma unroll
    for (int r = 0; r < 10; r++) {
        const uint32_t lo0 = 0xD2511F53u * c0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    o0 = c0;
    o1 = c1;
    o2 = c2;
    o3 = c3;
}

// Uniform in [0,1) and in (0,1] from 53 bits of a 64-bit word.
__device__ __forceinline__ double u53_lo(uint32_t hi, uint32_t lo)
{
    return (double)((((uint64_t)hi << 32) | lo) >> 11) * 0x1p-53;
}
__device__ __forceinline__ double u53_hi(uint32_t hi, uint32_t lo)
{
    return (double)(((((uint64_t)hi << 32) | lo) >> 11) + 1) * 0x1p-53;
}

// ln u for u in (0,1]: u = 2^e m with m in (sqrt(1/2), sqrt(2)], f = m - 1,
// s = f/(2+f), R = sum_{k=1..11} 2 s^(2k)/(2k+1) by Horner with fma,
// ln u = e*ln2_hi - ((f^2/2 - (s (f^2/2 + R) + e*ln2_lo)) - f), where
// ln2_hi = ln 2 rounded to 32 significant bits and ln2_lo the rest.
__device__ __forceinline__ double clock_ln(double u)
{
    constexpr double kLn2Hi = 0x1.62e42ffp-1;
    constexpr double kLn2Lo = -0x1.718432a1b0e26p-35;
    constexpr double kSqrt2 = 0x1.6a09e667f3bcdp+0;
    const uint64_t b = (uint64_t)__double_as_longlong(u);
    int e = (int)((b >> 52) & 0x7ff) - 1023;
    double m = __longlong_as_double((long long)((b & 0x000fffffffffffffull) | 0x3ff0000000000000ull));
    if (m > kSqrt2) {
        m = m * 0.5;
        e = e + 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double p = 2.0 / 23.0;
    p = __fma_rn(p, z, 2.0 / 21.0);
    p = __fma_rn(p, z, 2.0 / 19.0);
    p = __fma_rn(p, z, 2.0 / 17.0);
    p = __fma_rn(p, z, 2.0 / 15.0);
    p = __fma_rn(p, z, 2.0 / 13.0);
    p = __fma_rn(p, z, 2.0 / 11.0);
    p = __fma_rn(p, z, 2.0 / 9.0);
    p = __fma_rn(p, z, 2.0 / 7.0);
    p = __fma_rn(p, z, 2.0 / 5.0);
    p = __fma_rn(p, z, 2.0 / 3.0);
    const double R = z * p;
    const double hfsq = 0.5 * f * f;
    const double de = (double)e;
    return de * kLn2Hi - ((hfsq - (s * (hfsq + R) + de * kLn2Lo)) - f);
}

// Compiler barrier plus wait for this wave's LDS traffic.
__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ double wave_incl_scan(double v, int lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

// ----------------------------------------------------------------------------
// Brick geometry helpers.
struct Brick {
    int x0, y0, z0, wx, wy, wz;
    int64_t base;  // byte offset of the brick within its lattice
};

__device__ __forceinline__ Brick brick_of(const LatDesc& D, const int32_t* bounds, int bi, int bj,
                                          int bk)
{
    const int32_t* bx = bounds + D.bounds_off;
    const int32_t* by = bx + D.nsb[0] + 1;
    const int32_t* bz = by + D.nsb[1] + 1;
    Brick b;
    b.x0 = bx[bi];
    b.wx = bx[bi + 1] - b.x0;
    b.y0 = by[bj];
    b.wy = by[bj + 1] - b.y0;
    b.z0 = bz[bk];
    b.wz = bz[bk + 1] - b.z0;
    b.base = 3 * ((int64_t)b.z0 * D.L[1] * D.L[0] +
                  (int64_t)b.wz * ((int64_t)b.y0 * D.L[0] + (int64_t)b.wy * b.x0));
    return b;
}

__device__ __forceinline__ int brick_local(int t, int lx, int ly, int lz, int wx, int wy, int wz)
{
    const int V = wx * wy * wz;
    if (t == 0) return (lx * wz + lz) * wy + ly;
    if (t == 1) return V + (ly * wz + lz) * wx + lx;
    return 2 * V + (lz * wy + ly) * wx + lx;
}

// Storage offset (within the lattice) of canonical cell (i,j,k), type t.
__device__ __forceinline__ int64_t store_index(const LatDesc& D, const int32_t* bounds,
                                               const int32_t* c2s, int i, int j, int k, int t)
{
    const int32_t* m = c2s + D.c2s_off;
    const Brick b = brick_of(D, bounds, m[i], m[D.L[0] + j], m[D.L[0] + D.L[1] + k]);
    return b.base + brick_local(t, i - b.x0, j - b.y0, k - b.z0, b.wx, b.wy, b.wz);
}

__device__ __forceinline__ int is_gb(const LatDesc& D, int t, int cell_t)
{
    return (D.gb_period > 0 && ((D.gb_mask >> t) & 1) && (cell_t % D.gb_period) == 0) ? 1 : 0;
}

// ----------------------------------------------------------------------------
// Inclusive wavefront prefix sum of a binary64 value with DPP moves of its
// two 32-bit halves: row_shr 1,2,4,8 inside each 16-lane row, then
// row_bcast:15 and row_bcast:31 across rows.  The summands are exact
// multiples of one power of two, so every association gives the same sum.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_shifted(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_scan_dpp(double v)
{
    v += dpp_shifted<0x111, 0xF>(v);
    v += dpp_shifted<0x112, 0xF>(v);
    v += dpp_shifted<0x114, 0xF>(v);
    v += dpp_shifted<0x118, 0xF>(v);
    v += dpp_shifted<0x142, 0xA>(v);
    v += dpp_shifted<0x143, 0xC>(v);
    return v;
}

__device__ __forceinline__ double lane_value(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// ----------------------------------------------------------------------------
// Tile geometry.  A tile is the sub-block of fragment f with colour c; its
// footprint is the sub-block plus the +x face (type-0 sites of the next
// sub-block along x), the +y face (type 1) and the +z face (type 2).
// Segment k of the footprint: 0 = brick, 1..3 = faces; local index li of
// segment k lives at storage offset st[k] + li and at LDS byte lds[k] + li.
struct TileGeo {
    int wx, wy, wz;
    int ox, oy, oz;  // global cell of local cell (0,0,0)
    int64_t st0, st1, st2, st3;
    int lds0, lds1, lds2, lds3;
    int len0, len1, len2, len3;
};

// Segment accessors (selects, never a runtime-indexed local array).
__device__ __forceinline__ int64_t seg_st(const TileGeo& G, int k)
{
    return k == 0 ? G.st0 : (k == 1 ? G.st1 : (k == 2 ? G.st2 : G.st3));
}
__device__ __forceinline__ int seg_lds(const TileGeo& G, int k)
{
    return k == 0 ? G.lds0 : (k == 1 ? G.lds1 : (k == 2 ? G.lds2 : G.lds3));
}
__device__ __forceinline__ int seg_len(const TileGeo& G, int k)
{
    return k == 0 ? G.len0 : (k == 1 ? G.len1 : (k == 2 ? G.len2 : G.len3));
}

__device__ __forceinline__ TileGeo tile_geo_rec(const TileRec& R)
{
    TileGeo G;
    G.wx = R.wx;
    G.wy = R.wy;
    G.wz = R.wz;
    G.ox = R.ox;
    G.oy = R.oy;
    G.oz = R.oz;
    G.st0 = R.st[0];
    G.st1 = R.st[1];
    G.st2 = R.st[2];
    G.st3 = R.st[3];
    G.len0 = 3 * G.wx * G.wy * G.wz;
    G.len1 = G.wy * G.wz;
    G.len2 = G.wz * G.wx;
    G.len3 = G.wy * G.wx;
    G.lds0 = G.lds1 = G.lds2 = G.lds3 = 0;
    return G;
}

// LDS positions of the four segments in a wave's private footprint copy:
// consecutive 16-byte-aligned runs keeping each segment's HBM alignment.
__device__ __forceinline__ void tile_lds_private(TileGeo& G)
{
    int off = 0;
    G.lds0 = off + (int)(G.st0 & 15);
    off += ((int)(G.st0 & 15) + G.len0 + 15) & ~15;
    G.lds1 = off + (int)(G.st1 & 15);
    off += ((int)(G.st1 & 15) + G.len1 + 15) & ~15;
    G.lds2 = off + (int)(G.st2 & 15);
    off += ((int)(G.st2 & 15) + G.len2 + 15) & ~15;
    G.lds3 = off + (int)(G.st3 & 15);
}

// LDS positions when the whole lattice sits in LDS at its storage offsets.
__device__ __forceinline__ void tile_lds_resident(TileGeo& G)
{
    G.lds0 = (int)G.st0;
    G.lds1 = (int)G.st1;
    G.lds2 = (int)G.st2;
    G.lds3 = (int)G.st3;
}

__device__ __forceinline__ int fp_local(const TileGeo& G, int lx, int ly, int lz, int t, int& li)
{
    if (t == 0 && lx == G.wx) { li = lz * G.wy + ly; return 1; }
    if (t == 1 && ly == G.wy) { li = lz * G.wx + lx; return 2; }
    if (t == 2 && lz == G.wz) { li = ly * G.wx + lx; return 3; }
    li = brick_local(t, lx, ly, lz, G.wx, G.wy, G.wz);
    return 0;
}


__device__ __forceinline__ uint32_t pack_xyz(int X, int Y, int Z)
{
    return (uint32_t)X | ((uint32_t)Y << 10) | ((uint32_t)Z << 20);
}

// LDS position / storage offset of the site at packed local doubled coords.
__device__ __forceinline__ void xyz_where(const TileGeo& G, uint32_t xyz, int& lds, int64_t& st)
{
    const int X = xyz & 1023, Y = (xyz >> 10) & 1023, Z = xyz >> 20;
    int li;
    const int k = fp_local(G, X >> 1, Y >> 1, Z >> 1, site_type(X, Y), li);
    lds = seg_lds(G, k) + li;
    st = seg_st(G, k) + li;
}

// ----------------------------------------------------------------------------
// Per-wave LDS scratch: vacancy count, rate table, unsorted slots (canonical
// key + packed coordinates), sorted slot coordinates; then, for a tile whose
// lattice is not LDS-resident, the private footprint copy.
struct WaveScratch {
    int* cnt;
    double* k12;
    uint64_t* raw_key;
    uint32_t* raw_xyz;
    uint32_t* xyz;
    uint16_t* raw_idx;  // resident lattices: vacancy-list entry of each slot
    uint16_t* idx;
    unsigned char* occ;
};

__host__ __device__ constexpr int scratch_bytes() { return 112 + kMaxSlots * 20; }

__device__ __forceinline__ WaveScratch wave_scratch(unsigned char* base)
{
    WaveScratch w;
    w.cnt = (int*)base;
    w.k12 = (double*)(base + 16);
    w.raw_key = (uint64_t*)(base + 112);
    w.raw_xyz = (uint32_t*)(base + 112 + 8 * kMaxSlots);
    w.xyz = (uint32_t*)(base + 112 + 12 * kMaxSlots);
    w.raw_idx = (uint16_t*)(base + 112 + 16 * kMaxSlots);
    w.idx = (uint16_t*)(base + 112 + 18 * kMaxSlots);
    w.occ = base + scratch_bytes();
    return w;
}

// Record vacancy found at segment k, local index li.
__device__ __forceinline__ void add_slot(const TileGeo& G, const LatDesc& D, const WaveScratch& W,
                                         int k, int li)
{
    int lx, ly, lz, t;
    if (k == 0) {
        const int V = G.wx * G.wy * G.wz;
        t = li / V;
        const int r = li - t * V;
        if (t == 0) { ly = r % G.wy; lz = (r / G.wy) % G.wz; lx = r / (G.wy * G.wz); }
        else if (t == 1) { lx = r % G.wx; lz = (r / G.wx) % G.wz; ly = r / (G.wx * G.wz); }
        else { lx = r % G.wx; ly = (r / G.wx) % G.wy; lz = r / (G.wx * G.wy); }
    } else if (k == 1) {
        t = 0; lx = G.wx; ly = li % G.wy; lz = li / G.wy;
    } else if (k == 2) {
        t = 1; ly = G.wy; lx = li % G.wx; lz = li / G.wx;
    } else {
        t = 2; lz = G.wz; lx = li % G.wx; ly = li / G.wx;
    }
    int gi = G.ox + lx, gj = G.oy + ly, gk = G.oz + lz;
    if (gi >= D.L[0]) gi -= D.L[0];
    if (gj >= D.L[1]) gj -= D.L[1];
    if (gk >= D.L[2]) gk -= D.L[2];
    const uint64_t key = ((((uint64_t)gk * D.L[1] + gj) * D.L[0] + gi) * 3) + t;
    const int slot = atomicAdd(W.cnt, 1);
    if (slot < kMaxSlots) {
        W.raw_xyz[slot] = pack_xyz(2 * lx + (t != 0), 2 * ly + (t != 1), 2 * lz + (t != 2));
        W.raw_key[slot] = key;
    }
}

// Vacancy bytes (value 2) of one 16-byte chunk of segment k.
__device__ __forceinline__ void scan_chunk(const TileGeo& G, const LatDesc& D, const WaveScratch& W,
                                           int k, int chunk, int al, uint4 v)
{
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint32_t wq = q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w));
        const uint32_t x = wq ^ 0x02020202u;
        if (((x - 0x01010101u) & ~x & 0x80808080u) == 0) continue;
#pragma unroll
        for (int bb = 0; bb < 4; bb++) {
            if (((wq >> (8 * bb)) & 0xff) != kSpV) continue;
            const int li = 16 * chunk + 4 * q + bb - al;
            if (li < 0 || li >= seg_len(G, k)) continue;
            add_slot(G, D, W, k, li);
        }
    }
}

// Copy (kFromGlobal) or read in place the footprint's 16-byte chunks and
// collect its vacancies (unsorted).  All loads of a lane are issued before
// any of them is consumed.
__device__ __forceinline__ void collect_slots(const TileGeo& G, const LatDesc& D, const WaveScratch& W,
                                              const unsigned char* src, int lane, bool from_global)
{
    const int al0 = (int)(G.st0 & 15), al1 = (int)(G.st1 & 15), al2 = (int)(G.st2 & 15),
              al3 = (int)(G.st3 & 15);
    const int n0 = (al0 + G.len0 + 15) >> 4, n1 = (al1 + G.len1 + 15) >> 4,
              n2 = (al2 + G.len2 + 15) >> 4, n3 = (al3 + G.len3 + 15) >> 4;
    const int total = n0 + n1 + n2 + n3;
    for (int base = 0; base < total; base += 256) {
        uint4 v0, v1, v2, v3;
        int k0, k1, k2, k3, c0, c1, c2, c3;
        // locate chunk j: segment k, chunk index c within it
        auto locate = [&](int j, int& k, int& c) {
            k = -1;
            c = j;
            if (j >= total) return;
            if (c < n0) { k = 0; return; }
            c -= n0;
            if (c < n1) { k = 1; return; }
            c -= n1;
            if (c < n2) { k = 2; return; }
            c -= n2;
            k = 3;
        };
        auto fetch = [&](int k, int c) -> uint4 {
            const int64_t st = seg_st(G, k);
            const int a = (int)(st & 15);
            return *((const uint4*)(src + (st - a)) + c);
        };
        locate(base + lane, k0, c0);
        locate(base + lane + 64, k1, c1);
        locate(base + lane + 128, k2, c2);
        locate(base + lane + 192, k3, c3);
        if (k0 >= 0) v0 = fetch(k0, c0);
        if (k1 >= 0) v1 = fetch(k1, c1);
        if (k2 >= 0) v2 = fetch(k2, c2);
        if (k3 >= 0) v3 = fetch(k3, c3);
        auto take = [&](int k, int c, uint4 v) {
            if (k < 0) return;
            const int a = (int)(seg_st(G, k) & 15);
            if (from_global) *((uint4*)(W.occ + seg_lds(G, k) - a) + c) = v;
            scan_chunk(G, D, W, k, c, a, v);
        };
        take(k0, c0, v0);
        take(k1, c1, v1);
        take(k2, c2, v2);
        take(k3, c3, v3);
    }
    (void)al1;
    (void)al2;
    (void)al3;
}

// Order the slots by canonical site index (keys are distinct).
__device__ __forceinline__ void sort_slots(const WaveScratch& W, int n, int lane)
{
    for (int l = lane; l < n; l += 64) {
        const uint64_t key = W.raw_key[l];
        int rank = 0;
        for (int j = 0; j < n; j++) rank += W.raw_key[j] < key;
        W.xyz[rank] = W.raw_xyz[l];
        W.idx[rank] = W.raw_idx[l];
    }
}

// Resident lattices keep the global position of every vacancy in an LDS
// list (i | j << 10 | k << 20 | type << 30).  The slots of a tile are the
// list entries inside its footprint.
__device__ __forceinline__ void collect_from_list(const TileGeo& G, const LatDesc& D,
                                                  const WaveScratch& W, const uint32_t* vlist,
                                                  int nv, int lane)
{
    for (int v = lane; v < nv; v += 64) {
        const uint32_t g = vlist[v];
        const int i = g & 1023, j = (g >> 10) & 1023, k = (g >> 20) & 1023, t = g >> 30;
        int lx = i - G.ox, ly = j - G.oy, lz = k - G.oz;
        if (lx < 0) lx += D.L[0];
        if (ly < 0) ly += D.L[1];
        if (lz < 0) lz += D.L[2];
        const bool inx = lx < G.wx, iny = ly < G.wy, inz = lz < G.wz;
        const bool in = (inx && iny && inz) || (t == 0 && lx == G.wx && iny && inz) ||
                        (t == 1 && ly == G.wy && inx && inz) || (t == 2 && lz == G.wz && inx && iny);
        if (!in) continue;
        const int slot = atomicAdd(W.cnt, 1);
        if (slot < kMaxSlots) {
            W.raw_key[slot] = ((((uint64_t)k * D.L[1] + j) * D.L[0] + i) * 3) + t;
            W.raw_xyz[slot] = pack_xyz(2 * lx + (t != 0), 2 * ly + (t != 1), 2 * lz + (t != 2));
            W.raw_idx[slot] = (uint16_t)v;
        }
    }
}

// Write the final positions of a tile's vacancies back to the list.
__device__ __forceinline__ void update_list(const TileGeo& G, const LatDesc& D, const WaveScratch& W,
                                            uint32_t* vlist, int n, int lane)
{
    for (int l = lane; l < n; l += 64) {
        const uint32_t xyz = W.xyz[l];
        const int X = xyz & 1023, Y = (xyz >> 10) & 1023, Z = xyz >> 20;
        const int t = site_type(X, Y);
        int i = G.ox + (X >> 1), j = G.oy + (Y >> 1), k = G.oz + (Z >> 1);
        if (i >= D.L[0]) i -= D.L[0];
        if (j >= D.L[1]) j -= D.L[1];
        if (k >= D.L[2]) k -= D.L[2];
        vlist[W.idx[l]] = (uint32_t)i | ((uint32_t)j << 10) | ((uint32_t)k << 20) | ((uint32_t)t << 30);
    }
}

// Rate of event d of the vacancy at packed local doubled coordinates xyz:
// 0 when the hop edge's midpoint is outside the sub-block or the target
// holds a vacancy; else the table entry for (ion species, z step, boundary).
__device__ __forceinline__ double tile_rate(const TileGeo& G, const unsigned char* occl,
                                            const double* k12, const LatDesc& D, uint32_t xyz, int d)
{
    const int X = xyz & 1023, Y = (xyz >> 10) & 1023, Z = xyz >> 20;
    const int t = site_type(X, Y);
    int hx, hy, hz;
    hop_vec(t, d, hx, hy, hz);
    const int ox = (2 * X + hx) >> 2, oy = (2 * Y + hy) >> 2, oz = (2 * Z + hz) >> 2;
    if (ox < 0 || ox >= G.wx || oy < 0 || oy >= G.wy || oz < 0 || oz >= G.wz) return 0.0;
    const int tX = X + hx, tY = Y + hy, tZ = Z + hz;
    const int tt = site_type(tX, tY);
    int li;
    const int seg = fp_local(G, tX >> 1, tY >> 1, tZ >> 1, tt, li);
    const int sp = occl[seg_lds(G, seg) + li];
    if (sp == kSpV) return 0.0;
    int g = 0;
    if (D.gb_period > 0) {
        int cs = t == 0 ? G.ox + (X >> 1) : (t == 1 ? G.oy + (Y >> 1) : G.oz + (Z >> 1));
        int ct = tt == 0 ? G.ox + (tX >> 1) : (tt == 1 ? G.oy + (tY >> 1) : G.oz + (tZ >> 1));
        if (cs >= D.L[t]) cs -= D.L[t];
        if (ct >= D.L[tt]) ct -= D.L[tt];
        g = is_gb(D, t, cs) | is_gb(D, tt, ct);
    }
    return k12[(sp * 3 + hz + 1) * 2 + g];
}

__device__ __forceinline__ bool nn_site(uint32_t a, uint32_t b)
{
    const int dx = (int)(a & 1023) - (int)(b & 1023);
    const int dy = (int)((a >> 10) & 1023) - (int)((b >> 10) & 1023);
    const int dz = (int)(a >> 20) - (int)(b >> 20);
    return dx * dx + dy * dy + dz * dz == 2;
}

// Packed local doubled coordinates of the target of event d from xyz.
__device__ __forceinline__ uint32_t hop_target_xyz(uint32_t xyz, int d, int& hx, int& hy, int& hz)
{
    const int X = xyz & 1023, Y = (xyz >> 10) & 1023, Z = xyz >> 20;
    hop_vec(site_type(X, Y), d, hx, hy, hz);
    return pack_xyz(X + hx, Y + hy, Z + hz);
}

// BKL on one tile (Eqs. TransitionProb, eventSelection, TimeStep) until the
// next event would land after t_sync or no event is possible.  n sorted
// slots in W.xyz; event e = slot*8 + direction, in that order.
//  - n <= 8: lane e holds event e and its rate;
//  - n <= 64: lane l holds slot l and the rates of its 8 events;
//  - else: rates are recomputed from LDS at every step.
// The cumulative rates are a wavefront prefix sum; after a hop only the
// events whose vacancy moved or whose target changed are recomputed.
// Displacement changes are kept per moved particle in lane registers
// (origin, current site, accumulated hop) and written to HBM in two
// wave-wide passes (all reads, then all writes) when the 64 records fill up
// and at the end.
__device__ __forceinline__ void tile_bkl(const TileGeo& G_, const WaveScratch& W, unsigned char* occl,
                                         const LatDesc& D, int8_t* occ_lat, int4* disp_lat,
                                         uint32_t f, uint32_t cycle, uint32_t colour, double t_sync,
                                         int n, int lane, uint32_t& hops_o, uint32_t& hops_h,
                                         bool write_occ, bool& stores_pending)
{
    bool rv = false;
    uint32_t r_orig = 0, r_cur = 0;
    int ax = 0, ay = 0, az = 0;
    int4 r_old = make_int4(0, 0, 0, 0);  // origin's displacement, loaded when the record opens
    int nrec = 0;
    auto flush = [&]() {
        int lo;
        int64_t sf = 0;
        if (rv) xyz_where(G_, r_cur, lo, sf);
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): every lane's read is done
        __builtin_amdgcn_wave_barrier();
        if (rv) disp_lat[sf] = make_int4(r_old.x + ax, r_old.y + ay, r_old.z + az, 0);
        stores_pending = true;  // waited for before the next displacement read
        rv = false;
        ax = ay = az = 0;
        nrec = 0;
    };
    auto open_record = [&](uint32_t xyz) {
        int lo;
        int64_t so;
        rv = true;
        r_orig = xyz;
        r_cur = xyz;
        xyz_where(G_, xyz, lo, so);
        r_old = disp_lat[so];  // (pending writes of this wave were waited for above)
    };

    // mode 1: G lanes per slot (G = 8, 4, 2, 1 for n <= 8, 16, 32, 64), each
    // caching the rates of 8/G consecutive events; mode 2: recompute.
    const int mode = n <= 64 ? 1 : 2;
    const int G = n <= 8 ? 8 : (n <= 16 ? 4 : (n <= 32 ? 2 : 1));
    const int epl = 8 / G;
    const int my_slot = lane / G;
    const int my_d0 = (lane % G) * epl;
    const bool ev_valid = mode == 1 && my_slot < n;
    const int m = (n + 63) >> 6;
    const int s0 = lane * m < n ? lane * m : n;
    const int s1 = s0 + m < n ? s0 + m : n;
    uint32_t my_xyz = ev_valid ? W.xyz[my_slot] : 0u;
    double kk[8];
#pragma unroll
    for (int d = 0; d < 8; d++) kk[d] = 0.0;
    double ls = 0.0;
    auto refresh = [&]() {
        ls = 0.0;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            if (j < epl) {
                kk[j] = tile_rate(G_, occl, W.k12, D, my_xyz, my_d0 + j);
                ls += kk[j];
            }
        }
    };
    if (ev_valid) refresh();

    double tau = 0.0;
    uint32_t step = 0;
    for (;;) {
        if (mode == 2) {
            ls = 0.0;
            for (int s = s0; s < s1; s++) {
                const uint32_t xyz = W.xyz[s];
                for (int d = 0; d < 8; d++) ls += tile_rate(G_, occl, W.k12, D, xyz, d);
            }
        }
        const double incl = wave_scan_dpp(ls);
        const double R = lane_value(incl, 63);
        if (R == 0.0) break;
        uint32_t x0, x1, x2, x3;
        philox10(step, f, cycle, (colour << 8) | 2u, D.seed, D.lattice_id, x0, x1, x2, x3);
        const double u_sel = u53_lo(x0, x1);
        const double u_t = u53_hi(x2, x3);
        const double dt = -clock_ln(u_t) / R;
        const double tn = tau + dt;
        if (tn > t_sync) break;
        tau = tn;
        const double y = u_sel * R;
        const uint64_t mk = __ballot(incl > y);
        int sel;
        bool fallback = false;
        if (mk) {
            sel = __ffsll((unsigned long long)mk) - 1;
        } else {
            sel = 63 - __clzll((long long)__ballot(ls > 0.0));
            fallback = true;
        }
        // pick = packed vacancy coordinates | direction << 29; slot index
        int pick = 0, pslot = 0;
        if (lane == sel) {
            double C = incl - ls;
            int found = -1, last = -1;
            if (mode == 1) {
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    if (j < epl) {
                        if (kk[j] > 0.0) last = j;
                        C += kk[j];
                        if (!fallback && found < 0 && C > y) found = j;
                    }
                }
                pick = (int)(my_xyz | ((uint32_t)(my_d0 + (found >= 0 ? found : last)) << 29));
                pslot = my_slot;
            } else {
                uint32_t lx = 0;
                for (int s = s0; s < s1 && found < 0; s++) {
                    const uint32_t xyz = W.xyz[s];
                    for (int d = 0; d < 8; d++) {
                        const double k = tile_rate(G_, occl, W.k12, D, xyz, d);
                        if (k > 0.0) { last = s * 8 + d; lx = xyz; }
                        C += k;
                        if (!fallback && C > y) { found = s * 8 + d; lx = xyz; break; }
                    }
                }
                const int e = found >= 0 ? found : last;
                pick = (int)(lx | ((uint32_t)(e & 7) << 29));
                pslot = e >> 3;
            }
        }
        pick = __builtin_amdgcn_readlane(pick, sel);
        pslot = __builtin_amdgcn_readlane(pslot, sel);
        const uint32_t sx = (uint32_t)pick & 0x1FFFFFFFu;
        const int d = (int)((uint32_t)pick >> 29);
        int hx, hy, hz;
        const uint32_t tx = hop_target_xyz(sx, d, hx, hy, hz);
        int spos, tpos;
        int64_t sst, tst;
        xyz_where(G_, sx, spos, sst);
        xyz_where(G_, tx, tpos, tst);
        const int sp = occl[tpos];
        wave_lds_fence();
        if (lane == 0) {
            occl[spos] = (unsigned char)sp;
            occl[tpos] = (unsigned char)kSpV;
            W.xyz[pslot] = tx;
            if (write_occ) {
                occ_lat[sst] = (int8_t)sp;
                occ_lat[tst] = (int8_t)kSpV;
            }
        }
        // particle records: the vacancy moves sx -> tx, the ion tx -> sx
        uint64_t mv = __ballot(rv && r_cur == sx);
        uint64_t mi = __ballot(rv && r_cur == tx);
        if (nrec + (mv == 0) + (mi == 0) > 64) {
            flush();
            mv = 0;
            mi = 0;
        }
        int lv, lion;
        if (stores_pending && (mv == 0 || mi == 0)) {
            __builtin_amdgcn_s_waitcnt(0x0F70);
            __builtin_amdgcn_wave_barrier();
            stores_pending = false;
        }
        if (mv) {
            lv = __ffsll((unsigned long long)mv) - 1;
        } else {
            lv = nrec++;
            if (lane == lv) open_record(sx);
        }
        if (mi) {
            lion = __ffsll((unsigned long long)mi) - 1;
        } else {
            lion = nrec++;
            if (lane == lion) open_record(tx);
        }
        if (lane == lv) { r_cur = tx; ax += hx; ay += hy; az += hz; }
        if (lane == lion) { r_cur = sx; ax -= hx; ay -= hy; az -= hz; }
        if (sp == kSpO) hops_o++;
        else hops_h++;
        step++;
        wave_lds_fence();
        if (ev_valid) {
            if (my_slot == pslot) my_xyz = tx;
            if (my_slot == pslot || nn_site(my_xyz, sx) || nn_site(my_xyz, tx)) refresh();
        }
    }
    flush();
}

// ----------------------------------------------------------------------------
// Lockstep phase kernel: one wave per tile of colour `colour`, every
// fragment lattice of the set, footprint staged HBM -> LDS.
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_phase(DevPtrs P, int colour)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int tile = blockIdx.x * WAVES + wv;
    if (tile >= P.n_tiles) return;
    const int lat = P.n_lat == 1 ? 0 : P.tile2lat[tile];
    const LatDesc& D = P.desc[lat];
    LatState* S = P.state + lat;
    if (S->done) return;
    const uint32_t cycle = (uint32_t)S->cycles;
    const double t_sync = P.call[lat].t_sync;
    const WaveScratch W = wave_scratch(smem + wv * P.lds_wave_bytes);
    const int f = tile - D.tile0;
    TileGeo G = tile_geo_rec(P.tiles[(size_t)colour * P.n_tiles + tile]);
    tile_lds_private(G);
    if (lane == 0) *W.cnt = 0;
    if (lane < 12) W.k12[lane] = D.k12[lane];
    wave_lds_fence();
    collect_slots(G, D, W, (const unsigned char*)(P.occ + D.occ_off), lane, true);
    wave_lds_fence();
    const int n = *W.cnt;
    if (n == 0) return;
    if (n > kMaxSlots) {
        if (lane == 0) atomicOr(&S->err, 1u);
        return;
    }
    sort_slots(W, n, lane);
    wave_lds_fence();
    uint32_t ho = 0, hh = 0;
    bool pending = false;
    tile_bkl(G, W, W.occ, D, P.occ + D.occ_off, P.disp + D.disp_off, (uint32_t)f, cycle,
             (uint32_t)colour, t_sync, n, lane, ho, hh, true, pending);
    if (lane == 0 && (ho | hh)) {
        unsigned long long* b = P.buckets + ((size_t)lat * kHopBuckets + (f & (kHopBuckets - 1))) * 2;
        if (ho) atomicAdd(b, (unsigned long long)ho);
        if (hh) atomicAdd(b + 1, (unsigned long long)hh);
    }
}

// Persistent batched kernel: one workgroup per lattice runs the whole call
// (cycles of 8 phases, workgroup barrier between phases), so every lattice
// advances at its own pace.  A lattice that fits is kept in LDS for the
// whole call; otherwise each wave stages its tile's footprint from HBM.
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_batch(DevPtrs P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long hop_tot[2];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int nw = blockDim.x >> 6;
    const uint64_t t_begin = __builtin_amdgcn_s_memrealtime();
    const int lat = P.batch_ids[blockIdx.x];
    const LatDesc& D = P.desc[lat];
    LatState* S = P.state + lat;
    const LatCall* C = P.call + lat;
    const bool resident = D.resident != 0;
    unsigned char* slab = smem;
    const WaveScratch W = wave_scratch(smem + P.lds_resident_bytes + wv * P.lds_wave_bytes);
    int8_t* occ_lat = P.occ + D.occ_off;
    int4* disp_lat = P.disp + D.disp_off;
    const int64_t nbytes = D.n_sites;
    __shared__ int vlist_n;
    uint32_t* vlist = (uint32_t*)(slab + (((nbytes + 15) & ~(int64_t)15) + 32));
    if (threadIdx.x == 0) vlist_n = 0;
    if (resident) {
        const int nch = (int)((nbytes + 15) >> 4);
        for (int j = threadIdx.x; j < nch; j += blockDim.x)
            ((uint4*)slab)[j] = ((const uint4*)occ_lat)[j];
    }
    __syncthreads();
    if (resident) {
        // vacancy list, scanned in canonical order
        for (int64_t c = threadIdx.x; c < nbytes; c += blockDim.x) {
            const int t = (int)(c % 3);
            const int64_t cell = c / 3;
            const int i = (int)(cell % D.L[0]);
            const int j = (int)((cell / D.L[0]) % D.L[1]);
            const int k = (int)(cell / ((int64_t)D.L[0] * D.L[1]));
            if (slab[store_index(D, P.bounds, P.c2s, i, j, k, t)] != kSpV) continue;
            const int v = atomicAdd(&vlist_n, 1);
            if (v < D.n_vac)
                vlist[v] = (uint32_t)i | ((uint32_t)j << 10) | ((uint32_t)k << 20) | ((uint32_t)t << 30);
        }
    }
    if (threadIdx.x < 2) hop_tot[threadIdx.x] = 0;
    if (lane < 12) W.k12[lane] = D.k12[lane];
    __syncthreads();
    const int nv_list = vlist_n < D.n_vac ? vlist_n : D.n_vac;
    bool err = resident && vlist_n > D.n_vac;
    const double t_sync = C->t_sync;
    const uint64_t max_cycles = C->max_cycles, min_hops = C->min_hops;
    const uint64_t cycle0 = S->cycles;
    const int ntiles = D.nf[0] * D.nf[1] * D.nf[2];
    // A lattice with one tile per colour is run by wave 0 alone, without
    // workgroup barriers; otherwise every phase ends with one.
    const bool solo = ntiles == 1;
    bool pending = false;
    uint64_t ncyc = 0;
    if (!solo || wv == 0) {
        while (ncyc < max_cycles) {
            const uint32_t cycle = (uint32_t)(cycle0 + ncyc);
            for (int colour = 0; colour < 8; colour++) {
                uint32_t ho = 0, hh = 0;
                for (int f = wv; f < ntiles; f += nw) {
                    TileGeo G = tile_geo_rec(P.tiles[(size_t)colour * P.n_tiles + D.tile0 + f]);
                    if (lane == 0) *W.cnt = 0;
                    wave_lds_fence();
                    unsigned char* occl = resident ? slab : W.occ;
                    if (resident) {
                        tile_lds_resident(G);
                        collect_from_list(G, D, W, vlist, nv_list, lane);
                    } else {
                        tile_lds_private(G);
                        collect_slots(G, D, W, (const unsigned char*)occ_lat, lane, true);
                    }
                    wave_lds_fence();
                    const int n = *W.cnt;
                    if (n == 0) continue;
                    if (n > kMaxSlots) {
                        err = true;
                        continue;
                    }
                    sort_slots(W, n, lane);
                    wave_lds_fence();
                    tile_bkl(G, W, occl, D, occ_lat, disp_lat, (uint32_t)f, cycle, (uint32_t)colour,
                             t_sync, n, lane, ho, hh, !resident, pending);
                    if (resident) {
                        wave_lds_fence();
                        update_list(G, D, W, vlist, n, lane);
                    }
                }
                if (lane == 0 && (ho | hh)) {
                    atomicAdd(&hop_tot[0], (unsigned long long)ho);
                    atomicAdd(&hop_tot[1], (unsigned long long)hh);
                }
                if (solo) {
                    wave_lds_fence();
                } else {
                    __syncthreads();
                    pending = false;  // the barrier waited for every store
                }
            }
            ncyc++;
            const unsigned long long tot = hop_tot[0] + hop_tot[1];
            if (!solo) __syncthreads();
            if (min_hops > 0 && tot >= min_hops) break;
        }
    }
    __syncthreads();
    if (resident) {
        const int nch = (int)(nbytes >> 4);
        for (int j = threadIdx.x; j < nch; j += blockDim.x)
            ((uint4*)occ_lat)[j] = ((const uint4*)slab)[j];
        for (int64_t b = (int64_t)nch * 16 + threadIdx.x; b < nbytes; b += blockDim.x)
            occ_lat[b] = (int8_t)slab[b];
    }
    if (err && lane == 0) atomicOr(&S->err, 1u);
    if (threadIdx.x == 0) {
        S->busy_ticks = __builtin_amdgcn_s_memrealtime() - t_begin;
        S->cycles = cycle0 + ncyc;
        S->done = 1u;
        unsigned long long* b = P.buckets + (size_t)lat * kHopBuckets * 2;
        b[0] += hop_tot[0];
        b[1] += hop_tot[1];
    }
}

// Start (begin = 1) or end (begin = 0) of a cycle for every fragment
// lattice: one wave per lattice sums its hop buckets.
__global__ __launch_bounds__(64) void k_cycle(DevPtrs P, int begin)
{
    const int lat = blockIdx.x;
    const int lane = threadIdx.x;
    const LatDesc& D = P.desc[lat];
    if (D.plain) return;
    LatState* S = P.state + lat;
    LatCall* C = P.call + lat;
    if (!begin && S->done) return;
    unsigned long long so = 0, sh = 0;
    const unsigned long long* b = P.buckets + (size_t)lat * kHopBuckets * 2;
    for (int i = lane; i < kHopBuckets; i += 64) {
        so += b[2 * i];
        sh += b[2 * i + 1];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        so += __shfl_xor(so, off, 64);
        sh += __shfl_xor(sh, off, 64);
    }
    if (lane != 0) return;
    S->hops[0] = so;
    S->hops[1] = sh;
    if (begin) {
        C->hops_start = so + sh;
        C->cycles_start = S->cycles;
        S->done = C->max_cycles == 0 ? 1u : 0u;
        return;
    }
    S->cycles = S->cycles + 1;
    const uint64_t ncyc = S->cycles - C->cycles_start;
    const uint64_t nh = so + sh - C->hops_start;
    if ((C->min_hops > 0 && nh >= C->min_hops) || ncyc >= C->max_cycles) S->done = 1u;
}

// ----------------------------------------------------------------------------
// Plain (unfragmented) BKL: one 256-thread workgroup per lattice runs the
// whole call.  Vacancy slots in canonical order; occupancy read from HBM.
constexpr int kPlainThreads = 256;

struct PlainSlot {
    uint64_t packed;  // i | j << 16 | k << 32 | t << 48
};

__device__ __forceinline__ double plain_rate(const LatDesc& D, const DevPtrs& P, uint64_t pk,
                                             int d, int64_t& tgt_store)
{
    const int i = (int)(pk & 0xffff), j = (int)((pk >> 16) & 0xffff), k = (int)((pk >> 32) & 0xffff);
    const int t = (int)(pk >> 48);
    int hx, hy, hz;
    hop_vec(t, d, hx, hy, hz);
    int X = 2 * i + (t != 0) + hx, Y = 2 * j + (t != 1) + hy, Z = 2 * k + (t != 2) + hz;
    if (X < 0) X += 2 * D.L[0];
    if (X >= 2 * D.L[0]) X -= 2 * D.L[0];
    if (Y < 0) Y += 2 * D.L[1];
    if (Y >= 2 * D.L[1]) Y -= 2 * D.L[1];
    if (Z < 0) Z += 2 * D.L[2];
    if (Z >= 2 * D.L[2]) Z -= 2 * D.L[2];
    const int tt = site_type(X, Y);
    tgt_store = store_index(D, P.bounds, P.c2s, X >> 1, Y >> 1, Z >> 1, tt);
    const int sp = P.occ[D.occ_off + tgt_store];
    if (sp == kSpV) return 0.0;
    const int cs = t == 0 ? i : (t == 1 ? j : k);
    const int ct = tt == 0 ? (X >> 1) : (tt == 1 ? (Y >> 1) : (Z >> 1));
    const int g = is_gb(D, t, cs) | is_gb(D, tt, ct);
    return D.k12[(sp * 3 + hz + 1) * 2 + g];
}

__global__ __launch_bounds__(kPlainThreads) void k_plain(DevPtrs P, const int32_t* ids)
{
    __shared__ uint64_t slots[kMaxPlainSlots];
    __shared__ int wcount[kPlainThreads / 64];
    __shared__ double wsum[kPlainThreads / 64];
    __shared__ uint64_t wmask[kPlainThreads / 64];
    __shared__ uint64_t wnz[kPlainThreads / 64];
    __shared__ int n_sh;
    __shared__ int ev_sh;
    const int lat = ids[blockIdx.x];
    const LatDesc& D = P.desc[lat];
    LatState* S = P.state + lat;
    const LatCall* C = P.call + lat;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int NW = kPlainThreads / 64;

    // vacancy slots in ascending canonical index
    if (tid == 0) n_sh = 0;
    __syncthreads();
    const int64_t N = D.n_sites;
    for (int64_t base = 0; base < N; base += kPlainThreads) {
        const int64_t nidx = base + tid;
        bool v = false;
        uint64_t pk = 0;
        if (nidx < N) {
            const int t = (int)(nidx % 3);
            const int64_t cell = nidx / 3;
            const int i = (int)(cell % D.L[0]);
            const int j = (int)((cell / D.L[0]) % D.L[1]);
            const int k = (int)(cell / ((int64_t)D.L[0] * D.L[1]));
            v = P.occ[D.occ_off + store_index(D, P.bounds, P.c2s, i, j, k, t)] == kSpV;
            pk = (uint64_t)i | ((uint64_t)j << 16) | ((uint64_t)k << 32) | ((uint64_t)t << 48);
        }
        const uint64_t mk = __ballot(v);
        if (lane == 0) wcount[wv] = __popcll(mk);
        __syncthreads();
        int before = n_sh;
        for (int w = 0; w < wv; w++) before += wcount[w];
        if (v) {
            const int r = before + __popcll(mk & ((1ull << lane) - 1ull));
            if (r < kMaxPlainSlots) slots[r] = pk;
        }
        __syncthreads();
        if (tid == 0) {
            int tot = 0;
            for (int w = 0; w < NW; w++) tot += wcount[w];
            n_sh += tot;
        }
        __syncthreads();
    }
    const int n = n_sh;
    if (n > kMaxPlainSlots) {
        if (tid == 0) atomicOr(&S->err, 1u);
        return;
    }
    const int m = (n + kPlainThreads - 1) / kPlainThreads;
    const int s0 = tid * m < n ? tid * m : n;
    const int s1 = s0 + m < n ? s0 + m : n;
    double t = S->t;
    uint64_t draws = S->draws;
    const double horizon = C->t_sync;
    const double t_end = t + horizon;
    const uint64_t target = C->min_hops;
    uint64_t done = 0, ho = 0, hh = 0;
    while (done < target) {
        double ls = 0.0;
        for (int s = s0; s < s1; s++)
            for (int d = 0; d < 8; d++) {
                int64_t ts;
                ls += plain_rate(D, P, slots[s], d, ts);
            }
        double incl = wave_incl_scan(ls, lane);
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        double before = 0.0, R = 0.0;
        for (int w = 0; w < NW; w++) {
            if (w < wv) before += wsum[w];
            R += wsum[w];
        }
        incl += before;
        if (R == 0.0) break;
        uint32_t x0, x1, x2, x3;
        philox10((uint32_t)draws, (uint32_t)(draws >> 32), 0xFFFFFFFFu, 3u, D.seed, D.lattice_id,
                 x0, x1, x2, x3);
        draws++;
        const double u_sel = u53_lo(x0, x1);
        const double u_t = u53_hi(x2, x3);
        const double dt = -clock_ln(u_t) / R;
        const double tn = t + dt;
        if (horizon > 0.0 && tn > t_end) {
            t = t_end;
            break;
        }
        t = tn;
        const double y = u_sel * R;
        const uint64_t mk = __ballot(incl > y);
        const uint64_t nz = __ballot(ls > 0.0);
        if (lane == 0) {
            wmask[wv] = mk;
            wnz[wv] = nz;
        }
        __syncthreads();
        int sel = -1;
        bool fallback = false;
        for (int w = 0; w < NW && sel < 0; w++)
            if (wmask[w]) sel = w * 64 + __ffsll((unsigned long long)wmask[w]) - 1;
        if (sel < 0) {
            fallback = true;
            for (int w = NW - 1; w >= 0 && sel < 0; w--)
                if (wnz[w]) sel = w * 64 + 63 - __clzll((long long)wnz[w]);
        }
        if (tid == sel) {
            double Cc = incl - ls;
            int ev = -1, last = -1;
            for (int s = s0; s < s1 && ev < 0; s++)
                for (int d = 0; d < 8; d++) {
                    int64_t ts;
                    const double k = plain_rate(D, P, slots[s], d, ts);
                    if (k > 0.0) last = s * 8 + d;
                    Cc += k;
                    if (!fallback && Cc > y) { ev = s * 8 + d; break; }
                }
            if (ev < 0) ev = last;
            const int s = ev >> 3, d = ev & 7;
            const uint64_t pk = slots[s];
            int64_t ts;
            plain_rate(D, P, pk, d, ts);
            const int i = (int)(pk & 0xffff), j = (int)((pk >> 16) & 0xffff), k = (int)((pk >> 32) & 0xffff);
            const int tp = (int)(pk >> 48);
            const int64_t ss = store_index(D, P.bounds, P.c2s, i, j, k, tp);
            int hx, hy, hz;
            hop_vec(tp, d, hx, hy, hz);
            const int sp = P.occ[D.occ_off + ts];
            P.occ[D.occ_off + ss] = (int8_t)sp;
            P.occ[D.occ_off + ts] = (int8_t)kSpV;
            int4* dsrc = P.disp + (D.disp_off + ss);
            int4* dtgt = P.disp + (D.disp_off + ts);
            const int4 dv = *dsrc;
            const int4 di = *dtgt;
            *dtgt = make_int4(dv.x + hx, dv.y + hy, dv.z + hz, 0);
            *dsrc = make_int4(di.x - hx, di.y - hy, di.z - hz, 0);
            int X = 2 * i + (tp != 0) + hx, Y = 2 * j + (tp != 1) + hy, Z = 2 * k + (tp != 2) + hz;
            if (X < 0) X += 2 * D.L[0];
            if (X >= 2 * D.L[0]) X -= 2 * D.L[0];
            if (Y < 0) Y += 2 * D.L[1];
            if (Y >= 2 * D.L[1]) Y -= 2 * D.L[1];
            if (Z < 0) Z += 2 * D.L[2];
            if (Z >= 2 * D.L[2]) Z -= 2 * D.L[2];
            slots[s] = (uint64_t)(X >> 1) | ((uint64_t)(Y >> 1) << 16) | ((uint64_t)(Z >> 1) << 32) |
                       ((uint64_t)site_type(X, Y) << 48);
            ev_sh = sp;
            __threadfence_block();
        }
        __syncthreads();
        if (ev_sh == kSpO) ho++;
        else hh++;
        done++;
        __syncthreads();
    }
    if (tid == 0) {
        S->t = t;
        S->draws = draws;
        S->hops[0] += ho;
        S->hops[1] += hh;
    }
}

// ----------------------------------------------------------------------------
// Initial placement: one thread per lattice, rejection of occupied sites and
// of the biased low halves of the 128-bit product (exact uniform index).
__global__ void k_init(DevPtrs P, const uint64_t* counts, int n_lat)
{
    const int lat = blockIdx.x * blockDim.x + threadIdx.x;
    if (lat >= n_lat) return;
    const LatDesc& D = P.desc[lat];
    const uint64_t nv = counts[2 * lat], nh = counts[2 * lat + 1];
    const uint64_t N = (uint64_t)D.n_sites;
    const uint64_t thresh = (0ull - N) % N;
    uint64_t d = 0;
    for (uint64_t i = 0; i < nv + nh; i++) {
        const int8_t sp = i < nv ? (int8_t)kSpV : (int8_t)kSpH;
        for (;;) {
            uint32_t x0, x1, x2, x3;
            philox10((uint32_t)d, (uint32_t)(d >> 32), 0u, 1u, D.seed, D.lattice_id, x0, x1, x2, x3);
            d++;
            const uint64_t w = ((uint64_t)x0 << 32) | x1;
            const uint64_t lo = w * N;
            const uint64_t j = __umul64hi(w, N);
            if (lo < thresh) continue;
            const int t = (int)(j % 3);
            const uint64_t cell = j / 3;
            const int ci = (int)(cell % (uint64_t)D.L[0]);
            const int cj = (int)((cell / (uint64_t)D.L[0]) % (uint64_t)D.L[1]);
            const int ck = (int)(cell / ((uint64_t)D.L[0] * D.L[1]));
            int8_t* o = P.occ + D.occ_off + store_index(D, P.bounds, P.c2s, ci, cj, ck, t);
            if (*o != kSpO) continue;
            *o = sp;
            break;
        }
    }
}

// ----------------------------------------------------------------------------
// Per-species sums over one lattice: count, sum r, sum r_a r_b.
__global__ __launch_bounds__(256) void k_stats(DevPtrs P, int lat)
{
    const LatDesc& D = P.desc[lat];
    long long acc[3][kStatFields];
#pragma unroll
    for (int s = 0; s < 3; s++)
#pragma unroll
        for (int q = 0; q < kStatFields; q++) acc[s][q] = 0;
    const int64_t N = D.n_sites;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int sp = P.occ[D.occ_off + i];
        const int4 r = P.disp[D.disp_off + i];
        const long long x = r.x, y = r.y, z = r.z;
        const long long v[kStatFields] = {1, x, y, z, x * x, y * y, z * z, x * y, x * z, y * z};
#pragma unroll
        for (int s = 0; s < 3; s++)
            if (sp == s) {
#pragma unroll
                for (int q = 0; q < kStatFields; q++) acc[s][q] += v[q];
            }
    }
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int s = 0; s < 3; s++)
#pragma unroll
        for (int q = 0; q < kStatFields; q++) {
            long long v = acc[s][q];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0 && v != 0)
                atomicAdd((unsigned long long*)&P.stat_acc[((size_t)lat * 3 + s) * kStatFields + q],
                          (unsigned long long)v);
        }
}

// Canonical-order gather (read-out) and scatter (set occupancy).
__global__ void k_gather(DevPtrs P, int lat, int8_t* occ_c, int32_t* disp_c)
{
    const LatDesc& D = P.desc[lat];
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= D.n_sites) return;
    const int t = (int)(n % 3);
    const int64_t cell = n / 3;
    const int i = (int)(cell % D.L[0]);
    const int j = (int)((cell / D.L[0]) % D.L[1]);
    const int k = (int)(cell / ((int64_t)D.L[0] * D.L[1]));
    const int64_t s = store_index(D, P.bounds, P.c2s, i, j, k, t);
    occ_c[n] = P.occ[D.occ_off + s];
    if (disp_c) {
        const int4 r = P.disp[D.disp_off + s];
        disp_c[3 * n] = r.x;
        disp_c[3 * n + 1] = r.y;
        disp_c[3 * n + 2] = r.z;
    }
}

__global__ void k_scatter(DevPtrs P, int lat, const int8_t* occ_c)
{
    const LatDesc& D = P.desc[lat];
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= D.n_sites) return;
    const int t = (int)(n % 3);
    const int64_t cell = n / 3;
    const int i = (int)(cell % D.L[0]);
    const int j = (int)((cell / D.L[0]) % D.L[1]);
    const int k = (int)(cell / ((int64_t)D.L[0] * D.L[1]));
    const int64_t s = store_index(D, P.bounds, P.c2s, i, j, k, t);
    P.occ[D.occ_off + s] = occ_c[n];
    P.disp[D.disp_off + s] = make_int4(0, 0, 0, 0);
}

// ----------------------------------------------------------------------------
// Launchers.
int launch_init(const DevPtrs& P, const uint64_t* d_counts, int n_lat, void* stream)
{
    const int bs = 64;
    hipLaunchKernelGGL(k_init, dim3((n_lat + bs - 1) / bs), dim3(bs), 0, (hipStream_t)stream, P,
                       d_counts, n_lat);
    return (int)hipGetLastError();
}

int launch_phase(const DevPtrs& P, int colour, int lds_per_wave, void* stream)
{
    if (P.n_tiles == 0) return 0;
    if (4 * lds_per_wave <= kMaxLdsPerBlock) {
        const int blocks = (P.n_tiles + 3) / 4;
        hipLaunchKernelGGL(k_phase<4>, dim3(blocks), dim3(256), (size_t)lds_per_wave * 4,
                           (hipStream_t)stream, P, colour);
    } else {
        hipLaunchKernelGGL(k_phase<1>, dim3(P.n_tiles), dim3(64), (size_t)lds_per_wave,
                           (hipStream_t)stream, P, colour);
    }
    return (int)hipGetLastError();
}

int launch_batch(const DevPtrs& P, int n_batch, int waves, void* stream)
{
    if (n_batch == 0) return 0;
    const size_t lds = (size_t)P.lds_resident_bytes + (size_t)waves * P.lds_wave_bytes;
    hipError_t e = hipFuncSetAttribute((const void*)k_batch,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(k_batch, dim3(n_batch), dim3(64 * waves), lds, (hipStream_t)stream, P);
    return (int)hipGetLastError();
}

// A graph of `cycles` consecutive lockstep cycles (8 phase kernels and the
// cycle-end kernel each, chained), built from kernel nodes so that it can be
// launched on any stream.  Holds no memset or copy nodes.
int build_cycle_graph(const DevPtrs& P, int lds_per_wave, int cycles, hipGraphExec_t* out)
{
    hipGraph_t g;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return (int)e;
    DevPtrs args_p = P;  // argument values are copied into each node
    hipGraphNode_t prev = nullptr;
    const bool four = 4 * lds_per_wave <= kMaxLdsPerBlock;
    int colours[8] = {0, 1, 2, 3, 4, 5, 6, 7};
    int begin0 = 0;
    for (int c = 0; c < cycles && e == hipSuccess; c++) {
        for (int col = 0; col < 9 && e == hipSuccess; col++) {
            hipKernelNodeParams kp = {};
            void* argv[3];
            if (col < 8) {
                argv[0] = &args_p;
                argv[1] = &colours[col];
                kp.func = four ? (void*)k_phase<4> : (void*)k_phase<1>;
                kp.gridDim = four ? dim3((P.n_tiles + 3) / 4) : dim3(P.n_tiles);
                kp.blockDim = four ? dim3(256) : dim3(64);
                kp.sharedMemBytes = (unsigned)(lds_per_wave * (four ? 4 : 1));
            } else {
                argv[0] = &args_p;
                argv[1] = &begin0;
                kp.func = (void*)k_cycle;
                kp.gridDim = dim3(P.n_lat);
                kp.blockDim = dim3(64);
                kp.sharedMemBytes = 0;
            }
            kp.kernelParams = argv;
            kp.extra = nullptr;
            hipGraphNode_t node;
            e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
            prev = node;
        }
    }
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return (int)e;
}

int launch_cycle_end(const DevPtrs& P, void* stream)
{
    hipLaunchKernelGGL(k_cycle, dim3(P.n_lat), dim3(64), 0, (hipStream_t)stream, P, 0);
    return (int)hipGetLastError();
}

int launch_cycle_begin(const DevPtrs& P, void* stream)
{
    hipLaunchKernelGGL(k_cycle, dim3(P.n_lat), dim3(64), 0, (hipStream_t)stream, P, 1);
    return (int)hipGetLastError();
}

int launch_plain(const DevPtrs& P, const int32_t* d_plain_ids, int n_plain, void* stream)
{
    if (n_plain == 0) return 0;
    hipLaunchKernelGGL(k_plain, dim3(n_plain), dim3(kPlainThreads), 0, (hipStream_t)stream, P,
                       d_plain_ids);
    return (int)hipGetLastError();
}

int launch_stats(const DevPtrs& P, int lat, int64_t n_sites, void* stream)
{
    int64_t blocks = (n_sites + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_stats, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, P, lat);
    return (int)hipGetLastError();
}

int launch_gather(const DevPtrs& P, int lat, int64_t n_sites, int8_t* d_occ_canon,
                  int32_t* d_disp_canon, void* stream)
{
    const int64_t blocks = (n_sites + 255) / 256;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, P, lat,
                       d_occ_canon, d_disp_canon);
    return (int)hipGetLastError();
}

__global__ void k_scatter_disp(DevPtrs P, int lat, const int32_t* disp_c)
{
    const LatDesc& D = P.desc[lat];
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= D.n_sites) return;
    const int t = (int)(n % 3);
    const int64_t cell = n / 3;
    const int i = (int)(cell % D.L[0]);
    const int j = (int)((cell / D.L[0]) % D.L[1]);
    const int k = (int)(cell / ((int64_t)D.L[0] * D.L[1]));
    const int64_t s = store_index(D, P.bounds, P.c2s, i, j, k, t);
    P.disp[D.disp_off + s] = make_int4(disp_c[3 * n], disp_c[3 * n + 1], disp_c[3 * n + 2], 0);
}

int launch_scatter_disp(const DevPtrs& P, int lat, int64_t n_sites, const int32_t* d_disp_canon,
                        void* stream)
{
    const int64_t blocks = (n_sites + 255) / 256;
    hipLaunchKernelGGL(k_scatter_disp, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, P,
                       lat, d_disp_canon);
    return (int)hipGetLastError();
}

int launch_scatter(const DevPtrs& P, int lat, int64_t n_sites, const int8_t* d_occ_canon,
                   void* stream)
{
    const int64_t blocks = (n_sites + 255) / 256;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, P, lat,
                       d_occ_canon);
    return (int)hipGetLastError();
}

int phase_lds_per_wave(int max_footprint_bytes)
{
    // footprint segments each padded to 16 bytes, plus alignment slack
    return scratch_bytes() + ((max_footprint_bytes + 4 * 32 + 15) & ~15);
}

}  // namespace fkmc
