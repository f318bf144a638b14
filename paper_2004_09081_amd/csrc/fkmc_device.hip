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
                                         uint32_t k0, uint32_t k1, uint32_t out[4])
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
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
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
// Per-wave LDS layout of the fragment phase kernel.
struct WaveLds {
    int* cnt;            // vacancy count
    double* k12;         // rate table copy
    uint16_t* raw_pos;   // unsorted slots: LDS byte position
    uint32_t* raw_xyz;   //   local doubled coordinates
    uint64_t* raw_key;   //   canonical site index
    uint16_t* pos;       // sorted slots
    uint32_t* xyz;
    unsigned char* occ;  // footprint bytes
};

__device__ __forceinline__ WaveLds wave_lds(unsigned char* base)
{
    WaveLds w;
    w.cnt = (int*)base;
    w.k12 = (double*)(base + 16);
    w.raw_key = (uint64_t*)(base + 112);
    w.raw_xyz = (uint32_t*)(base + 112 + 8 * kMaxSlots);
    w.xyz = (uint32_t*)(base + 112 + 12 * kMaxSlots);
    w.raw_pos = (uint16_t*)(base + 112 + 16 * kMaxSlots);
    w.pos = (uint16_t*)(base + 112 + 18 * kMaxSlots);
    w.occ = base + ((112 + 20 * kMaxSlots + 15) & ~15);
    return w;
}

__host__ __device__ constexpr int slot_area_bytes() { return (112 + 20 * kMaxSlots + 15) & ~15; }

// Footprint: segment 0 = brick, 1 = +x face (type 0, x = wx), 2 = +y face
// (type 1, y = wy), 3 = +z face (type 2, z = wz).
struct Footprint {
    int wx, wy, wz;
    int ox, oy, oz;        // global cell of local (0,0,0)
    int64_t g[4];          // absolute byte offset of local index 0 (occ buffer)
    int len[4];
    int lds[4];            // LDS offset of local index 0
};

// Local cell + type -> (segment, local index).
__device__ __forceinline__ int fp_local(const Footprint& F, int lx, int ly, int lz, int t, int& li)
{
    if (t == 0 && lx == F.wx) { li = lz * F.wy + ly; return 1; }
    if (t == 1 && ly == F.wy) { li = lz * F.wx + lx; return 2; }
    if (t == 2 && lz == F.wz) { li = ly * F.wx + lx; return 3; }
    li = brick_local(t, lx, ly, lz, F.wx, F.wy, F.wz);
    return 0;
}

__device__ __forceinline__ int sel4(const int* a, int k)
{
    return k == 0 ? a[0] : (k == 1 ? a[1] : (k == 2 ? a[2] : a[3]));
}
__device__ __forceinline__ int64_t sel4(const int64_t* a, int k)
{
    return k == 0 ? a[0] : (k == 1 ? a[1] : (k == 2 ? a[2] : a[3]));
}

__device__ __forceinline__ uint32_t pack_xyz(int X, int Y, int Z)
{
    return (uint32_t)X | ((uint32_t)Y << 10) | ((uint32_t)Z << 20);
}

// Copy one segment HBM -> LDS in aligned 16-byte chunks and record its
// vacancies (unsorted).
__device__ __forceinline__ void load_segment(const Footprint& F, int k, const int8_t* occ_all,
                                             const WaveLds& W, const LatDesc& D, int lane)
{
    const int64_t g = F.g[k];
    const int al = (int)(g & 15);
    const int len = F.len[k];
    const int nch = (al + len + 15) >> 4;
    const uint4* src = (const uint4*)(occ_all + (g - al));
    uint4* dst = (uint4*)(W.occ + F.lds[k] - al);
    for (int j = lane; j < nch; j += 64) {
        const uint4 v = src[j];
        dst[j] = v;
        const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const uint32_t x = w4[q] ^ 0x02020202u;
            if (((x - 0x01010101u) & ~x & 0x80808080u) == 0) continue;
#pragma unroll
            for (int bb = 0; bb < 4; bb++) {
                if (((w4[q] >> (8 * bb)) & 0xff) != kSpV) continue;
                const int li = 16 * j + 4 * q + bb - al;
                if (li < 0 || li >= len) continue;
                int lx, ly, lz, t;
                if (k == 0) {
                    const int V = F.wx * F.wy * F.wz;
                    t = li / V;
                    const int r = li - t * V;
                    if (t == 0) { ly = r % F.wy; lz = (r / F.wy) % F.wz; lx = r / (F.wy * F.wz); }
                    else if (t == 1) { lx = r % F.wx; lz = (r / F.wx) % F.wz; ly = r / (F.wx * F.wz); }
                    else { lx = r % F.wx; ly = (r / F.wx) % F.wy; lz = r / (F.wx * F.wy); }
                } else if (k == 1) {
                    t = 0; lx = F.wx; ly = li % F.wy; lz = li / F.wy;
                } else if (k == 2) {
                    t = 1; ly = F.wy; lx = li % F.wx; lz = li / F.wx;
                } else {
                    t = 2; lz = F.wz; lx = li % F.wx; ly = li / F.wx;
                }
                const int X = 2 * lx + (t != 0), Y = 2 * ly + (t != 1), Z = 2 * lz + (t != 2);
                int gi = F.ox + lx, gj = F.oy + ly, gk = F.oz + lz;
                if (gi >= D.L[0]) gi -= D.L[0];
                if (gj >= D.L[1]) gj -= D.L[1];
                if (gk >= D.L[2]) gk -= D.L[2];
                const uint64_t key = ((((uint64_t)gk * D.L[1] + gj) * D.L[0] + gi) * 3) + t;
                const int slot = atomicAdd(W.cnt, 1);
                if (slot < kMaxSlots) {
                    W.raw_pos[slot] = (uint16_t)(F.lds[k] + li);
                    W.raw_xyz[slot] = pack_xyz(X, Y, Z);
                    W.raw_key[slot] = key;
                }
            }
        }
    }
}

// Rate of event d of the vacancy at local doubled coordinates xyz (0 when
// the edge is not owned by this tile or the target is a vacancy).  Also
// returns the target's local doubled coordinates and LDS position.
__device__ __forceinline__ double tile_rate(const Footprint& F, const WaveLds& W, const LatDesc& D,
                                            uint32_t xyz, int d, int& tX, int& tY, int& tZ,
                                            int& tpos)
{
    const int X = xyz & 1023, Y = (xyz >> 10) & 1023, Z = xyz >> 20;
    const int t = site_type(X, Y);
    int hx, hy, hz;
    hop_vec(t, d, hx, hy, hz);
    const int ox = (2 * X + hx) >> 2, oy = (2 * Y + hy) >> 2, oz = (2 * Z + hz) >> 2;
    if (ox < 0 || ox >= F.wx || oy < 0 || oy >= F.wy || oz < 0 || oz >= F.wz) return 0.0;
    tX = X + hx;
    tY = Y + hy;
    tZ = Z + hz;
    const int tt = site_type(tX, tY);
    int li;
    const int seg = fp_local(F, tX >> 1, tY >> 1, tZ >> 1, tt, li);
    tpos = sel4(F.lds, seg) + li;
    const int sp = W.occ[tpos];
    if (sp == kSpV) return 0.0;
    // grain-boundary flag of either end: type-a sites on planes normal to a
    const int cs = t == 0 ? (F.ox + (X >> 1)) : (t == 1 ? (F.oy + (Y >> 1)) : (F.oz + (Z >> 1)));
    const int ct = tt == 0 ? (F.ox + (tX >> 1)) : (tt == 1 ? (F.oy + (tY >> 1)) : (F.oz + (tZ >> 1)));
    const int Lt = D.L[t], Ltt = D.L[tt];
    const int g = is_gb(D, t, cs >= Lt ? cs - Lt : cs) | is_gb(D, tt, ct >= Ltt ? ct - Ltt : ct);
    return W.k12[(sp * 3 + hz + 1) * 2 + g];
}

template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_phase(DevPtrs P, int colour, int lds_per_wave)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int tile = blockIdx.x * WAVES + wv;
    if (tile >= P.n_tiles) return;
    const int lat = P.tile2lat[tile];
    const LatDesc& D = P.desc[lat];
    LatState* S = P.state + lat;
    if (S->done) return;
    const uint64_t cycle = S->cycles;
    const double t_sync = P.call[lat].t_sync;
    const WaveLds W = wave_lds(smem + wv * lds_per_wave);

    // tile -> fragment -> sub-block of this colour
    const int f = tile - D.tile0;
    const int nfx = D.nsb[0] >> 1, nfy = D.nsb[1] >> 1;
    const int fx = f % nfx, fy = (f / nfx) % nfy, fz = f / (nfx * nfy);
    const int bi = 2 * fx + (colour & 1), bj = 2 * fy + ((colour >> 1) & 1),
              bk = 2 * fz + ((colour >> 2) & 1);
    const Brick B = brick_of(D, P.bounds, bi, bj, bk);
    const int bin = bi + 1 == D.nsb[0] ? 0 : bi + 1;
    const int bjn = bj + 1 == D.nsb[1] ? 0 : bj + 1;
    const int bkn = bk + 1 == D.nsb[2] ? 0 : bk + 1;
    const Brick BX = brick_of(D, P.bounds, bin, bj, bk);
    const Brick BY = brick_of(D, P.bounds, bi, bjn, bk);
    const Brick BZ = brick_of(D, P.bounds, bi, bj, bkn);

    Footprint F;
    F.wx = B.wx; F.wy = B.wy; F.wz = B.wz;
    F.ox = B.x0; F.oy = B.y0; F.oz = B.z0;
    F.g[0] = D.occ_off + B.base;                                  F.len[0] = 3 * B.wx * B.wy * B.wz;
    F.g[1] = D.occ_off + BX.base;                                 F.len[1] = B.wy * B.wz;
    F.g[2] = D.occ_off + BY.base + (int64_t)BY.wx * BY.wy * BY.wz; F.len[2] = B.wz * B.wx;
    F.g[3] = D.occ_off + BZ.base + 2 * (int64_t)BZ.wx * BZ.wy * BZ.wz; F.len[3] = B.wy * B.wx;
    {
        int off = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int al = (int)(F.g[k] & 15);
            F.lds[k] = off + al;
            off += (al + F.len[k] + 15) & ~15;
        }
    }
    if (lane == 0) *W.cnt = 0;
    if (lane < 12) W.k12[lane] = D.k12[lane];
    wave_lds_fence();
#pragma unroll
    for (int k = 0; k < 4; k++) load_segment(F, k, P.occ, W, D, lane);
    wave_lds_fence();
    const int n = *W.cnt;
    if (n == 0) return;
    if (n > kMaxSlots) {
        if (lane == 0) atomicOr(&S->err, 1u);
        return;
    }
    // order the slots by canonical site index (keys are distinct)
    for (int l = lane; l < n; l += 64) {
        const uint64_t key = W.raw_key[l];
        int rank = 0;
        for (int j = 0; j < n; j++) rank += W.raw_key[j] < key;
        W.pos[rank] = W.raw_pos[l];
        W.xyz[rank] = W.raw_xyz[l];
    }
    wave_lds_fence();

    const int m = (n + 63) >> 6;
    const int s0 = lane * m < n ? lane * m : n;
    const int s1 = s0 + m < n ? s0 + m : n;
    const int64_t lat_disp = D.disp_off - D.occ_off;  // occ byte offset -> disp element
    double tau = 0.0;
    uint32_t step = 0;
    uint32_t hops_o = 0, hops_h = 0;
    for (;;) {
        double ls = 0.0;
        for (int s = s0; s < s1; s++) {
            const uint32_t xyz = W.xyz[s];
#pragma unroll
            for (int d = 0; d < 8; d++) {
                int a, b, c, p;
                ls += tile_rate(F, W, D, xyz, d, a, b, c, p);
            }
        }
        const double incl = wave_incl_scan(ls, lane);
        const double R = __shfl(incl, 63, 64);
        if (R == 0.0) break;
        uint32_t x[4];
        philox10(step, (uint32_t)f, (uint32_t)cycle, ((uint32_t)colour << 8) | 2u, D.seed,
                 D.lattice_id, x);
        const double u_sel = u53_lo(x[0], x[1]);
        const double u_t = u53_hi(x[2], x[3]);
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
            const uint64_t nz = __ballot(ls > 0.0);
            sel = 63 - __clzll((long long)nz);
            fallback = true;
        }
        int ev = -1;
        if (lane == sel) {
            double C = incl - ls;
            int last = -1;
            for (int s = s0; s < s1 && ev < 0; s++) {
                const uint32_t xyz = W.xyz[s];
                for (int d = 0; d < 8; d++) {
                    int a, b, c, p;
                    const double k = tile_rate(F, W, D, xyz, d, a, b, c, p);
                    if (k > 0.0) last = s * 8 + d;
                    C += k;
                    if (!fallback && C > y) { ev = s * 8 + d; break; }
                }
            }
            if (ev < 0) ev = last;
            // apply: swap vacancy and ion, move displacement entries
            const int s = ev >> 3, d = ev & 7;
            const uint32_t xyz = W.xyz[s];
            int tX, tY, tZ, tpos;
            tile_rate(F, W, D, xyz, d, tX, tY, tZ, tpos);
            const int X = xyz & 1023, Y = (xyz >> 10) & 1023, Z = xyz >> 20;
            const int t = site_type(X, Y);
            int hx, hy, hz;
            hop_vec(t, d, hx, hy, hz);
            int li_s, li_t;
            const int seg_s = fp_local(F, X >> 1, Y >> 1, Z >> 1, t, li_s);
            const int seg_t = fp_local(F, tX >> 1, tY >> 1, tZ >> 1, site_type(tX, tY), li_t);
            const int spos = sel4(F.lds, seg_s) + li_s;
            const int sp = W.occ[tpos];
            W.occ[spos] = (unsigned char)sp;
            W.occ[tpos] = (unsigned char)kSpV;
            W.pos[s] = (uint16_t)tpos;
            W.xyz[s] = pack_xyz(tX, tY, tZ);
            const int64_t gs = sel4(F.g, seg_s) + li_s;
            const int64_t gt = sel4(F.g, seg_t) + li_t;
            P.occ[gs] = (int8_t)sp;
            P.occ[gt] = (int8_t)kSpV;
            int4* ds = P.disp + (gs + lat_disp);
            int4* dtp = P.disp + (gt + lat_disp);
            const int4 dv = *ds;
            const int4 di = *dtp;
            *dtp = make_int4(dv.x + hx, dv.y + hy, dv.z + hz, 0);
            *ds = make_int4(di.x - hx, di.y - hy, di.z - hz, 0);
            ev = (ev & 0xffff) | (sp << 16);
        }
        ev = __shfl(ev, sel, 64);
        if ((ev >> 16) == kSpO) hops_o++;
        else hops_h++;
        wave_lds_fence();
        step++;
    }
    if (lane == 0 && (hops_o | hops_h)) {
        unsigned long long* b = P.buckets + ((size_t)lat * kHopBuckets + (f & (kHopBuckets - 1))) * 2;
        if (hops_o) atomicAdd(b, (unsigned long long)hops_o);
        if (hops_h) atomicAdd(b + 1, (unsigned long long)hops_h);
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
        uint32_t x[4];
        philox10((uint32_t)draws, (uint32_t)(draws >> 32), 0xFFFFFFFFu, 3u, D.seed, D.lattice_id, x);
        draws++;
        const double u_sel = u53_lo(x[0], x[1]);
        const double u_t = u53_hi(x[2], x[3]);
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
            uint32_t x[4];
            philox10((uint32_t)d, (uint32_t)(d >> 32), 0u, 1u, D.seed, D.lattice_id, x);
            d++;
            const uint64_t w = ((uint64_t)x[0] << 32) | x[1];
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
                           (hipStream_t)stream, P, colour, lds_per_wave);
    } else {
        hipLaunchKernelGGL(k_phase<1>, dim3(P.n_tiles), dim3(64), (size_t)lds_per_wave,
                           (hipStream_t)stream, P, colour, lds_per_wave);
    }
    return (int)hipGetLastError();
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
    return slot_area_bytes() + ((max_footprint_bytes + 4 * 32 + 15) & ~15);
}

}  // namespace fkmc
