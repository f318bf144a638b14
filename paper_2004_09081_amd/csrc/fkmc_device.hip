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
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
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

// Order this wave's LDS accesses across lanes without waiting for them: the
// LDS serves one wave's instructions in issue order, so a later read by any
// lane sees an earlier write by any other; the wavefront-scope fences only
// keep the compiler from moving accesses across this point.
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

// Index of local cell (lx,ly,lz), type t, in a brick of wx*wy*wz cells:
//   type 0: (x wz + z) wy + y;  type 1: V + (y wz + z) wx + x;
//   type 2: 2V + (z wy + y) wx + x   (V = wx wy wz).
// Written with selects only (no branches): plane t has the type's own axis
// slowest, then z (y for type 2), then y (type 0) or x.
__device__ __forceinline__ int brick_local(int t, int lx, int ly, int lz, int wx, int wy, int wz)
{
    const int a = t == 0 ? lx : (t == 1 ? ly : lz);
    const int b = t == 2 ? ly : lz;
    const int c = t == 0 ? ly : lx;
    const int mid = t == 2 ? wy : wz;
    const int fast = t == 0 ? wy : wx;
    return t * (wx * wy * wz) + (a * mid + b) * fast + c;
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

// Bit n of a boundary-site map (canonical site index).
__device__ __forceinline__ int gb_bit(const uint32_t* m, int64_t n)
{
    return (int)((m[n >> 5] >> (n & 31)) & 1u);
}

__device__ __forceinline__ int64_t canon_site(int L0, int L1, int i, int j, int k, int t)
{
    return (((int64_t)k * L1 + j) * L0 + i) * 3 + t;
}

// Boundary flag of the edge between site (i,j,k,t) and site (i2,j2,k2,t2):
// from the lattice's site map when it has one, else from its planes (cs, ct:
// the two sites' cell indices along their own type's axis).
__device__ __forceinline__ int edge_gb(const LatDesc& D, int i, int j, int k, int t, int i2, int j2, int k2,
                                       int t2, int cs, int ct)
{
    if (D.gb_map)
        return gb_bit(D.gb_map, canon_site(D.L[0], D.L[1], i, j, k, t)) |
               gb_bit(D.gb_map, canon_site(D.L[0], D.L[1], i2, j2, k2, t2));
    return is_gb(D, t, cs) | is_gb(D, t2, ct);
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

// Inclusive wavefront prefix maximum of non-negative binary64 values (the
// same DPP moves as the prefix sum; lanes moved in from outside read 0).
__device__ __forceinline__ double wave_max_dpp(double v)
{
    v = fmax(v, dpp_shifted<0x111, 0xF>(v));
    v = fmax(v, dpp_shifted<0x112, 0xF>(v));
    v = fmax(v, dpp_shifted<0x114, 0xF>(v));
    v = fmax(v, dpp_shifted<0x118, 0xF>(v));
    v = fmax(v, dpp_shifted<0x142, 0xA>(v));
    v = fmax(v, dpp_shifted<0x143, 0xC>(v));
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
    uint64_t ldsp;   // lds0..lds3 as 16-bit fields (LDS positions stay below 2^16)
};

// One of three or four values by a runtime index.  The operands are
// values (not struct lvalues), so the selection stays a register select
// and never becomes an indexed load from a private copy of the struct.
__device__ __forceinline__ int pick3(int k, int a, int b, int c)
{
    return k == 0 ? a : (k == 1 ? b : c);
}
__device__ __forceinline__ int pick4(int k, int a, int b, int c, int d)
{
    return k == 0 ? a : (k == 1 ? b : (k == 2 ? c : d));
}
__device__ __forceinline__ int64_t pick4(int k, int64_t a, int64_t b, int64_t c, int64_t d)
{
    return k == 0 ? a : (k == 1 ? b : (k == 2 ? c : d));
}

// Segment accessors (selects, never a runtime-indexed local array).
__device__ __forceinline__ int64_t seg_st(const TileGeo& G, int k)
{
    return pick4(k, G.st0, G.st1, G.st2, G.st3);
}
__device__ __forceinline__ int seg_lds(const TileGeo& G, int k)
{
    return (int)((G.ldsp >> (16 * k)) & 0xffffu);  // one shift, no select chain
}

__device__ __forceinline__ void pack_lds(TileGeo& G)
{
    G.ldsp = (uint64_t)(uint32_t)G.lds0 | ((uint64_t)(uint32_t)G.lds1 << 16) |
             ((uint64_t)(uint32_t)G.lds2 << 32) | ((uint64_t)(uint32_t)G.lds3 << 48);
}
// Sites of footprint segment k: the brick, then the three faces.
__device__ __forceinline__ int seg_len(const TileGeo& G, int k)
{
    return pick4(k, 3 * G.wx * G.wy * G.wz, G.wy * G.wz, G.wz * G.wx, G.wy * G.wx);
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
    G.lds0 = G.lds1 = G.lds2 = G.lds3 = 0;
    G.ldsp = 0;
    return G;
}

// Footprint segment and local index of local cell (lx,ly,lz), type t: the
// brick (0), or the +face of the type's own axis (1 + t) when that
// coordinate equals the sub-block width.  A face is ordered like one plane
// of the brick without its slowest axis, so both indices share the
// in-plane part.  Selects only, no branches.
__device__ __forceinline__ int fp_local(const TileGeo& G, int lx, int ly, int lz, int t, int& li)
{
    const int wx = G.wx, wy = G.wy, wz = G.wz;  // values: the selects below stay in registers
    const int a = pick3(t, lx, ly, lz);
    const int wa = pick3(t, wx, wy, wz);
    const int b = t == 2 ? ly : lz;
    const int c = t == 0 ? ly : lx;
    const int mid = t == 2 ? wy : wz;
    const int fast = t == 0 ? wy : wx;
    const int inplane = b * fast + c;
    const bool face = a == wa;
    li = face ? inplane : t * (wx * wy * wz) + a * mid * fast + inplane;
    return face ? t + 1 : 0;
}


__device__ __forceinline__ uint32_t pack_xyz(int X, int Y, int Z)
{
    return (uint32_t)X | ((uint32_t)Y << 10) | ((uint32_t)Z << 20);
}

// LDS position of the site at packed local doubled coords; its footprint
// segment and local index in k, li.
__device__ __forceinline__ int xyz_lds(const TileGeo& G, uint32_t xyz, int& k, int& li)
{
    const int X = xyz & 1023, Y = (xyz >> 10) & 1023, Z = xyz >> 20;
    k = fp_local(G, X >> 1, Y >> 1, Z >> 1, site_type(X, Y), li);
    return seg_lds(G, k) + li;
}

// ----------------------------------------------------------------------------
// ----------------------------------------------------------------------------
// Small quotient a / b for 0 <= a < 2^22, 1 <= b < 2^22: the float product
// with a one-ulp reciprocal lands within one of the true quotient, and one
// remainder test each way corrects it.
__device__ __forceinline__ int udiv22(int a, int b)
{
    int q = (int)((float)a * __builtin_amdgcn_rcpf((float)b));
    const int r = a - q * b;
    q += r >= b ? 1 : 0;
    q -= r < 0 ? 1 : 0;
    return q;
}

// What a tile needs of its lattice's rates: sizes for the boundary-plane
// test and the quantised table (an LDS copy).
struct RateCtx {
    int L0, L1, L2;
    int gbp, gbm;
    const double* k12;
    const uint32_t* gbmap;  // boundary-site map (replaces the planes), or nullptr
};

__device__ __forceinline__ int gb_flag(const RateCtx& C, int t, int cell)
{
    if (C.gbp <= 0 || !((C.gbm >> t) & 1)) return 0;
    return cell - udiv22(cell, C.gbp) * C.gbp == 0 ? 1 : 0;
}

// Rate of event d of the vacancy at packed local doubled coordinates xyz:
// 0 when the hop edge's midpoint is outside the sub-block or the target
// holds a vacancy; else the table entry for (ion species, z step, boundary).
// MAP: the lattice may have a boundary-site map (C.gbmap); without it the
// map branch is compiled out (the lockstep kernel keeps 128 VGPRs).
template <bool MAP = true>
__device__ __forceinline__ double tile_rate(const TileGeo& G, const unsigned char* occl,
                                            const RateCtx& C, uint32_t xyz, int d)
{
    const int X = xyz & 1023, Y = (xyz >> 10) & 1023, Z = xyz >> 20;
    const int t = site_type(X, Y);
    int hx, hy, hz;
    hop_vec(t, d, hx, hy, hz);
    const int ox = (2 * X + hx) >> 2, oy = (2 * Y + hy) >> 2, oz = (2 * Z + hz) >> 2;
    const bool in = ox >= 0 && ox < G.wx && oy >= 0 && oy < G.wy && oz >= 0 && oz < G.wz;
    const int tX = X + hx, tY = Y + hy, tZ = Z + hz;
    const int tt = site_type(tX, tY);
    int li;
    const int seg = fp_local(G, tX >> 1, tY >> 1, tZ >> 1, tt, li);
    // (an active edge's target is in the footprint; an inactive edge reads
    // the first brick byte instead, so every address stays in bounds)
    const int lds0 = G.lds0;
    const int sp = occl[in ? seg_lds(G, seg) + li : lds0];
    int g = 0;
    if (MAP && C.gbmap) {
        int si = G.ox + (X >> 1), sj = G.oy + (Y >> 1), sk = G.oz + (Z >> 1);
        int ti = G.ox + (tX >> 1), tj = G.oy + (tY >> 1), tk = G.oz + (tZ >> 1);
        si -= si >= C.L0 ? C.L0 : 0;
        sj -= sj >= C.L1 ? C.L1 : 0;
        sk -= sk >= C.L2 ? C.L2 : 0;
        ti -= ti >= C.L0 ? C.L0 : 0;
        tj -= tj >= C.L1 ? C.L1 : 0;
        tk -= tk >= C.L2 ? C.L2 : 0;
        // (an inactive edge may point outside the footprint: clamp its
        // indices into the lattice; its rate is 0 either way)
        ti = ti < 0 ? 0 : ti;
        tj = tj < 0 ? 0 : tj;
        tk = tk < 0 ? 0 : tk;
        g = gb_bit(C.gbmap, canon_site(C.L0, C.L1, si, sj, sk, t)) |
            gb_bit(C.gbmap, canon_site(C.L0, C.L1, ti, tj, tk, tt));
    } else if (C.gbp > 0) {
        int cs = pick3(t, G.ox + (X >> 1), G.oy + (Y >> 1), G.oz + (Z >> 1));
        int ct = pick3(tt, G.ox + (tX >> 1), G.oy + (tY >> 1), G.oz + (tZ >> 1));
        const int Ls = pick3(t, C.L0, C.L1, C.L2);
        const int Lt = pick3(tt, C.L0, C.L1, C.L2);
        if (cs >= Ls) cs -= Ls;
        if (ct >= Lt) ct -= Lt;
        g = gb_flag(C, t, cs) | gb_flag(C, tt, ct);
    }
    const int col = (hz + 1) * 2 + g;
    const double kO = C.k12[col], kH = C.k12[6 + col];
    return (!in || sp == kSpV) ? 0.0 : (sp == kSpO ? kO : kH);
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

// ----------------------------------------------------------------------------
// Displacement records.  A particle that hops gets a record in one lane of
// the wave: the displacement index of its current site, the index of the
// site it occupied when the record opened, and the hops since.  Records are
// keyed by displacement index, so they stay valid across tiles and phases
// for as long as one wave alone moves the lattice's particles.  Between two
// flushes only this wave writes the entries of the sites its records touch,
// and a record opens only for a particle on a site no hop has touched since
// the last flush, so every origin still holds its particle's displacement in
// HBM: a flush reads all origins (one round trip for all records, no load in
// flight between flushes), waits, then writes each particle's displacement
// to its current site.
struct Rec {
    int64_t cur;   // < 0: free
    int64_t orig;
    int ax, ay, az;
};

struct RecCtl {
    int n;         // records in use (wave-uniform)
    bool pending;  // stores of the last flush may still be in flight
};

__device__ __forceinline__ void rec_init(Rec& r, RecCtl& c)
{
    r.cur = -1;
    r.orig = 0;
    r.ax = r.ay = r.az = 0;
    c.n = 0;
    c.pending = false;
}

__device__ __forceinline__ void rec_flush(Rec& r, RecCtl& c, int4* disp)
{
    if (c.n == 0) return;
    if (c.pending) {
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the last flush's stores have landed
        __builtin_amdgcn_wave_barrier();
    }
    int4 o = make_int4(0, 0, 0, 0);
    if (r.cur >= 0) o = disp[r.orig];
    __builtin_amdgcn_s_waitcnt(0x0F70);  // every read has returned before any write
    __builtin_amdgcn_wave_barrier();
    if (r.cur >= 0) disp[r.cur] = make_int4(o.x + r.ax, o.y + r.ay, o.z + r.az, 0);
    r.cur = -1;
    r.ax = r.ay = r.az = 0;
    c.n = 0;
    c.pending = true;
}

// The vacancy at displacement index ks swaps with the ion at kt, the vacancy
// moving by h.  ks, kt and h are wave-uniform.
__device__ __forceinline__ void rec_hop(Rec& r, RecCtl& c, int4* disp, int lane, int64_t ks,
                                        int64_t kt, int hx, int hy, int hz)
{
    uint64_t mv = __ballot(r.cur == ks);
    uint64_t mi = __ballot(r.cur == kt);
    if (c.n + (mv == 0) + (mi == 0) > 64) {
        rec_flush(r, c, disp);
        mv = 0;
        mi = 0;
    }
    int lv, li;
    if (mv) {
        lv = __ffsll((unsigned long long)mv) - 1;
    } else {
        lv = c.n++;
        if (lane == lv) r.orig = ks;
    }
    if (mi) {
        li = __ffsll((unsigned long long)mi) - 1;
    } else {
        li = c.n++;
        if (lane == li) r.orig = kt;
    }
    const int sv = lane == lv ? 1 : (lane == li ? -1 : 0);
    r.cur = lane == lv ? kt : (lane == li ? ks : r.cur);
    r.ax += sv * hx;
    r.ay += sv * hy;
    r.az += sv * hz;
}

// ----------------------------------------------------------------------------
// Per-wave LDS scratch: slot counters (8 group tiles + 1 single tile), the
// group's tile records, the rate table, and slot lists of 128 entries
// (unsorted canonical key, packed coordinates, vacancy-list index; sorted
// coordinates and list index).  In group mode tile k owns entries
// [k*cap, k*cap + cap).
struct WaveLds {
    int* cnt;
    TileRec* rec;
    double* k12;
    uint64_t* raw_key;
    uint32_t* raw_xyz;
    uint32_t* xyz;
    uint16_t* raw_idx;
    uint16_t* idx;
};

// Byte offsets of the parts of a wave's scratch.
constexpr int kLdsRec = 64;                            // TileRec[8]
constexpr int kLdsK12 = kLdsRec + 8 * (int)sizeof(TileRec);
constexpr int kLdsRawKey = kLdsK12 + 96;               // uint64[128]
constexpr int kLdsRawXyz = kLdsRawKey + 1024;          // uint32[128]
constexpr int kLdsXyz = kLdsRawXyz + 512;              // uint32[128]
constexpr int kLdsRawIdx = kLdsXyz + 512;              // uint16[128]
constexpr int kLdsIdx = kLdsRawIdx + 256;              // uint16[128]
constexpr int kLdsEnd = kLdsIdx + 256;
static_assert(sizeof(TileRec) == 48, "tile record layout");
static_assert(kLdsK12 % 8 == 0 && kLdsRawKey % 8 == 0, "scratch alignment");
static_assert(kLdsEnd <= kWaveScratch && kWaveScratch % 16 == 0, "wave scratch size");
static_assert(kLdsRawIdx == kWaveScratchStaged && kLdsIdx > kLdsRawIdx,
              "the staged-tile scratch ends where the index arrays begin");

__device__ __forceinline__ WaveLds wave_lds(unsigned char* b)
{
    WaveLds w;
    w.cnt = (int*)b;
    w.rec = (TileRec*)(b + kLdsRec);
    w.k12 = (double*)(b + kLdsK12);
    w.raw_key = (uint64_t*)(b + kLdsRawKey);
    w.raw_xyz = (uint32_t*)(b + kLdsRawXyz);
    w.xyz = (uint32_t*)(b + kLdsXyz);
    w.raw_idx = (uint16_t*)(b + kLdsRawIdx);
    w.idx = (uint16_t*)(b + kLdsIdx);
    return w;
}

// LDS positions of a staged footprint: the four segments as consecutive
// 16-byte-aligned runs from `base`, each keeping its HBM alignment.
__device__ __forceinline__ void tile_lds_at(TileGeo& G, int base)
{
    int off = base;
    G.lds0 = off + (int)(G.st0 & 15);
    off += ((int)(G.st0 & 15) + seg_len(G, 0) + 15) & ~15;
    G.lds1 = off + (int)(G.st1 & 15);
    off += ((int)(G.st1 & 15) + seg_len(G, 1) + 15) & ~15;
    G.lds2 = off + (int)(G.st2 & 15);
    off += ((int)(G.st2 & 15) + seg_len(G, 2) + 15) & ~15;
    G.lds3 = off + (int)(G.st3 & 15);
    pack_lds(G);
}

// LDS positions when the whole lattice sits in LDS at its storage offsets.
__device__ __forceinline__ void tile_lds_resident(TileGeo& G)
{
    G.lds0 = (int)G.st0;
    G.lds1 = (int)G.st1;
    G.lds2 = (int)G.st2;
    G.lds3 = (int)G.st3;
    pack_lds(G);
}

// 16-byte chunk counts of the four staged segments.
__device__ __forceinline__ void seg_chunks(const TileGeo& G, int& n0, int& n1, int& n2, int& n3)
{
    n0 = ((int)(G.st0 & 15) + seg_len(G, 0) + 15) >> 4;
    n1 = ((int)(G.st1 & 15) + seg_len(G, 1) + 15) >> 4;
    n2 = ((int)(G.st2 & 15) + seg_len(G, 2) + 15) >> 4;
    n3 = ((int)(G.st3 & 15) + seg_len(G, 3) + 15) >> 4;
}

// Chunk c of the concatenated segments: segment k and chunk index within it.
__device__ __forceinline__ int locate_chunk(int c, int n0, int n1, int n2, int& cj)
{
    if (c < n0) { cj = c; return 0; }
    c -= n0;
    if (c < n1) { cj = c; return 1; }
    c -= n1;
    if (c < n2) { cj = c; return 2; }
    cj = c - n2;
    return 3;
}

// Local cell and type of local index li of footprint segment k.
__device__ __forceinline__ void seg_site(const TileGeo& G, int k, int li, int& lx, int& ly, int& lz,
                                         int& t)
{
    if (k == 0) {
        const int V = G.wx * G.wy * G.wz;
        t = li >= 2 * V ? 2 : (li >= V ? 1 : 0);
        const int r = li - t * V;
        const int inner = pick3(t, G.wy, G.wx, G.wx);  // fastest axis of the plane
        const int mid = pick3(t, G.wz, G.wz, G.wy);
        const int q1 = udiv22(r, inner);
        const int u = r - q1 * inner;
        const int w = udiv22(q1, mid);
        const int v = q1 - w * mid;
        if (t == 0) { ly = u; lz = v; lx = w; }       // (x wz + z) wy + y
        else if (t == 1) { lx = u; lz = v; ly = w; }  // (y wz + z) wx + x
        else { lx = u; ly = v; lz = w; }              // (z wy + y) wx + x
    } else if (k == 1) {
        t = 0; lx = G.wx; lz = udiv22(li, G.wy); ly = li - lz * G.wy;
    } else if (k == 2) {
        t = 1; ly = G.wy; lz = udiv22(li, G.wx); lx = li - lz * G.wx;
    } else {
        t = 2; lz = G.wz; ly = udiv22(li, G.wx); lx = li - ly * G.wx;
    }
}

// Append a vacancy at local cell (lx,ly,lz), type t of tile G to slot list
// `list` (entries [list*cap, list*cap + cap), counter cnt[ci]); vidx is its
// vacancy-list index, or < 0 for a staged tile (no index kept).
__device__ __forceinline__ void put_slot(const WaveLds& W, const TileGeo& G, int L0, int L1, int L2,
                                         int ci, int first, int cap, int lx, int ly, int lz, int t,
                                         int vidx)
{
    int gi = G.ox + lx, gj = G.oy + ly, gk = G.oz + lz;
    if (gi >= L0) gi -= L0;
    if (gj >= L1) gj -= L1;
    if (gk >= L2) gk -= L2;
    const uint64_t key = ((((uint64_t)gk * L1 + gj) * L0 + gi) * 3) + t;
    const int s = atomicAdd(&W.cnt[ci], 1);
    if (s < cap) {
        W.raw_key[first + s] = key;
        W.raw_xyz[first + s] = pack_xyz(2 * lx + (t != 0), 2 * ly + (t != 1), 2 * lz + (t != 2));
        if (vidx >= 0) W.raw_idx[first + s] = (uint16_t)vidx;
    }
}

// Vacancies of the footprint of tile G staged in LDS (positions G.lds*):
// every lane reads 16-byte chunks, and the rare chunk holding a vacancy
// byte (the only code with bit 1 set) is examined byte by byte.
__device__ __forceinline__ void scan_staged(const WaveLds& W, const TileGeo& G, const unsigned char* occl,
                                            int L0, int L1, int L2, int ci, int first, int cap,
                                            int lane)
{
    int n0, n1, n2, n3;
    seg_chunks(G, n0, n1, n2, n3);
    const int total = n0 + n1 + n2 + n3;
    const int base = G.lds0 - (int)(G.st0 & 15);
    for (int c = lane; c < total; c += 64) {
        const uint4 v = *(const uint4*)(occl + base + 16 * c);
        if (((v.x | v.y | v.z | v.w) & 0x02020202u) == 0) continue;
        int cj;
        const int k = locate_chunk(c, n0, n1, n2, cj);
        const int al = (int)(seg_st(G, k) & 15);
        const int len = seg_len(G, k);
        // bit b of m: byte b holds a vacancy (the product gathers bit 1 of
        // the four bytes of a word into its top nibble)
        uint32_t m = (((v.x >> 1) & 0x01010101u) * 0x10204080u) >> 28;
        m |= ((((v.y >> 1) & 0x01010101u) * 0x10204080u) >> 28) << 4;
        m |= ((((v.z >> 1) & 0x01010101u) * 0x10204080u) >> 28) << 8;
        m |= ((((v.w >> 1) & 0x01010101u) * 0x10204080u) >> 28) << 12;
        while (m) {
            const int b = __ffs(m) - 1;
            m &= m - 1;
            const int li = 16 * cj + b - al;
            if (li < 0 || li >= len) continue;
            int lx, ly, lz, t;
            seg_site(G, k, li, lx, ly, lz, t);
            put_slot(W, G, L0, L1, L2, ci, first, cap, lx, ly, lz, t, -1);
        }
    }
}

// 16-bit mask of the vacancy bytes of a 16-byte chunk (the only code with
// bit 1 set): a product gathers bit 1 of the four bytes of a word into its
// top nibble.
__device__ __forceinline__ uint32_t vacancy_mask16(uint4 v)
{
    uint32_t m = (((v.x >> 1) & 0x01010101u) * 0x10204080u) >> 28;
    m |= ((((v.y >> 1) & 0x01010101u) * 0x10204080u) >> 28) << 4;
    m |= ((((v.z >> 1) & 0x01010101u) * 0x10204080u) >> 28) << 8;
    m |= ((((v.w >> 1) & 0x01010101u) * 0x10204080u) >> 28) << 12;
    return m;
}

// Slots of the entries [0, n) of a group's vacancy list (tile k, chunk c of
// its staged footprint, byte b: k << 28 | c << 4 | b), one entry per lane:
// site, canonical key, append to tile k's slot list (entries
// [k*cap, k*cap + cap), counter cnt[k]).
__device__ __forceinline__ void group_slots(const WaveLds& W, const TileRec* R, const uint32_t* ent, int n,
                                            int fp, int fps, int L0, int L1, int L2, int cap, int lane)
{
    for (int e = lane; e < n; e += 64) {
        const uint32_t x = ent[e];
        const int k = (int)(x >> 28), c = (int)((x >> 4) & 0xFFFFFFu), b = (int)(x & 15u);
        TileGeo G = tile_geo_rec(R[k]);
        tile_lds_at(G, fp + k * fps);
        int n0, n1, n2, n3, cj;
        seg_chunks(G, n0, n1, n2, n3);
        const int sg = locate_chunk(c, n0, n1, n2, cj);
        const int li = 16 * cj + b - (int)(seg_st(G, sg) & 15);
        if (li < 0 || li >= seg_len(G, sg)) continue;
        int lx, ly, lz, t;
        seg_site(G, sg, li, lx, ly, lz, t);
        put_slot(W, G, L0, L1, L2, k, k * cap, cap, lx, ly, lz, t, -1);
    }
}

// Vacancies of the nt staged footprints of a group (tile k at LDS offset
// fp + k*fps, records R): every lane tests 16-byte chunks of all the
// footprints; the vacancy bytes found go to a compact list (W.xyz, not in
// use until the slots are sorted), which the whole wave then decodes one
// entry per lane.  The result equals scan_staged on each tile.
__device__ __forceinline__ void scan_group(const WaveLds& W, const TileRec* R, const unsigned char* occl,
                                           int nt, int fp, int fps, int L0, int L1, int L2, int cap, int lane)
{
    uint32_t* ent = W.xyz;  // 128 entries
    int n = 0;              // wave-uniform
    for (int k = 0; k < nt; k++) {
        TileGeo G = tile_geo_rec(R[k]);
        tile_lds_at(G, fp + k * fps);
        int n0, n1, n2, n3;
        seg_chunks(G, n0, n1, n2, n3);
        const int total = n0 + n1 + n2 + n3;
        const int base = G.lds0 - (int)(G.st0 & 15);
        for (int c0 = 0; c0 < total; c0 += 64) {
            const int c = c0 + lane;
            uint32_t m = 0;
            if (c < total) m = vacancy_mask16(*(const uint4*)(occl + base + 16 * c));
            for (;;) {
                const bool has = m != 0;
                const uint64_t mk = __ballot(has);
                if (mk == 0) break;
                if (has) {
                    const int pos = n + (int)__builtin_amdgcn_mbcnt_hi(
                                            (uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
                    ent[pos] = ((uint32_t)k << 28) | ((uint32_t)c << 4) | (uint32_t)(__ffs(m) - 1);
                    m &= m - 1;
                }
                n += __popcll(mk);
                if (n > 64) {
                    wave_lds_fence();
                    group_slots(W, R, ent, n, fp, fps, L0, L1, L2, cap, lane);
                    wave_lds_fence();
                    n = 0;
                }
            }
        }
    }
    wave_lds_fence();
    group_slots(W, R, ent, n, fp, fps, L0, L1, L2, cap, lane);
}

// Issue the 16-byte HBM->LDS copies of a tile's footprint straight into LDS
// (no registers): wave instruction i fills chunks [64 i, 64 i + 64).
__device__ __forceinline__ void stage_footprint(const TileGeo& G, const int8_t* occ_lat,
                                                unsigned char* occl, int lane)
{
    int n0, n1, n2, n3;
    seg_chunks(G, n0, n1, n2, n3);
    const int total = n0 + n1 + n2 + n3;
    const int base = __builtin_amdgcn_readfirstlane(G.lds0 - (int)(G.st0 & 15));
    for (int c0 = 0; c0 < total; c0 += 64) {
        const int c = c0 + lane;
        if (c < total) {
            int cj;
            const int k = locate_chunk(c, n0, n1, n2, cj);
            const int64_t st = seg_st(G, k);
            const int8_t* src = occ_lat + (st - (st & 15)) + 16 * cj;
            __builtin_amdgcn_global_load_lds(
                (const void*)src, (__attribute__((address_space(3))) void*)(occl + base + 16 * c0), 16,
                0, 0);
        }
    }
}

// Owner tile (fragment index) in colour c of the vacancy at global cell
// (i,j,k), type t, or -1; c2s holds the sub-block index of every cell
// (x cells, then y, then z).
__device__ __forceinline__ int owner_tile(const unsigned char* c2s, int L0, int L1, int L2, int nf0,
                                          int nf1, int colour, int i, int j, int k, int t)
{
    int sb0 = c2s[i], sb1 = c2s[L0 + j], sb2 = c2s[L0 + L1 + k];
    const int col = (sb0 & 1) | ((sb1 & 1) << 1) | ((sb2 & 1) << 2);
    if (col != colour) {
        if ((col ^ (1 << t)) != colour) return -1;
        // on the +t face of the sub-block below along t?
        const int ct = t == 0 ? i : (t == 1 ? j : k);
        const int Lt = t == 0 ? L0 : (t == 1 ? L1 : L2);
        const int off = t == 0 ? 0 : (t == 1 ? L0 : L0 + L1);
        const int sbt = t == 0 ? sb0 : (t == 1 ? sb1 : sb2);
        const int prev = c2s[off + (ct == 0 ? Lt - 1 : ct - 1)];
        if (prev == sbt) return -1;
        if (t == 0) sb0 = prev;
        else if (t == 1) sb1 = prev;
        else sb2 = prev;
    }
    return (sb0 >> 1) + nf0 * ((sb1 >> 1) + nf1 * (sb2 >> 1));
}

// Resident lattice: the slots of the group's tiles (or of tile `only`) from
// the LDS vacancy list (i | j << 10 | k << 20 | type << 30).
__device__ __forceinline__ void collect_list(const WaveLds& W, const TileRec* R, const LatDesc& D,
                                             const uint32_t* vlist, int nv, const unsigned char* c2s,
                                             int colour, int f0, int nt, int only, int cap, int lane)
{
    for (int v = lane; v < nv; v += 64) {
        const uint32_t g = vlist[v];
        const int i = g & 1023, j = (g >> 10) & 1023, k = (g >> 20) & 1023, t = g >> 30;
        const int f = owner_tile(c2s, D.L[0], D.L[1], D.L[2], D.nf[0], D.nf[1], colour, i, j, k, t);
        const int q = f - f0;
        if (f < 0 || q < 0 || q >= nt || (only >= 0 && q != only)) continue;
        const TileGeo G = tile_geo_rec(R[q]);
        int lx = i - G.ox, ly = j - G.oy, lz = k - G.oz;
        if (lx < 0) lx += D.L[0];
        if (ly < 0) ly += D.L[1];
        if (lz < 0) lz += D.L[2];
        const int list = only >= 0 ? 8 : q;
        put_slot(W, G, D.L[0], D.L[1], D.L[2], list, only >= 0 ? 0 : q * cap, cap, lx, ly, lz, t, v);
    }
}

// Order n slots of list [first, first+n) by canonical key (keys distinct);
// the vacancy-list indices follow for a resident lattice.
__device__ __forceinline__ void sort_list(const WaveLds& W, int first, int n, int l, bool with_idx)
{
    const uint64_t key = W.raw_key[first + l];
    int rank = 0;
    for (int j = 0; j < n; j++) rank += W.raw_key[first + j] < key;
    W.xyz[first + rank] = W.raw_xyz[first + l];
    if (with_idx) W.idx[first + rank] = W.raw_idx[first + l];
}

// Resident lattice: final position of slot l of list `first` back to the list.
__device__ __forceinline__ void list_update(const WaveLds& W, const TileGeo& G, const LatDesc& D,
                                            uint32_t* vlist, int first, int l)
{
    const uint32_t xyz = W.xyz[first + l];
    const int X = xyz & 1023, Y = (xyz >> 10) & 1023, Z = xyz >> 20;
    const int t = site_type(X, Y);
    int i = G.ox + (X >> 1), j = G.oy + (Y >> 1), k = G.oz + (Z >> 1);
    if (i >= D.L[0]) i -= D.L[0];
    if (j >= D.L[1]) j -= D.L[1];
    if (k >= D.L[2]) k -= D.L[2];
    vlist[W.idx[first + l]] = (uint32_t)i | ((uint32_t)j << 10) | ((uint32_t)k << 20) | ((uint32_t)t << 30);
}

// ----------------------------------------------------------------------------
// Segmented wavefront primitives over segments of S consecutive lanes.
//
// Inclusive prefix sum of a binary64 value: DPP row_shr 1,2,4,8 inside each
// 16-lane row (segments of 8 mask the moves that cross their start), then
// row_bcast:15 / row_bcast:31 across rows.  The summands are exact multiples
// of one power of two, so every association gives the same sum.
template <int S>
__device__ __forceinline__ double seg_scan(double v, int sl)
{
    double o = dpp_shifted<0x111, 0xF>(v);
    v += (S >= 16 || sl >= 1) ? o : 0.0;
    o = dpp_shifted<0x112, 0xF>(v);
    v += (S >= 16 || sl >= 2) ? o : 0.0;
    o = dpp_shifted<0x114, 0xF>(v);
    v += (S >= 16 || sl >= 4) ? o : 0.0;
    if (S >= 16) v += dpp_shifted<0x118, 0xF>(v);
    if (S >= 32) v += dpp_shifted<0x142, 0xA>(v);
    if (S >= 64) v += dpp_shifted<0x143, 0xC>(v);
    return v;
}

// Value of lane `src` (any lane of the wave) for every lane; all lanes active.
__device__ __forceinline__ int lane_pull(int v, int src)
{
    return __builtin_amdgcn_ds_bpermute(src << 2, v);
}

__device__ __forceinline__ double lane_pull(double v, int src)
{
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int l)
{
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Wave-uniform parameters of one group of tiles (all of one lattice).
struct GroupCall {
    int8_t* occ;       // the lattice's occupancy in HBM (write-through when staged)
    int4* disp;        // displacement buffer
    int64_t disp_off;  // the lattice's first displacement index
    uint32_t seed, lid, cycle, ctag;
    double t_sync;
    bool write_occ;
};

// ----------------------------------------------------------------------------
// BKL on K tiles at once (Eqs. TransitionProb, eventSelection, TimeStep),
// each until its next event would land after t_sync or no event is possible.
// Tile `seg` runs on lanes [seg*S, seg*S + S), S = 64/K, with its n sorted
// slots at sxyz (packed local coordinates), fragment index f, its own Philox
// stream (step, f, cycle, ctag) and clock; event e = slot*8 + direction, in
// that order.  With n <= S, each slot has G lanes (G = 8, 4, 2, 1 as n
// allows), each caching the rates of 8/G consecutive events; K = 1 with
// n > 64 recomputes the rates from LDS at every step.  After a hop only the
// events whose vacancy moved or whose target changed are recomputed.
template <int K, int E, bool TR, bool MAP = true>
__device__ __forceinline__ void group_bkl(const TileGeo& G, const RateCtx& C, unsigned char* occl,
                                          uint32_t* sxyz, int n, uint32_t f, const GroupCall& X,
                                          int lane, Rec& rec, RecCtl& rc, uint32_t& ho, uint32_t& hh)
{
    constexpr int S = 64 / K;  // E: most events cached per lane
    const int sl = lane & (S - 1);
    const int sb = lane & ~(S - 1);
    const uint64_t segmask = S == 64 ? ~0ull : (((1ull << (S & 63)) - 1ull) << sb);
    const bool cached = n * 8 <= S * E;
    int lg = 0;  // log2 lanes per slot
    if (cached && n > 0) lg = n * 8 <= S ? 3 : (n * 4 <= S ? 2 : (n * 2 <= S ? 1 : 0));
    const int epl = 8 >> lg;
    const int my_slot = sl >> lg;
    const int my_d0 = (sl & ((1 << lg) - 1)) * epl;
    const bool ev_valid = cached && my_slot < n;
    uint32_t my_xyz = ev_valid ? sxyz[my_slot] : 0u;
    // recompute mode (K == 1, n > 64): lane l covers slots [s0, s1)
    const int m = (n + 63) >> 6;
    const int s0 = lane * m < n ? lane * m : n;
    const int s1 = s0 + m < n ? s0 + m : n;
    double kk[E];
#pragma unroll
    for (int d = 0; d < E; d++) kk[d] = 0.0;
    double ls = 0.0;
    // (unrolled: each rate goes straight to its register; events past
    // this lane's epl are skipped, and a block no lane needs is branched
    // over)
    auto refresh = [&]() {
        ls = 0.0;
#pragma unroll
        for (int j = 0; j < E; j++) {
            if (j < epl) {
                kk[j] = tile_rate<MAP>(G, occl, C, my_xyz, my_d0 + j);
                ls += kk[j];
            }
        }
    };
    if (ev_valid) refresh();
    // with TR, when lanes cache several events: after a hop, the moved
    // vacancy's 8 rates are computed by 8 lanes at once and pulled by the
    // lanes that cache them, instead of each of those lanes computing its
    // events in turn (the same values; more registers, so the lockstep
    // kernel, whose tiles mostly cache one event per lane, leaves it off)
    const bool wide = TR && __ballot(ev_valid && epl > 1) != 0;

    double tau = 0.0;
    uint32_t step = 0;
    bool active = n > 0;
    // draws computed ahead: lane sl of a segment holds the draw of step
    // dbase + sl of its tile, refilled when the tile has used all S
    uint32_t dbase = 0;
    double dr_sel = 0.0, dr_ln = 0.0;
    {
        uint32_t x0, x1, x2, x3;
        philox10((uint32_t)sl, f, X.cycle, X.ctag, X.seed, X.lid, x0, x1, x2, x3);
        dr_sel = u53_lo(x0, x1);
        dr_ln = clock_ln(u53_hi(x2, x3));
    }
    for (;;) {
        if (__ballot(active) == 0) break;
        const bool refill = active && step - dbase >= (uint32_t)S;
        if (__ballot(refill)) {
            if (refill) {
                dbase = step;
                uint32_t x0, x1, x2, x3;
                philox10(step + (uint32_t)sl, f, X.cycle, X.ctag, X.seed, X.lid, x0, x1, x2, x3);
                dr_sel = u53_lo(x0, x1);
                dr_ln = clock_ln(u53_hi(x2, x3));
            }
        }
        if (K == 1 && !cached) {
            ls = 0.0;
            for (int s = s0; s < s1; s++) {
                const uint32_t xyz = sxyz[s];
                for (int d = 0; d < 8; d++) ls += tile_rate<MAP>(G, occl, C, xyz, d);
            }
        }
        const double lsv = active ? ls : 0.0;
        const double incl = seg_scan<S>(lsv, sl);
        const double R = S == 64 ? lane_value(incl, 63) : lane_pull(incl, lane | (S - 1));
        const int dl = (int)(step - dbase);  // < S for an active tile
        const double u_sel = S == 64 ? lane_value(dr_sel, dl) : lane_pull(dr_sel, sb + (dl & (S - 1)));
        const double lnu = S == 64 ? lane_value(dr_ln, dl) : lane_pull(dr_ln, sb + (dl & (S - 1)));
        const double dt = -lnu / R;
        const double tn = tau + dt;
        // a tile hops when it has an event (R > 0) and its next event lands
        // inside the window; the step that finds no tile hopping ends the
        // loop before any selection work
        const bool go = active && R != 0.0 && tn <= X.t_sync;
        active = go;
        if (__ballot(go) == 0) break;
        if (go) tau = tn;
        const double y = u_sel * R;
        const uint64_t mk_all = __ballot(go && incl > y);
        const uint64_t nz_all = __ballot(go && lsv > 0.0);
        bool fb;
        int sel;
        if (S < 64) {
            // this segment's bits as a 32-bit mask: selects, no branches
            const uint32_t sm = S >= 32 ? 0xffffffffu : ((1u << (S & 31)) - 1u);
            const uint32_t m = (uint32_t)(mk_all >> sb) & sm;
            const uint32_t z = (uint32_t)(nz_all >> sb) & sm;
            fb = m == 0u;
            sel = m ? sb + (int)__builtin_ctz(m) : (z ? sb + 31 - (int)__builtin_clz(z) : lane);
        } else {
            const uint64_t mk = mk_all & segmask;
            const uint64_t nz = nz_all & segmask;
            fb = mk == 0;
            sel = lane;
            if (mk) sel = __ffsll((unsigned long long)mk) - 1;
            else if (nz) sel = 63 - __clzll((long long)nz);
        }
        // the selected lane of each segment picks the event
        int pick = 0, pslot = 0;
        if (go && lane == sel) {
            double Cc = incl - lsv;
            int found = -1, last = -1;
            if (cached) {
#pragma unroll
                for (int j = 0; j < E; j++) {
                    if (j < epl) {
                        if (kk[j] > 0.0) last = j;
                        Cc += kk[j];
                        if (!fb && found < 0 && Cc > y) found = j;
                    }
                }
                pick = (int)(my_xyz | ((uint32_t)(my_d0 + (found >= 0 ? found : last)) << 29));
                pslot = my_slot;
            } else if (K == 1) {
                uint32_t lx = 0;
                for (int s = s0; s < s1 && found < 0; s++) {
                    const uint32_t xyz = sxyz[s];
                    for (int d = 0; d < 8; d++) {
                        const double k = tile_rate<MAP>(G, occl, C, xyz, d);
                        if (k > 0.0) { last = s * 8 + d; lx = xyz; }
                        Cc += k;
                        if (!fb && Cc > y) { found = s * 8 + d; lx = xyz; break; }
                    }
                }
                const int e = found >= 0 ? found : last;
                pick = (int)(lx | ((uint32_t)(e & 7) << 29));
                pslot = e >> 3;
            }
        }
        if (S == 64) {
            pick = __builtin_amdgcn_readlane(pick, sel);
            pslot = __builtin_amdgcn_readlane(pslot, sel);
        } else {
            pick = lane_pull(pick, sel);
            pslot = lane_pull(pslot, sel);
        }
        pick = go ? pick : 0;
        const uint32_t sx = (uint32_t)pick & 0x1FFFFFFFu;
        const int d = (int)((uint32_t)pick >> 29);
        int hx, hy, hz;
        const uint32_t tx = hop_target_xyz(sx, d, hx, hy, hz);
        // (a segment without a hop has pick 0: local site (0,0,0), inside
        // its footprint, so these addresses are valid either way)
        int sk, sli, tk, tli;
        const int spos = xyz_lds(G, sx, sk, sli);
        const int tpos = xyz_lds(G, tx, tk, tli);
        const int sp = occl[tpos];
        wave_lds_order();
        int64_t sst = 0, tst = 0;  // storage offsets, in the lanes that apply a hop
        if (go && sl == 0) {
            sst = seg_st(G, sk) + sli;
            tst = seg_st(G, tk) + tli;
            occl[spos] = (unsigned char)sp;
            occl[tpos] = (unsigned char)kSpV;
            sxyz[pslot] = tx;
            if (X.write_occ) {
                X.occ[sst] = (int8_t)sp;
                X.occ[tst] = (int8_t)kSpV;
            }
            if (sp == kSpO) ho++;
            else hh++;
        }
        // displacement records: the hops of this step one after another
        uint64_t hm = __ballot(go && sl == 0);
        if (hm) {
            const int64_t ks_l = X.disp_off + sst, kt_l = X.disp_off + tst;
            const int hp = (hx + 1) | ((hy + 1) << 2) | ((hz + 1) << 4);
            while (hm) {
                const int l = __ffsll((unsigned long long)hm) - 1;
                hm &= hm - 1;
                const int64_t ks = readlane64(ks_l, l), kt = readlane64(kt_l, l);
                const int h = __builtin_amdgcn_readlane(hp, l);
                rec_hop(rec, rc, X.disp, lane, ks, kt, (h & 3) - 1, ((h >> 2) & 3) - 1,
                        ((h >> 4) & 3) - 1);
            }
        }
        step += go ? 1u : 0u;
        wave_lds_order();
        if (wide) {
            const bool mover = ev_valid && go && my_slot == pslot;
            if (mover) my_xyz = tx;
            // the moved vacancy's 8 rates, one per lane of the segment's
            // first 8, pulled by the lanes that cache them
            if (__ballot(mover)) {
                double nk = 0.0;
                if (go && sl < 8) nk = tile_rate<MAP>(G, occl, C, tx, sl);
#pragma unroll
                for (int j = 0; j < E; j++) {
                    const double v = lane_pull(nk, sb + ((my_d0 + j) & 7));
                    if (mover && j < epl) kk[j] = v;
                }
            }
            // another vacancy next to either site (rare): all its cached events
            const bool nbr = ev_valid && go && !mover && (nn_site(my_xyz, sx) || nn_site(my_xyz, tx));
            if (__ballot(nbr)) {
                if (nbr) refresh();
            }
            if (mover) {
                ls = 0.0;
#pragma unroll
                for (int j = 0; j < E; j++)
                    if (j < epl) ls += kk[j];
            }
        } else if (ev_valid && go) {
            if (my_slot == pslot) my_xyz = tx;
            if (my_slot == pslot || nn_site(my_xyz, sx) || nn_site(my_xyz, tx)) refresh();
        }
    }
}

// ----------------------------------------------------------------------------
// One wave runs nt <= K tiles of colour `colour` of one lattice: fragments
// f0 .. f0+nt-1.  Streamed lattices stage their footprints from HBM into LDS
// at lds0 + fp (fps bytes apart); resident lattices find their slots in the
// LDS vacancy list.  The tiles run together, one per S = 64/K-lane segment;
// a tile with more vacancies than S/2 runs afterwards on the whole wave
// (E1 cached events per lane there).
// With `single`, every tile runs on the whole wave, one after another, and
// a streamed lattice stages one footprint at a time.
template <int K, int E1, bool TR, bool MAP = true>
__device__ __forceinline__ void run_group(const DevPtrs& P, const LatDesc& D, int f0, int nt, int colour,
                                          const GroupCall& X, const WaveLds& W, unsigned char* lds0,
                                          int fp, int fps, bool resident, bool single, uint32_t* vlist,
                                          int nv, const unsigned char* c2s, const TileRec* cached,
                                          int lane, Rec& rec, RecCtl& rc, uint32_t& ho, uint32_t& hh,
                                          bool& err)
{
    static_assert(K > 1, "tile groups of more than one tile");
    constexpr int S = 64 / K;
    constexpr int FIT = S / 2;  // vacancies a segment holds (4 cached events per lane)
    const int seg = lane / S, sl = lane & (S - 1);
    // tile records: an LDS cache of the whole call, or copied for this group
    const TileRec* R = cached;
    if (!cached) {
        const TileRec* trec = P.tiles + (size_t)colour * P.n_tiles + D.tile0 + f0;
        if (lane < nt) W.rec[lane] = trec[lane];
        R = W.rec;
    }
    if (lane < 16) W.cnt[lane] = 0;
    wave_lds_fence();
    // boundary planes: when no footprint of the group reaches a plane cell
    // (cells [o, o + w] along a masked axis, the +face included), every
    // boundary flag of its edges is 0 and the rates skip the test
    bool gb_live = false;
    if (D.gb_period > 0) {
        bool hit = false;
        if (lane < nt) {
            const TileRec& T = R[lane];
            const int o[3] = {T.ox, T.oy, T.oz}, w[3] = {T.wx, T.wy, T.wz};
#pragma unroll
            for (int a = 0; a < 3; a++) {
                const int hi = o[a] + w[a];
                hit |= ((D.gb_mask >> a) & 1) && (hi >= D.L[a] || (hi / D.gb_period) * D.gb_period >= o[a]);
            }
        }
        gb_live = __ballot(hit) != 0;
    }
    const RateCtx C = {D.L[0], D.L[1], D.L[2], gb_live ? D.gb_period : 0, D.gb_mask, W.k12, D.gb_map};
    int n_seg = 0;
    if (!single) {
        if (resident) {
            collect_list(W, R, D, vlist, nv, c2s, colour, f0, nt, -1, S, lane);
        } else {
            for (int k = 0; k < nt; k++) {
                TileGeo T = tile_geo_rec(R[k]);
                tile_lds_at(T, fp + k * fps);
                stage_footprint(T, X.occ, lds0, lane);
            }
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the staged footprints have landed
            __builtin_amdgcn_wave_barrier();
            scan_group(W, R, lds0, nt, fp, fps, D.L[0], D.L[1], D.L[2], S, lane);
        }
        wave_lds_fence();
        // this lane's tile
        TileGeo G = tile_geo_rec(R[seg < nt ? seg : 0]);
        if (resident) tile_lds_resident(G);
        else tile_lds_at(G, fp + seg * fps);
        n_seg = seg < nt ? W.cnt[seg] : 0;
        if (n_seg <= FIT && sl < n_seg) sort_list(W, seg * S, n_seg, sl, resident);
        wave_lds_fence();
        const int n_run = n_seg <= FIT ? n_seg : 0;
        group_bkl<K, 4, TR, MAP>(G, C, lds0, W.xyz + seg * S, n_run, (uint32_t)(f0 + seg), X, lane, rec, rc, ho,
                        hh);
        wave_lds_fence();
        if (resident && sl < n_run) list_update(W, G, D, vlist, seg * S, sl);
    }
    // tiles run on the whole wave: those that did not fit their segment, or all
    uint64_t todo = single ? (nt >= 64 ? ~0ull : ((1ull << nt) - 1ull))
                           : __ballot(sl == 0 && n_seg > FIT);
    while (todo) {
        wave_lds_fence();
        const int b = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        const int q = single ? b : b / S;
        if (lane == 0) W.cnt[8] = 0;
        TileGeo T = tile_geo_rec(R[q]);
        if (resident) {
            tile_lds_resident(T);
            wave_lds_fence();
            collect_list(W, R, D, vlist, nv, c2s, colour, f0, nt, q, 128, lane);
        } else {
            tile_lds_at(T, fp + (single ? 0 : q) * fps);
            if (single) {
                stage_footprint(T, X.occ, lds0, lane);
                __builtin_amdgcn_s_waitcnt(0x0F70);
                __builtin_amdgcn_wave_barrier();
            }
            wave_lds_fence();
            scan_staged(W, T, lds0, D.L[0], D.L[1], D.L[2], 8, 0, 128, lane);
        }
        wave_lds_fence();
        const int n1 = W.cnt[8];
        if (n1 > 128) {
            err = true;
            continue;
        }
        for (int l = lane; l < n1; l += 64) sort_list(W, 0, n1, l, resident);
        wave_lds_fence();
        group_bkl<1, E1, TR, MAP>(T, C, lds0, W.xyz, n1, (uint32_t)(f0 + q), X, lane, rec, rc, ho, hh);
        wave_lds_fence();
        if (resident)
            for (int l = lane; l < n1; l += 64) list_update(W, T, D, vlist, 0, l);
    }
    wave_lds_fence();
}

// ----------------------------------------------------------------------------
// Lockstep phase kernel: one wave per group of K tiles of colour `colour`
// (P.groups: lattice and first fragment), footprints staged HBM -> LDS.
// Without the boundary-site map branch the kernel is held to 128 VGPRs, so
// that 4 wavefronts share a SIMD (it fits without scratch).
template <int K, bool MAP>
__global__ __launch_bounds__(64 * kPhaseWaves) __attribute__((amdgpu_waves_per_eu(MAP ? 1 : 4)))
void k_phase(DevPtrs P, int colour)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + wv);
    if (g >= P.n_groups) return;
    const int2 gr = P.groups[g];
    const int lat = __builtin_amdgcn_readfirstlane(gr.x);
    const int f0 = __builtin_amdgcn_readfirstlane(gr.y);
    const LatDesc& D = P.desc[lat];
    LatState* St = P.state + lat;
    if (St->done) return;
    const int ntiles = D.nf[0] * D.nf[1] * D.nf[2];
    constexpr int KG = K == 1 ? 8 : K;  // K = 1: tiles one after another
    const int nt = ntiles - f0 < K ? ntiles - f0 : K;
    GroupCall X;
    X.occ = P.occ + D.occ_off;
    X.disp = P.disp;
    X.disp_off = D.disp_off;
    X.seed = D.seed;
    X.lid = D.lattice_id;
    X.cycle = (uint32_t)St->cycles;
    X.ctag = ((uint32_t)colour << 8) | 2u;
    X.t_sync = P.call[lat].t_sync;
    X.write_occ = true;
    unsigned char* base = smem + wv * P.lds_wave_bytes;
    const WaveLds W = wave_lds(base);
    Rec rec;
    RecCtl rc;
    rec_init(rec, rc);
    uint32_t ho = 0, hh = 0;
    bool err = false;
    if (lane < 12) W.k12[lane] = D.k12[lane];
    run_group<KG, 4, false, MAP>(P, D, f0, nt, colour, X, W, smem, (int)(base - smem) + kWaveScratchStaged, P.fp_stride,
                  false, K == 1, nullptr, 0, nullptr, nullptr, lane, rec, rc, ho, hh, err);
    rec_flush(rec, rc, P.disp);
    constexpr int S = K == 1 ? 64 : 64 / K;
    if ((lane & (S - 1)) == 0 && (ho | hh)) {
        const int f = f0 + lane / S;
        unsigned long long* b = P.buckets + ((size_t)lat * kHopBuckets + (f & (kHopBuckets - 1))) * 2;
        if (ho) atomicAdd(b, (unsigned long long)ho);
        if (hh) atomicAdd(b + 1, (unsigned long long)hh);
    }
    if (__ballot(err) && lane == 0) atomicOr(&St->err, 1u);
}

// ----------------------------------------------------------------------------
// Single-fragment lattices held in LDS, with at most 32 vacancies: the
// sub-blocks are the two halves of the lattice along each axis (lower half
// ceil(L/2) cells), one tile per colour, and one wave runs everything.
// A block of lanes owns each vacancy for the whole call (packed doubled
// coordinates) and caches the rates of its 8 events; the occupancy sits in
// LDS in canonical site order.  In each phase the slot order of the BKL
// domain is the canonical order of the vacancies at phase start: every lane
// computes its vacancy's rank once per phase, and each step moves the lane
// totals into event order (ds_permute) before the prefix sum.  Vacancies outside the
// phase's footprint have no active edge and contribute zero rates, which
// changes no partial sum and no selection.

__device__ __forceinline__ uint32_t pack_dbl(int X, int Y, int Z)
{
    return (uint32_t)X | ((uint32_t)Y << 11) | ((uint32_t)Z << 22);
}

// Canonical index of the site at doubled coordinates (X, Y, Z).
__device__ __forceinline__ int canon_dbl(int L0, int L1, int X, int Y, int Z)
{
    return (((Z >> 1) * L1 + (Y >> 1)) * L0 + (X >> 1)) * 3 + site_type(X, Y);
}

// Storage offset of canonical cell (i,j,k), type t, when the lattice is one
// fragment (sub-block bounds 0, ceil(L/2), L per axis).
__device__ __forceinline__ int store_index_1f(int L0, int L1, int L2, int i, int j, int k, int t)
{
    const int h0 = (L0 + 1) >> 1, h1 = (L1 + 1) >> 1, h2 = (L2 + 1) >> 1;
    const int x0 = i >= h0 ? h0 : 0, y0 = j >= h1 ? h1 : 0, z0 = k >= h2 ? h2 : 0;
    const int wx = i >= h0 ? L0 - h0 : h0, wy = j >= h1 ? L1 - h1 : h1, wz = k >= h2 ? L2 - h2 : h2;
    const int base = 3 * (z0 * L1 * L0 + wz * (y0 * L0 + wy * x0));
    return base + brick_local(t, i - x0, j - y0, k - z0, wx, wy, wz);
}

__device__ __forceinline__ int store_dbl_1f(int L0, int L1, int L2, int X, int Y, int Z)
{
    return store_index_1f(L0, L1, L2, X >> 1, Y >> 1, Z >> 1, site_type(X, Y));
}

// Rate of event d of the vacancy at doubled coordinates (X,Y,Z), every edge
// active: zero when the target holds a vacancy, else the table entry for
// (ion species, z step, boundary).
__device__ __forceinline__ double dbl_rate(const RateCtx& C, const unsigned char* slab, int X, int Y,
                                           int Z, int d)
{
    const int t = site_type(X, Y);
    int hx, hy, hz;
    hop_vec(t, d, hx, hy, hz);
    int TX = X + hx, TY = Y + hy, TZ = Z + hz;
    if (TX < 0) TX += 2 * C.L0;
    if (TX >= 2 * C.L0) TX -= 2 * C.L0;
    if (TY < 0) TY += 2 * C.L1;
    if (TY >= 2 * C.L1) TY -= 2 * C.L1;
    if (TZ < 0) TZ += 2 * C.L2;
    if (TZ >= 2 * C.L2) TZ -= 2 * C.L2;
    const int sp = slab[canon_dbl(C.L0, C.L1, TX, TY, TZ)];
    if (sp == kSpV) return 0.0;
    int g = 0;
    if (C.gbp > 0) {
        const int tt = site_type(TX, TY);
        g = gb_flag(C, t, pick3(t, X >> 1, Y >> 1, Z >> 1)) |
            gb_flag(C, tt, pick3(tt, TX >> 1, TY >> 1, TZ >> 1));
    }
    return C.k12[(sp * 3 + hz + 1) * 2 + g];
}

// Rate of event d in phase `colour`: zero unless the edge's owner cell (the
// cell of its midpoint) lies in the sub-block of that colour.
__device__ __forceinline__ double fast_rate(const RateCtx& C, const unsigned char* slab, int colour,
                                            int X, int Y, int Z, int d)
{
    const int t = site_type(X, Y);
    int hx, hy, hz;
    hop_vec(t, d, hx, hy, hz);
    int ox = (2 * X + hx) >> 2, oy = (2 * Y + hy) >> 2, oz = (2 * Z + hz) >> 2;
    if (ox < 0) ox += C.L0;
    if (oy < 0) oy += C.L1;
    if (oz < 0) oz += C.L2;
    const int col = (ox >= ((C.L0 + 1) >> 1) ? 1 : 0) | (oy >= ((C.L1 + 1) >> 1) ? 2 : 0) |
                    (oz >= ((C.L2 + 1) >> 1) ? 4 : 0);
    if (col != colour) return 0.0;
    return dbl_rate(C, slab, X, Y, Z, d);
}

// Periodic nearest neighbours (doubled coordinates differ by 1 on two axes).
__device__ __forceinline__ bool nn_dbl(int L0, int L1, int L2, uint32_t a, uint32_t b)
{
    int dx = (int)(a & 2047) - (int)(b & 2047);
    int dy = (int)((a >> 11) & 2047) - (int)((b >> 11) & 2047);
    int dz = (int)(a >> 22) - (int)(b >> 22);
    dx = dx < 0 ? -dx : dx;
    dy = dy < 0 ? -dy : dy;
    dz = dz < 0 ? -dz : dz;
    if (dx == 2 * L0 - 1) dx = 1;
    if (dy == 2 * L1 - 1) dy = 1;
    if (dz == 2 * L2 - 1) dz = 1;
    return dx * dx + dy * dy + dz * dz == 2;
}

// Runs the call's cycles on wave 0.  vlist holds the nv vacancies
// (i | j << 10 | k << 20 | t << 30); slab the canonical occupancy.  Each
// vacancy has G lanes (G = 8, 4, 2, 1 for nv <= 8, 16, 32, 64), lane q of
// its block caching the rates of directions [q*8/G, (q+1)*8/G).  The draws
// of a phase are computed ahead, one step per lane, 64 at a time.
__device__ __forceinline__ void solo_fast(const LatDesc& D, unsigned char* slab, const uint32_t* vlist,
                                          int nv, const RateCtx& C, GroupCall& X, uint64_t max_cycles,
                                          uint64_t min_hops, uint64_t cycle0, int lane, uint64_t& ncyc,
                                          unsigned long long& ho_tot, unsigned long long& hh_tot,
                                          Rec& rec, RecCtl& rc)
{
    const int L0 = D.L[0], L1 = D.L[1], L2 = D.L[2];
    const int lg = nv <= 8 ? 3 : (nv <= 16 ? 2 : (nv <= 32 ? 1 : 0));  // log2 G
    const int G = 1 << lg, epl = 8 >> lg;
    const int v = lane >> lg, q = lane & (G - 1), d0 = q * epl;
    const bool valid = v < nv;
    uint32_t pos = 0;
    if (valid) {
        const uint32_t g = vlist[v];
        const int i = g & 1023, j = (g >> 10) & 1023, k = (g >> 20) & 1023, t = g >> 30;
        pos = pack_dbl(2 * i + (t != 0), 2 * j + (t != 1), 2 * k + (t != 2));
    }
    double kk[8];
#pragma unroll
    for (int d = 0; d < 8; d++) kk[d] = 0.0;
    double tot = 0.0;
    int colour = 0;
    auto rates = [&]() {
        tot = 0.0;
        const int Xs = pos & 2047, Ys = (pos >> 11) & 2047, Zs = pos >> 22;
#pragma nounroll
        for (int j = 0; j < epl; j++) {
            const double r = fast_rate(C, slab, colour, Xs, Ys, Zs, d0 + j);
            tot += r;
#pragma unroll
            for (int u = 0; u < 8; u++) kk[u] = u == j ? r : kk[u];
        }
    };
    unsigned long long ho = 0, hh = 0;
    while (ncyc < max_cycles) {
        X.cycle = (uint32_t)(cycle0 + ncyc);
        for (colour = 0; colour < 8; colour++) {
            const uint32_t ctag = ((uint32_t)colour << 8) | 2u;
            // slot order: canonical order of the vacancies at phase start
            const int Xs = pos & 2047, Ys = (pos >> 11) & 2047, Zs = pos >> 22;
            const int key = valid ? canon_dbl(L0, L1, Xs, Ys, Zs) : 0x7fffffff;
            int rank = 0;
            for (int j = 0; j < nv; j++) rank += (__builtin_amdgcn_readlane(key, j << lg) < key) ? 1 : 0;
            const int dst = valid ? ((rank << lg) | q) : lane;  // unused lanes keep their place
            const int inv = __builtin_amdgcn_ds_permute(dst << 2, lane);  // source lane of each place
            if (valid) rates();
            double tau = 0.0;
            uint32_t step = 0;
            double dr_sel = 0.0, dr_ln = 0.0;  // draw of step (step & ~63) + lane
            for (;;) {
                if ((step & 63) == 0) {
                    uint32_t x0, x1, x2, x3;
                    philox10(step + (uint32_t)lane, 0u, X.cycle, ctag, X.seed, X.lid, x0, x1, x2, x3);
                    dr_sel = u53_lo(x0, x1);
                    dr_ln = clock_ln(u53_hi(x2, x3));
                }
                const int lo = __builtin_amdgcn_ds_permute(dst << 2, __double2loint(tot));
                const int hi = __builtin_amdgcn_ds_permute(dst << 2, __double2hiint(tot));
                const double srt = __hiloint2double(hi, lo);  // lane totals in event order
                const double incl = wave_scan_dpp(srt);
                const double R = lane_value(incl, 63);
                if (R == 0.0) break;
                const int sl = (int)(step & 63);
                const double u_sel = lane_value(dr_sel, sl);
                const double dt = -lane_value(dr_ln, sl) / R;
                const double tn = tau + dt;
                if (tn > X.t_sync) break;
                tau = tn;
                const double y = u_sel * R;
                const uint64_t mk = __ballot(incl > y);
                int r;
                bool fb = false;
                if (mk) {
                    r = __ffsll((unsigned long long)mk) - 1;
                } else {
                    r = 63 - __clzll((long long)__ballot(srt > 0.0));
                    fb = true;
                }
                const int owner = __builtin_amdgcn_readlane(inv, r);
                const double c0 = lane_value(incl, r) - lane_value(srt, r);
                int dsel = 0;
                if (lane == owner) {
                    double cc = c0;
                    int found = -1, last = -1;
#pragma unroll
                    for (int j = 0; j < 8; j++) {
                        if (j < epl) {
                            if (kk[j] > 0.0) last = j;
                            cc += kk[j];
                            if (!fb && found < 0 && cc > y) found = j;
                        }
                    }
                    dsel = d0 + (found >= 0 ? found : last);
                }
                const int d = __builtin_amdgcn_readlane(dsel, owner);
                const uint32_t sx = (uint32_t)__builtin_amdgcn_readlane((int)pos, owner);
                const int SX = sx & 2047, SY = (sx >> 11) & 2047, SZ = sx >> 22;
                int hx, hy, hz;
                hop_vec(site_type(SX, SY), d, hx, hy, hz);
                int TX = SX + hx, TY = SY + hy, TZ = SZ + hz;
                if (TX < 0) TX += 2 * L0;
                if (TX >= 2 * L0) TX -= 2 * L0;
                if (TY < 0) TY += 2 * L1;
                if (TY >= 2 * L1) TY -= 2 * L1;
                if (TZ < 0) TZ += 2 * L2;
                if (TZ >= 2 * L2) TZ -= 2 * L2;
                const uint32_t tx = pack_dbl(TX, TY, TZ);
                const int cs = canon_dbl(L0, L1, SX, SY, SZ), ct = canon_dbl(L0, L1, TX, TY, TZ);
                const int sp = slab[ct];
                wave_lds_order();
                if (lane == 0) {
                    slab[cs] = (unsigned char)sp;
                    slab[ct] = (unsigned char)kSpV;
                }
                const bool mover = valid && (lane >> lg) == (owner >> lg);
                if (mover) pos = tx;
                if (sp == kSpO) ho++;
                else hh++;
                rec_hop(rec, rc, X.disp, lane, X.disp_off + store_dbl_1f(L0, L1, L2, SX, SY, SZ),
                        X.disp_off + store_dbl_1f(L0, L1, L2, TX, TY, TZ), hx, hy, hz);
                step++;
                wave_lds_order();
                if (valid && (mover || nn_dbl(L0, L1, L2, pos, sx) || nn_dbl(L0, L1, L2, pos, tx)))
                    rates();
            }
        }
        ncyc++;
        if (min_hops > 0 && ho + hh >= min_hops) break;
    }
    ho_tot = ho;
    hh_tot = hh;
}

// ----------------------------------------------------------------------------
// Plain BKL (Eqs. TransitionProb, eventSelection, TimeStep) on a lattice held
// in LDS, 2 bits per site in canonical order, with at most 512 vacancies, on
// one wave.  The slots are the vacancies in canonical order at the start of
// the call (a slot follows its vacancy); lane l holds the P = 1, 2, 4 or 8
// consecutive slots l*P .. l*P+P-1 with their rate totals, the lane's total
// and the inclusive prefix of the lane totals.  The 8 rates of every slot
// and the species of its 8 targets sit in LDS.  After a hop one 16-lane pass
// reads the neighbours of both sites: lanes 0-7 give the moved vacancy its
// new rates, and a vacancy found next to either site (rare) has its slot
// recomputed; the prefix sums of a changed lane and every later one move by
// the change of its total.  The rates are multiples of one power of two with
// every partial sum below 2^53 of them, so these updates give exactly the
// sums of a fresh pass in event order.

// Storage offset in plain mode: the whole lattice is one brick.
__device__ __forceinline__ int64_t plain_offset(int L0, int L1, int L2, int i, int j, int k, int t)
{
    const int64_t V = (int64_t)L0 * L1 * L2;
    if (t == 0) return ((int64_t)i * L2 + k) * L1 + j;
    if (t == 1) return V + ((int64_t)j * L2 + k) * L0 + i;
    return 2 * V + ((int64_t)k * L1 + j) * L0 + i;
}

// 2-bit species of canonical site c.
__device__ __forceinline__ int pk_get(const uint32_t* ps, int c)
{
    return (int)((ps[c >> 4] >> ((c & 15) << 1)) & 3u);
}

// Set the 2-bit species of site c: two LDS atomics without return (clear,
// then set), so nothing waits for a read of the word.  The word address
// carries a zero from a register the compiler cannot see into, so it is
// not known to be uniform and the atomics are issued as written (a
// uniform-address atomic gets a wavefront-combining wrapper, five more
// instructions each, even when only one lane is active).
__device__ __forceinline__ void pk_set(uint32_t* ps, int c, int v)
{
    int z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    uint32_t* w = ps + ((c >> 4) + z);
    const int sh = (c & 15) << 1;
    atomicAnd(w, ~(3u << sh));
    atomicOr(w, (uint32_t)v << sh);
}

// Neighbour d of the site at packed doubled coordinates p: its canonical
// index and packed coordinates, and the column of the rate table (z step,
// boundary flag): the rate for ion species X is k12[X*6 + col].
__device__ __forceinline__ int plain_nb(const RateCtx& C, uint32_t p, int d, uint32_t& np, int& col,
                                        int& hx, int& hy, int& hz)
{
    const int X = p & 2047, Y = (p >> 11) & 2047, Z = p >> 22;
    const int t = site_type(X, Y);
    hop_vec(t, d, hx, hy, hz);
    int TX = X + hx, TY = Y + hy, TZ = Z + hz;
    if (TX < 0) TX += 2 * C.L0;
    if (TX >= 2 * C.L0) TX -= 2 * C.L0;
    if (TY < 0) TY += 2 * C.L1;
    if (TY >= 2 * C.L1) TY -= 2 * C.L1;
    if (TZ < 0) TZ += 2 * C.L2;
    if (TZ >= 2 * C.L2) TZ -= 2 * C.L2;
    np = pack_dbl(TX, TY, TZ);
    int g = 0;
    if (__builtin_expect(C.gbp > 0, 0)) {
        const int tt = site_type(TX, TY);
        g = gb_flag(C, t, pick3(t, X >> 1, Y >> 1, Z >> 1)) |
            gb_flag(C, tt, pick3(tt, TX >> 1, TY >> 1, TZ >> 1));
    }
    col = (hz + 1) * 2 + g;
    return canon_dbl(C.L0, C.L1, TX, TY, TZ);
}

__device__ __forceinline__ int plain_nb(const RateCtx& C, uint32_t p, int d, uint32_t& np, int& col)
{
    int hx, hy, hz;
    return plain_nb(C, p, d, np, col, hx, hy, hz);
}

// Storage offset in plain mode for a lattice held in LDS (fewer than 2^31
// sites, so 32-bit arithmetic): the whole lattice is one brick, so this is
// the brick index with the lattice as the brick (selects, no branches).
__device__ __forceinline__ int plain_offset32(int L0, int L1, int L2, int i, int j, int k, int t)
{
    return brick_local(t, i, j, k, L0, L1, L2);
}

// Storage offset (within the lattice) of canonical site c in plain mode.
__device__ __forceinline__ int plain_site_offset(uint32_t c, uint32_t L0, uint32_t L1, uint32_t L2)
{
    const uint32_t cell = c / 3u, t = c - 3u * cell;
    const uint32_t row = cell / L0, i = cell - row * L0;
    const uint32_t k = row / L1, j = row - k * L1;
    return plain_offset32((int)L0, (int)L1, (int)L2, (int)i, (int)j, (int)k, (int)t);
}

// Displacement records of the plain path in LDS, as the tile path keeps
// them (one record per lane, for the particle now at site cur that started
// the open run at site orig, with its displacement since), keyed by
// canonical site index: the storage offsets are worked out only when the
// records are written back, by every lane at once.
struct PlainRec {
    int cur;  // < 0: free
    int orig;
    int ax, ay, az;
    int n;         // records in use (wave-uniform)
    bool pending;  // stores of the last flush may still be in flight
};

__device__ __forceinline__ void prec_flush(PlainRec& r, int4* disp, int64_t disp_off, int L0, int L1, int L2)
{
    if (r.n == 0) return;
    if (r.pending) {
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the last flush's stores have landed
        __builtin_amdgcn_wave_barrier();
    }
    int4 o = make_int4(0, 0, 0, 0);
    int64_t dst = 0;
    if (r.cur >= 0) {
        o = disp[disp_off + plain_site_offset((uint32_t)r.orig, L0, L1, L2)];
        dst = disp_off + plain_site_offset((uint32_t)r.cur, L0, L1, L2);
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // every read has returned before any write
    __builtin_amdgcn_wave_barrier();
    if (r.cur >= 0) disp[dst] = make_int4(o.x + r.ax, o.y + r.ay, o.z + r.az, 0);
    r.cur = -1;
    r.ax = r.ay = r.az = 0;
    r.n = 0;
    r.pending = true;
}

// The vacancy at canonical site cs swaps with the ion at ct, the vacancy
// moving by h (all wave-uniform).
__device__ __forceinline__ void prec_hop(PlainRec& r, int4* disp, int64_t disp_off, int L0, int L1, int L2,
                                         int lane, int cs, int ct, int hx, int hy, int hz)
{
    uint64_t mv = __ballot(r.cur == cs);
    uint64_t mi = __ballot(r.cur == ct);
    if (__builtin_expect(r.n + (mv == 0) + (mi == 0) > 64, 0)) {
        prec_flush(r, disp, disp_off, L0, L1, L2);
        mv = 0;
        mi = 0;
    }
    // a site without a record opens one in the next free lane (selects)
    const int lv = mv ? __ffsll((unsigned long long)mv) - 1 : r.n;
    const int n1 = r.n + (mv == 0);
    const int li = mi ? __ffsll((unsigned long long)mi) - 1 : n1;
    r.n = n1 + (mi == 0);
    r.orig = lane == lv && mv == 0 ? cs : (lane == li && mi == 0 ? ct : r.orig);
    const int sv = lane == lv ? 1 : (lane == li ? -1 : 0);
    r.cur = lane == lv ? ct : (lane == li ? cs : r.cur);
    r.ax += sv * hx;
    r.ay += sv * hy;
    r.az += sv * hz;
}

// Rate of a hop onto a target holding species sp (0 for a vacancy); the
// table entries of both ions are read together with the target.
__device__ __forceinline__ double plain_rate_of(const RateCtx& C, const uint32_t* ps, int cn, int col, int& sp)
{
    const double kO = C.k12[col], kH = C.k12[6 + col];
    sp = pk_get(ps, cn);
    return sp == kSpO ? kO : (sp == kSpH ? kH : 0.0);
}

// Lanes 0-7: rate and target species of direction `lane` of the vacancy at
// packed doubled coordinates p, stored for slot `slot`.  Returns the slot
// total (wave-uniform).  All lanes must be active.
__device__ __forceinline__ double plain_slot_rates(const RateCtx& C, const uint32_t* ps, double* krate,
                                                   unsigned char* kspec, int slot, uint32_t p, int lane)
{
    double k = 0.0;
    if (lane < 8) {
        uint32_t np;
        int col, sp;
        const int cn = plain_nb(C, p, lane, np, col);
        k = plain_rate_of(C, ps, cn, col, sp);
        krate[slot * 8 + lane] = k;
        kspec[slot * 8 + lane] = (unsigned char)sp;
    }
    return lane_value(seg_scan<8>(k, lane & 7), 7);
}

// Load a plain lattice's occupancy into LDS at 2 bits per site in canonical
// order (16 sites per word) and list its vacancies (i | j << 10 | k << 20 |
// t << 30, in no particular order) up to `cap` of them; every thread of the
// workgroup takes part.
__device__ __forceinline__ void plain_pack_load(const LatDesc& D, const int8_t* occ_lat, uint32_t* pslab,
                                                uint32_t* vlist, int* vlist_n, int cap)
{
    const int64_t nbytes = D.n_sites;
    const int n_words = (int)((nbytes + 15) >> 4);
    for (int w = threadIdx.x; w < n_words; w += blockDim.x) {
        uint32_t word = 0;
        for (int b = 0; b < 16; b++) {
            const int64_t c = 16 * (int64_t)w + b;
            if (c >= nbytes) break;
            const int t = (int)(c % 3);
            const int64_t cell = c / 3;
            const int i = (int)(cell % D.L[0]);
            const int j = (int)((cell / D.L[0]) % D.L[1]);
            const int k = (int)(cell / ((int64_t)D.L[0] * D.L[1]));
            const uint32_t sp = (uint32_t)occ_lat[plain_offset(D.L[0], D.L[1], D.L[2], i, j, k, t)] & 3u;
            word |= sp << (2 * b);
            if (sp == (uint32_t)kSpV) {
                const int v = atomicAdd(vlist_n, 1);
                if (v < cap)
                    vlist[v] = (uint32_t)i | ((uint32_t)j << 10) | ((uint32_t)k << 20) | ((uint32_t)t << 30);
            }
        }
        pslab[w] = word;
    }
}

// Write a packed plain lattice back to its storage; every thread takes part.
__device__ __forceinline__ void plain_pack_store(const LatDesc& D, int8_t* occ_lat, const uint32_t* pslab)
{
    const int64_t nbytes = D.n_sites;
    for (int64_t c = threadIdx.x; c < nbytes; c += blockDim.x) {
        const int t = (int)(c % 3);
        const int64_t cell = c / 3;
        const int i = (int)(cell % D.L[0]);
        const int j = (int)((cell / D.L[0]) % D.L[1]);
        const int k = (int)(cell / ((int64_t)D.L[0] * D.L[1]));
        occ_lat[plain_offset(D.L[0], D.L[1], D.L[2], i, j, k, t)] = (int8_t)pk_get(pslab, (int)c);
    }
}

// Slots of a plain lattice held in LDS: vlist (nv entries, i | j << 10 |
// k << 20 | t << 30) is rewritten in ascending canonical index as packed
// doubled coordinates, so slot s is the vacancy of rank s.  One wave.
template <int P>
__device__ __forceinline__ void plain_rank_slots(uint32_t* vlist, int nv, int L0, int L1, int lane)
{
    uint32_t pv[P];
    int key[P], rank[P];
#pragma unroll
    for (int q = 0; q < P; q++) {
        const int v = lane + 64 * q;
        pv[q] = 0;
        key[q] = 0x7fffffff;
        rank[q] = 0;
        if (v < nv) {
            const uint32_t g = vlist[v];
            const int i = g & 1023, j = (g >> 10) & 1023, k = (g >> 20) & 1023, t = g >> 30;
            pv[q] = pack_dbl(2 * i + (t != 0), 2 * j + (t != 1), 2 * k + (t != 2));
            key[q] = ((k * L1 + j) * L0 + i) * 3 + t;
        }
    }
#pragma unroll
    for (int qq = 0; qq < P; qq++) {
        const int n_q = nv - 64 * qq < 64 ? nv - 64 * qq : 64;
        for (int l = 0; l < n_q; l++) {
            const int kv = __builtin_amdgcn_readlane(key[qq], l);
#pragma unroll
            for (int q = 0; q < P; q++) rank[q] += kv < key[q] ? 1 : 0;
        }
    }
    wave_lds_fence();
#pragma unroll
    for (int q = 0; q < P; q++)
        if (lane + 64 * q < nv) vlist[rank[q]] = pv[q];
    wave_lds_fence();
}

// Runs the call: exactly min_hops hops, stopping early when the next event
// would land after t + t_sync (t_sync > 0; the clock then takes that value
// and the draw is spent) or no event is possible.  Draw d uses Philox
// counter (d_lo, d_hi, 0xFFFFFFFF, 3); draws are computed 64 ahead, one per
// lane.  vlist holds the nv vacancies (i | j << 10 | k << 20 | t << 30) and
// is rewritten here as the packed doubled coordinates of each slot.
//
// The 8P events of lane l's slots are entries l*8P .. l*8P+8P-1 of the rate
// table, in event order.  Each lane keeps the total of its block and the
// inclusive prefix of the block totals over the lanes, so a selection is
// one ballot over the prefixes (the block), one read of the block's rates
// into lanes 0 .. 8P-1, their prefix sum and a second ballot (the event).
// HZ: the call has a horizon (t_sync > 0), so every step needs its clock.
// Without one, a step records its total rate in the lane of its draw, and
// the clock takes the steps' increments -ln(u)/R every 64 steps (and at the
// end), one division for all of them and the additions in step order: the
// same operations in the same order, with the divisions off the path from
// one selection to the next.
template <int P, bool HZ>
__device__ __forceinline__ void solo_plain(const LatDesc& D, uint32_t* ps, uint32_t* vlist, int nv,
                                           double* krate, unsigned char* kspec, const RateCtx& C, int4* disp,
                                           LatState* St, const LatCall* Cl, int lane)
{
    constexpr int NE = 8 * P;  // events per block
    // descriptor fields in registers: the loop stores to global memory, so
    // fields read through D would be loaded again (and waited for) each step
    const int L0 = D.L[0], L1 = D.L[1], L2 = D.L[2];
    const int64_t disp_off = D.disp_off;
    const uint32_t seed = D.seed, lid = D.lattice_id;
    // slot = canonical rank at call start
    plain_rank_slots<P>(vlist, nv, L0, L1, lane);
    // the rates of every slot (zero past the last vacancy: a block read
    // covers whole blocks) and the block totals
    double bsum = 0.0;
#pragma nounroll
    for (int q = 0; q < P; q++) {
        const int sidx = lane * P + q;
        const bool v = sidx < nv;
        const uint32_t p = v ? vlist[sidx] : 0u;
#pragma nounroll
        for (int d = 0; d < 8; d++) {
            double k = 0.0;
            int sp = kSpV;
            if (v) {
                uint32_t np;
                int col;
                k = plain_rate_of(C, ps, plain_nb(C, p, d, np, col), col, sp);
            }
            krate[sidx * 8 + d] = k;
            kspec[sidx * 8 + d] = (unsigned char)sp;
            bsum += k;
        }
    }
    double bincl = wave_scan_dpp(bsum);
    double R = lane_value(bincl, 63);
    PlainRec pr;
    pr.cur = -1;
    pr.orig = 0;
    pr.ax = pr.ay = pr.az = 0;
    pr.n = 0;
    pr.pending = false;
    double t = St->t;
    uint64_t draws = St->draws;
    const double horizon = Cl->t_sync;
    const double t_end = t + horizon;
    const uint64_t target = Cl->min_hops;
    uint64_t done = 0;
    unsigned long long ho = 0, hh = 0;
    int sl = 64;
    double dr_sel = 0.0, dr_ln = 0.0;  // draw sl + (draws at the refill) is in lane sl
    double r_step = 0.0;               // (no horizon) total rate of the step that used this lane's draw
    int n_pend = 0;                    // (no horizon) steps whose clock increment is pending
    auto settle = [&]() {
        const double dtl = -dr_ln / r_step;
        for (int l = 0; l < n_pend; l++) t += lane_value(dtl, l);
        n_pend = 0;
    };
    while (done < target) {
        if (R == 0.0) break;
        if (sl == 64) {
            if (!HZ) settle();
            const uint64_t di = draws + (uint64_t)lane;
            uint32_t x0, x1, x2, x3;
            philox10((uint32_t)di, (uint32_t)(di >> 32), 0xFFFFFFFFu, 3u, seed, lid, x0, x1, x2, x3);
            dr_sel = u53_lo(x0, x1);
            dr_ln = clock_ln(u53_hi(x2, x3));
            sl = 0;
        }
        const double u_sel = lane_value(dr_sel, sl);
        if (HZ) {
            const double tn = t + -lane_value(dr_ln, sl) / R;
            if (tn > t_end) {
                t = t_end;
                draws++;
                break;
            }
            t = tn;
        } else {
            r_step = lane == sl ? R : r_step;
            n_pend++;
        }
        sl++;
        draws++;
        // the event whose inclusive prefix first exceeds y: its block from
        // one ballot, then the event inside the block from a second; when y
        // rounded up to R, the last event with a positive rate
        // (both ballots of each choice are taken, and the choice is a
        // select: the step runs without branches)
        const double y = u_sel * R;
        const uint64_t mb = __ballot(bincl > y);
        const uint64_t nzb = __ballot(bsum > 0.0);
        const bool fb = mb == 0;
        const int r = fb ? 63 - __clzll((long long)nzb) : __ffsll((unsigned long long)mb) - 1;
        const double c0 = lane_value(bincl, r) - lane_value(bsum, r);
        // lane l < NE: event l of the block (its slot's position, rate and
        // target species); every lane reads inside the block (lanes past NE
        // repeat it and are masked by value), and a slot past the last
        // vacancy, whose events have zero rates, takes position 0
        const int eb = r * NE;
        const int le = lane & (NE - 1);
        const bool in_blk = NE == 64 || lane < NE;
        const double kraw = krate[eb + le];
        const double kv = in_blk ? kraw : 0.0;
        const int kspv = (int)kspec[eb + le];
        const int slot_l = r * P + (le >> 3);
        const uint32_t pv_l = vlist[slot_l];
        const uint32_t pos = slot_l < nv ? pv_l : 0u;
        // every lane works out its event's target while the scan runs: the
        // selected one is then read from its lane
        uint32_t np_l;
        int col_l, hx_l, hy_l, hz_l;
        const int ct_l = plain_nb(C, pos, le & 7, np_l, col_l, hx_l, hy_l, hz_l);
        const int cs_l = canon_dbl(L0, L1, pos & 2047, (pos >> 11) & 2047, pos >> 22);
        const int hv_l = (hx_l + 1) | ((hy_l + 1) << 2) | ((hz_l + 1) << 4);
        const double cs = seg_scan<NE>(kv, le) + c0;
        const uint64_t me = __ballot(in_blk && cs > y);
        const uint64_t nze = __ballot(in_blk && kv > 0.0);
        const int e = !fb && me ? __ffsll((unsigned long long)me) - 1 : 63 - __clzll((long long)nze);
        const int j = e >> 3;
        const int slot = r * P + j;
        const int sp = __builtin_amdgcn_readlane(kspv, e);
        // the slot's old total: its 8 events in the block's prefix sum
        const double cs_hi = lane_value(cs, (j << 3) | 7), cs_lo = lane_value(cs, j ? (j << 3) - 1 : 0);
        const double tot_old = cs_hi - (j ? cs_lo : c0);
        const uint32_t sx = (uint32_t)__builtin_amdgcn_readlane((int)pos, e);
        const uint32_t tx = (uint32_t)__builtin_amdgcn_readlane((int)np_l, e);
        const int ct_i = __builtin_amdgcn_readlane(ct_l, e);
        const int cs_i = __builtin_amdgcn_readlane(cs_l, e);
        const int hv = __builtin_amdgcn_readlane(hv_l, e);
        const int hx = (hv & 3) - 1, hy = ((hv >> 2) & 3) - 1, hz = ((hv >> 4) & 3) - 1;
        if (lane == 0) {
            pk_set(ps, cs_i, sp);
            pk_set(ps, ct_i, kSpV);
            vlist[slot] = tx;
        }
        if (sp == kSpO) ho++;
        else hh++;
        prec_hop(pr, disp, disp_off, L0, L1, L2, lane, cs_i, ct_i, hx, hy, hz);
        done++;
        // one pass over the neighbours of both sites: lanes 0-7 around the
        // moved vacancy's new site (its new rates), lanes 8-15 around its old
        // site (now the ion); a vacancy there (other than the mover) has
        // changed events
        uint32_t nb = 0;
        int spn = kSpO;
        double kn = 0.0;
        if (lane < 16) {
            int col;
            const int cn = plain_nb(C, lane < 8 ? tx : sx, lane & 7, nb, col);
            // (the rate table entries in all 16 lanes: read with the
            // occupancy word, one LDS round trip)
            kn = plain_rate_of(C, ps, cn, col, spn);
        }
        kn = lane < 8 ? kn : 0.0;
        if (lane < 8) {
            krate[slot * 8 + lane] = kn;
            kspec[slot * 8 + lane] = (unsigned char)spn;
        }
        {
            const double delta = lane_value(seg_scan<8>(kn, lane & 7), 7) - tot_old;
            if (lane == r) bsum += delta;
            if (lane >= r) bincl += delta;
            R += delta;
        }
        uint64_t aff = __ballot(lane < 16 && spn == kSpV && nb != tx);
        while (aff) {
            const int l = __ffsll((unsigned long long)aff) - 1;
            aff &= aff - 1;
            const uint32_t pa = (uint32_t)__builtin_amdgcn_readlane((int)nb, l);
            // its slot, from the lanes' slot positions
            int hit = -1;
#pragma unroll
            for (int q = 0; q < P; q++)
                if (lane * P + q < nv && vlist[lane * P + q] == pa) hit = q;
            const uint64_t m = __ballot(hit >= 0);
            if (m) {
                const int al = __ffsll((unsigned long long)m) - 1;
                const int a = al * P + __builtin_amdgcn_readlane(hit, al);
                const double ko = lane < 8 ? krate[a * 8 + lane] : 0.0;
                const double old = lane_value(seg_scan<8>(ko, lane & 7), 7);
                const double dl = plain_slot_rates(C, ps, krate, kspec, a, pa, lane) - old;
                if (lane == al) bsum += dl;
                if (lane >= al) bincl += dl;
                R += dl;
            }
        }
    }
    if (!HZ) settle();
    prec_flush(pr, disp, disp_off, L0, L1, L2);
    if (lane == 0) {
        St->t = t;
        St->draws = draws;
        St->hops[0] += ho;
        St->hops[1] += hh;
    }
}

template <int P>
__device__ __forceinline__ void solo_plain_call(const LatDesc& D, uint32_t* ps, uint32_t* vlist, int nv,
                                                double* krate, unsigned char* kspec, const RateCtx& C,
                                                int4* disp, LatState* St, const LatCall* Cl, int lane)
{
    if (Cl->t_sync > 0.0) solo_plain<P, true>(D, ps, vlist, nv, krate, kspec, C, disp, St, Cl, lane);
    else solo_plain<P, false>(D, ps, vlist, nv, krate, kspec, C, disp, St, Cl, lane);
}

// ----------------------------------------------------------------------------
// Atom-selection fragment kMC with null events (Sec. "Atomic-based fragment
// kMC method", Eqs. AtomP and TimeStepFrg) on a plain lattice held in LDS,
// one wave.  An atom is a vacancy (its 8 hops are its events).  A stage:
//  - every slot's 8 rates at the start of the stage into the rate table;
//    the total K = sum_i k_i and R^max = max over slots of the slot total;
//  - lane j < n_frg selects slot a = floor(x0 nv / 2^32) from Philox counter
//    (stage_lo, stage_hi, j, 4), and its first event whose cumulative rate
//    exceeds u R^max (u from x2, x3, in [0,1)), or a null event;
//  - the events are taken in selection order; one whose vacancy or target
//    site an earlier taken event of the stage touched becomes null;
//  - the clock moves by N_updated (-ln r') / K, r' from counter
//    (stage_lo, stage_hi, 0xFFFFFFFF, 4), u in (0,1].
// Slots are the vacancies in canonical order at the call start, following
// their vacancies; the stage counter is the lattice's draw counter.  Runs
// n_stages stages, fewer when no event is possible.
// Hashed bit of cell (i, j, k) in a mark bitmap of 2^B bits.
template <int B>
__device__ __forceinline__ uint32_t cell_mark_bit(int i, int j, int k)
{
    return ((uint32_t)i * 0x9E3779B1u ^ (uint32_t)j * 0x85EBCA77u ^ (uint32_t)k * 0xC2B2AE3Du) >> (32 - B);
}

// Mark the cells that hold the neighbours of the site at doubled coordinates
// (X, Y, Z): a neighbour differs by one in two of them, so along each axis
// it lies in cell (X-1)/2 or (X+1)/2 (periodic), 8 cells in all.
template <int B>
__device__ __forceinline__ void mark_neighbour_cells(uint32_t* marks, int L0, int L1, int L2, int X, int Y,
                                                     int Z)
{
    const int x0 = (X == 0 ? 2 * L0 - 1 : X - 1) >> 1, x1 = (X + 1 == 2 * L0 ? 0 : X + 1) >> 1;
    const int y0 = (Y == 0 ? 2 * L1 - 1 : Y - 1) >> 1, y1 = (Y + 1 == 2 * L1 ? 0 : Y + 1) >> 1;
    const int z0 = (Z == 0 ? 2 * L2 - 1 : Z - 1) >> 1, z1 = (Z + 1 == 2 * L2 ? 0 : Z + 1) >> 1;
#pragma unroll
    for (int c = 0; c < 8; c++) {
        const uint32_t h = cell_mark_bit<B>(c & 1 ? x1 : x0, c & 2 ? y1 : y0, c & 4 ? z1 : z0);
        atomicOr(marks + (h >> 5), 1u << (h & 31));
    }
}

template <int P>
__device__ __forceinline__ void atomic_stages(const LatDesc& D, uint32_t* ps, uint32_t* vlist, int nv,
                                              double* krate, unsigned char* kspec, double* stot,
                                              uint32_t* marks, uint16_t* fresh, const RateCtx& C,
                                              int4* disp, LatState* St,
                                              uint32_t n_frg, uint64_t n_stages, int lane)
{
    const int L0 = D.L[0], L1 = D.L[1], L2 = D.L[2];
    const int64_t disp_off = D.disp_off;
    const uint32_t seed = D.seed, lid = D.lattice_id;
    plain_rank_slots<P>(vlist, nv, L0, L1, lane);
    PlainRec pr;
    pr.cur = -1;
    pr.orig = 0;
    pr.ax = pr.ay = pr.az = 0;
    pr.n = 0;
    pr.pending = false;
    double t = St->t;
    uint64_t stage = St->draws;
    unsigned long long ho = 0, hh = 0;
    // the 8 rates and the total of slot sidx (zero past the last vacancy)
    auto slot_rates = [&](int sidx) {
        const bool v = sidx < nv;
        const uint32_t p = v ? vlist[sidx] : 0u;
        double ri = 0.0;
#pragma nounroll
        for (int d = 0; d < 8; d++) {
            double kd = 0.0;
            int sp = kSpV;
            if (v) {
                uint32_t np;
                int col;
                kd = plain_rate_of(C, ps, plain_nb(C, p, d, np, col), col, sp);
            }
            krate[sidx * 8 + d] = kd;
            kspec[sidx * 8 + d] = (unsigned char)sp;
            ri += kd;
        }
        stot[sidx] = ri;
    };
#pragma nounroll
    for (int q = 0; q < P; q++) slot_rates(lane * P + q);
    for (int w = lane; w < 2 * kAtomMarkWords; w += 64) marks[w] = 0u;
    wave_lds_order();
    for (uint64_t k = 0; k < n_stages; k++) {
        // rates at the start of the stage: new ones for the slots in cells
        // the last stage marked
        if (k > 0) {
            // list them (ballot prefix), then recompute the list densely
            const uint32_t* seen = marks + ((k + 1) & 1) * kAtomMarkWords;
            int nf = 0;
#pragma nounroll
            for (int q = 0; q < P; q++) {
                const int sidx = lane * P + q;
                bool f = false;
                if (sidx < nv) {
                    const uint32_t p = vlist[sidx];
                    const uint32_t h = cell_mark_bit<kAtomMarkBits>(
                        (int)((p & 2047) >> 1), (int)(((p >> 11) & 2047) >> 1), (int)(p >> 23));
                    f = (seen[h >> 5] >> (h & 31)) & 1u;
                }
                const uint64_t fm = __ballot(f);
                if (f) fresh[nf + __popcll(fm & ((1ull << lane) - 1ull))] = (uint16_t)sidx;
                nf += __popcll(fm);
            }
            wave_lds_order();
#pragma nounroll
            for (int x = lane; x < nf; x += 64) slot_rates(fresh[x]);
            wave_lds_order();
        }
        double lsum = 0.0, lmax = 0.0;
#pragma nounroll
        for (int q = 0; q < P; q++) {
            const double ri = stot[lane * P + q];
            lsum += ri;
            lmax = fmax(lmax, ri);
        }
        const double K = lane_value(wave_scan_dpp(lsum), 63);
        const double Rmax = lane_value(wave_max_dpp(lmax), 63);
        if (K == 0.0) break;
        // the last stage's marks are read: clear them for the next
        for (int w = lane; w < kAtomMarkWords; w += 64) marks[((k + 1) & 1) * kAtomMarkWords + w] = 0u;
        wave_lds_order();
        // selection j in lane j: an atom, then its event or a null event
        int a = 0, e = -1;
        if ((uint32_t)lane < n_frg) {
            uint32_t x0, x1, x2, x3;
            philox10((uint32_t)stage, (uint32_t)(stage >> 32), (uint32_t)lane, 4u, seed, lid, x0, x1, x2,
                     x3);
            a = (int)(((uint64_t)x0 * (uint64_t)(uint32_t)nv) >> 32);
            const double y = u53_lo(x2, x3) * Rmax;
            double cum = 0.0;
#pragma unroll
            for (int d = 0; d < 8; d++) {
                cum += krate[a * 8 + d];
                if (e < 0 && cum > y) e = d;
            }
        }
        const bool ev = e >= 0;
        uint32_t tx = 0;
        int cs = -1, ct = -1, sp = kSpO, hx = 0, hy = 0, hz = 0;
        if (ev) {
            const uint32_t sx = vlist[a];
            int col;
            ct = plain_nb(C, sx, e, tx, col, hx, hy, hz);
            cs = canon_dbl(L0, L1, sx & 2047, (sx >> 11) & 2047, sx >> 22);
            sp = kspec[a * 8 + e];
        }
        // conflicts, in selection order
        bool taken = false;
        uint64_t evm = __ballot(ev);
        while (evm) {
            const int j = __ffsll((unsigned long long)evm) - 1;
            evm &= evm - 1;
            const int sj = __builtin_amdgcn_readlane(cs, j), tj = __builtin_amdgcn_readlane(ct, j);
            const bool hit = __ballot(taken && (cs == sj || cs == tj || ct == sj || ct == tj)) != 0;
            if (!hit && lane == j) taken = true;
        }
        wave_lds_order();
        if (taken) {
            pk_set(ps, cs, sp);
            pk_set(ps, ct, kSpV);
            const uint32_t sx = vlist[a];
            vlist[a] = tx;
            uint32_t* mark = marks + (k & 1) * kAtomMarkWords;
            mark_neighbour_cells<kAtomMarkBits>(mark, L0, L1, L2, (int)(sx & 2047), (int)((sx >> 11) & 2047),
                                                (int)(sx >> 22));
            mark_neighbour_cells<kAtomMarkBits>(mark, L0, L1, L2, (int)(tx & 2047), (int)((tx >> 11) & 2047),
                                                (int)(tx >> 22));
        }
        uint64_t tm = __ballot(taken);
        const int n_upd = __popcll(tm);
        const int n_o = __popcll(__ballot(taken && sp == kSpO));
        ho += (unsigned long long)n_o;
        hh += (unsigned long long)(n_upd - n_o);
        while (tm) {
            const int j = __ffsll((unsigned long long)tm) - 1;
            tm &= tm - 1;
            prec_hop(pr, disp, disp_off, L0, L1, L2, lane, __builtin_amdgcn_readlane(cs, j),
                     __builtin_amdgcn_readlane(ct, j), __builtin_amdgcn_readlane(hx, j),
                     __builtin_amdgcn_readlane(hy, j), __builtin_amdgcn_readlane(hz, j));
        }
        // Eq. TimeStepFrg
        {
            uint32_t x0, x1, x2, x3;
            philox10((uint32_t)stage, (uint32_t)(stage >> 32), 0xFFFFFFFFu, 4u, seed, lid, x0, x1, x2, x3);
            const double dt = -clock_ln(u53_hi(x2, x3)) / K;
            t = t + dt * (double)n_upd;
        }
        stage++;
        wave_lds_order();
    }
    prec_flush(pr, disp, disp_off, L0, L1, L2);
    if (lane == 0) {
        St->t = t;
        St->draws = stage;
        St->hops[0] += ho;
        St->hops[1] += hh;
    }
}

// One workgroup per plain lattice of `ids`: the occupancy is packed into LDS
// by every thread, wave 0 runs the stages, and every thread writes it back.
__global__ __launch_bounds__(256) void k_atomic(DevPtrs P, const int32_t* ids, uint32_t n_frg,
                                                uint64_t n_stages)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int vlist_n;
    __shared__ double k12[12];
    const int lane = threadIdx.x & 63;
    const uint64_t t_begin = __builtin_amdgcn_s_memrealtime();
    const int lat = ids[blockIdx.x];
    const LatDesc& D = P.desc[lat];
    LatState* St = P.state + lat;
    int8_t* occ_lat = P.occ + D.occ_off;
    const int n_words = (int)((D.n_sites + 15) >> 4);
    uint32_t* pslab = (uint32_t*)smem;
    uint32_t* vlist = (uint32_t*)(smem + ((4 * n_words + 15) & ~15));
    const int slots = D.n_vac <= 64 ? 64 : (D.n_vac <= 128 ? 128 : (D.n_vac <= 256 ? 256 : 512));
    double* krate = (double*)(vlist + ((D.n_vac + 3) & ~3));
    unsigned char* kspec = (unsigned char*)(krate + 8 * slots);
    double* stot = (double*)(kspec + 8 * slots);
    uint32_t* marks = (uint32_t*)(stot + slots);
    uint16_t* fresh = (uint16_t*)(marks + 2 * kAtomMarkWords);
    if (threadIdx.x == 0) vlist_n = 0;
    if (threadIdx.x < 12) k12[threadIdx.x] = D.k12[threadIdx.x];
    __syncthreads();
    plain_pack_load(D, occ_lat, pslab, vlist, &vlist_n, D.n_vac);
    __syncthreads();
    const int nv = vlist_n < D.n_vac ? vlist_n : D.n_vac;
    if (threadIdx.x < 64) {
        const RateCtx C = {D.L[0], D.L[1], D.L[2], D.gb_period, D.gb_mask, k12};
        if (slots == 64)
            atomic_stages<1>(D, pslab, vlist, nv, krate, kspec, stot, marks, fresh, C, P.disp, St, n_frg, n_stages,
                             lane);
        else if (slots == 128)
            atomic_stages<2>(D, pslab, vlist, nv, krate, kspec, stot, marks, fresh, C, P.disp, St, n_frg, n_stages,
                             lane);
        else if (slots == 256)
            atomic_stages<4>(D, pslab, vlist, nv, krate, kspec, stot, marks, fresh, C, P.disp, St, n_frg, n_stages,
                             lane);
        else
            atomic_stages<8>(D, pslab, vlist, nv, krate, kspec, stot, marks, fresh, C, P.disp, St, n_frg, n_stages,
                             lane);
    }
    __syncthreads();
    plain_pack_store(D, occ_lat, pslab);
    if (threadIdx.x == 0) {
        if (vlist_n != D.n_vac) atomicOr(&St->err, 1u);
        St->busy_ticks = __builtin_amdgcn_s_memrealtime() - t_begin;
    }
}

// Persistent batched kernel: one workgroup per lattice runs the whole call
// (cycles of 8 phases, workgroup barrier between phases), so every lattice
// advances at its own pace.  A lattice that fits is kept in LDS for the
// whole call with a list of its vacancies; otherwise each wave stages its
// tiles' footprints from HBM.  Each wave runs groups of D.group tiles.  A
// lattice whose phase is one group runs on wave 0 alone, without barriers,
// and keeps its displacement records across phases.  Plain lattices held in
// LDS run plain BKL on wave 0.
template <bool MAP>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void k_batch(DevPtrs P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long hop_tot[2];
    __shared__ int vlist_n;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const uint64_t t_begin = __builtin_amdgcn_s_memrealtime();
    const int lat = P.batch_ids[blockIdx.x];
    const LatDesc& D = P.desc[lat];
    LatState* St = P.state + lat;
    const LatCall* Cl = P.call + lat;
    const bool resident = D.resident != 0;
    const int K = D.group;
    unsigned char* region = smem;
    const WaveLds W = wave_lds(smem + P.lds_region_bytes + wv * kWaveScratch);
    int8_t* occ_lat = P.occ + D.occ_off;
    const int64_t nbytes = D.n_sites;
    // resident slab: occupancy, vacancy list, cell -> sub-block maps
    uint32_t* vlist = (uint32_t*)(region + ((nbytes + 15) & ~(int64_t)15));
    unsigned char* c2s = (unsigned char*)(vlist + ((D.n_vac + 3) & ~3));
    if (threadIdx.x == 0) vlist_n = 0;
    const bool fast = D.fast != 0;
    // plain lattice held in LDS: 2 bits per site in canonical order (16
    // sites per word), then the vacancy list, the slots' rates and the
    // species of their targets
    const bool packed = fast && D.plain;
    const int n_words = (int)((nbytes + 15) >> 4);
    uint32_t* pslab = (uint32_t*)region;
    const int plain_slots = D.n_vac <= 64 ? 64 : (D.n_vac <= 128 ? 128 : (D.n_vac <= 256 ? 256 : 512));
    if (packed) {
        vlist = (uint32_t*)(region + ((4 * n_words + 15) & ~15));
        c2s = (unsigned char*)(vlist + ((D.n_vac + 3) & ~3));
    }
    __syncthreads();
    if (packed) {
        plain_pack_load(D, occ_lat, pslab, vlist, &vlist_n, D.n_vac);
    } else if (resident && fast) {
        // canonical order
        for (int64_t c = threadIdx.x; c < nbytes; c += blockDim.x) {
            const int t = (int)(c % 3);
            const int64_t cell = c / 3;
            const int i = (int)(cell % D.L[0]);
            const int j = (int)((cell / D.L[0]) % D.L[1]);
            const int k = (int)(cell / ((int64_t)D.L[0] * D.L[1]));
            region[c] = (unsigned char)occ_lat[store_index_1f(D.L[0], D.L[1], D.L[2], i, j, k, t)];
        }
    } else if (resident) {
        const int nch = (int)((nbytes + 15) >> 4);
        for (int j = threadIdx.x; j < nch; j += blockDim.x)
            ((uint4*)region)[j] = ((const uint4*)occ_lat)[j];
        const int32_t* m = P.c2s + D.c2s_off;
        for (int j = threadIdx.x; j < D.L[0] + D.L[1] + D.L[2]; j += blockDim.x)
            c2s[j] = (unsigned char)m[j];
    }
    __syncthreads();
    if (resident && !packed) {
        for (int64_t c = threadIdx.x; c < nbytes; c += blockDim.x) {
            const int t = (int)(c % 3);
            const int64_t cell = c / 3;
            const int i = (int)(cell % D.L[0]);
            const int j = (int)((cell / D.L[0]) % D.L[1]);
            const int k = (int)(cell / ((int64_t)D.L[0] * D.L[1]));
            if (region[fast ? c : store_index(D, P.bounds, P.c2s, i, j, k, t)] != kSpV) continue;
            const int v = atomicAdd(&vlist_n, 1);
            if (v < D.n_vac)
                vlist[v] = (uint32_t)i | ((uint32_t)j << 10) | ((uint32_t)k << 20) | ((uint32_t)t << 30);
        }
    }
    if (threadIdx.x < 2) hop_tot[threadIdx.x] = 0;
    if (lane < 12) W.k12[lane] = D.k12[lane];
    const int ntiles = D.nf[0] * D.nf[1] * D.nf[2];
    const int ngroups = (ntiles + K - 1) / K;
    const bool solo = ngroups == 1;
    // a lattice run by one wave keeps every colour's tile records in LDS
    TileRec* rcache = (TileRec*)(smem + P.lds_region_bytes + nw * kWaveScratch);
    if (solo && !D.plain)
        for (int j = threadIdx.x; j < 8 * ntiles; j += blockDim.x)
            rcache[j] = P.tiles[(size_t)(j / ntiles) * P.n_tiles + D.tile0 + j % ntiles];
    __syncthreads();
    const int nv_list = vlist_n < D.n_vac ? vlist_n : D.n_vac;
    bool err = resident && vlist_n > D.n_vac;
    GroupCall X;
    X.occ = occ_lat;
    X.disp = P.disp;
    X.disp_off = D.disp_off;
    X.seed = D.seed;
    X.lid = D.lattice_id;
    X.t_sync = Cl->t_sync;
    X.write_occ = !resident;
    const uint64_t max_cycles = Cl->max_cycles, min_hops = Cl->min_hops;
    const uint64_t cycle0 = St->cycles;
    unsigned char* occl = resident ? region : smem;
    const int fp = resident ? 0 : wv * (K == 1 ? 1 : K) * D.fp_stride;
    Rec rec;
    RecCtl rc;
    rec_init(rec, rc);
    uint64_t ncyc = 0;
    if (packed) {
        if (wv == 0) {
            const RateCtx C = {D.L[0], D.L[1], D.L[2], D.gb_period, D.gb_mask, W.k12};
            double* krate = (double*)c2s;
            unsigned char* kspec = (unsigned char*)(krate + 8 * plain_slots);
            if (plain_slots == 64)
                solo_plain_call<1>(D, pslab, vlist, nv_list, krate, kspec, C, P.disp, St, Cl, lane);
            else if (plain_slots == 128)
                solo_plain_call<2>(D, pslab, vlist, nv_list, krate, kspec, C, P.disp, St, Cl, lane);
            else if (plain_slots == 256)
                solo_plain_call<4>(D, pslab, vlist, nv_list, krate, kspec, C, P.disp, St, Cl, lane);
            else
                solo_plain_call<8>(D, pslab, vlist, nv_list, krate, kspec, C, P.disp, St, Cl, lane);
        }
    } else if (fast) {
        if (wv == 0) {
            const RateCtx C = {D.L[0], D.L[1], D.L[2], D.gb_period, D.gb_mask, W.k12};
            unsigned long long fo = 0, fh = 0;
            solo_fast(D, region, vlist, nv_list, C, X, max_cycles, min_hops, cycle0, lane, ncyc, fo, fh, rec,
                      rc);
            if (lane == 0) {
                hop_tot[0] = fo;
                hop_tot[1] = fh;
            }
        }
    } else if (!solo || wv == 0) {
        while (ncyc < max_cycles) {
            X.cycle = (uint32_t)(cycle0 + ncyc);
            for (int colour = 0; colour < 8; colour++) {
                X.ctag = ((uint32_t)colour << 8) | 2u;
                uint32_t ho = 0, hh = 0;
                for (int g = wv; g < ngroups; g += nw) {
                    const int f0 = g * K;
                    const int nt = ntiles - f0 < K ? ntiles - f0 : K;
                    if (K == 4)
                        run_group<4, 8, true, MAP>(P, D, f0, nt, colour, X, W, occl, fp, D.fp_stride, resident, false,
                                        vlist, nv_list, c2s, solo ? rcache + colour * ntiles : nullptr,
                                        lane, rec, rc, ho, hh, err);
                    else
                        run_group<8, 8, true, MAP>(P, D, f0, nt, colour, X, W, occl, fp, D.fp_stride, resident, K == 1,
                                        vlist, nv_list, c2s, solo ? rcache + colour * ntiles : nullptr,
                                        lane, rec, rc, ho, hh, err);
                }
                // per-lane counts of segment leaders to the workgroup totals
                if (ho) atomicAdd(&hop_tot[0], (unsigned long long)ho);
                if (hh) atomicAdd(&hop_tot[1], (unsigned long long)hh);
                if (solo) {
                    wave_lds_fence();
                } else {
                    rec_flush(rec, rc, P.disp);
                    __syncthreads();
                    rc.pending = false;  // the barrier waited for every store
                }
            }
            ncyc++;
            const unsigned long long tot = hop_tot[0] + hop_tot[1];
            if (!solo) __syncthreads();
            if (min_hops > 0 && tot >= min_hops) break;
        }
    }
    rec_flush(rec, rc, P.disp);
    __syncthreads();
    if (packed) {
        plain_pack_store(D, occ_lat, pslab);
    } else if (resident && fast) {
        for (int64_t c = threadIdx.x; c < nbytes; c += blockDim.x) {
            const int t = (int)(c % 3);
            const int64_t cell = c / 3;
            const int i = (int)(cell % D.L[0]);
            const int j = (int)((cell / D.L[0]) % D.L[1]);
            const int k = (int)(cell / ((int64_t)D.L[0] * D.L[1]));
            occ_lat[store_index_1f(D.L[0], D.L[1], D.L[2], i, j, k, t)] = (int8_t)region[c];
        }
    } else if (resident) {
        const int nch = (int)(nbytes >> 4);
        for (int j = threadIdx.x; j < nch; j += blockDim.x)
            ((uint4*)occ_lat)[j] = ((const uint4*)region)[j];
        for (int64_t b = (int64_t)nch * 16 + threadIdx.x; b < nbytes; b += blockDim.x)
            occ_lat[b] = (int8_t)region[b];
    }
    if (__ballot(err) && lane == 0) atomicOr(&St->err, 1u);
    if (threadIdx.x == 0) {
        St->busy_ticks = __builtin_amdgcn_s_memrealtime() - t_begin;
        St->cycles = cycle0 + ncyc;
        St->done = 1u;
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

__device__ __forceinline__ int64_t plain_store(const LatDesc& D, int i, int j, int k, int t)
{
    return plain_offset(D.L[0], D.L[1], D.L[2], i, j, k, t);
}

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
    tgt_store = plain_store(D, X >> 1, Y >> 1, Z >> 1, tt);
    const int sp = P.occ[D.occ_off + tgt_store];
    if (sp == kSpV) return 0.0;
    const int cs = t == 0 ? i : (t == 1 ? j : k);
    const int ct = tt == 0 ? (X >> 1) : (tt == 1 ? (Y >> 1) : (Z >> 1));
    const int g = edge_gb(D, i, j, k, t, X >> 1, Y >> 1, Z >> 1, tt, cs, ct);
    return D.k12[(sp * 3 + hz + 1) * 2 + g];
}

// Periodic nearest neighbours among packed cell/type positions.
__device__ __forceinline__ bool plain_adjacent(const LatDesc& D, uint64_t a, uint64_t b)
{
    const int ta = (int)(a >> 48), tb = (int)(b >> 48);
    int dX = (2 * (int)(a & 0xffff) + (ta != 0)) - (2 * (int)(b & 0xffff) + (tb != 0));
    int dY = (2 * (int)((a >> 16) & 0xffff) + (ta != 1)) - (2 * (int)((b >> 16) & 0xffff) + (tb != 1));
    int dZ = (2 * (int)((a >> 32) & 0xffff) + (ta != 2)) - (2 * (int)((b >> 32) & 0xffff) + (tb != 2));
    dX = dX < 0 ? -dX : dX;
    dY = dY < 0 ? -dY : dY;
    dZ = dZ < 0 ? -dZ : dZ;
    if (dX == 2 * D.L[0] - 1) dX = 1;
    if (dY == 2 * D.L[1] - 1) dY = 1;
    if (dZ == 2 * D.L[2] - 1) dZ = 1;
    return dX * dX + dY * dY + dZ * dZ == 2;
}

// Each thread owns a contiguous range of slots; the total rate of every
// slot is kept in LDS, so a step sums m <= 32 totals per thread, scans the
// workgroup, evaluates the 8 rates of the selected slot only, and after the
// hop re-evaluates just the slots next to its two sites.
// Vacancy slots of a plain lattice in ascending canonical index, as packed
// cell/type positions (at most cap are stored); every thread of the
// workgroup calls it and gets the vacancy count.
__device__ int plain_collect_slots(const LatDesc& D, const DevPtrs& P, uint64_t* slots, int* wcount,
                                   int* n_sh, int tid, int cap)
{
    const int lane = tid & 63, wv = tid >> 6;
    constexpr int NW = kPlainThreads / 64;
    if (tid == 0) *n_sh = 0;
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
            v = P.occ[D.occ_off + plain_store(D, i, j, k, t)] == kSpV;
            pk = (uint64_t)i | ((uint64_t)j << 16) | ((uint64_t)k << 32) | ((uint64_t)t << 48);
        }
        const uint64_t mk = __ballot(v);
        if (lane == 0) wcount[wv] = __popcll(mk);
        __syncthreads();
        int before = *n_sh;
        for (int w = 0; w < wv; w++) before += wcount[w];
        if (v) {
            const int r = before + __popcll(mk & ((1ull << lane) - 1ull));
            if (r < cap) slots[r] = pk;
        }
        __syncthreads();
        if (tid == 0) {
            int tot = 0;
            for (int w = 0; w < NW; w++) tot += wcount[w];
            *n_sh += tot;
        }
        __syncthreads();
    }
    return *n_sh;
}

__global__ __launch_bounds__(kPlainThreads) void k_plain(DevPtrs P, const int32_t* ids, int cap)
{
    extern __shared__ __align__(16) unsigned char psm[];
    uint64_t* slots = (uint64_t*)psm;                     // [cap]
    double* stot = (double*)(psm + 8 * (size_t)cap);      // [cap]
    __shared__ int wcount[kPlainThreads / 64];
    __shared__ double wsum[kPlainThreads / 64];
    __shared__ uint64_t wmask[kPlainThreads / 64];
    __shared__ uint64_t wnz[kPlainThreads / 64];
    __shared__ int n_sh;
    __shared__ int ev_sh;
    __shared__ int hop_slot;
    __shared__ uint64_t hop_s, hop_t;  // packed positions of the hop's two sites
    const uint64_t t_begin = __builtin_amdgcn_s_memrealtime();
    const int lat = ids[blockIdx.x];
    const LatDesc& D = P.desc[lat];
    LatState* S = P.state + lat;
    const LatCall* C = P.call + lat;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int NW = kPlainThreads / 64;

    const int n = plain_collect_slots(D, P, slots, wcount, &n_sh, tid, cap);
    if (n > cap) {
        if (tid == 0) atomicOr(&S->err, 1u);
        return;
    }
    const int m = (n + kPlainThreads - 1) / kPlainThreads;
    const int s0 = tid * m < n ? tid * m : n;
    const int s1 = s0 + m < n ? s0 + m : n;
    auto slot_total = [&](int sidx) {
        double r = 0.0;
        for (int d = 0; d < 8; d++) {
            int64_t ts;
            r += plain_rate(D, P, slots[sidx], d, ts);
        }
        return r;
    };
    for (int sidx = s0; sidx < s1; sidx++) stot[sidx] = slot_total(sidx);
    __syncthreads();
    double t = S->t;
    uint64_t draws = S->draws;
    const double horizon = C->t_sync;
    const double t_end = t + horizon;
    const uint64_t target = C->min_hops;
    uint64_t done = 0, ho = 0, hh = 0;
    while (done < target) {
        double ls = 0.0;
        for (int sidx = s0; sidx < s1; sidx++) ls += stot[sidx];
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
            // the slot, then the direction, where the cumulative rate first exceeds y
            double Cc = incl - ls;
            int sp_slot = -1, last = -1;
            for (int sidx = s0; sidx < s1; sidx++) {
                if (stot[sidx] > 0.0) last = sidx;
                if (!fallback && sp_slot < 0 && Cc + stot[sidx] > y) {
                    sp_slot = sidx;
                    break;
                }
                Cc += stot[sidx];
            }
            if (sp_slot < 0) sp_slot = last;
            const uint64_t pk = slots[sp_slot];
            int dsel = -1, dlast = -1;
            for (int d = 0; d < 8; d++) {
                int64_t ts;
                const double k = plain_rate(D, P, pk, d, ts);
                if (k > 0.0) dlast = d;
                Cc += k;
                if (!fallback && dsel < 0 && Cc > y) dsel = d;
            }
            const int d = dsel >= 0 ? dsel : dlast;
            int64_t ts;
            plain_rate(D, P, pk, d, ts);
            const int i = (int)(pk & 0xffff), j = (int)((pk >> 16) & 0xffff), k = (int)((pk >> 32) & 0xffff);
            const int tp = (int)(pk >> 48);
            const int64_t ss = plain_store(D, i, j, k, tp);
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
            const uint64_t npk = (uint64_t)(X >> 1) | ((uint64_t)(Y >> 1) << 16) |
                                 ((uint64_t)(Z >> 1) << 32) | ((uint64_t)site_type(X, Y) << 48);
            slots[sp_slot] = npk;
            hop_slot = sp_slot;
            hop_s = pk;
            hop_t = npk;
            ev_sh = sp;
        }
        // the barrier's workgroup-scope fence makes the hop's HBM writes
        // visible to every wave of this workgroup, the only readers
        __syncthreads();
        if (ev_sh == kSpO) ho++;
        else hh++;
        done++;
        // slots whose events changed: the moved vacancy and those next to its two sites
        const uint64_t ps = hop_s, pt = hop_t;
        const int mv = hop_slot;
        for (int sidx = s0; sidx < s1; sidx++)
            if (sidx == mv || plain_adjacent(D, slots[sidx], ps) || plain_adjacent(D, slots[sidx], pt))
                stot[sidx] = slot_total(sidx);
        __syncthreads();
    }
    if (tid == 0) {
        S->t = t;
        S->draws = draws;
        S->hops[0] += ho;
        S->hops[1] += hh;
        S->busy_ticks = __builtin_amdgcn_s_memrealtime() - t_begin;
    }
}

// ----------------------------------------------------------------------------
// Plain BKL with site-energy interactions (Sec. "Oxygen vacancy diffusion
// with dopant and defect interaction", Table TABLEadd01): the hop rate is
// k = A exp(-(Ea + dE_site/2 + field and boundary terms)/(k_B T)), with
// dE_site the vacancy's site energy at the target (without itself at the
// origin) minus that at the origin.  A site energy sums the pair energies
// (integers in meV) of the Fe dopants on B sites within squared doubled
// distance 1, 5, 9, 13 and of the other vacancies on O sites within 2, 4, 6,
// 8, 10, 16.  The host tabulates every rate as the quantised product of the
// Arrhenius rate and exp(-dE/(2 k_B T)) for |dE| <= window, so sums stay
// exact and a rate is one table entry.  One workgroup per lattice, the
// occupancy in HBM; per vacancy slot the LDS holds its position, its total
// rate and the table indices of its 8 events.  A slot's events are
// evaluated by the whole workgroup: 9 site energies (origin and 8 targets)
// over 92 lattice points each, summed with LDS integer atomics.  After a hop
// only the slots within squared doubled distance 29 of its two sites (the
// reach of an energy change onto a slot's origin or targets) are evaluated
// again.  Draws, clock and selection are those of plain BKL (k_plain).
constexpr int kSiteOffsets = 96;  // interacting lattice points around an anion site (92)

__device__ __forceinline__ int site_shell(bool bsite, int n)
{
    if (bsite) return n == 1 ? 0 : (n == 5 ? 1 : (n == 9 ? 2 : (n == 13 ? 3 : -1)));
    return n == 2 ? 0 : (n == 4 ? 1 : (n == 6 ? 2 : (n == 8 ? 3 : (n == 10 ? 4 : (n == 16 ? 5 : -1)))));
}

__device__ __forceinline__ int wrap2(int v, int L2)
{
    v = v < 0 ? v + L2 : v;
    return v >= L2 ? v - L2 : v;
}

// Squared doubled distance between two packed plain positions (minimum image).
__device__ __forceinline__ int plain_dist2(const LatDesc& D, uint64_t a, uint64_t b)
{
    const int ta = (int)(a >> 48), tb = (int)(b >> 48);
    int d[3];
    d[0] = (2 * (int)(a & 0xffff) + (ta != 0)) - (2 * (int)(b & 0xffff) + (tb != 0));
    d[1] = (2 * (int)((a >> 16) & 0xffff) + (ta != 1)) - (2 * (int)((b >> 16) & 0xffff) + (tb != 1));
    d[2] = (2 * (int)((a >> 32) & 0xffff) + (ta != 2)) - (2 * (int)((b >> 32) & 0xffff) + (tb != 2));
    int r = 0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        int v = d[k] < 0 ? -d[k] : d[k];
        const int L2 = 2 * D.L[k];
        v = v > L2 - v ? L2 - v : v;
        r += v * v;
    }
    return r;
}

// The interacting lattice points of each anion type as packed offsets (the
// order is irrelevant: the energies are integer sums); n_off zeroed and
// published by the caller's barriers.  Every thread of the workgroup calls it.
__device__ __forceinline__ void site_offsets(const LatDesc& D, uint16_t* offs, int* n_off, int tid)
{
    for (int c = tid; c < 729; c += kPlainThreads) {
        const int dX = c % 9 - 4, dY = (c / 9) % 9 - 4, dZ = c / 81 - 4;
        const int n = dX * dX + dY * dY + dZ * dZ;
        if (n == 0 || n > 16) continue;
        for (int t = 0; t < 3; t++) {
            const int odd = ((t != 0) + dX) & 1;
            const int odd_y = ((t != 1) + dY) & 1;
            const int odd_z = ((t != 2) + dZ) & 1;
            const int nodd = odd + odd_y + odd_z;
            const bool bsite = nodd == 3;
            if (nodd < 2) continue;
            const int sh = site_shell(bsite, n);
            if (sh < 0) continue;
            const int e = bsite ? D.site_e_fe[sh] : D.site_e_vv[sh];
            if (e == 0) continue;
            const int k = atomicAdd(&n_off[t], 1);
            if (k < kSiteOffsets)
                offs[t * kSiteOffsets + k] =
                    (uint16_t)((dX + 4) | ((dY + 4) << 4) | ((dZ + 4) << 8) | ((bsite ? 1 : 0) << 12) | (sh << 13));
        }
    }
}

__global__ __launch_bounds__(kPlainThreads) void k_plain_site(DevPtrs P, const int32_t* ids)
{
    extern __shared__ __align__(16) unsigned char psm[];
    uint64_t* slots = (uint64_t*)psm;                           // [kMaxSiteSlots]
    double* stot = (double*)(psm + 8 * kMaxSiteSlots);          // [kMaxSiteSlots]
    uint16_t* eidx = (uint16_t*)(psm + 16 * kMaxSiteSlots);     // [kMaxSiteSlots][8]
    uint16_t* offs = (uint16_t*)(psm + 32 * kMaxSiteSlots);     // [3][kSiteOffsets]
    __shared__ int wcount[kPlainThreads / 64];
    __shared__ double wsum[kPlainThreads / 64];
    __shared__ uint64_t wmask[kPlainThreads / 64];
    __shared__ uint64_t wnz[kPlainThreads / 64];
    __shared__ int n_sh, ev_sh, hop_slot, n_off[3], Eacc[9], tsp[8], tcol[8], n_aff, err_sh;
    __shared__ uint64_t hop_s, hop_t, tpk[8];
    __shared__ int16_t aff[kPlainThreads];
    const uint64_t t_begin = __builtin_amdgcn_s_memrealtime();
    const int lat = ids[blockIdx.x];
    const LatDesc& D = P.desc[lat];
    LatState* S = P.state + lat;
    const LatCall* C = P.call + lat;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int NW = kPlainThreads / 64;
    const int W = D.site_window;
    const int WW = 2 * W + 1;
    const int8_t* occ = P.occ + D.occ_off;

    if (tid < 3) n_off[tid] = 0;
    if (tid == 0) err_sh = 0;
    __syncthreads();
    site_offsets(D, offs, n_off, tid);
    const int n = plain_collect_slots(D, P, slots, wcount, &n_sh, tid, kMaxSiteSlots);
    if (n > kMaxSiteSlots) {
        if (tid == 0) atomicOr(&S->err, 1u);
        return;
    }
    const int noff_max = max(n_off[0], max(n_off[1], n_off[2]));

    // events of slot sidx: 9 site energies by the whole workgroup, then the
    // 8 table indices and the slot total (all threads call it together)
    auto eval_slot = [&](int sidx) {
        const uint64_t pk = slots[sidx];
        if (tid < 9) Eacc[tid] = 0;
        if (tid < 8) {
            int64_t ts;
            const int i = (int)(pk & 0xffff), j = (int)((pk >> 16) & 0xffff), k = (int)((pk >> 32) & 0xffff);
            const int t = (int)(pk >> 48);
            int hx, hy, hz;
            hop_vec(t, tid, hx, hy, hz);
            const int X = wrap2(2 * i + (t != 0) + hx, 2 * D.L[0]);
            const int Y = wrap2(2 * j + (t != 1) + hy, 2 * D.L[1]);
            const int Z = wrap2(2 * k + (t != 2) + hz, 2 * D.L[2]);
            const int tt = site_type(X, Y);
            ts = plain_store(D, X >> 1, Y >> 1, Z >> 1, tt);
            const int sp = occ[ts];
            const int cs = t == 0 ? i : (t == 1 ? j : k);
            const int ct = tt == 0 ? (X >> 1) : (tt == 1 ? (Y >> 1) : (Z >> 1));
            const int g = edge_gb(D, i, j, k, t, X >> 1, Y >> 1, Z >> 1, tt, cs, ct);
            tpk[tid] = (uint64_t)(X >> 1) | ((uint64_t)(Y >> 1) << 16) | ((uint64_t)(Z >> 1) << 32) |
                       ((uint64_t)tt << 48);
            tsp[tid] = sp;
            tcol[tid] = (sp * 3 + hz + 1) * 2 + g;
        }
        __syncthreads();
        for (int w = tid; w < 9 * noff_max; w += kPlainThreads) {
            const int c = w / noff_max, kk = w - c * noff_max;
            if (c > 0 && tsp[c - 1] == kSpV) continue;
            const uint64_t ck = c == 0 ? pk : tpk[c - 1];
            const int t = (int)(ck >> 48);
            if (kk >= n_off[t]) continue;
            const int o = offs[t * kSiteOffsets + kk];
            const int X = wrap2(2 * (int)(ck & 0xffff) + (t != 0) + (o & 15) - 4, 2 * D.L[0]);
            const int Y = wrap2(2 * (int)((ck >> 16) & 0xffff) + (t != 1) + ((o >> 4) & 15) - 4, 2 * D.L[1]);
            const int Z = wrap2(2 * (int)((ck >> 32) & 0xffff) + (t != 2) + ((o >> 8) & 15) - 4, 2 * D.L[2]);
            const int sh = o >> 13;
            int e = 0;
            if ((o >> 12) & 1) {
                const int64_t cell = ((int64_t)(Z >> 1) * D.L[1] + (Y >> 1)) * D.L[0] + (X >> 1);
                if ((D.site_fe[cell >> 5] >> (cell & 31)) & 1u) e = D.site_e_fe[sh];
            } else {
                const int tt = site_type(X, Y);
                // the origin's own vacancy is never a partner (it is the one hopping)
                const uint64_t upk = (uint64_t)(X >> 1) | ((uint64_t)(Y >> 1) << 16) |
                                     ((uint64_t)(Z >> 1) << 32) | ((uint64_t)tt << 48);
                if (upk != pk && occ[plain_store(D, X >> 1, Y >> 1, Z >> 1, tt)] == kSpV)
                    e = D.site_e_vv[sh];
            }
            if (e) atomicAdd(&Eacc[c], e);
        }
        __syncthreads();
        if (tid < 8) {
            int ix = 0xFFFF;
            if (tsp[tid] != kSpV) {
                const int dE = Eacc[1 + tid] - Eacc[0];
                if (dE < -W || dE > W) err_sh = 1;
                else ix = tcol[tid] * WW + dE + W;
            }
            eidx[sidx * 8 + tid] = (uint16_t)ix;
        }
        __syncthreads();
        if (tid == 0) {
            double r = 0.0;
            for (int d = 0; d < 8; d++) {
                const int ix = eidx[sidx * 8 + d];
                r += ix == 0xFFFF ? 0.0 : D.site_table[ix];
            }
            stot[sidx] = r;
        }
        __syncthreads();
    };
    for (int sidx = 0; sidx < n; sidx++) eval_slot(sidx);

    const int m = (n + kPlainThreads - 1) / kPlainThreads;
    const int s0 = tid * m < n ? tid * m : n;
    const int s1 = s0 + m < n ? s0 + m : n;
    double t = S->t;
    uint64_t draws = S->draws;
    const double horizon = C->t_sync;
    const double t_end = t + horizon;
    const uint64_t target = C->min_hops;
    uint64_t done = 0, ho = 0, hh = 0;
    while (done < target && !err_sh) {
        double ls = 0.0;
        for (int sidx = s0; sidx < s1; sidx++) ls += stot[sidx];
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
            int sp_slot = -1, last = -1;
            for (int sidx = s0; sidx < s1; sidx++) {
                if (stot[sidx] > 0.0) last = sidx;
                if (!fallback && sp_slot < 0 && Cc + stot[sidx] > y) {
                    sp_slot = sidx;
                    break;
                }
                Cc += stot[sidx];
            }
            if (sp_slot < 0) sp_slot = last;
            int dsel = -1, dlast = -1;
            for (int d = 0; d < 8; d++) {
                const int ix = eidx[sp_slot * 8 + d];
                const double k = ix == 0xFFFF ? 0.0 : D.site_table[ix];
                if (k > 0.0) dlast = d;
                Cc += k;
                if (!fallback && dsel < 0 && Cc > y) dsel = d;
            }
            const int d = dsel >= 0 ? dsel : dlast;
            const uint64_t pk = slots[sp_slot];
            const int i = (int)(pk & 0xffff), j = (int)((pk >> 16) & 0xffff), k = (int)((pk >> 32) & 0xffff);
            const int tp = (int)(pk >> 48);
            int hx, hy, hz;
            hop_vec(tp, d, hx, hy, hz);
            const int X = wrap2(2 * i + (tp != 0) + hx, 2 * D.L[0]);
            const int Y = wrap2(2 * j + (tp != 1) + hy, 2 * D.L[1]);
            const int Z = wrap2(2 * k + (tp != 2) + hz, 2 * D.L[2]);
            const int tt = site_type(X, Y);
            const int64_t ss = plain_store(D, i, j, k, tp);
            const int64_t ts = plain_store(D, X >> 1, Y >> 1, Z >> 1, tt);
            const int sp = P.occ[D.occ_off + ts];
            P.occ[D.occ_off + ss] = (int8_t)sp;
            P.occ[D.occ_off + ts] = (int8_t)kSpV;
            int4* dsrc = P.disp + (D.disp_off + ss);
            int4* dtgt = P.disp + (D.disp_off + ts);
            const int4 dv = *dsrc;
            const int4 di = *dtgt;
            *dtgt = make_int4(dv.x + hx, dv.y + hy, dv.z + hz, 0);
            *dsrc = make_int4(di.x - hx, di.y - hy, di.z - hz, 0);
            const uint64_t npk = (uint64_t)(X >> 1) | ((uint64_t)(Y >> 1) << 16) | ((uint64_t)(Z >> 1) << 32) |
                                 ((uint64_t)tt << 48);
            slots[sp_slot] = npk;
            hop_slot = sp_slot;
            hop_s = pk;
            hop_t = npk;
            ev_sh = sp;
        }
        if (tid == 0) n_aff = 0;
        // the barrier's workgroup-scope fence makes the hop's HBM writes
        // visible to every wave of this workgroup, the only readers
        __syncthreads();
        if (ev_sh == kSpO) ho++;
        else hh++;
        done++;
        // slots whose events can have changed: within squared doubled
        // distance 29 of either site (energies reach 16, a target is 2 away)
        const uint64_t ps = hop_s, pt = hop_t;
        for (int sidx = s0; sidx < s1; sidx++)
            if (sidx == hop_slot || plain_dist2(D, slots[sidx], ps) <= 29 || plain_dist2(D, slots[sidx], pt) <= 29) {
                const int a = atomicAdd(&n_aff, 1);
                if (a < kPlainThreads) aff[a] = (int16_t)sidx;
            }
        __syncthreads();
        const int na = n_aff;
        if (na > kPlainThreads) {
            for (int sidx = 0; sidx < n; sidx++) eval_slot(sidx);
        } else {
            for (int a = 0; a < na; a++) eval_slot(aff[a]);
        }
    }
    __syncthreads();
    if (tid == 0) {
        if (err_sh) atomicOr(&S->err, 4u);
        S->t = t;
        S->draws = draws;
        S->hops[0] += ho;
        S->hops[1] += hh;
        S->busy_ticks = __builtin_amdgcn_s_memrealtime() - t_begin;
    }
}

// ----------------------------------------------------------------------------
// Fragment kMC with site energies, one phase per launch: one 256-thread
// workgroup per sub-block of colour `colour` of a lattice with a site model
// (P.site_groups: lattice, fragment).  Its BKL domain is the sub-block's
// edges (an edge belongs to the sub-block that holds its midpoint cell),
// its slots the footprint's vacancies in canonical order, its draws the
// fragment's Philox stream (step, f, cycle, colour * 256 + 2) and its clock
// the phase's own, ending at t_sync (Eqs. TransitionProb, eventSelection,
// TimeStep); every rate is the site-model table entry of k_plain_site,
// evaluated from the occupancy in HBM.  The host admits a site model on a
// fragment lattice only when every sub-block is wider than the
// vacancy-vacancy reach (4 w^2 above the squared doubled distance of the
// farthest nonzero shell): no rate of a sub-block then reads a site that
// another sub-block of the phase changes, so the workgroups need no frozen
// halo and no order.
constexpr int kSiteTileSlots = 256;  // vacancies per footprint

__global__ __launch_bounds__(kPlainThreads) void k_phase_site(DevPtrs P, int colour)
{
    __shared__ uint64_t slots[kSiteTileSlots];  // packed positions, canonical order
    __shared__ uint64_t ukey[kSiteTileSlots];   // canonical index, collection order
    __shared__ uint64_t upos[kSiteTileSlots];
    __shared__ double stot[kSiteTileSlots];
    __shared__ uint16_t eidx[kSiteTileSlots * 8];
    __shared__ uint16_t offs[3 * kSiteOffsets];
    __shared__ double wsum[kPlainThreads / 64];
    __shared__ uint64_t wmask[kPlainThreads / 64];
    __shared__ uint64_t wnz[kPlainThreads / 64];
    __shared__ int n_sh, ev_sh, hop_slot, n_off[3], Eacc[9], tsp[8], tcol[8], n_aff, err_sh;
    __shared__ uint64_t hop_s, hop_t, tpk[8];
    __shared__ int16_t aff[kPlainThreads];
    const int2 gr = P.site_groups[blockIdx.x];
    const int lat = gr.x, f = gr.y;
    const LatDesc& D = P.desc[lat];
    LatState* S = P.state + lat;
    if (S->done) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int NW = kPlainThreads / 64;
    const int W = D.site_window;
    const int WW = 2 * W + 1;
    const int L0 = D.L[0], L1 = D.L[1], L2 = D.L[2];
    const TileRec& T = P.tiles[(size_t)colour * P.n_tiles + D.tile0 + f];
    const int o0 = T.ox, o1 = T.oy, o2 = T.oz, w0 = T.wx, w1 = T.wy, w2 = T.wz;
    int8_t* occ = P.occ + D.occ_off;
    auto store = [&](int i, int j, int k, int t) { return store_index(D, P.bounds, P.c2s, i, j, k, t); };

    if (tid < 3) n_off[tid] = 0;
    if (tid == 0) {
        err_sh = 0;
        n_sh = 0;
    }
    __syncthreads();
    site_offsets(D, offs, n_off, tid);
    // the footprint's vacancies: the sub-block's sites and the +face of each
    // axis (type a at cell o_a + w_a), from the box of (w+1)^3 cells
    const int e0 = w0 + 1, e1 = w1 + 1, e2 = w2 + 1;
    const int nbox = 3 * e0 * e1 * e2;
    for (int m = tid; m < nbox; m += kPlainThreads) {
        const int t = m % 3, c = m / 3;
        const int di = c % e0, dj = (c / e0) % e1, dk = c / (e0 * e1);
        const int fx = di == w0, fy = dj == w1, fz = dk == w2;
        const bool in = fx + fy + fz == 0 || (fx + fy + fz == 1 && (t == 0 ? fx : (t == 1 ? fy : fz)));
        if (!in) continue;
        int i = o0 + di, j = o1 + dj, k = o2 + dk;
        i -= i >= L0 ? L0 : 0;
        j -= j >= L1 ? L1 : 0;
        k -= k >= L2 ? L2 : 0;
        if (occ[store(i, j, k, t)] != kSpV) continue;
        const int a = atomicAdd(&n_sh, 1);
        if (a < kSiteTileSlots) {
            ukey[a] = (uint64_t)canon_site(L0, L1, i, j, k, t);
            upos[a] = (uint64_t)i | ((uint64_t)j << 16) | ((uint64_t)k << 32) | ((uint64_t)t << 48);
        }
    }
    __syncthreads();
    const int n = n_sh;
    if (n > kSiteTileSlots) {
        if (tid == 0) atomicOr(&S->err, 1u);
        return;
    }
    // canonical order: each slot's rank among the distinct keys
    for (int a = tid; a < n; a += kPlainThreads) {
        int r = 0;
        for (int b = 0; b < n; b++) r += ukey[b] < ukey[a] ? 1 : 0;
        slots[r] = upos[a];
    }
    __syncthreads();
    const int noff_max = max(n_off[0], max(n_off[1], n_off[2]));

    // events of slot sidx (as k_plain_site): an event whose edge the
    // sub-block does not own, or whose target holds a vacancy, has no rate
    auto eval_slot = [&](int sidx) {
        const uint64_t pk = slots[sidx];
        if (tid < 9) Eacc[tid] = 0;
        if (tid < 8) {
            const int i = (int)(pk & 0xffff), j = (int)((pk >> 16) & 0xffff), k = (int)((pk >> 32) & 0xffff);
            const int t = (int)(pk >> 48);
            int hx, hy, hz;
            hop_vec(t, tid, hx, hy, hz);
            const int X0 = 2 * i + (t != 0), Y0 = 2 * j + (t != 1), Z0 = 2 * k + (t != 2);
            // the edge's midpoint cell, relative to the sub-block's origin
            int ox = ((2 * X0 + hx) >> 2) - o0, oy = ((2 * Y0 + hy) >> 2) - o1, oz = ((2 * Z0 + hz) >> 2) - o2;
            ox += ox < 0 ? L0 : 0;
            oy += oy < 0 ? L1 : 0;
            oz += oz < 0 ? L2 : 0;
            ox -= ox >= L0 ? L0 : 0;
            oy -= oy >= L1 ? L1 : 0;
            oz -= oz >= L2 ? L2 : 0;
            const bool own = ox < w0 && oy < w1 && oz < w2;
            const int X = wrap2(X0 + hx, 2 * L0), Y = wrap2(Y0 + hy, 2 * L1), Z = wrap2(Z0 + hz, 2 * L2);
            const int tt = site_type(X, Y);
            const int sp = own ? (int)occ[store(X >> 1, Y >> 1, Z >> 1, tt)] : kSpV;
            const int cs = t == 0 ? i : (t == 1 ? j : k);
            const int ct = tt == 0 ? (X >> 1) : (tt == 1 ? (Y >> 1) : (Z >> 1));
            const int g = edge_gb(D, i, j, k, t, X >> 1, Y >> 1, Z >> 1, tt, cs, ct);
            tpk[tid] = (uint64_t)(X >> 1) | ((uint64_t)(Y >> 1) << 16) | ((uint64_t)(Z >> 1) << 32) |
                       ((uint64_t)tt << 48);
            tsp[tid] = sp;
            tcol[tid] = (sp * 3 + hz + 1) * 2 + g;
        }
        __syncthreads();
        for (int w = tid; w < 9 * noff_max; w += kPlainThreads) {
            const int c = w / noff_max, kk = w - c * noff_max;
            if (c > 0 && tsp[c - 1] == kSpV) continue;
            const uint64_t ck = c == 0 ? pk : tpk[c - 1];
            const int t = (int)(ck >> 48);
            if (kk >= n_off[t]) continue;
            const int o = offs[t * kSiteOffsets + kk];
            const int X = wrap2(2 * (int)(ck & 0xffff) + (t != 0) + (o & 15) - 4, 2 * L0);
            const int Y = wrap2(2 * (int)((ck >> 16) & 0xffff) + (t != 1) + ((o >> 4) & 15) - 4, 2 * L1);
            const int Z = wrap2(2 * (int)((ck >> 32) & 0xffff) + (t != 2) + ((o >> 8) & 15) - 4, 2 * L2);
            const int sh = o >> 13;
            int e = 0;
            if ((o >> 12) & 1) {
                const int64_t cell = ((int64_t)(Z >> 1) * L1 + (Y >> 1)) * L0 + (X >> 1);
                if ((D.site_fe[cell >> 5] >> (cell & 31)) & 1u) e = D.site_e_fe[sh];
            } else {
                const int tt = site_type(X, Y);
                // the origin's own vacancy is never a partner (it is the one hopping)
                const uint64_t upk = (uint64_t)(X >> 1) | ((uint64_t)(Y >> 1) << 16) |
                                     ((uint64_t)(Z >> 1) << 32) | ((uint64_t)tt << 48);
                if (upk != pk && occ[store(X >> 1, Y >> 1, Z >> 1, tt)] == kSpV) e = D.site_e_vv[sh];
            }
            if (e) atomicAdd(&Eacc[c], e);
        }
        __syncthreads();
        if (tid < 8) {
            int ix = 0xFFFF;
            if (tsp[tid] != kSpV) {
                const int dE = Eacc[1 + tid] - Eacc[0];
                if (dE < -W || dE > W) err_sh = 1;
                else ix = tcol[tid] * WW + dE + W;
            }
            eidx[sidx * 8 + tid] = (uint16_t)ix;
        }
        __syncthreads();
        if (tid == 0) {
            double r = 0.0;
            for (int d = 0; d < 8; d++) {
                const int ix = eidx[sidx * 8 + d];
                r += ix == 0xFFFF ? 0.0 : D.site_table[ix];
            }
            stot[sidx] = r;
        }
        __syncthreads();
    };
    for (int sidx = 0; sidx < n; sidx++) eval_slot(sidx);

    const int m = (n + kPlainThreads - 1) / kPlainThreads;
    const int s0 = tid * m < n ? tid * m : n;
    const int s1 = s0 + m < n ? s0 + m : n;
    const double t_sync = P.call[lat].t_sync;
    const uint32_t cyc = (uint32_t)S->cycles;
    const uint32_t ctag = ((uint32_t)colour << 8) | 2u;
    double tau = 0.0;
    uint32_t step = 0;
    unsigned long long ho = 0, hh = 0;
    while (!err_sh) {
        double ls = 0.0;
        for (int sidx = s0; sidx < s1; sidx++) ls += stot[sidx];
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
        philox10(step, (uint32_t)f, cyc, ctag, D.seed, D.lattice_id, x0, x1, x2, x3);
        const double u_sel = u53_lo(x0, x1);
        const double tn = tau + -clock_ln(u53_hi(x2, x3)) / R;
        if (tn > t_sync) break;
        tau = tn;
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
            int sp_slot = -1, last = -1;
            for (int sidx = s0; sidx < s1; sidx++) {
                if (stot[sidx] > 0.0) last = sidx;
                if (!fallback && sp_slot < 0 && Cc + stot[sidx] > y) {
                    sp_slot = sidx;
                    break;
                }
                Cc += stot[sidx];
            }
            if (sp_slot < 0) sp_slot = last;
            int dsel = -1, dlast = -1;
            for (int d = 0; d < 8; d++) {
                const int ix = eidx[sp_slot * 8 + d];
                const double k = ix == 0xFFFF ? 0.0 : D.site_table[ix];
                if (k > 0.0) dlast = d;
                Cc += k;
                if (!fallback && dsel < 0 && Cc > y) dsel = d;
            }
            const int d = dsel >= 0 ? dsel : dlast;
            const uint64_t pk = slots[sp_slot];
            const int i = (int)(pk & 0xffff), j = (int)((pk >> 16) & 0xffff), k = (int)((pk >> 32) & 0xffff);
            const int tp = (int)(pk >> 48);
            int hx, hy, hz;
            hop_vec(tp, d, hx, hy, hz);
            const int X = wrap2(2 * i + (tp != 0) + hx, 2 * L0);
            const int Y = wrap2(2 * j + (tp != 1) + hy, 2 * L1);
            const int Z = wrap2(2 * k + (tp != 2) + hz, 2 * L2);
            const int tt = site_type(X, Y);
            const int64_t ss = store(i, j, k, tp);
            const int64_t ts = store(X >> 1, Y >> 1, Z >> 1, tt);
            const int sp = occ[ts];
            occ[ss] = (int8_t)sp;
            occ[ts] = (int8_t)kSpV;
            int4* dsrc = P.disp + (D.disp_off + ss);
            int4* dtgt = P.disp + (D.disp_off + ts);
            const int4 dv = *dsrc;
            const int4 di = *dtgt;
            *dtgt = make_int4(dv.x + hx, dv.y + hy, dv.z + hz, 0);
            *dsrc = make_int4(di.x - hx, di.y - hy, di.z - hz, 0);
            const uint64_t npk = (uint64_t)(X >> 1) | ((uint64_t)(Y >> 1) << 16) | ((uint64_t)(Z >> 1) << 32) |
                                 ((uint64_t)tt << 48);
            slots[sp_slot] = npk;
            hop_slot = sp_slot;
            hop_s = pk;
            hop_t = npk;
            ev_sh = sp;
        }
        if (tid == 0) n_aff = 0;
        // the barrier's workgroup-scope fence makes the hop's HBM writes
        // visible to every wave of this workgroup, the only readers
        __syncthreads();
        if (ev_sh == kSpO) ho++;
        else hh++;
        step++;
        // slots whose events can have changed: within squared doubled
        // distance 29 of either site (energies reach 16, a target is 2 away)
        const uint64_t ps = hop_s, pt = hop_t;
        for (int sidx = s0; sidx < s1; sidx++)
            if (sidx == hop_slot || plain_dist2(D, slots[sidx], ps) <= 29 || plain_dist2(D, slots[sidx], pt) <= 29) {
                const int a = atomicAdd(&n_aff, 1);
                if (a < kPlainThreads) aff[a] = (int16_t)sidx;
            }
        __syncthreads();
        const int na = n_aff;
        for (int a = 0; a < na; a++) eval_slot(aff[a]);
    }
    __syncthreads();
    if (tid == 0) {
        if (err_sh) atomicOr(&S->err, 4u);
        if (ho | hh) {
            unsigned long long* b = P.buckets + ((size_t)lat * kHopBuckets + (f & (kHopBuckets - 1))) * 2;
            if (ho) atomicAdd(b, ho);
            if (hh) atomicAdd(b + 1, hh);
        }
    }
}

// Cells whose slots need new totals after a stage: a hashed bitmap of
// 2^kMarkBits bits per stage (collisions only cost recomputations).
constexpr int kMarkBits = 14;
constexpr int kMarkWords = 1 << (kMarkBits - 5);
static_assert(kMaxPlainSlots <= 65536, "slot indices of the refresh list are 16-bit");
// Atom-selection stages (Sec. "Atomic-based fragment kMC method", Eqs. AtomP
// and TimeStepFrg) on a plain lattice whose occupancy stays in HBM: one
// workgroup per lattice, its vacancy slots and their totals R_I in LDS, the
// slots in ascending canonical index at the call start, each following its
// vacancy.  Each stage reduces the totals to K (sum) and R^max (maximum);
// wave 0 draws the selections, one per lane, resolves the conflicts in
// selection order, makes the taken hops in place and marks the cells around
// their sites; the next stage recomputes the totals of the slots in marked
// cells only.  Two mark bitmaps alternate, so that one is cleared while the
// other is written.
__global__ __launch_bounds__(kPlainThreads) void k_atomic_hbm(DevPtrs P, const int32_t* ids, int cap,
                                                              uint32_t n_frg, uint64_t n_stages)
{
    extern __shared__ __align__(16) unsigned char psm[];
    uint64_t* slots = (uint64_t*)psm;                           // [cap]
    double* stot = (double*)(psm + 8 * (size_t)cap);            // [cap]
    uint32_t* marks = (uint32_t*)(psm + 16 * (size_t)cap);      // [2][kMarkWords]
    uint16_t* fresh = (uint16_t*)(marks + 2 * kMarkWords);     // [cap] slots to recompute
    __shared__ int n_fresh;
    __shared__ int wcount[kPlainThreads / 64];
    __shared__ double wsum[kPlainThreads / 64];
    __shared__ double wmax[kPlainThreads / 64];
    __shared__ int n_sh;
    const uint64_t t_begin = __builtin_amdgcn_s_memrealtime();
    const int lat = ids[blockIdx.x];
    const LatDesc& D = P.desc[lat];
    LatState* S = P.state + lat;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int NW = kPlainThreads / 64;
    const int n = plain_collect_slots(D, P, slots, wcount, &n_sh, tid, cap);
    if (n > cap) {
        if (tid == 0) atomicOr(&S->err, 1u);
        return;
    }
    const int m = (n + kPlainThreads - 1) / kPlainThreads;
    const int s0 = tid * m < n ? tid * m : n;
    const int s1 = s0 + m < n ? s0 + m : n;
    int8_t* occ = P.occ + D.occ_off;
    auto slot_total = [&](int sidx) {
        double r = 0.0;
        for (int d = 0; d < 8; d++) {
            int64_t ts;
            r += plain_rate(D, P, slots[sidx], d, ts);
        }
        return r;
    };
    for (int w = tid; w < 2 * kMarkWords; w += kPlainThreads) marks[w] = 0u;
    if (tid == 0) n_fresh = 0;
    for (int sidx = s0; sidx < s1; sidx++) stot[sidx] = slot_total(sidx);
    __syncthreads();
    double t = S->t;
    uint64_t stage = S->draws;
    unsigned long long ho = 0, hh = 0;
    for (uint64_t st = 0; st < n_stages; st++) {
        // rates at the start of the stage: new totals for the slots in cells
        // the last stage marked, listed first and then shared out evenly
        if (st > 0) {
            const uint32_t* seen = marks + ((st + 1) & 1) * kMarkWords;
            for (int sidx = s0; sidx < s1; sidx++) {
                const uint64_t pk = slots[sidx];
                const uint32_t h = cell_mark_bit<kMarkBits>((int)(pk & 0xffff), (int)((pk >> 16) & 0xffff),
                                                            (int)((pk >> 32) & 0xffff));
                if ((seen[h >> 5] >> (h & 31)) & 1u) fresh[atomicAdd(&n_fresh, 1)] = (uint16_t)sidx;
            }
            __syncthreads();
            const int nf = n_fresh;
            for (int x = tid; x < nf; x += kPlainThreads) stot[fresh[x]] = slot_total(fresh[x]);
            __syncthreads();
        }
        double ls = 0.0, lm = 0.0;
        for (int sidx = s0; sidx < s1; sidx++) {
            const double r = stot[sidx];
            ls += r;
            lm = fmax(lm, r);
        }
        ls = lane_value(wave_scan_dpp(ls), 63);
        lm = lane_value(wave_max_dpp(lm), 63);
        if (lane == 0) {
            wsum[wv] = ls;
            wmax[wv] = lm;
        }
        __syncthreads();
        double K = 0.0, Rmax = 0.0;
        for (int w = 0; w < NW; w++) {
            K += wsum[w];
            Rmax = fmax(Rmax, wmax[w]);
        }
        if (K == 0.0) break;
        // nobody reads the last stage's marks or list any more: clear them
        for (int w = tid; w < kMarkWords; w += kPlainThreads) marks[((st + 1) & 1) * kMarkWords + w] = 0u;
        if (tid == 0) n_fresh = 0;
        if (wv == 0) {
            uint32_t* mark = marks + (st & 1) * kMarkWords;
            // selection j in lane j: an atom, then its event or a null event
            int a = 0, e = -1;
            int64_t cs = -1, ct = -1;
            uint64_t pk = 0;
            if ((uint32_t)lane < n_frg) {
                uint32_t x0, x1, x2, x3;
                philox10((uint32_t)stage, (uint32_t)(stage >> 32), (uint32_t)lane, 4u, D.seed,
                         D.lattice_id, x0, x1, x2, x3);
                a = (int)(((uint64_t)x0 * (uint64_t)(uint32_t)n) >> 32);
                pk = slots[a];
                const double y = u53_lo(x2, x3) * Rmax;
                double cum = 0.0;
                for (int d = 0; d < 8; d++) {
                    int64_t ts;
                    cum += plain_rate(D, P, pk, d, ts);
                    if (e < 0 && cum > y) {
                        e = d;
                        ct = ts;
                    }
                }
            }
            const bool ev = e >= 0;
            int sp = kSpO;
            if (ev) {
                cs = plain_store(D, (int)(pk & 0xffff), (int)((pk >> 16) & 0xffff),
                                 (int)((pk >> 32) & 0xffff), (int)(pk >> 48));
                sp = occ[ct];
            }
            // conflicts, in selection order
            bool taken = false;
            uint64_t evm = __ballot(ev);
            while (evm) {
                const int j = __ffsll((unsigned long long)evm) - 1;
                evm &= evm - 1;
                const int64_t sj = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(cs >> 32), j) << 32) |
                                             (uint32_t)__builtin_amdgcn_readlane((int)cs, j));
                const int64_t tj = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(ct >> 32), j) << 32) |
                                             (uint32_t)__builtin_amdgcn_readlane((int)ct, j));
                const bool hit = __ballot(taken && (cs == sj || cs == tj || ct == sj || ct == tj)) != 0;
                if (!hit && lane == j) taken = true;
            }
            if (taken) {
                // the taken hops touch disjoint sites: each lane swaps its own pair
                const int i = (int)(pk & 0xffff), jj = (int)((pk >> 16) & 0xffff),
                          k = (int)((pk >> 32) & 0xffff), tp = (int)(pk >> 48);
                int hx, hy, hz;
                hop_vec(tp, e, hx, hy, hz);
                occ[cs] = (int8_t)sp;
                occ[ct] = (int8_t)kSpV;
                int4* dsrc = P.disp + (D.disp_off + cs);
                int4* dtgt = P.disp + (D.disp_off + ct);
                const int4 dv = *dsrc;
                const int4 di = *dtgt;
                *dtgt = make_int4(dv.x + hx, dv.y + hy, dv.z + hz, 0);
                *dsrc = make_int4(di.x - hx, di.y - hy, di.z - hz, 0);
                int X = 2 * i + (tp != 0) + hx, Y = 2 * jj + (tp != 1) + hy, Z = 2 * k + (tp != 2) + hz;
                if (X < 0) X += 2 * D.L[0];
                if (X >= 2 * D.L[0]) X -= 2 * D.L[0];
                if (Y < 0) Y += 2 * D.L[1];
                if (Y >= 2 * D.L[1]) Y -= 2 * D.L[1];
                if (Z < 0) Z += 2 * D.L[2];
                if (Z >= 2 * D.L[2]) Z -= 2 * D.L[2];
                slots[a] = (uint64_t)(X >> 1) | ((uint64_t)(Y >> 1) << 16) | ((uint64_t)(Z >> 1) << 32) |
                           ((uint64_t)site_type(X, Y) << 48);
                mark_neighbour_cells<kMarkBits>(mark, D.L[0], D.L[1], D.L[2], 2 * i + (tp != 0),
                                                2 * jj + (tp != 1), 2 * k + (tp != 2));
                mark_neighbour_cells<kMarkBits>(mark, D.L[0], D.L[1], D.L[2], X, Y, Z);
            }
            const int n_upd = __popcll(__ballot(taken));
            const int n_o = __popcll(__ballot(taken && sp == kSpO));
            ho += (unsigned long long)n_o;
            hh += (unsigned long long)(n_upd - n_o);
            // Eq. TimeStepFrg
            uint32_t x0, x1, x2, x3;
            philox10((uint32_t)stage, (uint32_t)(stage >> 32), 0xFFFFFFFFu, 4u, D.seed, D.lattice_id, x0,
                     x1, x2, x3);
            const double dt = -clock_ln(u53_hi(x2, x3)) / K;
            t = t + dt * (double)n_upd;
        }
        stage++;
        // the barrier's workgroup-scope fence makes the hops' HBM writes
        // visible to every wave of this workgroup, the only readers
        __syncthreads();
    }
    if (tid == 0) {
        S->t = t;
        S->draws = stage;
        S->hops[0] += ho;
        S->hops[1] += hh;
        S->busy_ticks = __builtin_amdgcn_s_memrealtime() - t_begin;
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

// Canonical-order gather (read-out) and scatter (set occupancy) over the
// canonical sites [begin, begin + count); the canonical arrays hold only those.
__device__ __forceinline__ int64_t canon_store(const DevPtrs& P, const LatDesc& D, int64_t n)
{
    const int t = (int)(n % 3);
    const int64_t cell = n / 3;
    const int i = (int)(cell % D.L[0]);
    const int j = (int)((cell / D.L[0]) % D.L[1]);
    const int k = (int)(cell / ((int64_t)D.L[0] * D.L[1]));
    return store_index(D, P.bounds, P.c2s, i, j, k, t);
}

__global__ void k_gather(DevPtrs P, int lat, int64_t begin, int64_t count, int8_t* occ_c, int32_t* disp_c)
{
    const LatDesc& D = P.desc[lat];
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= count || begin + m >= D.n_sites) return;
    const int64_t s = canon_store(P, D, begin + m);
    occ_c[m] = P.occ[D.occ_off + s];
    if (disp_c) {
        const int4 r = P.disp[D.disp_off + s];
        disp_c[3 * m] = r.x;
        disp_c[3 * m + 1] = r.y;
        disp_c[3 * m + 2] = r.z;
    }
}

__global__ void k_scatter(DevPtrs P, int lat, int64_t begin, int64_t count, const int8_t* occ_c)
{
    const LatDesc& D = P.desc[lat];
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= count || begin + m >= D.n_sites) return;
    const int64_t s = canon_store(P, D, begin + m);
    P.occ[D.occ_off + s] = occ_c[m];
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

using PhaseFn = void (*)(DevPtrs, int);

// The lockstep kernel for a group size; the variant with the boundary-site
// map branch only when a lattice of the set has a map.
static PhaseFn phase_fn(int group, bool map)
{
    if (map)
        return group == 8 ? k_phase<8, true>
                          : (group == 4 ? k_phase<4, true> : (group == 2 ? k_phase<2, true> : k_phase<1, true>));
    return group == 8 ? k_phase<8, false>
                      : (group == 4 ? k_phase<4, false> : (group == 2 ? k_phase<2, false> : k_phase<1, false>));
}

// Allow the lockstep workgroup's dynamic LDS beyond the default 64 KB.
static hipError_t phase_lds_attr(int group, bool map, size_t lds)
{
    static size_t granted[2][9] = {{0}};
    if (lds <= 65536 || lds <= granted[map][group]) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)phase_fn(group, map),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) granted[map][group] = lds;
    return e;
}

// Waves per lockstep workgroup: kPhaseWaves while their LDS stays below
// 64 KB (every staged footprint then has an LDS address below 2^16), else 1.
static int phase_waves(const DevPtrs& P)
{
    return (size_t)P.lds_wave_bytes * kPhaseWaves <= 65536 ? kPhaseWaves : 1;
}

int launch_phase(const DevPtrs& P, int colour, int group, void* stream)
{
    if (P.n_groups == 0) return 0;
    const int wpb = phase_waves(P);
    const size_t lds = (size_t)P.lds_wave_bytes * wpb;
    hipError_t e = phase_lds_attr(group, P.gb_maps != 0, lds);
    if (e != hipSuccess) return (int)e;
    const int blocks = (P.n_groups + wpb - 1) / wpb;
    hipLaunchKernelGGL(phase_fn(group, P.gb_maps != 0), dim3(blocks), dim3(64 * wpb), lds, (hipStream_t)stream, P,
                       colour);
    return (int)hipGetLastError();
}

int launch_atomic(const DevPtrs& P, const int32_t* d_ids, int n, size_t lds, uint32_t n_frg,
                  uint64_t n_stages, void* stream)
{
    if (n == 0) return 0;
    hipError_t e = hipFuncSetAttribute((const void*)k_atomic, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(k_atomic, dim3(n), dim3(256), lds, (hipStream_t)stream, P, d_ids, n_frg, n_stages);
    return (int)hipGetLastError();
}

int launch_batch(const DevPtrs& P, int n_batch, int waves, void* stream)
{
    if (n_batch == 0) return 0;
    const size_t lds = (size_t)P.lds_region_bytes + (size_t)waves * kWaveScratch + kRecCache;
    // the variant with the boundary-site map branch only when a lattice has a map
    const auto fn = P.gb_maps ? k_batch<true> : k_batch<false>;
    hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(fn, dim3(n_batch), dim3(64 * waves), lds, (hipStream_t)stream, P);
    return (int)hipGetLastError();
}

// A graph of `cycles` consecutive lockstep cycles (8 phase kernels and the
// cycle-end kernel each, chained), built from kernel nodes so that it can be
// launched on any stream.  Holds no memset or copy nodes.
int build_cycle_graph(const DevPtrs& P, int group, int cycles, hipGraphExec_t* out)
{
    const int wpb = phase_waves(P);
    const size_t lds = (size_t)P.lds_wave_bytes * wpb;
    hipError_t e = phase_lds_attr(group, P.gb_maps != 0, lds);
    if (e != hipSuccess) return (int)e;
    hipGraph_t g;
    e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return (int)e;
    DevPtrs args_p = P;  // argument values are copied into each node
    hipGraphNode_t prev = nullptr;
    int colours[8] = {0, 1, 2, 3, 4, 5, 6, 7};
    int begin0 = 0;
    for (int c = 0; c < cycles && e == hipSuccess; c++) {
        for (int col = 0; col < 9 && e == hipSuccess; col++) {
            hipKernelNodeParams kp = {};
            void* argv[3];
            argv[0] = &args_p;
            if (col < 8) {
                argv[1] = &colours[col];
                kp.func = (void*)phase_fn(group, P.gb_maps != 0);
                kp.gridDim = dim3((P.n_groups + wpb - 1) / wpb);
                kp.blockDim = dim3(64 * wpb);
                kp.sharedMemBytes = (unsigned)lds;
            } else {
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

int launch_plain(const DevPtrs& P, const int32_t* d_plain_ids, int n_plain, int cap, void* stream)
{
    if (n_plain == 0) return 0;
    if (cap < 1 || cap > kMaxPlainSlots) return (int)hipErrorInvalidValue;
    const size_t lds = (size_t)16 * cap;
    hipError_t e = hipFuncSetAttribute((const void*)k_plain, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(k_plain, dim3(n_plain), dim3(kPlainThreads), lds, (hipStream_t)stream, P,
                       d_plain_ids, cap);
    return (int)hipGetLastError();
}

int launch_plain_site(const DevPtrs& P, const int32_t* d_ids, int n, void* stream)
{
    if (n == 0) return 0;
    const size_t lds = (size_t)32 * kMaxSiteSlots + 2 * 3 * kSiteOffsets;
    hipError_t e = hipFuncSetAttribute((const void*)k_plain_site, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(k_plain_site, dim3(n), dim3(kPlainThreads), lds, (hipStream_t)stream, P, d_ids);
    return (int)hipGetLastError();
}

int launch_phase_site(const DevPtrs& P, int colour, void* stream)
{
    if (P.n_site_groups == 0) return 0;
    hipLaunchKernelGGL(k_phase_site, dim3(P.n_site_groups), dim3(kPlainThreads), 0, (hipStream_t)stream, P,
                       colour);
    return (int)hipGetLastError();
}

int launch_atomic_hbm(const DevPtrs& P, const int32_t* d_ids, int n, int cap, uint32_t n_frg,
                      uint64_t n_stages, void* stream)
{
    if (n == 0) return 0;
    if (cap < 1 || cap > kMaxPlainSlots) return (int)hipErrorInvalidValue;
    const size_t lds = (size_t)18 * cap + (size_t)8 * kMarkWords;
    hipError_t e = hipFuncSetAttribute((const void*)k_atomic_hbm, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(k_atomic_hbm, dim3(n), dim3(kPlainThreads), lds, (hipStream_t)stream, P, d_ids,
                       cap, n_frg, n_stages);
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

int launch_gather(const DevPtrs& P, int lat, int64_t begin, int64_t count, int8_t* d_occ_canon,
                  int32_t* d_disp_canon, void* stream)
{
    const int64_t blocks = (count + 255) / 256;
    if (blocks < 1) return 0;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, P, lat, begin,
                       count, d_occ_canon, d_disp_canon);
    return (int)hipGetLastError();
}

__global__ void k_scatter_disp(DevPtrs P, int lat, int64_t begin, int64_t count, const int32_t* disp_c)
{
    const LatDesc& D = P.desc[lat];
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= count || begin + m >= D.n_sites) return;
    const int64_t s = canon_store(P, D, begin + m);
    P.disp[D.disp_off + s] = make_int4(disp_c[3 * m], disp_c[3 * m + 1], disp_c[3 * m + 2], 0);
}

int launch_scatter_disp(const DevPtrs& P, int lat, int64_t begin, int64_t count,
                        const int32_t* d_disp_canon, void* stream)
{
    const int64_t blocks = (count + 255) / 256;
    if (blocks < 1) return 0;
    hipLaunchKernelGGL(k_scatter_disp, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, P,
                       lat, begin, count, d_disp_canon);
    return (int)hipGetLastError();
}

int launch_scatter(const DevPtrs& P, int lat, int64_t begin, int64_t count, const int8_t* d_occ_canon,
                   void* stream)
{
    const int64_t blocks = (count + 255) / 256;
    if (blocks < 1) return 0;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, P, lat, begin,
                       count, d_occ_canon);
    return (int)hipGetLastError();
}

__global__ void k_fill_zero(unsigned char* p, size_t bytes)
{
    const size_t n16 = bytes / 16;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        ((int4*)p)[i] = make_int4(0, 0, 0, 0);
    const size_t t = n16 * 16 + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0 && t < bytes) p[t] = 0;
}

int launch_fill_zero(void* p, size_t bytes, void* stream)
{
    if (bytes == 0) return 0;
    size_t blocks = (bytes / 16 + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 8192 ? 8192 : blocks);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (unsigned char*)p, bytes);
    return (int)hipGetLastError();
}

int footprint_stride(int max_footprint_bytes)
{
    // four segments, each padded to whole 16-byte chunks from its alignment
    return (max_footprint_bytes + 4 * 30 + 15) & ~15;
}

}  // namespace fkmc
