/*
 * Reference (oracle) implementation of fragment kinetic Monte Carlo for
 * vacancy-mediated anion diffusion in a cubic ABO3 perovskite
 * (Nakata, "Development of a fragment kinetic Monte Carlo method for
 * efficient prediction of ionic diffusion in perovskite crystals",
 * arXiv:2004.09081).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is plain, serial, deliberately slow C.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no source, header, table or constant with the HIP
 * library; both follow the same written numerics specification.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC
 *   (no FMA contraction: every rounding below is the one written here).
 *
 * What is computed (paper references by section / equation):
 *  - Arrhenius rate k = A exp(-Ea/(k_B T)) of each vacancy hop
 *    (Sec. "Summary of the conventional kMC method", Eq. RateCnst1), with the
 *    electrostatic-potential term of Sec. "Computational details" (the rate
 *    constant with Ea + dE_pot) taken as a uniform field, half of the hop's
 *    energy change added to the barrier, and an extra barrier on
 *    grain-boundary sites (Sec. "Oxygen vacancy diffusion ... applied voltage").
 *  - Rejection-free selection of one event with probability k_i / sum_j k_j
 *    (Eqs. TransitionProb and eventSelection) and the residence-time clock
 *    t += -ln(r') / sum_i k_i (Eq. TimeStep).
 *  - The fragment decomposition: the lattice is split into spatial fragments
 *    that each advance independently to a synchronisation time; hops that
 *    cross fragment boundaries are reconciled by an 8-colour edge splitting
 *    (each fragment is halved per axis, every hop edge belongs to the
 *    half-block containing its midpoint, and the 8 colour classes run one
 *    after another).  The paper leaves the boundary rule unstated (Sec.
 *    "Atomic-based fragment kMC method": the event lists are gathered and
 *    updated); this edge splitting is the reading used here.
 *  - The paper's own atom-selection scheme with null events (Eqs. AtomP and
 *    TimeStepFrg) over a whole lattice, with its open points read as
 *    written at or_advance_atomic.
 *
 * Parity status: Philox is pinned against an independent library
 * implementation; ln against libm / mpmath; the BKL step and clock against
 * the exact master equation on a 2x2x2 lattice; the phase splitting against
 * the exact product of phase propagators on a 4x4x4 lattice; the single
 * vacancy diffusion coefficient and the biased drift against closed forms;
 * the atom-selection scheme with one selection per stage against the exact
 * master equation, and its single-vacancy diffusion against the closed form.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define SP_O 0
#define SP_H 1
#define SP_V 2

#define TAG_INIT 1u
#define TAG_BKL 2u
#define TAG_PLAIN 3u
#define TAG_ATOM 4u

/* Boltzmann constant in eV/K: k_B/e from the exact SI values
 * k_B = 1.380649e-23 J/K and e = 1.602176634e-19 C, rounded to nearest
 * binary64.  The paper's Eq. RateCnst1 writes the gas constant R, but its
 * barriers are per-event energies in eV, so R here is k_B. */
static const double KB_EV = 0x1.696fe94e2cf9ep-14;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11).  Round: two 32x32->64 products of the counter
 * words 0 and 2 with the multipliers, outputs permuted and xor-ed with the
 * key; the key is bumped by the two Weyl constants between rounds. */
static const uint32_t PH_M0 = 0xD2511F53u;
static const uint32_t PH_M1 = 0xCD9E8D57u;
static const uint32_t PH_W0 = 0x9E3779B9u;
static const uint32_t PH_W1 = 0xBB67AE85u;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int r;
    for (r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)PH_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PH_M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        if (r < 9) { k0 += PH_W0; k1 += PH_W1; }
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniforms from two 32-bit words: u in [0,1) and u in (0,1]. */
static double u53_open1(uint32_t hi, uint32_t lo)
{
    uint64_t w = ((uint64_t)hi << 32) | lo;
    return (double)(w >> 11) * 0x1p-53;
}
static double u53_open0(uint32_t hi, uint32_t lo)
{
    uint64_t w = ((uint64_t)hi << 32) | lo;
    return (double)((w >> 11) + 1) * 0x1p-53;
}

/* ------------------------------------------------------------------------ */
/* Natural logarithm for u in (0,1], built only from correctly rounded IEEE
 * operations so that any conforming machine gives the same bits:
 *   u = 2^e * m, m reduced to (sqrt(1/2), sqrt(2)], f = m - 1 (exact);
 *   ln m = 2 atanh(s), s = f/(2+f); with 2s = f - s f this is
 *   ln m = f - (f^2/2 - s (f^2/2 + R)),  R = sum_{k=1..11} 2 s^(2k)/(2k+1);
 *   ln u = e*ln2_hi - ((f^2/2 - (s (f^2/2 + R) + e*ln2_lo)) - f)
 * (Cody & Waite split of ln 2; the arrangement keeps the exact term f
 * outermost so the result stays within one ulp).  ln2_hi is ln 2 rounded to
 * 32 significant bits (so e*ln2_hi is exact for |e| < 2^21); ln2_lo is
 * ln 2 - ln2_hi rounded to nearest double.  Both are printed by
 * gen_ln_constants.py (mpmath, 200-bit).  Polynomial coefficients are
 * 2/(2k+1) rounded to nearest, evaluated by Horner's rule with fused
 * multiply-adds. */
static const double OR_LN2_HI = 0x1.62e42ffp-1;
static const double OR_LN2_LO = -0x1.718432a1b0e26p-35;
static const double OR_SQRT2 = 0x1.6a09e667f3bcdp+0;

void or_ln_constants(double out[3])
{
    out[0] = OR_LN2_HI; out[1] = OR_LN2_LO; out[2] = OR_SQRT2;
}

double or_ln(double u)
{
    uint64_t bits;
    int e;
    double m, f, s, z, P, R, hfsq, de;
    memcpy(&bits, &u, 8);
    e = (int)((bits >> 52) & 0x7ff) - 1023;
    bits = (bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
    memcpy(&m, &bits, 8);
    if (m > OR_SQRT2) { m = m * 0.5; e = e + 1; }
    f = m - 1.0;
    s = f / (2.0 + f);
    z = s * s;
    P = 2.0 / 23.0;
    P = fma(P, z, 2.0 / 21.0);
    P = fma(P, z, 2.0 / 19.0);
    P = fma(P, z, 2.0 / 17.0);
    P = fma(P, z, 2.0 / 15.0);
    P = fma(P, z, 2.0 / 13.0);
    P = fma(P, z, 2.0 / 11.0);
    P = fma(P, z, 2.0 / 9.0);
    P = fma(P, z, 2.0 / 7.0);
    P = fma(P, z, 2.0 / 5.0);
    P = fma(P, z, 2.0 / 3.0);
    R = z * P;
    hfsq = 0.5 * f * f;
    de = (double)e;
    return de * OR_LN2_HI - ((hfsq - (s * (hfsq + R) + de * OR_LN2_LO)) - f);
}

/* ------------------------------------------------------------------------ */
/* Geometry.  Cubic perovskite ABO3, A at the cube corner, B at the body
 * centre, the three O (anion) sites at the face centres (Sec. "Computational
 * details", the crystal-structure figure).  Positions in doubled integer
 * coordinates (1 unit = a/2): type 0 at (2i, 2j+1, 2k+1), type 1 at
 * (2i+1, 2j, 2k+1), type 2 at (2i+1, 2j+1, 2k).  Canonical site index
 * n = ((k*Ly + j)*Lx + i)*3 + type. */
typedef struct {
    int32_t L[3];
    int32_t frag[3];         /* fragment edge in cells; 0 = one domain     */
    double a_angstrom;
    uint32_t seed, lattice_id;
    int32_t gb_period_cells; /* 0 = no grain-boundary planes              */
    int32_t gb_axes_mask;    /* bit a: planes normal to axis a            */
    const uint8_t* gb_map;   /* NULL, or one byte per site in canonical
                                order, 1 = boundary site (Voronoi grain
                                boundaries); replaces the planes         */
} or_geom;

static const int TYPE_OFF[3][3] = {{0, 1, 1}, {1, 0, 1}, {1, 1, 0}};

/* The 8 nearest-neighbour hops of each site type (|h|^2 = 2 in doubled
 * units, distance a/sqrt(2)), in ascending lexicographic order of (hx,hy,hz).
 * Filled by enumeration in or_hops() rather than typed in. */
static int HOPS[3][8][3];
static int hops_ready = 0;

static int is_site_parity(int px, int py, int pz)
{
    /* a doubled coordinate triple is an anion site iff exactly one is even */
    int ev = (px == 0) + (py == 0) + (pz == 0);
    return ev == 1;
}

static void or_hops(void)
{
    int t, hx, hy, hz, n;
    if (hops_ready) return;
    for (t = 0; t < 3; t++) {
        n = 0;
        for (hx = -1; hx <= 1; hx++)
            for (hy = -1; hy <= 1; hy++)
                for (hz = -1; hz <= 1; hz++) {
                    int px, py, pz;
                    if (hx * hx + hy * hy + hz * hz != 2) continue;
                    px = (TYPE_OFF[t][0] + hx) & 1;
                    py = (TYPE_OFF[t][1] + hy) & 1;
                    pz = (TYPE_OFF[t][2] + hz) & 1;
                    if (!is_site_parity(px, py, pz)) continue;
                    HOPS[t][n][0] = hx; HOPS[t][n][1] = hy; HOPS[t][n][2] = hz;
                    n++;
                }
    }
    hops_ready = 1;
}

void or_hop_table(int32_t out[3][8][3])
{
    int t, d, a;
    or_hops();
    for (t = 0; t < 3; t++)
        for (d = 0; d < 8; d++)
            for (a = 0; a < 3; a++) out[t][d][a] = HOPS[t][d][a];
}

static int64_t n_sites(const or_geom* g)
{
    return 3LL * g->L[0] * g->L[1] * g->L[2];
}

static void site_coords(const or_geom* g, int64_t n, int c[3], int* t)
{
    int64_t cell = n / 3;
    *t = (int)(n % 3);
    c[0] = (int)(cell % g->L[0]);
    c[1] = (int)((cell / g->L[0]) % g->L[1]);
    c[2] = (int)(cell / ((int64_t)g->L[0] * g->L[1]));
}

static int64_t site_index(const or_geom* g, const int c[3], int t)
{
    return (((int64_t)c[2] * g->L[1] + c[1]) * g->L[0] + c[0]) * 3 + t;
}

static int floordiv(int a, int b)
{
    int q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q--;
    return q;
}
static int modp(int a, int b)
{
    int r = a % b;
    return r < 0 ? r + b : r;
}

/* Target of hop d from site (c,t): returns its index and fills its cell. */
static int64_t hop_target(const or_geom* g, const int c[3], int t, int d, int tc[3], int* tt)
{
    int a, X[3];
    for (a = 0; a < 3; a++) {
        X[a] = modp(2 * c[a] + TYPE_OFF[t][a] + HOPS[t][d][a], 2 * g->L[a]);
        tc[a] = X[a] / 2;
    }
    if (X[0] % 2 == 0) *tt = 0;
    else if (X[1] % 2 == 0) *tt = 1;
    else *tt = 2;
    return site_index(g, tc, *tt);
}

/* Cell owning the hop edge {s, s+h}: the cell containing its midpoint. */
static void edge_owner(const or_geom* g, const int c[3], int t, int d, int own[3])
{
    int a;
    for (a = 0; a < 3; a++) {
        int X = 2 * c[a] + TYPE_OFF[t][a];
        own[a] = modp(floordiv(2 * X + HOPS[t][d][a], 4), g->L[a]);
    }
}

/* Grain-boundary sites: planes normal to axis a through cells with
 * index = 0 mod P; on such a plane lie the sites whose doubled coordinate
 * along a is even (type a). */
static int is_gb_site(const or_geom* g, const int c[3], int t)
{
    int P = g->gb_period_cells;
    if (g->gb_map) return g->gb_map[site_index(g, c, t)] != 0;
    if (P <= 0) return 0;
    if (!(g->gb_axes_mask & (1 << t))) return 0;
    return (c[t] % P) == 0;
}

/* ------------------------------------------------------------------------ */
/* Rate table (Eq. RateCnst1 with the ESP and boundary terms).  Entry
 * [X][dz+1][g] for ion species X in {O,H} exchanging with the vacancy, the
 * vacancy's z step dz in doubled units, and g = 1 when either end of the hop
 * lies on a grain-boundary site.  The hop changes the vacancy's electrostatic
 * energy by dE = -q E_z dz (a/2); half of it shifts the barrier, so that
 * forward and backward rates obey detailed balance. */
typedef struct {
    double nu, T, Ea_O, Ea_H, E_z, q;
    int32_t gb_period_cells, gb_axes_mask;
    double gb_dE;
} or_rates;

void or_rate_raw(const or_rates* p, double a_angstrom, double out[12])
{
    int X, dzi, g;
    for (X = 0; X < 2; X++)
        for (dzi = 0; dzi < 3; dzi++)
            for (g = 0; g < 2; g++) {
                double Ea = (X == 0) ? p->Ea_O : p->Ea_H;
                double dz = (double)(dzi - 1);
                double hs = a_angstrom * 1e-10 / 2.0;
                double dEf = -(p->q * p->E_z * dz * hs);
                double b = Ea + dEf / 2.0 + (double)g * p->gb_dE;
                out[(X * 3 + dzi) * 2 + g] = p->nu * exp(-b / (KB_EV * p->T));
            }
}

static int ceil_log2_u64(uint64_t n)
{
    int e = 0;
    while (((uint64_t)1 << e) < n) e++;
    return e;
}

/* Quantise the rates to integer multiples of q = 2^e, with e chosen so that a
 * sum of n_ev entries stays below 2^53 q: every partial sum of quantised rates
 * is then exact in binary64, whatever the summation order.  Returns 0, or -4
 * if a nonzero rate would keep fewer than 10 significant bits.
 * Also returns the maximum relative quantisation error. */
int or_quantise(const double raw[12], uint64_t n_ev, double out[12], double* q_out, double* max_rel)
{
    double kmax = 0.0, q;
    int i, e, ex;
    for (i = 0; i < 12; i++) {
        if (!(raw[i] >= 0.0) || isinf(raw[i])) return -1;
        if (raw[i] > kmax) kmax = raw[i];
    }
    if (n_ev < 1) n_ev = 1;
    *max_rel = 0.0;
    if (kmax == 0.0) {
        for (i = 0; i < 12; i++) out[i] = 0.0;
        *q_out = 0.0;
        return 0;
    }
    frexp(kmax, &ex);  /* kmax = f 2^ex, f in [0.5,1): ceil(log2 kmax) = ex, or ex-1 if f = 0.5 */
    if (ldexp(1.0, ex - 1) == kmax) ex = ex - 1;
    e = ex - 53 + ceil_log2_u64(n_ev);
    q = ldexp(1.0, e);
    for (i = 0; i < 12; i++) {
        double m = rint(raw[i] / q);
        out[i] = m * q;
        if (raw[i] > 0.0) {
            double rel = fabs(out[i] - raw[i]) / raw[i];
            if (m < 1024.0) return -4;
            if (rel > *max_rel) *max_rel = rel;
        }
    }
    *q_out = q;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Initial configuration: exactly n_vac vacancies, then n_h H, on distinct
 * uniformly chosen anion sites; all other sites O.  Draw d (d = 0, 1, ...)
 * uses Philox counter (d_lo, d_hi, 0, TAG_INIT) and key (seed, lattice_id);
 * its first two words give a 64-bit w, mapped to [0, N) by the 128-bit
 * product w*N (upper half), rejecting the low-half values that would bias it
 * (Lemire's method).  A draw hitting an occupied site is rejected too. */
int or_init_random(const or_geom* g, int8_t* occ, uint64_t n_vac, uint64_t n_h, uint64_t* draws_used)
{
    int64_t N = n_sites(g);
    uint64_t d = 0, i;
    uint32_t key[2], ctr[4], x[4];
    uint64_t thresh;
    if (n_vac + n_h > (uint64_t)N) return -1;
    memset(occ, SP_O, (size_t)N);
    key[0] = g->seed; key[1] = g->lattice_id;
    thresh = (0ull - (uint64_t)N) % (uint64_t)N;  /* 2^64 mod N */
    for (i = 0; i < n_vac + n_h; i++) {
        int8_t sp = (i < n_vac) ? SP_V : SP_H;
        for (;;) {
            uint64_t w;
            unsigned __int128 prod;
            uint64_t lo, j;
            ctr[0] = (uint32_t)d; ctr[1] = (uint32_t)(d >> 32); ctr[2] = 0; ctr[3] = TAG_INIT;
            d++;
            or_philox4x32_10(ctr, key, x);
            w = ((uint64_t)x[0] << 32) | x[1];
            prod = (unsigned __int128)w * (uint64_t)N;
            lo = (uint64_t)prod;
            j = (uint64_t)(prod >> 64);
            if (lo < thresh) continue;
            if (occ[j] != SP_O) continue;
            occ[j] = sp;
            break;
        }
    }
    if (draws_used) *draws_used = d;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Fragment decomposition along one axis: fragments of F cells, a remainder
 * r >= 2 forms its own fragment, r = 1 joins the last one; F <= 0 or F >= L
 * gives one fragment.  Each fragment is halved (lower ceil, upper floor). */
static int frag_count(int L, int F)
{
    int nf, r;
    if (F <= 0 || F >= L) return 1;
    nf = L / F;
    r = L - nf * F;
    if (r >= 2) nf++;
    return nf;
}
static void frag_range(int L, int F, int f, int* lo, int* hi)
{
    int nf = frag_count(L, F);
    if (nf == 1) { *lo = 0; *hi = L; return; }
    *lo = f * F;
    *hi = (f == nf - 1) ? L : (f + 1) * F;
}

int or_num_fragments(const or_geom* g)
{
    return frag_count(g->L[0], g->frag[0]) * frag_count(g->L[1], g->frag[1]) *
           frag_count(g->L[2], g->frag[2]);
}

/* Sub-block of fragment f with colour c: box [lo, hi) in cells. */
static void sub_block(const or_geom* g, int f, int c, int lo[3], int hi[3])
{
    int a, fi[3], nf[3];
    for (a = 0; a < 3; a++) nf[a] = frag_count(g->L[a], g->frag[a]);
    fi[0] = f % nf[0];
    fi[1] = (f / nf[0]) % nf[1];
    fi[2] = f / (nf[0] * nf[1]);
    for (a = 0; a < 3; a++) {
        int flo, fhi, mid, b = (c >> a) & 1;
        frag_range(g->L[a], g->frag[a], fi[a], &flo, &fhi);
        mid = flo + (fhi - flo + 1) / 2;
        if (b == 0) { lo[a] = flo; hi[a] = mid; }
        else { lo[a] = mid; hi[a] = fhi; }
    }
}

static int in_box(const int c[3], const int lo[3], const int hi[3])
{
    return c[0] >= lo[0] && c[0] < hi[0] && c[1] >= lo[1] && c[1] < hi[1] && c[2] >= lo[2] &&
           c[2] < hi[2];
}

/* Footprint of a sub-block: its own sites plus the sites that an edge owned
 * by one of its cells can reach outside it.  Decided by brute force over the
 * neighbouring cells, directly from the edge-ownership rule. */
static int in_footprint(const or_geom* g, const int c[3], int t, const int lo[3], const int hi[3])
{
    int d;
    if (in_box(c, lo, hi)) return 1;
    for (d = 0; d < 8; d++) {
        int own[3];
        edge_owner(g, c, t, d, own);
        if (in_box(own, lo, hi)) return 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One BKL step's event list over a fixed, ordered list of vacancy slots.
 * Event e = slot*8 + direction.  rate = 0 unless the hop edge is active (its
 * owner cell lies in box [lo,hi), or always when box == NULL) and the target
 * holds an ion (O or H). */
typedef struct site_ctx site_ctx;
static int site_failed(const site_ctx* X);

typedef struct {
    const or_geom* g;
    const double* k12;
    int8_t* occ;
    int32_t* disp; /* [N][3] */
    int64_t* slot_site;
    int n_slots;
    const int* lo;
    const int* hi;
    site_ctx* site; /* site-energy interactions (NULL: none) */
} step_ctx;

static double site_event_rate(const step_ctx* S, int64_t s, int64_t tgt, int X, int dzi, int g);

static double event_rate(const step_ctx* S, int64_t s, int d)
{
    int c[3], t, tc[3], tt, g, dzi, X;
    int64_t tgt;
    site_coords(S->g, s, c, &t);
    if (S->lo) {
        int own[3];
        edge_owner(S->g, c, t, d, own);
        if (!in_box(own, S->lo, S->hi)) return 0.0;
    }
    tgt = hop_target(S->g, c, t, d, tc, &tt);
    X = S->occ[tgt];
    if (X == SP_V) return 0.0;
    g = is_gb_site(S->g, c, t) || is_gb_site(S->g, tc, tt);
    dzi = HOPS[t][d][2] + 1;
    if (S->site) return site_event_rate(S, s, tgt, X, dzi, g);
    return S->k12[(X * 3 + dzi) * 2 + g];
}

/* Apply event e: swap the vacancy and the ion; each site's displacement
 * entry travels with its occupant (vacancy += h, ion -= h). */
static void apply_event(step_ctx* S, int e, uint64_t hops[2])
{
    int slot = e / 8, d = e % 8, c[3], t, tc[3], tt, a;
    int64_t s = S->slot_site[slot], tgt;
    int32_t dv[3], di[3];
    int X;
    site_coords(S->g, s, c, &t);
    tgt = hop_target(S->g, c, t, d, tc, &tt);
    X = S->occ[tgt];
    for (a = 0; a < 3; a++) {
        dv[a] = S->disp[s * 3 + a] + HOPS[t][d][a];
        di[a] = S->disp[tgt * 3 + a] - HOPS[t][d][a];
    }
    S->occ[s] = (int8_t)X;
    S->occ[tgt] = SP_V;
    for (a = 0; a < 3; a++) {
        S->disp[tgt * 3 + a] = dv[a];
        S->disp[s * 3 + a] = di[a];
    }
    hops[X]++;
    S->slot_site[slot] = tgt;
}

/* One BKL step (Eqs. TransitionProb, eventSelection, TimeStep).
 * Returns 0 = hop applied, 1 = no event possible, 2 = the next event falls
 * after the window end (draw discarded; waiting times are memoryless).
 * tau: window-relative clock; t_end: window length (<= 0: none). */
static int bkl_step(step_ctx* S, const uint32_t ctr[4], const uint32_t key[2], double* tau,
                    double t_end, uint64_t hops[2])
{
    int ne = S->n_slots * 8, e, last_pos = -1;
    double* k = (double*)malloc(sizeof(double) * (size_t)(ne > 0 ? ne : 1));
    double R = 0.0, u_sel, u_t, dt, tn, y, C;
    uint32_t x[4];
    for (e = 0; e < ne; e++) {
        k[e] = event_rate(S, S->slot_site[e / 8], e % 8);
        R = R + k[e];
        if (k[e] > 0.0) last_pos = e;
    }
    if (R == 0.0) { free(k); return 1; }
    or_philox4x32_10(ctr, key, x);
    u_sel = u53_open1(x[0], x[1]);
    u_t = u53_open0(x[2], x[3]);
    dt = -or_ln(u_t) / R;
    tn = *tau + dt;
    if (t_end > 0.0 && tn > t_end) { free(k); return 2; }
    *tau = tn;
    /* selected event: the first l whose cumulative rate exceeds u_sel * R */
    y = u_sel * R;
    C = 0.0;
    for (e = 0; e < ne; e++) {
        C = C + k[e];
        if (C > y) break;
    }
    if (e == ne) e = last_pos; /* u_sel*R rounded up to R */
    free(k);
    apply_event(S, e, hops);
    return 0;
}

static int cmp_i64(const void* a, const void* b)
{
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

/* One phase: sub-block of fragment f with colour c, during cycle n.
 * Every endpoint of an edge owned by a cell of the sub-block lies in the
 * owner cell or in its +1 neighbour along one axis, so the footprint is
 * contained in the box [lo, hi] (one extra cell layer, periodic); the
 * candidates are taken from that box and filtered by in_footprint(). */
static int phase_run(const or_geom* g, const double k12[12], site_ctx* X, int8_t* occ, int32_t* disp,
                     double t_sync, uint64_t n, int c, int f, uint64_t hops[2], uint64_t* steps_out);

int or_phase(const or_geom* g, const double k12[12], int8_t* occ, int32_t* disp, double t_sync,
             uint64_t n, int c, int f, uint64_t hops[2], uint64_t* steps_out)
{
    return phase_run(g, k12, NULL, occ, disp, t_sync, n, c, f, hops, steps_out);
}

/* The phase itself; with a site-energy context X the rates are those of the
 * site model (k12 unused), and the phase ends early when an event's |dE|
 * exceeded the window (X->err). */
static int phase_run(const or_geom* g, const double k12[12], site_ctx* X, int8_t* occ, int32_t* disp,
                     double t_sync, uint64_t n, int c, int f, uint64_t hops[2], uint64_t* steps_out)
{
    int lo[3], hi[3], a, cc[3], t, ext[3], i, j, k, w;
    int n_slots = 0, cap = 64, m;
    int64_t* slots = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
    step_ctx S;
    double tau = 0.0;
    uint32_t step = 0, key[2], ctr[4];
    or_hops();
    sub_block(g, f, c, lo, hi);
    for (a = 0; a < 3; a++) {
        ext[a] = hi[a] - lo[a] + 1;
        if (ext[a] > g->L[a]) ext[a] = g->L[a];
    }
    /* slots: vacancies of the footprint, ascending canonical index */
    for (k = 0; k < ext[2]; k++)
        for (j = 0; j < ext[1]; j++)
            for (i = 0; i < ext[0]; i++)
                for (t = 0; t < 3; t++) {
                    int64_t s;
                    cc[0] = (lo[0] + i) % g->L[0];
                    cc[1] = (lo[1] + j) % g->L[1];
                    cc[2] = (lo[2] + k) % g->L[2];
                    s = site_index(g, cc, t);
                    if (occ[s] != SP_V) continue;
                    if (!in_footprint(g, cc, t, lo, hi)) continue;
                    if (n_slots == cap) {
                        cap *= 2;
                        slots = (int64_t*)realloc(slots, sizeof(int64_t) * (size_t)cap);
                    }
                    slots[n_slots++] = s;
                }
    qsort(slots, (size_t)n_slots, sizeof(int64_t), cmp_i64);
    /* drop duplicates (none unless the extended box wraps onto itself) */
    for (m = 0, w = 0; m < n_slots; m++)
        if (w == 0 || slots[w - 1] != slots[m]) slots[w++] = slots[m];
    n_slots = w;
    S.g = g; S.k12 = k12; S.occ = occ; S.disp = disp;
    S.slot_site = slots; S.n_slots = n_slots; S.lo = lo; S.hi = hi; S.site = X;
    key[0] = g->seed; key[1] = g->lattice_id;
    for (;;) {
        int r;
        ctr[0] = step; ctr[1] = (uint32_t)f; ctr[2] = (uint32_t)n; ctr[3] = ((uint32_t)c << 8) | TAG_BKL;
        r = bkl_step(&S, ctr, key, &tau, t_sync, hops);
        if (r != 0) break;
        step++;
        if (X && site_failed(X)) break;
    }
    if (steps_out) *steps_out = step;
    free(slots);
    return 0;
}

/* Fragment kMC: cycles of 8 phases (colours 0..7 in order, fragments in
 * ascending index); each phase advances every sub-block of that colour to the
 * window end t_sync independently.  Cycles are numbered from cycle0.  Stops
 * after a cycle once hops in this call >= min_hops (min_hops > 0), or after
 * max_cycles cycles. */
int or_advance_frag(const or_geom* g, const double k12[12], int8_t* occ, int32_t* disp,
                    double t_sync, uint64_t cycle0, uint64_t max_cycles, uint64_t min_hops,
                    uint64_t hops[2], uint64_t* cycles_done)
{
    int nf = or_num_fragments(g), c, f;
    uint64_t n = 0;
    hops[0] = hops[1] = 0;
    while (n < max_cycles) {
        for (c = 0; c < 8; c++)
            for (f = 0; f < nf; f++) or_phase(g, k12, occ, disp, t_sync, cycle0 + n, c, f, hops, NULL);
        n++;
        if (min_hops > 0 && hops[0] + hops[1] >= min_hops) break;
    }
    *cycles_done = n;
    return 0;
}

/* Plain (unfragmented) BKL over the whole lattice.  Slots: all vacancies in
 * ascending canonical index at the start of the call.  Draw number d (a
 * persistent counter) uses Philox counter (d_lo, d_hi, 0xFFFFFFFF,
 * TAG_PLAIN).  The clock t advances by -ln(u)/R per hop (Eq. TimeStep).
 * Performs exactly n_hops hops, unless t_horizon > 0 and the next event would
 * fall after t_end = t + t_horizon (then t = t_end, the draw is consumed),
 * or no event is possible. */
int or_advance_plain(const or_geom* g, const double k12[12], int8_t* occ, int32_t* disp,
                     uint64_t* draws, double* t, double t_horizon, uint64_t n_hops, uint64_t hops[2])
{
    int64_t N = n_sites(g), s;
    int n_slots = 0;
    int64_t* slots;
    step_ctx S;
    uint32_t key[2], ctr[4];
    uint64_t done = 0;
    double t_end;
    or_hops();
    for (s = 0; s < N; s++) n_slots += (occ[s] == SP_V);
    slots = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_slots > 0 ? n_slots : 1));
    n_slots = 0;
    for (s = 0; s < N; s++)
        if (occ[s] == SP_V) slots[n_slots++] = s;
    S.g = g; S.k12 = k12; S.occ = occ; S.disp = disp;
    S.slot_site = slots; S.n_slots = n_slots; S.lo = NULL; S.hi = NULL; S.site = NULL;
    key[0] = g->seed; key[1] = g->lattice_id;
    hops[0] = hops[1] = 0;
    t_end = t_horizon > 0.0 ? *t + t_horizon : 0.0;
    while (done < n_hops) {
        int r;
        double tau = *t;
        ctr[0] = (uint32_t)*draws; ctr[1] = (uint32_t)(*draws >> 32);
        ctr[2] = 0xFFFFFFFFu; ctr[3] = TAG_PLAIN;
        r = bkl_step(&S, ctr, key, &tau, t_end, hops);
        if (r == 1) break;
        *draws = *draws + 1;
        if (r == 2) { *t = t_end; break; }
        *t = tau;
        done++;
    }
    free(slots);
    return 0;
}

/* Atom-selection fragment kMC with null events (Sec. "Atomic-based fragment
 * kMC method", Eqs. AtomP and TimeStepFrg), over the whole lattice.
 *
 * Readings of the paper (it leaves these open):
 *  - an "atom" I is a vacancy: every event of this model is a vacancy hop,
 *    so R_I is the sum of the rates of a vacancy's 8 hops, and R^max the
 *    largest R_I at the start of the stage;
 *  - a stage selects N^frg atoms, each uniformly and independently (with
 *    replacement) among the vacancies, slot a = floor(x0 * n / 2^32);
 *  - each selected atom takes its event i with probability k_i / R^max,
 *    else a null event: the first event whose cumulative rate exceeds
 *    u * R^max, none when u * R^max >= R_I;
 *  - every selection is decided on the rates at the start of the stage; the
 *    non-null events are then applied in selection order, and one whose
 *    vacancy or target site an earlier applied event of the stage touched
 *    becomes null (this covers an atom selected twice);
 *  - t advances by N^updated * (-ln r') / sum_i k_i with one r' per stage
 *    and the total rate at the stage start (Eq. TimeStepFrg).
 * Slots are the vacancies in ascending canonical index at the start of the
 * call, each following its vacancy.  Stage number n (a persistent counter)
 * draws selection j from Philox counter (n_lo, n_hi, j, TAG_ATOM) (x0: the
 * atom, x2 x3: u in [0,1)) and r' from (n_lo, n_hi, 0xFFFFFFFF, TAG_ATOM)
 * (x2 x3: u in (0,1]).  Runs n_stages stages, fewer when no event is
 * possible. */
int or_advance_atomic(const or_geom* g, const double k12[12], int8_t* occ, int32_t* disp,
                      uint64_t* stages, double* t, uint32_t n_frg, uint64_t n_stages,
                      uint64_t hops[2])
{
    int64_t N = n_sites(g), s;
    int n_slots = 0, j, a, d;
    int64_t *slots, *touched;
    double *k, *RI;
    int *sel_slot, *sel_ev;
    step_ctx S;
    uint32_t key[2], ctr[4], x[4];
    uint64_t st;
    or_hops();
    for (s = 0; s < N; s++) n_slots += (occ[s] == SP_V);
    slots = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_slots > 0 ? n_slots : 1));
    k = (double*)malloc(sizeof(double) * (size_t)(n_slots > 0 ? 8 * n_slots : 1));
    RI = (double*)malloc(sizeof(double) * (size_t)(n_slots > 0 ? n_slots : 1));
    sel_slot = (int*)malloc(sizeof(int) * (size_t)(n_frg > 0 ? n_frg : 1));
    sel_ev = (int*)malloc(sizeof(int) * (size_t)(n_frg > 0 ? n_frg : 1));
    touched = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * (n_frg > 0 ? n_frg : 1)));
    n_slots = 0;
    for (s = 0; s < N; s++)
        if (occ[s] == SP_V) slots[n_slots++] = s;
    S.g = g; S.k12 = k12; S.occ = occ; S.disp = disp;
    S.slot_site = slots; S.n_slots = n_slots; S.lo = NULL; S.hi = NULL; S.site = NULL;
    key[0] = g->seed; key[1] = g->lattice_id;
    hops[0] = hops[1] = 0;
    for (st = 0; st < n_stages; st++) {
        double Rmax = 0.0, K = 0.0, u, dt;
        int n_touched = 0, n_upd = 0;
        /* rates at the start of the stage: R_I, R^max and sum_i k_i */
        for (a = 0; a < n_slots; a++) {
            RI[a] = 0.0;
            for (d = 0; d < 8; d++) {
                k[a * 8 + d] = event_rate(&S, slots[a], d);
                RI[a] = RI[a] + k[a * 8 + d];
            }
            if (RI[a] > Rmax) Rmax = RI[a];
            K = K + RI[a];
        }
        if (K == 0.0) break;
        /* N^frg atoms, each with an event of probability k_i / R^max or null */
        for (j = 0; j < (int)n_frg; j++) {
            double y, C = 0.0;
            ctr[0] = (uint32_t)*stages; ctr[1] = (uint32_t)(*stages >> 32);
            ctr[2] = (uint32_t)j; ctr[3] = TAG_ATOM;
            or_philox4x32_10(ctr, key, x);
            a = (int)(((uint64_t)x[0] * (uint64_t)n_slots) >> 32);
            y = u53_open1(x[2], x[3]) * Rmax;
            sel_slot[j] = a;
            sel_ev[j] = -1;
            for (d = 0; d < 8; d++) {
                C = C + k[a * 8 + d];
                if (C > y) { sel_ev[j] = d; break; }
            }
        }
        /* apply in selection order; a hop onto or from a site an earlier
         * hop of this stage touched is null */
        for (j = 0; j < (int)n_frg; j++) {
            int c[3], tt, tc[3], tq, m, clash = 0;
            int64_t src, tgt;
            if (sel_ev[j] < 0) continue;
            src = slots[sel_slot[j]];
            site_coords(g, src, c, &tt);
            tgt = hop_target(g, c, tt, sel_ev[j], tc, &tq);
            for (m = 0; m < n_touched; m++)
                if (touched[m] == src || touched[m] == tgt) clash = 1;
            if (clash) continue;
            apply_event(&S, sel_slot[j] * 8 + sel_ev[j], hops);
            touched[n_touched++] = src;
            touched[n_touched++] = tgt;
            n_upd++;
        }
        /* Eq. TimeStepFrg */
        ctr[0] = (uint32_t)*stages; ctr[1] = (uint32_t)(*stages >> 32);
        ctr[2] = 0xFFFFFFFFu; ctr[3] = TAG_ATOM;
        or_philox4x32_10(ctr, key, x);
        u = u53_open0(x[2], x[3]);
        dt = -or_ln(u) / K;
        *t = *t + dt * (double)n_upd;
        *stages = *stages + 1;
    }
    free(slots); free(k); free(RI); free(sel_slot); free(sel_ev); free(touched);
    return 0;
}

/* Footprint membership query, exposed for the tests of the decomposition. */
int or_footprint_sites(const or_geom* g, int f, int c, int64_t* out, int64_t cap)
{
    int lo[3], hi[3], cc[3], t;
    int64_t N = n_sites(g), s, n = 0;
    or_hops();
    sub_block(g, f, c, lo, hi);
    for (s = 0; s < N; s++) {
        site_coords(g, s, cc, &t);
        if (in_footprint(g, cc, t, lo, hi)) {
            if (n < cap) out[n] = s;
            n++;
        }
    }
    return (int)n;
}

/* Edge owner and activity, exposed for the tests of the decomposition. */
int or_edge_active(const or_geom* g, int64_t s, int d, int f, int c)
{
    int lo[3], hi[3], cc[3], t, own[3];
    or_hops();
    sub_block(g, f, c, lo, hi);
    site_coords(g, s, cc, &t);
    edge_owner(g, cc, t, d, own);
    return in_box(own, lo, hi);
}

int64_t or_hop_target(const or_geom* g, int64_t s, int d)
{
    int cc[3], t, tc[3], tt;
    or_hops();
    site_coords(g, s, cc, &t);
    return hop_target(g, cc, t, d, tc, &tt);
}

int or_is_gb_site(const or_geom* g, int64_t s)
{
    int cc[3], t;
    site_coords(g, s, cc, &t);
    return is_gb_site(g, cc, t);
}

void or_sub_block(const or_geom* g, int f, int c, int32_t lo[3], int32_t hi[3])
{
    int l[3], h[3], a;
    sub_block(g, f, c, l, h);
    for (a = 0; a < 3; a++) { lo[a] = l[a]; hi[a] = h[a]; }
}

/* ------------------------------------------------------------------------ */
/* Site-energy interactions (Sec. "Oxygen vacancy diffusion with dopant and
 * defect interaction", Table TABLEadd01).  The hop rate becomes
 * k = A exp(-(Ea + dE_site/2 + field and boundary terms)/(k_B T)), where
 * dE_site is the vacancy's site energy at the target minus that at its
 * origin, and a site energy sums pair energies over the Fe dopants (on B
 * sites, the cube centres) and the other vacancies within the tabulated
 * shells: E_site(s) = sum_shell (number of Fe in the shell) e_Fe[shell] +
 * sum_shell (number of other vacancies in the shell) e_VV[shell].
 *
 * Shells by squared distance in (a/2)^2, minimum image:
 *  - vacancy-Fe (O site to B site): 1, 5, 9, 13 (a/2, 1.12 a, 1.5 a, 1.80 a);
 *  - vacancy-vacancy (O site to O site): 2, 4, 6, 8, 10, 16 (a/sqrt2, a,
 *    1.22 a, 1.41 a, 1.58 a, 2 a); any other distance contributes 0.
 * Energies are integers in meV, so site energies and their differences are
 * exact.  The hopping vacancy does not interact with itself: the target's
 * energy is taken without the vacancy at the origin.  Rates are
 * k = quantise(k12raw[X][dz][g] * f[dE]), f[dE] = exp(-dE meV / (2 k_B T)),
 * for |dE| <= window meV; the quantum is set by the largest product, as in
 * or_quantise.  The draws, clock and selection are those of plain BKL
 * (or_advance_plain): with all pair energies zero the trajectory is plain
 * BKL's, bit for bit. */
typedef struct {
    int32_t e_fe[4];
    int32_t e_vv[6];
    int32_t window;
} or_site_params;

struct site_ctx {
    const uint8_t* fe;      /* [L2][L1][L0] cells: 1 = Fe on the cell's B site */
    const or_site_params* sp;
    const double* raw12;    /* unquantised rates of Eq. RateCnst1 (zeroed absent species) */
    const double* f;        /* [2 window + 1] */
    double q;
    int err;                /* a hop's |dE| exceeded the window */
};

static int shell_fe(int n)
{
    return n == 1 ? 0 : (n == 5 ? 1 : (n == 9 ? 2 : (n == 13 ? 3 : -1)));
}

static int shell_vv(int n)
{
    return n == 2 ? 0 : (n == 4 ? 1 : (n == 6 ? 2 : (n == 8 ? 3 : (n == 10 ? 4 : (n == 16 ? 5 : -1)))));
}

/* Site energy (meV) of a vacancy on O site s: Fe pairs and vacancy pairs,
 * leaving out the vacancy on site `skip` (and s itself).  Brute force over
 * every lattice point within squared doubled distance 16. */
int32_t or_site_energy(const or_geom* g, const int8_t* occ, const uint8_t* fe, const or_site_params* sp,
                       int64_t s, int64_t skip)
{
    int c[3], t, P[3], dX, dY, dZ, a;
    int32_t E = 0;
    site_coords(g, s, c, &t);
    P[0] = 2 * c[0] + (t != 0);
    P[1] = 2 * c[1] + (t != 1);
    P[2] = 2 * c[2] + (t != 2);
    for (dX = -4; dX <= 4; dX++)
        for (dY = -4; dY <= 4; dY++)
            for (dZ = -4; dZ <= 4; dZ++) {
                int n = dX * dX + dY * dY + dZ * dZ, Q[3], odd = 0;
                if (n == 0 || n > 16) continue;
                Q[0] = modp(P[0] + dX, 2 * g->L[0]);
                Q[1] = modp(P[1] + dY, 2 * g->L[1]);
                Q[2] = modp(P[2] + dZ, 2 * g->L[2]);
                for (a = 0; a < 3; a++) odd += Q[a] & 1;
                if (odd == 3) {          /* B site: the centre of cell Q/2 */
                    int sh = shell_fe(n);
                    int64_t cell = ((int64_t)(Q[2] >> 1) * g->L[1] + (Q[1] >> 1)) * g->L[0] + (Q[0] >> 1);
                    if (sh >= 0 && fe[cell]) E += sp->e_fe[sh];
                } else if (odd == 2) {   /* O site: type = the even coordinate */
                    int sh = shell_vv(n), cc[3], tt = (Q[0] & 1) == 0 ? 0 : ((Q[1] & 1) == 0 ? 1 : 2);
                    int64_t u;
                    cc[0] = Q[0] >> 1;
                    cc[1] = Q[1] >> 1;
                    cc[2] = Q[2] >> 1;
                    u = site_index(g, cc, tt);
                    if (sh >= 0 && u != skip && u != s && occ[u] == SP_V) E += sp->e_vv[sh];
                }
            }
    return E;
}

static double site_event_rate(const step_ctx* S, int64_t s, int64_t tgt, int X, int dzi, int g)
{
    site_ctx* C = S->site;
    const int32_t W = C->sp->window;
    const int32_t dE = or_site_energy(S->g, S->occ, C->fe, C->sp, tgt, s) -
                       or_site_energy(S->g, S->occ, C->fe, C->sp, s, s);
    double k;
    if (dE < -W || dE > W) {
        C->err = 1;
        return 0.0;
    }
    k = C->raw12[(X * 3 + dzi) * 2 + g] * C->f[dE + W];
    return rint(k / C->q) * C->q;
}

/* Factors f[j] = exp(-(j - window) meV / (2 k_B T)), j = 0 .. 2 window, and
 * the quantum of the products raw12[i] * f[j] (as or_quantise: q = 2^e,
 * e = ceil(log2 kmax) - 53 + ceil(log2 n_ev)).  Returns -4 when a nonzero
 * product would keep fewer than 10 significant bits, -1 on bad input. */
int or_site_table(const double raw12[12], double T, int32_t window, uint64_t n_ev, double* f, double* q_out,
                  double* max_rel)
{
    double kmax = 0.0, q, rmax = 0.0;
    int i, e, ex;
    int32_t j;
    if (window < 0 || !(T > 0.0)) return -1;
    for (j = 0; j <= 2 * window; j++) f[j] = exp(-((double)(j - window) * 1e-3) / (2.0 * KB_EV * T));
    for (i = 0; i < 12; i++) {
        if (!(raw12[i] >= 0.0) || isinf(raw12[i])) return -1;
        if (raw12[i] > rmax) rmax = raw12[i];
    }
    *max_rel = 0.0;
    *q_out = 0.0;
    if (rmax == 0.0) return 0;
    kmax = rmax * f[0];
    if (n_ev < 1) n_ev = 1;
    frexp(kmax, &ex);
    if (ldexp(1.0, ex - 1) == kmax) ex = ex - 1;
    e = ex - 53 + ceil_log2_u64(n_ev);
    q = ldexp(1.0, e);
    for (i = 0; i < 12; i++) {
        if (raw12[i] == 0.0) continue;
        for (j = 0; j <= 2 * window; j++) {
            double k = raw12[i] * f[j], m = rint(k / q);
            double rel = fabs(m * q - k) / k;
            if (m < 1024.0) return -4;
            if (rel > *max_rel) *max_rel = rel;
        }
    }
    *q_out = q;
    return 0;
}

/* Plain BKL (as or_advance_plain: same draws, clock and selection) with
 * site-energy interactions.  Returns 0, or -4 when an event's |dE| exceeded
 * the window (its rate was taken as 0; the call stops after that step, and
 * the trajectory no longer follows the method). */
int or_advance_plain_site(const or_geom* g, const double raw12[12], const double* f, double q,
                          const uint8_t* fe, const or_site_params* sp, int8_t* occ, int32_t* disp,
                          uint64_t* draws, double* t, double t_horizon, uint64_t n_hops, uint64_t hops[2])
{
    int64_t N = n_sites(g), s;
    int n_slots = 0, rc = 0;
    int64_t* slots;
    step_ctx S;
    site_ctx X;
    uint32_t key[2], ctr[4];
    uint64_t done = 0;
    double t_end;
    or_hops();
    for (s = 0; s < N; s++) n_slots += (occ[s] == SP_V);
    slots = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_slots > 0 ? n_slots : 1));
    n_slots = 0;
    for (s = 0; s < N; s++)
        if (occ[s] == SP_V) slots[n_slots++] = s;
    X.fe = fe; X.sp = sp; X.raw12 = raw12; X.f = f; X.q = q; X.err = 0;
    S.g = g; S.k12 = NULL; S.occ = occ; S.disp = disp;
    S.slot_site = slots; S.n_slots = n_slots; S.lo = NULL; S.hi = NULL; S.site = &X;
    key[0] = g->seed; key[1] = g->lattice_id;
    hops[0] = hops[1] = 0;
    t_end = t_horizon > 0.0 ? *t + t_horizon : 0.0;
    while (done < n_hops) {
        int r;
        double tau = *t;
        ctr[0] = (uint32_t)*draws; ctr[1] = (uint32_t)(*draws >> 32);
        ctr[2] = 0xFFFFFFFFu; ctr[3] = TAG_PLAIN;
        r = bkl_step(&S, ctr, key, &tau, t_end, hops);
        if (X.err) { rc = -4; break; }
        if (r == 1) break;
        *draws = *draws + 1;
        if (r == 2) { *t = t_end; break; }
        *t = tau;
        done++;
    }
    free(slots);
    return rc;
}

static int site_failed(const site_ctx* X)
{
    return X->err;
}

/* Squared doubled distance of the farthest vacancy-vacancy shell with a
 * nonzero energy (0 when there is none). */
int or_site_vv_reach(const or_site_params* sp)
{
    static const int N[6] = {2, 4, 6, 8, 10, 16};
    int k, r = 0;
    for (k = 0; k < 6; k++)
        if (sp->e_vv[k] != 0) r = N[k];
    return r;
}

/* Fragment kMC (or_advance_frag: the same cycles, phases, draws and clock)
 * with the site-energy interactions of or_advance_plain_site.  The rates of
 * a sub-block's edges read site energies at its footprint's sites, which
 * sum over vacancies within the vacancy-vacancy reach (the Fe dopants do
 * not move).  Along an axis, a footprint spans doubled coordinates
 * [2o, 2o + 2w] and the nearest footprint of the same colour begins 2w'
 * further on, w' the width of the sub-block between them; when 4 w'^2
 * exceeds the reach for every sub-block, no sub-block's rates read a site
 * that another sub-block of the same colour changes, and the sub-blocks of
 * a phase are independent (any order of them gives the same result)
 * without a frozen halo.  Returns 0; -1 when a sub-block is too narrow for
 * the reach; -4 when an event's |dE| exceeded the window (its rate was
 * taken as 0; the call stops after that phase, and the trajectory no
 * longer follows the method). */
int or_advance_frag_site(const or_geom* g, const double raw12[12], const double* f, double q,
                         const uint8_t* fe, const or_site_params* sp, int8_t* occ, int32_t* disp,
                         double t_sync, uint64_t cycle0, uint64_t max_cycles, uint64_t min_hops,
                         uint64_t hops[2], uint64_t* cycles_done)
{
    int nf = or_num_fragments(g), c, fi, a, k, reach = or_site_vv_reach(sp);
    uint64_t n = 0;
    site_ctx X;
    *cycles_done = 0;
    hops[0] = hops[1] = 0;
    for (a = 0; a < 3; a++) {
        int nfa = frag_count(g->L[a], g->frag[a]);
        for (k = 0; k < nfa; k++) {
            int flo, fhi, w;
            frag_range(g->L[a], g->frag[a], k, &flo, &fhi);
            w = (fhi - flo) / 2;  /* the narrower sub-block of the fragment */
            if (4 * w * w <= reach) return -1;
        }
    }
    X.fe = fe; X.sp = sp; X.raw12 = raw12; X.f = f; X.q = q; X.err = 0;
    while (n < max_cycles) {
        for (c = 0; c < 8; c++) {
            for (fi = 0; fi < nf; fi++) phase_run(g, NULL, &X, occ, disp, t_sync, cycle0 + n, c, fi, hops, NULL);
            if (X.err) {
                *cycles_done = n;
                return -4;
            }
        }
        n++;
        if (min_hops > 0 && hops[0] + hops[1] >= min_hops) break;
    }
    *cycles_done = n;
    return 0;
}

/* One phase of or_advance_frag_site (sub-block of fragment f, colour c,
 * cycle n), for tests of the order of a phase's sub-blocks; no width check.
 * Returns 0, or -4 when an event's |dE| exceeded the window. */
int or_phase_site(const or_geom* g, const double raw12[12], const double* f, double q, const uint8_t* fe,
                  const or_site_params* sp, int8_t* occ, int32_t* disp, double t_sync, uint64_t n, int c,
                  int fi, uint64_t hops[2])
{
    site_ctx X;
    X.fe = fe; X.sp = sp; X.raw12 = raw12; X.f = f; X.q = q; X.err = 0;
    hops[0] = hops[1] = 0;
    phase_run(g, NULL, &X, occ, disp, t_sync, n, c, fi, hops, NULL);
    return X.err ? -4 : 0;
}

/* Rate of event d of the vacancy on site s under the site-energy model
 * (0 when the target holds a vacancy; -1 when |dE| exceeds the window). */
double or_site_rate(const or_geom* g, const double raw12[12], const double* f, double q, const uint8_t* fe,
                    const or_site_params* sp, const int8_t* occ, int64_t s, int d)
{
    step_ctx S;
    site_ctx X;
    double k;
    or_hops();
    X.fe = fe; X.sp = sp; X.raw12 = raw12; X.f = f; X.q = q; X.err = 0;
    S.g = g; S.k12 = NULL; S.occ = (int8_t*)occ; S.disp = NULL;
    S.slot_site = NULL; S.n_slots = 0; S.lo = NULL; S.hi = NULL; S.site = &X;
    k = event_rate(&S, s, d);
    return X.err ? -1.0 : k;
}
