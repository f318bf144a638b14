/*
 * fkmc.h - C ABI of the MI355X fragment kinetic Monte Carlo library.
 *
 * The library simulates vacancy-mediated diffusion of O and H on the anion
 * sublattice of a cubic ABO3 perovskite with rejection-free (BKL) kinetic
 * Monte Carlo (Nakata, arXiv:2004.09081, Sec. "Summary of the conventional
 * kMC method", Eqs. RateCnst1, TransitionProb, eventSelection, TimeStep),
 * split into spatial fragments that advance independently to a
 * synchronisation time (Sec. "Atomic-based fragment kMC method"; the
 * boundary rule is an 8-colour edge splitting, below).
 *
 * A handle holds a SET of n >= 1 independent lattices that advance together
 * (n = 1 is a single lattice; n > 1 is the batched ensemble).  All device
 * memory is owned by the caller (e.g. allocated through PyTorch) and passed in
 * at creation; the library keeps only host-side plans and tables.  Nothing in
 * this header uses C++ or framework types.
 *
 * Conventions
 *  - Every function returns fkmc_status: FKMC_OK (0) or a negative code.
 *    A failed call leaves the handle's state unchanged, except that an
 *    asynchronous device error is reported by the next fkmc_sync/read call.
 *    fkmc_last_error() returns a message for the calling thread.
 *  - Device work is enqueued on the HIP stream given at creation; calls that
 *    return data to the host synchronise that stream.
 *  - Handles are not thread-safe.  Two handles may share a device.
 *
 * Physics conventions
 *  - Species codes (int8): O = 0, H = 1, vacancy V = 2.
 *  - Lattice of L[0] x L[1] x L[2] cubic cells, periodic, 3 anion sites per
 *    cell: type 0 at (0, a/2, a/2), type 1 at (a/2, 0, a/2), type 2 at
 *    (a/2, a/2, 0) relative to the cell corner.  CANONICAL site order:
 *    n = ((k*L[1] + j)*L[0] + i)*3 + type.  Each site has 8 neighbours at
 *    a/sqrt(2); a hop swaps a vacancy with a neighbouring O or H.
 *  - Displacements are int32 triples in units of a/2, unwrapped; each site's
 *    entry travels with its occupant (the vacancy gains h, the ion -h).
 *  - Rate of a hop (Eq. RateCnst1 with the ESP term of the biased run):
 *    k = nu exp(-(Ea_X + dE/2 + g dE_gb)/(k_B T)), X the ion species,
 *    dE = -q E_z dz (a/2) the vacancy's electrostatic energy change for a z
 *    step dz in {-1,0,+1} (units of a/2), g = 1 when either end lies on a
 *    grain-boundary site.  Rates are rounded to integer multiples of a power
 *    of two q chosen so that any sum of the rates of one domain is exact in
 *    binary64; results are therefore independent of summation order.
 *  - Fragment mode (frag > 0): fragments of frag[a] cells per axis (a last
 *    remainder of >= 2 cells is its own fragment, 1 cell joins the last),
 *    each halved per axis into 8 sub-blocks of colour bx + 2 by + 4 bz.  A
 *    hop edge belongs to the sub-block holding its midpoint.  One CYCLE runs
 *    colours 0..7 in order; in each PHASE every sub-block of that colour
 *    advances its own BKL clock from 0 to t_sync (a draw landing after
 *    t_sync is discarded), and the sub-blocks of one colour never share a
 *    site.  The lattice clock then advances by t_sync per cycle.
 *  - Plain mode (frag all 0): one BKL domain over the whole lattice with a
 *    continuous clock (the conventional kMC of the paper).  Plain lattices
 *    can also run the paper's atom-selection scheme with null events
 *    (fkmc_advance_atomic).
 *  - Random numbers: Philox4x32-10 with key (seed, lattice_id).
 */
#ifndef FKMC_H
#define FKMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fkmc_status;
#define FKMC_OK 0
#define FKMC_E_INVALID -1     /* bad argument (null pointer, size, range) */
#define FKMC_E_STATE -2       /* call not valid in the current state */
#define FKMC_E_DEVICE -3      /* HIP runtime error */
#define FKMC_E_RANGE -4       /* rate below the quantisation floor, slot or
                                 counter overflow detected on the device */
#define FKMC_E_NOMEM -5       /* caller buffer too small or misaligned */
#define FKMC_E_UNSUPPORTED -6 /* configuration outside the supported limits */

typedef struct fkmc_lattice fkmc_lattice; /* opaque handle */

/* Geometry of one lattice.  L[a] >= 2.  frag[a] = 0 for all a selects plain
 * mode; otherwise every frag[a] must be > 0 (a value >= L[a] means one
 * fragment along that axis).  Sub-block edges must not exceed 100 cells. */
typedef struct {
    int32_t L[3];
    int32_t frag[3];
    double a_angstrom;   /* lattice constant, Angstrom */
    uint32_t seed;       /* Philox key word 0 */
    uint32_t lattice_id; /* Philox key word 1 */
} fkmc_geometry;

/* Rate parameters of one lattice (Eq. RateCnst1 plus field and boundary
 * terms).  Grain-boundary planes: normal to axis a when bit a of
 * gb_axes_mask is set, through every cell whose index along a is a multiple
 * of gb_period_cells (0 = none); the sites on such a plane are those of type
 * a in those cells. */
typedef struct {
    double nu;     /* attempt frequency, 1/s */
    double T;      /* temperature, K */
    double Ea_O;   /* O-vacancy exchange barrier, eV */
    double Ea_H;   /* H-vacancy exchange barrier, eV */
    double E_z;    /* uniform field along z, V/m */
    double q;      /* vacancy charge, units of e (+2 for an oxygen vacancy) */
    int32_t gb_period_cells;
    int32_t gb_axes_mask;
    double gb_dE;  /* extra barrier on boundary hops, eV */
} fkmc_rate_params;

/* Caller-owned device buffers (one allocation each, covering all lattices).
 * occ and work must be 256-byte aligned, disp 16-byte aligned. */
typedef struct {
    void* occ;   /* int8 occupancy, library storage order (not canonical) */
    void* disp;  /* int32x4 per site (x, y, z, unused), library order */
    void* work;  /* descriptors, counters, tables, and a staging slice for the
                    canonical-order transfers of fkmc_set_occupancy,
                    fkmc_read_state and fkmc_restore (up to 2^19 sites per
                    chunk, 13 bytes per site): the library allocates no
                    device memory of its own */
    size_t bytes[3];
} fkmc_buffers;

/* Statistics of one lattice, species index 0 = O, 1 = H, 2 = V. */
typedef struct {
    double t;              /* simulated time, s */
    uint64_t cycles;       /* fragment cycles completed (0 in plain mode) */
    uint64_t draws;        /* plain-mode random draws consumed */
    uint64_t hops[2];      /* hops of O and of H (vacancy hops = sum) */
    uint64_t count[3];     /* particles per species */
    int64_t sum_r[3][3];   /* sum of displacements, units of a/2 */
    int64_t sum_rr[3][6];  /* sum of r_a r_b: xx yy zz xy xz yz, (a/2)^2 */
    double msd[3];         /* mean square displacement, Angstrom^2 */
    double D[3];           /* tracer diffusion coefficient MSD/(6t), A^2/s */
    double drift[3][3];    /* mean velocity, Angstrom/s */
    double Dtensor[3][6];  /* (<r_a r_b> - <r_a><r_b>)/(2t), A^2/s */
    double busy_ms;        /* persistent schedule or fkmc_advance_atomic:
                              device time this lattice's workgroup took in
                              the last such call (ms) */
    uint32_t lds_resident; /* 1 if the last fkmc_advance ran the persistent
                              schedule with this lattice held in LDS (or the
                              last call was fkmc_advance_atomic) */
    uint32_t tile_group;   /* tiles a wavefront ran at once in the last
                              fkmc_advance on the persistent schedule (8, 4
                              or 1; 0 for other runs and plain lattices) */
} fkmc_stats;

/* Required byte sizes of the occ, disp and work buffers for n lattices. */
fkmc_status fkmc_query_sizes(const fkmc_geometry* geoms, uint32_t n, size_t bytes_out[3]);

/* Create a handle over n lattices in the given buffers; hip_stream may be
 * NULL (the null stream).  Zeroes occupancy (all O) and displacements. */
fkmc_status fkmc_create(const fkmc_geometry* geoms, uint32_t n, const fkmc_buffers* buf,
                        void* hip_stream, fkmc_lattice** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * handle as fkmc_create, but the work buffer is a static array of 64 MiB per
 * device held by the library (it stays allocated on every device the library
 * runs on until the process ends).  The caller passes only the occupancy and
 * displacement buffers (sizes and alignment as fkmc_query_sizes and
 * fkmc_buffers state; the work size it reports must not exceed 64 MiB, else
 * FKMC_E_NOMEM).  The call allocates nothing on the device or in pinned host
 * memory.  One such handle per device at a time: a second one while the
 * first lives returns FKMC_E_STATE (two handles on one array would race);
 * fkmc_destroy releases it.  The array keeps the previous handle's contents,
 * so creation clears all of it that the handle uses.  Every other call works
 * on the handle as on one from fkmc_create, with identical results. */
fkmc_status fkmc_create_static(const fkmc_geometry* geoms, uint32_t n, void* occ, size_t occ_bytes,
                               void* disp, size_t disp_bytes, void* hip_stream, fkmc_lattice** out);

/* Never frees the caller's buffers. */
fkmc_status fkmc_destroy(fkmc_lattice* lat);

uint32_t fkmc_count(const fkmc_lattice* lat);

/* Place exactly n_vac[i] vacancies then n_h[i] H on uniformly chosen
 * distinct sites of lattice i (all others O) and zero its displacements,
 * clock and counters.  Draw d uses Philox counter (d_lo, d_hi, 0, 1); its
 * first two words form a 64-bit w mapped to a site by the upper half of the
 * 128-bit product w*N, rejecting the low halves below 2^64 mod N, and
 * rejecting occupied sites.  Invalidates the rate tables. */
fkmc_status fkmc_init_random(fkmc_lattice* lat, const uint64_t* n_vac, const uint64_t* n_h);

/* Copy occupancy (canonical order, n bytes = 3 L0 L1 L2) into lattice i and
 * zero its displacements, clock and counters.  Values must be 0, 1 or 2
 * (checked on the host before any device work).  The data pass through the
 * work buffer's staging slice in chunks of at most 2^19 sites.  Invalidates
 * the rate tables. */
fkmc_status fkmc_set_occupancy(fkmc_lattice* lat, uint32_t i, const int8_t* host, size_t n);

/* Build and quantise the 12-entry rate table of every lattice from params[i]
 * (entry (X*3 + dz+1)*2 + g).  Entries of an ion species absent from the
 * lattice are set to zero first (hops conserve the species counts).  The
 * quantum is q = 2^e with
 * e = ceil(log2 kmax) - 53 + ceil(log2 n_ev), n_ev = 8 min(N_V, S), S the
 * largest number of sites in one BKL domain.  FKMC_E_RANGE when a nonzero
 * rate would keep fewer than 10 significant bits. */
fkmc_status fkmc_set_rates(fkmc_lattice* lat, const fkmc_rate_params* params);

/* Same quantisation applied to a caller-supplied raw table of lattice i. */
fkmc_status fkmc_set_rate_table(fkmc_lattice* lat, uint32_t i, const double* k12, size_t n);

/* Site-energy interactions (Sec. "Oxygen vacancy diffusion with dopant and
 * defect interaction", with the pair energies of its Table TABLEadd01 as
 * inputs), for lattices of at least 5 cells per axis: plain lattices with at
 * most 2048 vacancies, and fragment lattices whose sub-blocks are all wider
 * than the vacancy-vacancy reach (below).  The rate of a hop becomes
 * k = nu exp(-(Ea_X + dE/2 + g dE_gb + dE_site/2)/(k_B T)) with dE_site the
 * vacancy's site energy at the target minus that at its origin.  The site
 * energy of an anion site sums integer pair energies (meV) over the Fe
 * dopants on B sites (cube centres) at squared distance 1, 5, 9, 13 (a/2)^2
 * (e_fe[0..3]) and over the other vacancies at 2, 4, 6, 8, 10, 16 (a/2)^2
 * (e_vv[0..5]); the hopping vacancy does not interact with itself.  Every
 * possible rate, |dE_site| <= window_meV (0..2047), is tabulated as
 * quantise(k_Arrhenius x exp(-dE_site/(2 k_B T))) with the quantum of the
 * largest (FKMC_E_RANGE when a rate would keep fewer than 10 bits: narrow
 * the window).  A hop whose |dE_site| exceeds the window sets FKMC_E_RANGE
 * (the event counted as impossible; the trajectory no longer follows the
 * method).  Draws, clock and selection are those of the lattice's mode in
 * fkmc_advance (plain BKL, or the fragment cycle: phase c of cycle n in
 * fragment f, step s uses Philox counter (s, f, n, c*256 + 2), the domain a
 * sub-block's edges and its slots its footprint's vacancies), so with all
 * pair energies zero the run equals the same mode without them bit for bit
 * (fragment lattices: when the quanta agree, i.e. N_V is at most the
 * smallest footprint's site count).  A fragment lattice with a site model
 * runs the lockstep schedule whatever fkmc_set_schedule chose, one
 * workgroup per sub-block and phase, its occupancy in HBM; a footprint with
 * more than 256 vacancies sets FKMC_E_RANGE.  The rates of a sub-block read
 * site energies at its footprint's sites, which reach the vacancies within
 * the squared doubled distance of the farthest vacancy-vacancy shell with a
 * nonzero energy (the reach: 16 when e_vv[5] != 0, 10 when only e_vv[0..4]
 * are nonzero, ...); the footprint of the next sub-block of the same colour
 * lies 2w doubled units away, w the width of the sub-block between them, so
 * 4 w^2 > reach for every sub-block keeps the sub-blocks of a phase from
 * reading each other's sites (no frozen halo is needed).
 * Returns the bytes of the caller-owned device buffer that holds lattice
 * i's Fe bitmap and rate table for a given window. */
fkmc_status fkmc_site_model_bytes(const fkmc_lattice* lat, uint32_t i, int32_t window_meV, size_t* bytes);

/* Enable site energies on lattice i: fe (host, L0 L1 L2 bytes in
 * canonical cell order (k L1 + j) L0 + i, 1 = Fe on that cell's B site),
 * pair energies and window as above, dev a caller-owned device buffer of
 * fkmc_site_model_bytes bytes (256-byte aligned) that must outlive the
 * model.  Call after fkmc_set_rates (FKMC_E_STATE otherwise; the table
 * uses those parameters); fkmc_set_rates, fkmc_set_rate_table,
 * fkmc_init_random, fkmc_set_occupancy and fkmc_restore remove it.
 * FKMC_E_UNSUPPORTED for L < 5, a plain lattice of more than 2048
 * vacancies, or a fragment lattice with a sub-block of width w and
 * 4 w^2 <= the reach; fkmc_advance_atomic refuses lattices with a model. */
fkmc_status fkmc_set_site_model(fkmc_lattice* lat, uint32_t i, const uint8_t* fe, const int32_t e_fe[4],
                                const int32_t e_vv[6], int32_t window_meV, void* dev, size_t bytes);

/* Grain boundaries as a site map (Sec. "Oxygen diffusion in micro-scale
 * BaTiO3 model": grains from a Voronoi tessellation, separated by a
 * boundary layer whose hops carry the extra barrier gb_dE).  map (host, n
 * bytes in canonical site order, 1 = boundary site) replaces lattice i's
 * boundary planes: an edge with either end on a boundary site takes gb_dE
 * from its rate parameters.  dev is caller-owned device memory of
 * fkmc_gb_map_bytes bytes (256-byte aligned) that must outlive the map;
 * map = NULL removes it (the planes apply again).  Lattices with a map run
 * the tile-group fragment paths (both schedules) and, when plain, the HBM
 * plain kernel or the site-energy kernel; fkmc_advance_atomic refuses
 * them.  Results equal the oracle's with the same map. */
fkmc_status fkmc_gb_map_bytes(const fkmc_lattice* lat, uint32_t i, size_t* bytes);
fkmc_status fkmc_set_gb_map(fkmc_lattice* lat, uint32_t i, const uint8_t* map, void* dev, size_t bytes);

/* Current quantised table of lattice i (12 doubles). */
fkmc_status fkmc_get_rate_table(const fkmc_lattice* lat, uint32_t i, double* k12, size_t n);

/* Host-only: raw rates and their quantisation for one parameter set, the way
 * fkmc_set_rates computes them (no device needed).  q_out and max_rel_out
 * (maximum relative rounding error) may be NULL. */
fkmc_status fkmc_rate_table_host(const fkmc_rate_params* p, double a_angstrom, uint64_t n_ev,
                                 double raw_out[12], double quant_out[12], double* q_out,
                                 double* max_rel_out);

/* Largest number of sites of one BKL domain of a geometry (whole lattice in
 * plain mode, else the largest sub-block plus its three +faces). */
fkmc_status fkmc_max_domain_sites(const fkmc_geometry* g, uint64_t* out);

/* Advance every lattice (asynchronous on the stream).
 * Fragment lattices: run cycles with window t_sync[i] until the hops made in
 * this call reach min_hops (checked after each cycle; min_hops = 0 means no
 * hop target) or max_cycles cycles have run.  Cycle numbers continue across
 * calls.  Phase c of cycle n in fragment f, BKL step s uses Philox counter
 * (s, f, n, c*256 + 2).
 * Plain lattices: make exactly min_hops hops, stopping early when the next
 * event would land after t_start + t_sync[i] (t_sync[i] > 0; the clock is then
 * set to that time) or no event is possible.  Draw d uses Philox counter
 * (d_lo, d_hi, 0xFFFFFFFF, 3).  max_cycles is ignored.
 * t_sync may be NULL for plain-only sets (no horizon).
 * FKMC_E_RANGE when a BKL domain (a fragment lattice's sub-block plus its
 * three +faces) holds more than 128 vacancies, or a plain lattice on the
 * HBM kernel more than 8192; such a domain makes no hop in that phase, so
 * the trajectory no longer follows the method.  The error stays set: every
 * later advance, sync or read of the set reports it until fkmc_init_random
 * or fkmc_set_occupancy initialises that lattice again. */
fkmc_status fkmc_advance(fkmc_lattice* lat, const double* t_sync, uint64_t max_cycles,
                         uint64_t min_hops);

/* Atom-selection fragment kMC with null events (Sec. "Atomic-based fragment
 * kMC method", Eqs. AtomP and TimeStepFrg), for sets whose lattices are all
 * plain (fragment edge 0) with at most 8192 vacancies.  Runs n_stages
 * stages on every lattice (fewer when no event is possible), one workgroup
 * per lattice: a lattice that fits in LDS (at most 512 vacancies, occupancy
 * at 2 bits per site plus the rate table within 64 KB) runs there on one
 * wavefront unless fkmc_set_plain_lds turned that off; any other keeps its
 * occupancy in HBM and its vacancy slots in LDS.  Results are identical
 * either way.  An atom is a vacancy, its events its 8 hops.  A stage takes
 * the rates at its start (K = sum of all rates, R^max = largest vacancy
 * total), then n_frg (1..64) selections: selection j picks vacancy slot
 * floor(x0 * n_vac / 2^32) and its first hop whose cumulative rate exceeds
 * u * R^max, or a null event (Philox counter (n_lo, n_hi, j, 4) at stage n;
 * u from words 2 and 3, in [0,1)).  The hops are taken in selection order,
 * and one whose vacancy or target site an earlier taken hop of the stage
 * touched becomes null.  The clock moves by N_updated * (-ln r') / K with r'
 * from counter (n_lo, n_hi, 0xFFFFFFFF, 4).  Slots are the vacancies in
 * canonical order at the call start, each following its vacancy; the stage
 * counter is the lattice's draw counter (fkmc_stats.draws).  With n_frg = 1
 * the trajectory is an exact kMC trajectory; with more, simultaneous
 * selections make it the paper's parallel approximation.  Synchronous.
 * FKMC_E_UNSUPPORTED for a fragment lattice or one of more than 8192
 * vacancies; FKMC_E_STATE when rates are not set. */
fkmc_status fkmc_advance_atomic(fkmc_lattice* lat, uint32_t n_frg, uint64_t n_stages);

/* Scheduling of fragment lattices (results are identical under every
 * schedule):
 *  FKMC_SCHEDULE_LOCKSTEP: one kernel launch per phase covering every tile
 *    of every lattice, all lattices advancing cycle by cycle together (best
 *    for one large lattice);
 *  FKMC_SCHEDULE_PERSISTENT: one launch per fkmc_advance call, one
 *    workgroup of `waves` wavefronts per lattice running all its cycles,
 *    small lattices held entirely in LDS (best for ensembles);
 *  FKMC_SCHEDULE_AUTO (default): persistent for a set of at least 32
 *    fragment lattices, of several lattices of at most 49152 sites each, or
 *    of several lattices that the GPU can give a compute unit each (no
 *    more lattices than compute units) whose fragment lattices have at most
 *    128 tiles per colour; lockstep otherwise.
 *  waves in 1..8; 0 keeps the current value.  Until a value is set the
 *  persistent workgroups are sized per call: 8 wavefronts for a set that
 *  has at most one lattice per compute unit and at most 128 tiles per
 *  colour in each fragment lattice, else 4. */
#define FKMC_SCHEDULE_AUTO 0
#define FKMC_SCHEDULE_LOCKSTEP 1
#define FKMC_SCHEDULE_PERSISTENT 2
fkmc_status fkmc_set_schedule(fkmc_lattice* lat, int32_t schedule, int32_t waves);

/* Tile groups: a wavefront runs `group` tiles of a phase at once, each on
 * 64/group lanes with that many vacancy slots; a tile with more vacancies
 * runs afterwards on the whole wavefront.  group = 0 (default) chooses per
 * lattice from the mean vacancy count of a footprint (the lockstep schedule
 * then halves it while a launch would have fewer than 8 wavefronts per
 * compute unit); otherwise the
 * lockstep schedule uses group (1, 2, 4 or 8) and the persistent schedule
 * uses 8 or 4 when group is 8 or 4 and 1 (whole wavefront per tile) for any
 * other value, or when the staged footprints of that many tiles per
 * wavefront do not fit its LDS.  Results are identical for every group
 * size. */
fkmc_status fkmc_set_group(fkmc_lattice* lat, int32_t group);

/* Plain lattices (Eqs. TransitionProb, eventSelection, TimeStep over the
 * whole lattice): with enable = 1 (default) a plain lattice of at most 512
 * vacancies whose occupancy (2 bits per site) and per-slot rates fit in the
 * persistent kernel's LDS share (x and y edges up to 1023 cells, z up to
 * 512) runs there on one wavefront, in the same launch as the fragment
 * lattices when those use the persistent schedule; every other plain lattice
 * runs the HBM-resident plain kernel.  enable = 0 sends every plain lattice
 * to the HBM kernel, in fkmc_advance_atomic too.  Results are identical
 * either way. */
fkmc_status fkmc_set_plain_lds(fkmc_lattice* lat, int32_t enable);

/* Lockstep schedule: replay batches of 8 cycles from a prebuilt HIP graph
 * (1, default) or enqueue every kernel separately (0).  Results are
 * identical; event timing (fkmc_set_timing) always uses separate launches. */
fkmc_status fkmc_set_graph(fkmc_lattice* lat, int32_t enable);

/* Run exactly one phase (colour c of the current cycle) on every fragment
 * lattice, without completing the cycle: the lattice is left mid-cycle, and
 * only fkmc_run_phase or reads may follow until the 8 colours are done.
 * For checking single phases against the reference. */
fkmc_status fkmc_run_phase(fkmc_lattice* lat, const double* t_sync, int32_t colour);

/* Wait for the stream; report device-side errors. */
fkmc_status fkmc_sync(fkmc_lattice* lat);

/* Occupancy (n bytes) and displacements (3n int32) of lattice i in canonical
 * order; synchronises.  disp may be NULL.  The data pass through the work
 * buffer's staging slice in chunks of at most 2^19 sites. */
fkmc_status fkmc_read_state(fkmc_lattice* lat, uint32_t i, int8_t* occ, int32_t* disp, size_t n);

/* Statistics of every lattice (out[n]); synchronises. */
fkmc_status fkmc_read_stats(fkmc_lattice* lat, fkmc_stats* out);

/* Checkpoint of lattice i into a host buffer of fkmc_checkpoint_size()
 * bytes: geometry and key, canonical occupancy and displacements, clock,
 * cycle and draw counters, hop counters and the quantised rate table.
 * Synchronises.  fkmc_restore() puts it back into lattice i of a handle with
 * the same geometry and key; the run then continues exactly as the original
 * would (the random numbers are indexed by the counters, not by a state). */
fkmc_status fkmc_checkpoint_size(const fkmc_lattice* lat, uint32_t i, size_t* bytes);
fkmc_status fkmc_checkpoint(fkmc_lattice* lat, uint32_t i, void* host, size_t bytes);
fkmc_status fkmc_restore(fkmc_lattice* lat, uint32_t i, const void* host, size_t bytes);

/* Enable (1) or disable (0) HIP-event timing of each phase launch of the
 * following fkmc_advance calls (at most 2048 launches per call are timed). */
fkmc_status fkmc_set_timing(fkmc_lattice* lat, int32_t enable);

/* Average duration in milliseconds of the timed phase kernels of the last
 * fkmc_advance call, measured with HIP events on the handle's stream, and
 * the number of timed launches (0 if timing was off). */
fkmc_status fkmc_phase_timing(const fkmc_lattice* lat, double* avg_ms, uint64_t* launches);

/* Rate quantum q and maximum relative rounding error of lattice i's table. */
fkmc_status fkmc_quantisation(const fkmc_lattice* lat, uint32_t i, double* q, double* max_rel);

const char* fkmc_last_error(void);

/* ------------------------------------------------------------------------
 * Learned surrogate: an ensemble of `members` MLPs 4 -> 128 -> 128 -> 2
 * (SiLU) mapping (1000/T, x_H, log10 x_V, E_z / 1e7 V/m) to
 * (log10 D_O, log10 D_H), trained on diffusion coefficients measured by the
 * kMC engine.  Weights are used in BF16 with FP32 accumulation (MFMA on the
 * 128x128 layer), Adam (0.9, 0.999, 1e-8) on FP32 master weights, loss =
 * sum over outputs of the masked mean square error of standardised targets
 * (inputs and valid targets standardised by their mean and population
 * standard deviation over the data set).  Parameter vector of one member:
 * W1[4][128], b1[128], W2[128][128] (input-major), b2[128], W3[128][2],
 * b3[2]; 17410 floats.  All data pointers below are DEVICE pointers unless
 * named host; the work buffer is caller-owned device memory (256-byte
 * aligned).  Initialisation: He-normal weights from Philox (key seed),
 * zero biases. */
typedef struct fkmc_mlp fkmc_mlp;
uint32_t fkmc_mlp_param_count(void);
fkmc_status fkmc_mlp_query_sizes(uint32_t members, uint32_t max_samples, size_t* bytes);
fkmc_status fkmc_mlp_create(uint32_t members, uint32_t seed, uint32_t max_samples, void* work,
                            size_t bytes, void* hip_stream, fkmc_mlp** out);
fkmc_status fkmc_mlp_destroy(fkmc_mlp* h);
/* Training data: X[n][4], Y[n][2] targets, mask[n][2] (1 = valid label,
 * 0 = ignored); computes the standardisation.  The arrays must stay valid
 * while the handle trains on them. */
fkmc_status fkmc_mlp_set_data(fkmc_mlp* h, const float* X, const float* Y, const float* mask,
                              uint32_t n);
/* `steps` Adam steps with learning rate lr; each step uses `batch` samples
 * drawn uniformly with replacement from Philox (independent streams per
 * member: a bootstrap per step), or the whole set in order when batch = 0.
 * batch <= 1024.  loss_host (may be NULL) receives each member's loss of
 * the last step. */
fkmc_status fkmc_mlp_train(fkmc_mlp* h, uint32_t steps, uint32_t batch, float lr, float* loss_host);
/* Loss and gradient over the whole data set at the current parameters, no
 * update: grads_host[members][17410], loss_host[members] (may be NULL). */
fkmc_status fkmc_mlp_grad(fkmc_mlp* h, float* grads_host, float* loss_host);
/* Ensemble prediction for X[n][4]: mean[n][2] and population standard
 * deviation std[n][2] across members, in de-standardised units; each
 * (may be NULL) receives every member's output [members][n][2]. */
fkmc_status fkmc_mlp_predict(fkmc_mlp* h, const float* X, uint32_t n, float* mean, float* stdev,
                             float* each);
fkmc_status fkmc_mlp_get_params(fkmc_mlp* h, float* host, size_t n);
/* Replace all members' parameters (n = members * 17410) and reset Adam. */
fkmc_status fkmc_mlp_set_params(fkmc_mlp* h, const float* host, size_t n);
/* Standardisation: x mean[4], x std[4], y mean[2], y std[2]. */
fkmc_status fkmc_mlp_get_norm(fkmc_mlp* h, float* host12);

#ifdef __cplusplus
}
#endif
#endif
