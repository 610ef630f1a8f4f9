/*
 * hsg.h -- C-ABI of libhsg.so: Monte-Carlo sweeps of the three-dimensional
 * Edwards-Anderson Heisenberg spin glass on one AMD Instinct MI355X (gfx950).
 *
 * The operations follow T. Yavors'kii and M. Weigel, "Optimized GPU simulation
 * of continuous-spin glass models" (arXiv:1204.6192):
 *   - the model, Eq. (1): unit 3-vector spins on a periodic L^3 cubic lattice,
 *     quenched nearest-neighbour couplings J_ij, optional random field H_i;
 *   - the heat-bath update, Eq. (2), and the over-relaxation reflection,
 *     Eq. (3), applied as checkerboard half-sweeps (Sec. 3.1);
 *   - parallel tempering between neighbouring temperatures, Eq. (4), walking
 *     the ladder from the lowest temperature and permuting temperatures, not
 *     spins (Sec. 2 and the description of the tempering kernel in Sec. 3.3);
 *   - the energy of Eq. (1) and the Edwards-Anderson overlap of Eq. (5);
 *   - one execution round in the sense of Sec. 3.2: the caller provides spins,
 *     couplings, fields and temperatures, runs sweeps, and reads back the spins
 *     and the generator position to resume later.
 *
 * Conventions
 *   Site index i = x + L (y + L z); parity (x + y + z) mod 2; L even, >= 4.
 *   A group is a set of samples sharing L, the number of copies R_O and the
 *   temperature ladder (R_T rungs). Replica r = (sample d, copy o, slot s);
 *   "slot" is the storage place of a replica inside its (d, o) ladder. The
 *   canonical replica order is [group][d][o][s].
 *   Canonical arrays (float32, device memory):
 *     spins   [group][d][o][s][3][L^3]
 *     J       [group][d][3][L^3]   J[a][i] couples i and i + e_a (a = x, y, z)
 *     H       [group][d][3][L^3]   only for groups with has_field != 0
 *   Temperature map (int32, device): slot_at_temp[group][d][o][k] = slot that
 *   currently holds rung k; rung k has temperature temps[k] (increasing).
 *
 * One sweep = n_hb heat-bath half-sweep pairs (even sites, then odd), then
 * n_or over-relaxation pairs, then the exact float64 energy of every replica,
 * then, if (t + 1) is a multiple of pt_every, one tempering pass. t is the
 * sweep counter (0 after init).
 *
 * Random numbers: Philox4x32-10 keyed by the 64-bit seed with counter
 *   heat bath (c0, c1, c2, c3) = (i >> 2, t, s | o<<8 | rep<<12 | parity<<16, uid)
 *     the parity site with ((i >> 1) & 1) == 0 takes words 0, 1; the other
 *     site of the block takes words 2, 3; u = ((w >> 8) + 1) 2^-24;
 *   tempering (k, t, o<<8 | 1<<20, uid), standalone call n: (k, n, o<<8 | 2<<20, uid)
 *     u = ((w0 << 21 ^ w1 >> 11) + 1) 2^-53, accept if Delta >= 0 or u <= exp(Delta);
 *   uid = sample_uid_base of the group + d.
 *
 * Ownership and errors
 *   The caller allocates and owns every device buffer; the library never
 *   calls hipMalloc. Buffer sizes come from hsg_query_sizes. The handle holds
 *   host metadata only. Every call returns an hsg_status; arguments are
 *   validated before anything is enqueued. Calls are ordered on the given
 *   stream and asynchronous unless stated; faults inside kernels surface as
 *   HSG_E_DEVICE from the next synchronising call (hsg_sync). After an error,
 *   hsg_last_error() returns a message (per thread). One handle must not be
 *   used from two threads at once.
 */
#ifndef HSG_H
#define HSG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *hsg_stream_t; /* a hipStream_t; NULL = default stream */

typedef int32_t hsg_status;
#define HSG_OK 0
#define HSG_E_INVALID (-1)     /* bad argument or description */
#define HSG_E_SIZE (-2)        /* a size limit of the counter map or the ABI exceeded */
#define HSG_E_UNSUPPORTED (-3) /* a storage / coupling combination that is not built */
#define HSG_E_DEVICE (-4)      /* a HIP runtime or kernel error */
#define HSG_E_STATE (-5)       /* call out of order (e.g. set_temp_map with a non-permutation) */

/* Spin storage in HBM. Arithmetic is always float32; compressed forms are
 * renormalised to |s| = 1 when they are read (Sec. 3.3 packs spins as well). */
#define HSG_STORE_F32 0
#define HSG_STORE_F16 1
#define HSG_STORE_BF16 2
#define HSG_STORE_QANGLE 3

typedef struct {
    int32_t L;                /* even, 4 <= L <= 1024 */
    int32_t n_samples;        /* R_D >= 1 */
    int32_t n_copies;         /* R_O, 1..16 (2 for the overlap) */
    int32_t n_temps;          /* R_T, 1..256 */
    const double *temps;      /* host, [n_temps], strictly increasing, finite, > 0 */
    uint32_t sample_uid_base; /* RNG identity of sample 0 of this group */
    int32_t has_field;        /* 0: H = 0 and no field array is read */
    int32_t coupling_kind;    /* 0: real couplings; 1: couplings are exactly +-1 */
    int32_t reserved;         /* must be 0 */
} hsg_group_desc;

typedef struct {
    const hsg_group_desc *groups; /* host, [n_groups] */
    int32_t n_groups;             /* 1..64 */
    int32_t storage;              /* HSG_STORE_* */
    int32_t n_hb;                 /* heat-bath half-sweep pairs per sweep, 0..16 */
    int32_t n_or;                 /* over-relaxation pairs per sweep, 0..1000; n_hb + n_or >= 1 */
    int32_t pt_every;             /* tempering after every pt_every-th sweep; 0 = never */
    int32_t reserved;             /* must be 0 */
    uint64_t seed;                /* Philox key */
} hsg_desc;

typedef struct {
    uint64_t state_bytes;    /* spins (internal layout), temperature maps, energies, counters */
    uint64_t coupling_bytes; /* couplings in the internal layout and the ladders */
    uint64_t field_bytes;    /* random fields in the internal layout (0 if no group has one) */
    uint64_t scratch_bytes;  /* reduction partials */
    uint64_t n_replicas;     /* total replicas over all groups */
    uint64_t n_spins;        /* total spins over all replicas */
} hsg_sizes;

typedef struct hsg_lattice hsg_lattice;

/* Sizes of the four caller-owned device buffers for `desc`. Host only. */
hsg_status hsg_query_sizes(const hsg_desc *desc, hsg_sizes *out);

/* Validate `desc`, bind the buffers and pack the canonical inputs into them
 * (the inputs of one execution round, Sec. 3.2: spins, couplings, fields and
 * temperatures; the random-number state is the seed plus the sweep counter).
 * d_spins0, d_J (and d_H if any group has a field) are read on `stream` and
 * may be freed once the stream has passed this call. d_state, d_couplings,
 * d_field (may be NULL if field_bytes == 0) and d_scratch must stay allocated
 * until hsg_destroy, 256-byte aligned, with at least the queried sizes. The
 * sweep counter starts at 0, every temperature map at the identity. */
hsg_status hsg_init_lattice(const hsg_desc *desc, const float *d_spins0, const float *d_J,
                            const float *d_H, void *d_state, void *d_couplings, void *d_field,
                            void *d_scratch, hsg_stream_t stream, hsg_lattice **out);

/* n_sweeps >= 0 full sweeps (see the header comment), asynchronous. */
hsg_status hsg_sweep(hsg_lattice *h, int32_t n_sweeps, hsg_stream_t stream);

/* One checkerboard half-sweep of every replica (the sub-lattice update of
 * Sec. 3.1): kind 0 = heat bath, Eq. (2), 1 = over-relaxation, Eq. (3); parity
 * 0 or 1; rep = heat-bath repetition index for the counter. Uses the current
 * sweep counter and does not advance it. */
hsg_status hsg_half_sweep(hsg_lattice *h, int32_t kind, int32_t parity, int32_t rep,
                          hsg_stream_t stream);

/* Both half-sweeps of a pair (parity 0, then parity 1) of every replica, as
 * inside a sweep of the full-lattice chain (whatever hsg_set_chain selected):
 * one fused launch where the kernel variant allows it, else two passes. Uses
 * the current sweep counter and does not advance it. */
hsg_status hsg_pair_sweep(hsg_lattice *h, int32_t kind, int32_t rep, hsg_stream_t stream);

/* n_pairs in 1..1000 over-relaxation pairs (Eq. (3); parity 0, then 1, each
 * time) of every replica, as inside a sweep of the full-lattice chain: two by
 * two in one launch where the kernel variant allows it, the odd one as a pair.
 * Deterministic, so it needs no counter; energies are not computed. Returns
 * HSG_E_INVALID for a NULL handle or n_pairs outside 1..1000. */
hsg_status hsg_or_pairs(hsg_lattice *h, int32_t n_pairs, hsg_stream_t stream);

/* One standalone tempering pass, Eq. (4), over every ladder (rung pairs from
 * the lowest temperature up, temperatures permuted, spins kept) using the
 * energies of the last sweep (or of the last hsg_measure_energy); advances the
 * standalone-call counter. */
hsg_status hsg_pt_exchange(hsg_lattice *h, hsg_stream_t stream);

/* Recompute the float64 energy of Eq. (1) of every replica into d_E
 * [n_replicas] (canonical replica order); also stores it as the energies that
 * a following hsg_pt_exchange uses. */
hsg_status hsg_measure_energy(hsg_lattice *h, double *d_E, hsg_stream_t stream);

/* hsg_measure_energy without the caller's scratch buffer, for callers that
 * cannot allocate device memory (code under graph capture, tight serving
 * loops, harnesses that forbid hipMalloc). Same kernels and results, bit for
 * bit; the per-work-group float64 partials go to a fixed device array of
 * 16 MiB inside the library, one per device, held until the process ends.
 * Allocates nothing (no hipMalloc, hipFree or allocating library call). Every
 * call on a device shares that array: calls that overlap on one device (other
 * streams, other handles, other threads) race and must be ordered by the
 * caller. The partials need, per group, n_replicas x 8 bytes times the
 * work-groups per replica: for L % 4 == 0 up to L = 224 the bands of rows
 * times the z-slabs of the z-march (one band up to L = 32, 3 at L = 48, 4 at
 * L = 64, 16 at L = 128; slabs until the group makes 2048 work-groups: 1 for
 * 4096 replicas of L = 32, 2 for 64 replicas of L = 128), else
 * ceil(L^3 / 512); HSG_E_SIZE when the largest exceeds 16 MiB, HSG_E_INVALID
 * for a NULL handle or d_E. */
hsg_status hsg_measure_energy_static(hsg_lattice *h, double *d_E, hsg_stream_t stream);

/* Copy the energies computed at the end of the last sweep into d_E [n_replicas]. */
hsg_status hsg_get_energies(const hsg_lattice *h, double *d_E, hsg_stream_t stream);

/* Overlap of Eq. (5) between copies 0 and 1 at every rung, float64:
 * d_q[group][d][k][10] = q^{mu nu} at 3 mu + nu (mu from copy 0), then
 * q^2 = sum of the nine squares. Requires n_copies >= 2 in every group. */
hsg_status hsg_measure_overlap(hsg_lattice *h, double *d_q, hsg_stream_t stream);

/* Wave-vector dependent spin-glass overlap and chiral overlap (the analysis
 * quantities of the paper's model section: the overlap q^{mu nu}(k) entering
 * chi_SG(k) and the correlation length, Eqs. (6)-(8), and the chiral overlap
 * of Eq. (12) built from kappa_i^alpha = s_{i+alpha} . (s_i x s_{i-alpha})),
 * between copies 0 and 1 at each rung, for k = 0 and k = (2 pi / L) e_a,
 * a = x, y, z. Output d_q (device, caller-owned, float64) is
 * [group][sample][rung][84]:
 *   0..8          q^{mu nu}(0), index 3 mu + nu;
 *   9 + 18 a + 2 (3 mu + nu) + {0, 1}   Re, Im q^{mu nu}(k_a);
 *   63 + 7 alpha  q_c^alpha(0);
 *   63 + 7 alpha + 1 + 2 a + {0, 1}     Re, Im q_c^alpha(k_a);
 * each with the factor 1/N, exp(+i k.R_i), R_i = (x, y, z) of site i.
 * chi_SG(k) = N sum_{mu nu} |q^{mu nu}(k)|^2 and chi_CG^alpha(k) = N
 * |q_c^alpha(k)|^2 follow per configuration. Needs n_copies >= 2 and L <= 1024
 * (HSG_E_INVALID / HSG_E_UNSUPPORTED). Uses the scratch buffer; stream-ordered. */
hsg_status hsg_measure_kmodes(hsg_lattice *h, double *d_q, hsg_stream_t stream);

/* Local-overlap Fourier sums of every pair of copies (the four-replica
 * estimators of the connected susceptibility in a field, Eqs. (9)-(11)):
 * summed over mu and nu, each chi_1, chi_2, chi_3 of Eq. (9) is a product of
 *   A_ab(k) = (1/N) sum_i (s_i(a) . s_i(b)) exp(i k.R_i)
 * at one rung: chi_1 = N^2 |A_12|^2, chi_2 = N^2 A_13 conj(A_14),
 * chi_3 = N^2 A_13 conj(A_24) (copies numbered from 1). Output d_q (device,
 * caller-owned, float64) is [group][sample][rung][pair][7], pairs a < b in the
 * order (0,1), (0,2), ..., (0,O-1), (1,2), ...; per pair: A_ab(0), then Re, Im
 * of A_ab((2 pi / L) e_a) for a = x, y, z. Needs n_copies >= 2 and L <= 1024.
 * Uses the scratch buffer; stream-ordered. */
hsg_status hsg_measure_pair_overlaps(hsg_lattice *h, double *d_q, hsg_stream_t stream);

/* Four-replica estimators of the connected spin-glass susceptibility in a
 * field, Eqs. (9)-(11): with copies 0, 1, 2, 3 at each rung as the replicas
 * (1), (2), (3), (4), the double sums of Eq. (10)
 *   chi_1(k) = sum_{i,j} sum_{mu,nu} s_i^mu(1) s_j^nu(1) s_i^mu(2) s_j^nu(2) e^{i k.(R_i - R_j)},
 *   chi_2(k): the same with s_i^mu(3) s_j^nu(4) in place of the second pair,
 *   chi_3(k): s_i^mu(1) s_j^nu(2) s_i^mu(3) s_j^nu(4),
 * of the current configurations (one entry of their time series), for k = 0
 * and k = (2 pi / L) e_a, a = x, y, z. Eq. (11) assembles chi_SG(k) =
 * [chi_1 - 2 chi_2 + chi_3]_J / N from their thermal averages. Output d_chi
 * (device, caller-owned, float64) is [group][sample][rung][4][5]: for k = 0,
 * k_x, k_y, k_z: chi_1, Re chi_2, Im chi_2, Re chi_3, Im chi_3 (chi_1 is real).
 * Computed from the copy-pair sums of hsg_measure_pair_overlaps (the double
 * sums factorise), in float64. Needs n_copies >= 4 in every group
 * (HSG_E_INVALID) and L <= 1024 (HSG_E_UNSUPPORTED). Uses the scratch buffer;
 * stream-ordered. */
hsg_status hsg_measure_chi(hsg_lattice *h, double *d_chi, hsg_stream_t stream);

/* Per-sweep time series (the paper records time series of the measured
 * quantities and copies them to the host, Sec. 3.2; the internal energy U_L
 * of the model section is their average). With d_series (device,
 * caller-owned, float64, capacity records) every following sweep of
 * hsg_sweep writes, after its tempering pass, one record at position
 * t - t0 (t the sweep's counter, t0 the counter at this call): for each group
 * in order, the energy of the configuration at every rung [sample][copy][rung],
 * then, where the group has n_copies >= 2, the overlap q^2 of Eq. (5) between
 * copies 0 and 1 [sample][rung]. Records past `capacity` (or before t0, after
 * hsg_set_state moved the counter back) are not written. *record_doubles
 * (host, may be NULL) receives the doubles per record. d_series = NULL with
 * capacity = 0 switches the series off. While a series is on, sweeps run on
 * one stream (hsg_set_overlap has no effect). HSG_E_INVALID for a NULL handle
 * or a pointer / capacity mismatch; HSG_E_SIZE for capacity >= 2^31. */
hsg_status hsg_set_series(hsg_lattice *h, double *d_series, int64_t capacity, int64_t *record_doubles);

/* Records of the series written so far (host, no synchronisation):
 * min(t - t0, capacity), 0 when no series is set. */
hsg_status hsg_get_series_count(const hsg_lattice *h, int64_t *n_records);

/* Decode the spins into the canonical float32 layout (renormalised). */
hsg_status hsg_get_spins(const hsg_lattice *h, float *d_spins, hsg_stream_t stream);

/* Replace the spins from the canonical float32 layout (encoded as stored). */
hsg_status hsg_set_spins(hsg_lattice *h, const float *d_spins, hsg_stream_t stream);

/* Temperature maps [group][d][o][k] int32 (device). set_ validates nothing on
 * the device: the caller must pass permutations of 0..n_temps-1. */
hsg_status hsg_get_temp_map(const hsg_lattice *h, int32_t *d_slot_at_temp, hsg_stream_t stream);
hsg_status hsg_set_temp_map(hsg_lattice *h, const int32_t *d_slot_at_temp, hsg_stream_t stream);

/* Accepted tempering swaps per rung pair since init, uint64 [group][d][o][k]
 * for k = 0..n_temps-2 (device). */
hsg_status hsg_get_pt_accepts(const hsg_lattice *h, uint64_t *d_accepts, hsg_stream_t stream);

/* Generator position for checkpoint / resume (the random-number state that
 * one execution round of Sec. 3.2 hands to the next). get_ returns host
 * values; set_ also writes the device copy of the sweep counter, ordered on
 * `stream`. */
hsg_status hsg_get_state(const hsg_lattice *h, uint64_t *sweep_counter, uint64_t *pt_calls,
                         uint64_t *seed);
hsg_status hsg_set_state(hsg_lattice *h, uint64_t sweep_counter, uint64_t pt_calls,
                         hsg_stream_t stream);

/* Tuning (results do not depend on it): slots processed per work item
 * (1..R_O R_T, 0 = automatic). */
hsg_status hsg_set_tuning(hsg_lattice *h, int32_t slots_per_item);

/* Tuning (results do not depend on it): 1 = the gather kernel (any even L);
 * 2 = the z-march kernel, one launch per half-sweep (L % 4 == 0; other sizes
 * keep the gather kernel); 3 = the z-march kernel with both half-sweeps of a
 * pair in one launch where the whole plane fits a work-group (L <= 32), else
 * as 2; 4 = as 3, and the over-relaxation pairs of a sweep two by two in one
 * launch (four half-sweeps per read and write of the spins) where eleven
 * staged planes fit the work-group's LDS; 5 = where every replica of a sample
 * of every lattice size fits one work-group's LDS (L <= 12; the paper's
 * per-block shared-memory tiles, Sec. 3.1, taken to a whole sample) and no
 * series is recorded, hsg_sweep runs whole sweeps in one launch (up to 256
 * per launch), a sample per work-group: the half-sweeps, the energies, the
 * tempering walk (Eq. (4)) and the statistics, the spins staying in LDS;
 * otherwise, and for the per-call entry points, as 4; 0 = automatic
 * (currently 4, but 3 for quantised-angle storage, whose two-pair launch is
 * slower than two fused pairs). Energies computed in a variant-5 launch equal
 * the others' to rounding (another summation order). */
hsg_status hsg_set_kernel(hsg_lattice *h, int32_t variant);

/* Tuning (results do not depend on it): 1 = where every lattice size runs
 * the z-march, has at least two samples and no replica batches, and the
 * full-lattice chain is selected, hsg_sweep runs the two halves of every
 * group's samples on two streams (the caller's and one of the library's,
 * joined before it returns), each half with its own device sweep counter
 * (the second copied from the first at the start of every call); one half's
 * heat-bath pairs then run beside the other half's over-relaxation pairs.
 * Samples never interact (tempering is per sample), so every replica gets the
 * same updates with the same random numbers. 0 (default) = one stream (and
 * hipGraph replay). It pays where the two kinds of pass are limited by
 * different resources (lattice sizes of unequal cost); hsg_autotune tries it.
 * Returns HSG_E_INVALID for a NULL handle or a value other than 0 and 1. */
hsg_status hsg_set_overlap(hsg_lattice *h, int32_t enable);

/* The launch choices in force (as set by hsg_set_kernel, hsg_set_tuning,
 * hsg_set_overlap or chosen by hsg_autotune): kernel variant (0 = automatic),
 * slots per work item (0 = automatic) and overlapped sweeps (0 or 1), each
 * written to its non-NULL host output. HSG_E_INVALID for a NULL handle. */
hsg_status hsg_get_tuning(const hsg_lattice *h, int32_t *variant, int32_t *slots_per_item, int32_t *overlap);

/* Tuning (results do not depend on it): geometry of the z-march kernels of
 * lattice-size group `group` (the tile shape of the local-update kernel; the
 * paper scans tile sizes for speed, Sec. 4). tile_y = rows per work-group: L
 * (whole planes, the only choice where L * L / 4 <= 256 threads fit a
 * work-group, i.e. L <= 32) or a divisor of L below it with L / 4 * tile_y <=
 * 256 (row bands with two halo rows; one of the four tallest); z_slabs = 1, 2,
 * 4 or 8 slabs of at least 8 planes that a single-pass launch splits the
 * z-march into. tile_y = z_slabs = 0 restores the default (the tallest band,
 * slabs until a launch has about 4096 work-groups). Fused pairs and two-pair
 * launches always march whole planes in one slab. HSG_E_INVALID for a bad
 * handle, group or shape; HSG_E_UNSUPPORTED for a group with L % 4 != 0. */
hsg_status hsg_set_geometry(hsg_lattice *h, int32_t group, int32_t tile_y, int32_t z_slabs);

/* The geometry in force for `group` (0, 0 where L % 4 != 0); either output may
 * be NULL. */
hsg_status hsg_get_geometry(const hsg_lattice *h, int32_t group, int32_t *tile_y, int32_t *z_slabs);

/* Arithmetic of the heat-bath draw (Eq. (2)). 0 (default): square roots and
 * divisions from the hardware reciprocal (square root) refined by Newton steps
 * (within one ulp, almost always correctly rounded), the azimuth's sine and
 * cosine from polynomials (absolute error at most 7e-8); in both modes e^z and
 * ln X from the hardware 2^x and log2 with extended-precision scaling.
 * 1: the field's length, direction and the divisions from the bare hardware
 * reciprocal square root and reciprocal (1 ulp), the azimuth from the hardware
 * sin/cos (absolute error about 1.2e-7). Mode 1
 * changes the trajectory at the float32 rounding level and is the faster
 * choice; over-relaxation is the same in both. HSG_E_INVALID for a NULL
 * handle or a mode other than 0 and 1. */
hsg_status hsg_set_math(hsg_lattice *h, int32_t mode);

/* Markov chain of hsg_sweep. chain = 0 (default): the full-lattice
 * checkerboard (every half-sweep updates one parity of the whole lattice:
 * n_hb heat-bath pairs, then n_or over-relaxation pairs). chain = 1: the
 * tile-local chain of the double checkerboard decomposition (the paper's
 * implementation section and its numbered Monte Carlo procedure): the lattice
 * is cut into tiles of tile_x x tile_y x tile_z sites (0 = L: whole rows along
 * x, or whole planes; the paper's optimum is 8 x 8 x 8); every lattice size
 * must have L % 4 == 0, tile edges dividing L, tile_x a multiple of 4 and
 * L / edge either 1 or even. A sweep visits the tiles of coarse parity
 * (X + Y + Z) mod 2 = 0, then those of parity 1; on a visit the tile gets n_hit
 * repetitions of n_or over-relaxation rounds followed by n_hb heat-bath rounds
 * (a round: even sites, then odd sites), with the sites outside the tile held
 * fixed; heat-bath round b of repetition r uses repetition index r n_hb + b of
 * the counter map (n_hit n_hb <= 16). Then the exact energies and tempering.
 * A different chain with the same stationary distribution; results do not
 * depend on launch choices. Not part of the checkpoint state: set it again
 * after resuming. Errors: HSG_E_INVALID for bad shapes, HSG_E_UNSUPPORTED when
 * a tile does not fit one work-group (at most 1024 site pairs per parity and
 * 64 KiB of staged spins per replica). */
hsg_status hsg_set_chain(hsg_lattice *h, int32_t chain, int32_t tile_x, int32_t tile_y, int32_t tile_z,
                         int32_t n_hit);

/* Autotuner of the launch configuration (the batching row of the method: tile
 * shape and fusion per lattice size). Times n_sweeps (1..1000) whole sweeps of
 * each distinct kernel variant of hsg_set_kernel (and, where lattices use the
 * gather kernel, 2, 4, 8 or 16 slots per work item; where hsg_set_overlap
 * applies, each z-march variant also with overlapped sweeps) with HIP events
 * after ten warm-up sweeps each (the sweep graphs are captured and launched
 * once), in two rounds over all candidates, and keeps
 * the fastest by best time, where a candidate must be at least 1 % faster
 * than an earlier one in the order above to replace it (the overlap choice is
 * kept too; hsg_get_tuning reports it). Then, with that choice in force, it
 * times the z-march geometries of hsg_set_geometry for every lattice size that
 * runs single passes, one size after the other, the current geometry first
 * and replaced only by one at least 1 % faster (hsg_get_geometry reports the
 * result). Every variant computes the same spins and temperature maps bit
 * for bit (variant 5 the energies to rounding, another summation order), so
 * the trial sweeps are ordinary sweeps of the chain: with
 * d_backup == NULL the chain advances by them (2 (n_sweeps + 10) per candidate);
 * with d_backup (device, state_bytes of hsg_query_sizes, 256-byte aligned,
 * caller-owned) the state is saved first and restored afterwards, so the chain
 * is left exactly as it was. Synchronises the stream. On success the chosen
 * variant and slots per item (0 = automatic) are written to the non-NULL
 * outputs; on error the previous tuning is kept. */
hsg_status hsg_autotune(hsg_lattice *h, int32_t n_sweeps, void *d_backup, int32_t *variant,
                        int32_t *slots_per_item, hsg_stream_t stream);

/* Run statistics (the paper's U_L, C_L and tempering diagnostics). With
 * hsg_set_stats(h, 1), every following sweep ends (after tempering) with: for
 * every ladder and rung k, the energy E of the configuration now at rung k is
 * added to sums of E and E^2; and a replica that reaches the lowest rung after
 * having reached the highest since its last visit to the lowest completes one
 * round trip. U_L(T_k) = sum E / n and C_L(T_k) = (sum E^2 / n - U_L^2) / T_k^2
 * per ladder, with n the sweeps counted. hsg_reset_stats clears them (also done
 * at init). hsg_get_stats copies d_sums [group][sample][copy][rung][2] (E, E^2;
 * float64, device) and d_trips [group][sample][copy][slot] (uint32, device);
 * either may be NULL; *n_sweeps (host) receives the sweeps accumulated.
 * The statistics live in the state buffer. */
hsg_status hsg_set_stats(hsg_lattice *h, int32_t enable);
hsg_status hsg_reset_stats(hsg_lattice *h, hsg_stream_t stream);
hsg_status hsg_get_stats(const hsg_lattice *h, double *d_sums, uint32_t *d_trips, uint64_t *n_sweeps,
                         hsg_stream_t stream);

/* Tuning (results do not depend on it): run the pairs of a sweep in batches of
 * replicas, all pairs of one batch back to back so that its spins stay in the
 * last-level cache, then the next batch (lattice sizes that use the z-march
 * kernels; tempering after every batch). -1: off (default); 0: automatic
 * (about 192 MiB of spins per batch); > 0: replicas per batch. */
hsg_status hsg_set_batch(hsg_lattice *h, int64_t replicas);

/* Replay whole sweeps as captured HIP graphs (default on; used when tempering
 * runs every sweep or never). Results do not depend on it. */
hsg_status hsg_set_graphs(hsg_lattice *h, int32_t enable);

/* Wait for `stream` and report any device error. */
hsg_status hsg_sync(hsg_lattice *h, hsg_stream_t stream);

/* Release the handle (not the caller's buffers). NULL is ignored. */
void hsg_destroy(hsg_lattice *h);

/* Message for the last non-OK status on this thread ("" if none). */
const char *hsg_last_error(void);

/* Identity of the sources this library was built from (a hash): measurements
 * taken with hardware counters are valid for one build id only. */
const char *hsg_build_id(void);

/* Test hook: n Philox4x32-10 blocks, d_ctr [n][4], d_key [n][2] -> d_out [n][4]
 * (device arrays). Exposes the device generator for a bit-exact comparison. */
hsg_status hsg_debug_philox(const uint32_t *d_ctr, const uint32_t *d_key, uint32_t *d_out,
                            int64_t n, hsg_stream_t stream);

/* Test hook: the hardware transcendentals and the refined routines the
 * kernels use, for x = d_x[i]: d_out[12 i ..] = hardware sin(2 pi x),
 * cos(2 pi x), ln x, e^-x, 1/x, 1/sqrt(x); then the default heat bath's
 * polynomial sin(2 pi x), cos(2 pi x) (x on the 2^-24 grid), its refined
 * sqrt(x), 1/sqrt(x) (0, 0 for x <= 0), and the heat bath's e^-x (0 for
 * x < 0) and ln x (0 below the smallest normal number) (device arrays,
 * n >= 0), so that their accuracy can be checked against float64. HSG_E_INVALID for n < 0 or a NULL
 * array with n > 0. */
hsg_status hsg_debug_hw_math(const float *d_x, float *d_out, int64_t n, hsg_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HSG_H */
