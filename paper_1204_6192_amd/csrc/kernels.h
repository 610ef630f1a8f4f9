// kernels.h -- host-side launchers of the device kernels (internal to libhsg.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsg {

constexpr int kBlock = 256;  // work-group size of the sweep and reduction kernels (4 waves)

// Internal layouts (per group; d = sample, r = replica in canonical order):
//   spins  [r][parity][3][Nh]      storage type per codec, Nh = L^3 / 2,
//                                  element j of parity p = canonical site i with
//                                  parity(i) = p and i >> 1 = j
//   J6     [d][parity][6][Nh]      float32, the six couplings of each site in
//                                  neighbour order +x, -x, +y, -y, +z, -z
//   Hp     [d][parity][3][Nh]      float32
struct SweepArgs {
    void *spins;
    const float *J6;
    const float *Hp;             // nullptr when the group has no field
    const int32_t *temp_of_slot; // [D][O][T] rung of each slot
    const float *beta32;         // [T]
    double *e_partials;          // [replica][n_pb] when the pass computes energies
    int64_t Nh;
    int32_t L, Lh;
    int32_t slots_per_sample;    // O * T
    int32_t T;
    int32_t chunk, n_chunks, n_pb, n_blocks;
    const uint32_t *tptr;        // device sweep counter (read at launch time)
    uint32_t rep, parity;
    uint32_t key0, key1, uid_base;
};

// kind 0 = heat bath, 1 = over-relaxation.
hipError_t launch_half_sweep(const SweepArgs &a, int storage, int kind, bool field, bool energy,
                             hipStream_t s);

// z-march variant (L divisible by 4): a work-group owns RB replicas x TY rows
// and walks the zlen planes of one z-slab; P = L / 4 site pairs per row; rows =
// TY (whole plane in LDS) or TY + 2 (with halo rows). Energy partials are
// [replica][n_ytiles][n_zslabs]. The fused pair kernel takes one slab.
struct StreamArgs {
    void *spins;
    const float *J6;
    const uint8_t *Jbits;  // non-null: couplings are +-1, bit n of byte j set <=> J_n(j) = -1
    const float *Hp;
    const int32_t *temp_of_slot;
    const float *beta32;
    double *e_partials;
    int64_t Nh, n_rep;  // n_rep: end of the replica range of the launch
    int64_t r_base;     // first replica of the range (canonical order within the group)
    int32_t L, Lh, P, TY, RB, rows, n_ytiles, n_blocks;
    int32_t n_zslabs, zlen;
    int32_t slots_per_sample, T;
    const uint32_t *tptr;  // device sweep counter
    uint32_t t_offset;     // added to it (sweeps of a persistent launch; 0 otherwise)
    uint32_t rep, parity;
    uint32_t key0, key1, uid_base;
};
// Tile-local chain: one launch visits every tile of coarse parity `phase` of
// one group. Tiles are TX x TY x TZ sites; BX = L / TX, BY = L / TY, BZ = L / TZ
// tiles per axis; hx, hy, hz = 1 when that axis is tiled (a halo of one site
// row / plane; in x two half-indices on either side, to keep pairs aligned),
// else 0; RXh = TX / 2 + 4 hx staged half-indices per row, RY = TY + 2 hy rows,
// RZ = TZ + 2 hz planes; P = TZ TY TX / 4 site pairs per parity of a tile; RB
// replicas of one sample per work-group, in n_chunks chunks per sample.
// Blocks: [sample][tile of the phase][chunk].
struct TileArgs {
    void *spins;
    const float *J6;
    const uint8_t *Jbits;
    const float *Hp;
    const int32_t *temp_of_slot;
    const float *beta32;
    const uint32_t *tptr;
    int64_t Nh;
    int32_t L, Lh, TX, TY, TZ, BX, BY, BZ, hx, hy, hz, RXh, RY, RZ, P, RB, n_chunks;
    int32_t phase, n_tiles_phase, n_blocks;
    int32_t n_or, n_hb, n_hit;
    int32_t slots_per_sample, T;
    uint32_t key0, key1, uid_base;
};
hipError_t launch_tile_visit(const TileArgs &a, int storage, bool field, bool jb, bool hw, unsigned threads,
                             size_t lds, hipStream_t s);

// Up to kMaxStreamGroups lattice-size groups in one launch: group k owns the
// blocks [block_start[k], block_start[k + 1]).
constexpr int kMaxStreamGroups = 8;
struct MultiStreamArgs {
    int32_t n_groups, n_blocks;
    int32_t block_start[kMaxStreamGroups + 1];
    StreamArgs g[kMaxStreamGroups];
};
// fuse = 0: one half-sweep of parity a.parity; 1: both parities of a pair;
// 2: two over-relaxation pairs (kind 1). Fused launches need whole planes
// (TY = L) in every group.
hipError_t launch_half_sweep_stream(const MultiStreamArgs &m, int storage, int kind, bool energy, int fuse,
                                    unsigned threads, size_t lds_bytes, hipStream_t s);

// *flag = 1 if any of the n values is not exactly +1 or -1, else 0.
hipError_t launch_check_pm1(const float *v, int64_t n, int32_t *flag, hipStream_t s);

// Six coupling sign bits per site, [d][parity][Nh] bytes, from canonical J.
hipError_t launch_pack_jbits(const float *J_can, uint8_t *Jbits, int64_t D, int32_t L, hipStream_t s);

// E[r] = sum over the n_pb partials of replica r, for n_rep replicas.
hipError_t launch_reduce_partials(const double *partials, int n_pb, int64_t n_rep, double *E,
                                  hipStream_t s);

struct PtArgs {
    int32_t *slot_at_temp;       // [D][O][T]
    int32_t *temp_of_slot;       // [D][O][T]
    const double *E;             // [D][O][T] by slot
    const double *beta64;        // [T]
    unsigned long long *accepts; // [D][O][T-1]
    int32_t D, O, T;
    const uint32_t *tptr;  // in-sweep passes read the counter here; nullptr: use ctr1
    uint32_t ctr1, purpose;
    uint32_t key0, key1, uid_base;
};
hipError_t launch_pt(const PtArgs &a, hipStream_t s);

// Run statistics: sum [D][O][T][2] (E, E^2 by rung), flag and trips [D][O][T] by slot.
struct StatsArgs {
    const int32_t *slot_at_temp;
    const double *E;
    double *sum;
    int32_t *flag;
    uint32_t *trips;
    int32_t D, O, T;
};
hipError_t launch_stats(const StatsArgs &a, bool clear, hipStream_t s);


// Whole sweeps of small lattices, a sample per work-group with its spins in LDS
// (resident.hip): n_sweeps sweeps of the D samples of one group, each with
// n_hb heat-bath pairs, n_or over-relaxation pairs, the energy of the last
// pass, tempering when (t + 1) % pt_every == 0 and (stats) the run statistics;
// t = *tptr + i for sweep i. The caller advances the device counter. `groups`
// replica groups of Nh / 2 threads each; launch with groups * Nh / 2 <= threads.
struct ResidentArgs {
    void *spins;
    const float *J6;
    const float *Hp;
    int32_t *slot_at_temp, *temp_of_slot;  // [D][O][T]
    double *E;                             // [D][O][T] by slot
    const float *beta32;
    const double *beta64;
    unsigned long long *accepts;           // [D][O][T-1]
    double *stat_sum;                      // [D][O][T][2]
    int32_t *stat_flag;
    uint32_t *stat_trips;
    const uint32_t *tptr;
    int64_t Nh;
    int32_t L, Lh, D, O, T, slots_per_sample, groups;
    int32_t n_sweeps, n_hb, n_or, pt_every, stats;
    uint32_t key0, key1, uid_base;
};
// LDS bytes a work-group of the resident kernel needs.
size_t resident_lds_bytes(int storage, int64_t Nh, int32_t slots_per_sample);
hipError_t launch_resident(const ResidentArgs &a, int storage, bool field, bool hw, unsigned threads, size_t lds,
                           hipStream_t s);

struct PackArgs {
    void *spins_int;
    float *spins_can;  // canonical [r][3][N]
    const float *J_can;
    float *J6;
    const float *H_can;
    float *Hp;
    int64_t n_rep, D;
    int32_t L;
};
hipError_t launch_pack_spins(const PackArgs &a, int storage, hipStream_t s);
hipError_t launch_unpack_spins(const PackArgs &a, int storage, hipStream_t s);
hipError_t launch_pack_couplings(const PackArgs &a, hipStream_t s);
hipError_t launch_pack_field(const PackArgs &a, hipStream_t s);

// Exact float64 energy of every replica: partials [r][n_pb], n_pb = ceil(Nh / 256).
struct EnergyArgs {
    const void *spins;
    const float *J6;
    const float *Hp;
    double *partials;
    int64_t Nh, n_rep;
    int32_t L, Lh, slots_per_sample, n_pb;
};
hipError_t launch_energy(const EnergyArgs &a, int storage, hipStream_t s);
// The partials per replica that launch_energy writes (n_pb): one per band and
// z-slab of the z-march where kmode_rows(L) > 0 (march_slabs(L, n_rep)), else
// one per 256 parity-0 sites.
int64_t energy_partials(int L, int64_t n_rep, int64_t n_pb_site);

// Overlap of copies 0 and 1 at every rung: partials [d][k][n_pb][9] -> q [d][k][10];
// work-group pb covers the half-indices [pb * chunk, (pb + 1) * chunk).
struct OverlapArgs {
    const void *spins;
    const int32_t *slot_at_temp;
    double *partials;
    double *q;
    int64_t Nh;
    int32_t D, O, T, n_pb, chunk;
    int32_t L;
};
// Where kmode_rows(L) > 0 a z-march runs instead (k_overlap_stream): partial pb
// is z-slab pb % S of band pb / S, and n_pb must be march_partials(L, D T, .).
hipError_t launch_overlap(const OverlapArgs &a, int storage, hipStream_t s);

// Wave-vector dependent and chiral overlaps: partials [D T][n_pb][84], q [D T][84].
// Gathering passes: block pb covers canonical sites [pb chunk, (pb + 1) chunk).
// z-marches (kmode_rows(L) > 0): partial pb is band pb of kmode_rows(L) rows,
// and n_pb must be kmode_partials(L, .).
struct KmodeArgs {
    const void *spins;
    const int32_t *slot_at_temp;
    double *partials;
    double *q;
    int64_t Nh;
    int32_t L, D, O, T, n_pb, chunk;
};
hipError_t launch_kmodes(const KmodeArgs &a, int storage, hipStream_t s);

// Rows per work-group of the k-mode z-marches: four sites per thread, at most
// kBlock threads, a divisor of L, and the chiral march's LDS (two buffers x two
// copies x three components x (rows + two halo rows) x L floats) within 64 KiB.
// 0 where the marches do not apply (L % 4 != 0, or L > 224); the gathering
// passes run there.
__host__ __device__ inline int kmode_rows(int L)
{
    if (L < 4 || L % 4 != 0 || L / 4 > kBlock) return 0;
    int ty = kBlock / (L / 4);
    if (ty > L) ty = L;
    while (L % ty != 0) --ty;
    return (int64_t)2 * 2 * 3 * (ty + 2) * L * 4 <= 65536 ? ty : 0;
}

// z-slabs per band of the z-marches: n_items work items ((sample, rung) pairs,
// or replicas) with L / kmode_rows(L) bands each are split along z into the
// fewest slabs (a power of two dividing L, at least 4 planes each) that make
// 2048 work-groups, so that lattices with few items still fill the device.
__host__ __device__ inline int march_slabs(int L, int64_t n_items)
{
    const int rows = kmode_rows(L);
    if (rows <= 0) return 1;
    const int64_t blocks = n_items * (L / rows);
    int s = 1;
    while (blocks * s < 2048 && L % (2 * s) == 0 && L / (2 * s) >= 4) s *= 2;
    return s;
}

// Copy-pair local-overlap sums: partials [D T][n_pb][7 P], q [D T][P][7],
// P = O (O - 1) / 2 pairs a < b in the order (0,1), (0,2), ..., (1,2), ...
// q may be nullptr. With chi != nullptr (O >= 4) the sums of copies 0..3 also
// give the four-replica estimators, chi [D T][4 wave vectors][5]: chi_1, Re and
// Im chi_2, Re and Im chi_3 (each with the factor N^2 of the double sums).
struct PairOvArgs {
    const void *spins;
    const int32_t *slot_at_temp;
    double *partials;
    double *q;
    double *chi;
    int64_t Nh;
    int32_t L, D, O, T, n_pb, chunk;
};

// Per-sweep record of one group into a caller-owned series: at position
// p = *tptr - t0 (skipped when p >= capacity), out[p stride + m] holds the
// energies by rung [D][O][T], then (q != nullptr) q^2 [D][T] from the overlap
// output q [D][T][10].
struct SeriesArgs {
    const int32_t *slot_at_temp;
    const double *E;
    const double *q;
    double *out;
    const uint32_t *tptr;
    uint32_t t0;
    int64_t capacity, stride;
    int32_t D, O, T;
};
hipError_t launch_series(const SeriesArgs &a, hipStream_t s);
hipError_t launch_pair_overlaps(const PairOvArgs &a, int storage, hipStream_t s);
// The partials per (sample, rung) that launch_pair_overlaps and launch_overlap
// expect (n_pb): one
// per band and z-slab of the z-march where kmode_rows(L) > 0
// (march_slabs(L, D T)), else the overlap's work-groups (q_pb).
int64_t march_partials(int L, int64_t n_items, int64_t q_pb);
// The same for launch_kmodes, whose marches take whole z: one per band.
int64_t kmode_partials(int L, int64_t q_pb);

hipError_t launch_fill_identity_maps(int32_t *slot_at_temp, int32_t *temp_of_slot, int64_t n_lad,
                                     int32_t T, hipStream_t s);
hipError_t launch_invert_maps(const int32_t *slot_at_temp, int32_t *temp_of_slot, int64_t n_lad,
                              int32_t T, hipStream_t s);
// Advance the device sweep counter by one (end of a sweep).
hipError_t launch_advance(uint32_t *tptr, hipStream_t s);
hipError_t launch_set_u32(uint32_t *ptr, uint32_t value, hipStream_t s);
hipError_t launch_copy_u32(const uint32_t *src, uint32_t *dst, hipStream_t s);
hipError_t launch_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n,
                         hipStream_t s);
hipError_t launch_hw_math(const float *x, float *out, int64_t n, hipStream_t s);

}  // namespace hsg
