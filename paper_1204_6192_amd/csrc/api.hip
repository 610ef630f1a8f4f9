// api.hip -- the C-ABI of libhsg.so (declared in include/hsg.h).
//
// Host side only: validation, buffer carving, and the order of launches that
// makes one sweep (heat-bath pairs, over-relaxation pairs with the energy of
// Eq. (1) fused into the last pass, tempering per Eq. (4)). No device memory is
// allocated here; every buffer belongs to the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hsg.h"
#include "kernels.h"

namespace {

thread_local std::string g_err;

hsg_status fail(hsg_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
hsg_status fail(hsg_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

hsg_status hip_fail(hipError_t e, const char *what)
{
    return fail(HSG_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

}  // namespace

// Fixed device scratch of the allocation-free energy measurement
// (hsg_measure_energy_static): one copy per device, held until the process
// ends. In host code `scratch` only names the symbol; its device address comes
// from hipGetSymbolAddress, resolved once per device (static_scratch_ptr).
constexpr size_t kStaticScratchBytes = 16u << 20;
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (current), resolved on first use.
hipError_t static_scratch_ptr(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Bytes of stored spin per site: 3 float32, 3 x 16-bit, or one 32-bit angle word.
int bytes_per_spin(int storage)
{
    switch (storage) {
    case HSG_STORE_F32: return 12;
    case HSG_STORE_F16:
    case HSG_STORE_BF16: return 6;
    default: return 4;
    }
}

struct Group {
    int32_t L, D, O, T;
    int64_t N, Nh;
    uint32_t uid_base;
    bool field;
    int32_t ckind;
    std::vector<double> temps;
    int64_t rep0;  // first replica of the group in canonical order
    int64_t n_rep;
    int64_t can_spin0;  // element offset of the group in the canonical spin array
    int64_t can_site0;  // element offset of the group in the canonical J and H arrays
    // byte offsets
    uint64_t o_spins, o_sat, o_tos, o_E, o_acc;  // state
    uint64_t o_ssum, o_sflag, o_strips;          // run statistics
    uint64_t o_J6, o_b64, o_b32, o_Jbits;        // couplings
    uint64_t o_H;                                // field
    uint64_t o_scr;                              // scratch
    uint64_t o_scr_q;                            // overlap output of the per-sweep series (in scratch)
    int32_t n_pb_sweep;                          // blocks of 256 site pairs per replica
    int32_t n_pb_site;                           // blocks of 256 sites per replica half
    int32_t q_pb, q_chunk;                       // overlap: work-groups per rung pair, sites each
    // z-march geometry (L divisible by 4), see hsg::StreamArgs
    bool stream_ok;
    int32_t s_TY, s_RB, s_rows, s_ytiles, s_zslabs;
    int32_t s_max_pb;  // most energy partials per replica any allowed geometry makes (scratch sizing)
    // tile-local chain geometry, see hsg::TileArgs (set by hsg_set_chain)
    int32_t t_TX, t_TY, t_TZ, t_BX, t_BY, t_BZ, t_hx, t_hy, t_hz, t_RXh, t_RY, t_RZ, t_P, t_RB, t_chunks, t_threads;
    size_t t_lds;
};

// z-march geometry (L % 4 == 0): TY rows per work-group, either the whole plane
// (TY = L, when L * L / 4 <= 256 threads; several replicas per group for small
// L) or a row band of TY rows with two halo rows, and the number of z-slabs of
// a single-pass launch (each slab reads one extra plane at either end). Returns
// false for a shape the kernels do not take.
bool apply_geometry(Group &g, int ty, int zslabs)
{
    const int P = g.L / 4;
    if (ty == g.L) {
        if (P * g.L > hsg::kBlock) return false;
        g.s_rows = g.L;
    } else {
        if (ty < 2 || ty > g.L || g.L % ty != 0 || P * ty > hsg::kBlock || P * g.L <= hsg::kBlock) return false;
        g.s_rows = ty + 2;
    }
    if (zslabs < 1 || zslabs > 8 || (zslabs & (zslabs - 1)) != 0 || g.L % zslabs != 0 ||
        (zslabs > 1 && g.L / zslabs < 8))
        return false;
    g.s_TY = ty;
    g.s_RB = hsg::kBlock / (P * ty);
    g.s_ytiles = g.L / ty;
    g.s_zslabs = zslabs;
    return true;
}

// The geometries the autotuner tries for a lattice size: the whole plane where
// it fits a work-group, else the four tallest row bands; 1, 2, 4 or 8 z-slabs
// of at least 8 planes. The default comes first.
std::vector<std::pair<int, int>> geometry_candidates(const Group &g)
{
    std::vector<std::pair<int, int>> out;
    if (!g.stream_ok) return out;
    const int P = g.L / 4;
    std::vector<int> tys;
    if (P * g.L <= hsg::kBlock) {
        tys.push_back(g.L);
    } else {
        for (int c = g.L - 1; c >= 2 && tys.size() < 4; --c)
            if (g.L % c == 0 && P * c <= hsg::kBlock) tys.push_back(c);
    }
    for (int ty : tys)
        for (int z = 1; z <= 8; z *= 2)
            if (z == 1 || (g.L % z == 0 && g.L / z >= 8)) out.emplace_back(ty, z);
    return out;
}

// Default z-march geometry for lattice size L: the whole plane where it fits,
// otherwise the tallest row band; single half-sweeps split z into slabs until
// the launch has about 4096 work-groups, keeping slabs >= 16 planes.
void stream_geometry(Group &g)
{
    g.stream_ok = (g.L % 4) == 0;
    if (!g.stream_ok) return;
    const std::vector<std::pair<int, int>> cands = geometry_candidates(g);
    if (cands.empty()) {
        g.stream_ok = false;
        return;
    }
    const int ty = cands.front().first;
    const int rb = hsg::kBlock / ((g.L / 4) * ty);
    const int64_t base = (g.n_rep + rb - 1) / rb * (g.L / ty);
    int zs = 1;
    while (base * zs < 4096 && g.L % (2 * zs) == 0 && g.L / (2 * zs) >= 16 && 2 * zs <= 8) zs *= 2;
    g.s_max_pb = 1;
    for (const auto &c : cands) g.s_max_pb = std::max(g.s_max_pb, (g.L / c.first) * c.second);
    (void)apply_geometry(g, ty, zs);
}

struct Layout {
    std::vector<Group> g;
    hsg_sizes sz{};
};

hsg_status build_layout(const hsg_desc *desc, Layout &lay)
{
    if (desc == nullptr) return fail(HSG_E_INVALID, "desc is NULL");
    if (desc->reserved != 0) return fail(HSG_E_INVALID, "desc.reserved must be 0");
    if (desc->n_groups < 1 || desc->n_groups > 64)
        return fail(HSG_E_INVALID, "n_groups = %d, need 1..64", desc->n_groups);
    if (desc->groups == nullptr) return fail(HSG_E_INVALID, "groups is NULL");
    if (desc->storage < HSG_STORE_F32 || desc->storage > HSG_STORE_QANGLE)
        return fail(HSG_E_INVALID, "storage = %d is not an HSG_STORE_* value", desc->storage);
    if (desc->n_hb < 0 || desc->n_hb > 16) return fail(HSG_E_SIZE, "n_hb = %d, need 0..16", desc->n_hb);
    if (desc->n_or < 0 || desc->n_or > 1000) return fail(HSG_E_SIZE, "n_or = %d, need 0..1000", desc->n_or);
    if (desc->n_hb + desc->n_or < 1) return fail(HSG_E_INVALID, "a sweep needs n_hb + n_or >= 1");
    if (desc->pt_every < 0) return fail(HSG_E_INVALID, "pt_every = %d < 0", desc->pt_every);
    lay.g.clear();
    // the state buffer starts with a control block: the device sweep counter
    uint64_t st = kAlign, cp = 0, fd = 0, sc = 0;
    int64_t rep0 = 0, spins = 0, sites = 0;
    for (int gi = 0; gi < desc->n_groups; ++gi) {
        const hsg_group_desc &gd = desc->groups[gi];
        Group g{};
        if (gd.reserved != 0) return fail(HSG_E_INVALID, "group %d: reserved must be 0", gi);
        if (gd.L < 4 || gd.L > 1024 || (gd.L & 1))
            return fail(HSG_E_INVALID, "group %d: L = %d must be even and in 4..1024", gi, gd.L);
        if (gd.n_samples < 1) return fail(HSG_E_INVALID, "group %d: n_samples = %d < 1", gi, gd.n_samples);
        if (gd.n_copies < 1 || gd.n_copies > 16)
            return fail(HSG_E_SIZE, "group %d: n_copies = %d, need 1..16", gi, gd.n_copies);
        if (gd.n_temps < 1 || gd.n_temps > 256)
            return fail(HSG_E_SIZE, "group %d: n_temps = %d, need 1..256", gi, gd.n_temps);
        if (gd.temps == nullptr) return fail(HSG_E_INVALID, "group %d: temps is NULL", gi);
        for (int k = 0; k < gd.n_temps; ++k) {
            const double T = gd.temps[k];
            if (!(std::isfinite(T) && T > 0.0))
                return fail(HSG_E_INVALID, "group %d: temps[%d] = %g is not finite and > 0", gi, k, T);
            if (k > 0 && !(T > gd.temps[k - 1]))
                return fail(HSG_E_INVALID, "group %d: temps must be strictly increasing (k = %d)", gi, k);
        }
        if (gd.coupling_kind != 0 && gd.coupling_kind != 1)
            return fail(HSG_E_INVALID, "group %d: coupling_kind = %d", gi, gd.coupling_kind);
        if ((uint64_t)gd.sample_uid_base + (uint64_t)gd.n_samples > 0x100000000ull)
            return fail(HSG_E_SIZE, "group %d: sample uids exceed 32 bits", gi);
        g.L = gd.L;
        g.D = gd.n_samples;
        g.O = gd.n_copies;
        g.T = gd.n_temps;
        g.N = (int64_t)g.L * g.L * g.L;
        g.Nh = g.N / 2;
        g.uid_base = gd.sample_uid_base;
        g.field = gd.has_field != 0;
        g.ckind = gd.coupling_kind;
        g.temps.assign(gd.temps, gd.temps + gd.n_temps);
        g.rep0 = rep0;
        g.can_spin0 = spins * 3;
        g.can_site0 = sites * 3;
        g.n_rep = (int64_t)g.D * g.O * g.T;
        const int64_t pairs = g.Nh / 2;
        g.n_pb_sweep = (int32_t)((pairs + hsg::kBlock - 1) / hsg::kBlock);
        g.n_pb_site = (int32_t)((g.Nh + hsg::kBlock - 1) / hsg::kBlock);
        {  // about 4096 work-groups in all for the overlap, each over whole blocks of 256 sites
            const int64_t pairs = (int64_t)g.D * g.T;
            int64_t qpb = (4096 + pairs - 1) / pairs;
            if (qpb > g.n_pb_site) qpb = g.n_pb_site;
            if (qpb < 1) qpb = 1;
            const int64_t per = (g.Nh + qpb - 1) / qpb;
            g.q_chunk = (int32_t)((per + hsg::kBlock - 1) / hsg::kBlock * hsg::kBlock);
            g.q_pb = (int32_t)((g.Nh + g.q_chunk - 1) / g.q_chunk);
        }
        stream_geometry(g);
        // state
        g.o_spins = st;
        st = align_up(st + (uint64_t)g.n_rep * 2 * g.Nh * bytes_per_spin(desc->storage));
        g.o_sat = st;
        st = align_up(st + (uint64_t)g.n_rep * 4);
        g.o_tos = st;
        st = align_up(st + (uint64_t)g.n_rep * 4);
        g.o_E = st;
        st = align_up(st + (uint64_t)g.n_rep * 8);
        g.o_acc = st;
        st = align_up(st + (uint64_t)g.D * g.O * (g.T > 1 ? g.T - 1 : 1) * 8);
        // run statistics: sums of E and E^2 per (ladder, rung), flag and round trips per slot
        g.o_ssum = st;
        st = align_up(st + (uint64_t)g.n_rep * 2 * 8);
        g.o_sflag = st;
        st = align_up(st + (uint64_t)g.n_rep * 4);
        g.o_strips = st;
        st = align_up(st + (uint64_t)g.n_rep * 4);
        // couplings and ladder
        g.o_J6 = cp;
        cp = align_up(cp + (uint64_t)g.D * 2 * 6 * g.Nh * 4);
        g.o_b64 = cp;
        cp = align_up(cp + (uint64_t)g.T * 8);
        g.o_b32 = cp;
        cp = align_up(cp + (uint64_t)g.T * 4);
        g.o_Jbits = cp;
        if (g.ckind == 1) cp = align_up(cp + (uint64_t)g.D * 2 * g.Nh);
        // field
        g.o_H = fd;
        if (g.field) fd = align_up(fd + (uint64_t)g.D * 2 * 3 * g.Nh * 4);
        // scratch: the largest of the reductions of this group
        g.o_scr = sc;
        const int64_t n_pb_stream = g.stream_ok ? (int64_t)g.s_max_pb : 1;
        const uint64_t e_sweep = (uint64_t)g.n_rep * (g.n_pb_sweep > n_pb_stream ? g.n_pb_sweep : n_pb_stream) * 8;
        const int64_t e_pb = hsg::energy_partials(g.L, g.n_rep, g.n_pb_site);
        const uint64_t e_full = (uint64_t)g.n_rep * (e_pb > g.n_pb_site ? e_pb : g.n_pb_site) * 8;
        const uint64_t q_full = (uint64_t)g.D * g.T * hsg::march_partials(g.L, (int64_t)g.D * g.T, g.q_pb) * 9 * 8;
        // k modes and copy pairs: the overlap's blocks, or one partial per band of the z-marches
        const int64_t k_pb = hsg::kmode_partials(g.L, g.q_pb);
        const int64_t p_pb = hsg::march_partials(g.L, (int64_t)g.D * g.T, g.q_pb);
        const uint64_t k_full = (uint64_t)g.D * g.T * k_pb * 84 * 8;
        const uint64_t p_full = (uint64_t)g.D * g.T * p_pb * 7 * (g.O * (g.O - 1) / 2) * 8;
        uint64_t need = e_sweep > e_full ? e_sweep : e_full;
        // the per-sweep series stages the overlap [D][T][10] after its partials
        g.o_scr_q = g.o_scr + align_up(q_full);
        const uint64_t series_need = align_up(q_full) + (uint64_t)g.D * g.T * 10 * 8;
        if (series_need > need) need = series_need;
        if (q_full > need) need = q_full;
        if (k_full > need) need = k_full;
        if (p_full > need) need = p_full;
        sc = align_up(sc + need);
        rep0 += g.n_rep;
        spins += g.n_rep * g.N;
        sites += (int64_t)g.D * g.N;
        lay.g.push_back(std::move(g));
    }
    lay.sz.state_bytes = st;
    lay.sz.coupling_bytes = cp;
    lay.sz.field_bytes = fd;
    lay.sz.scratch_bytes = sc;
    lay.sz.n_replicas = (uint64_t)rep0;
    lay.sz.n_spins = (uint64_t)spins;
    return HSG_OK;
}

}  // namespace

struct hsg_lattice {
    Layout lay;
    int32_t storage = 0, n_hb = 1, n_or = 4, pt_every = 1;
    uint64_t seed = 0;
    uint64_t t = 0, pt_calls = 0;
    char *state = nullptr, *coup = nullptr, *field = nullptr, *scratch = nullptr;
    int32_t slots_per_item = 0;
    // 0 automatic (= 4), 1 gather, 2 z-march, 3 z-march with fused pairs, 4 fused pairs and
    // over-relaxation pairs fused two by two
    int32_t kernel_variant = 0;
    size_t max_lds = 64 * 1024;  // LDS bytes per work-group the device allows
    int device = 0;              // the device current at init (the buffers live there)
    bool hw_math = false;        // heat bath with the hardware transcendentals (kernel kind 2)
    int64_t batch = -1;   // replicas per sweep batch: -1 off, 0 automatic (about 192 MiB of spins)
    bool stats = false;   // accumulate run statistics after every sweep
    uint64_t n_stats = 0;  // sweeps accumulated since the last reset
    // per-sweep series (hsg_set_series): record of sweep t at position t - series_t0
    double *series = nullptr;
    int64_t series_cap = 0, series_rec = 0;
    uint64_t series_t0 = 0;
    // Markov chain: 0 the full-lattice checkerboard, 1 the tile-local chain
    int32_t chain = 0, tile_x = 0, tile_y = 0, tile_z = 0, n_hit = 1;
    bool have_energies = false;
    // hipGraph replay of whole sweeps (tempering every sweep or never)
    bool use_graphs = true;
    // Overlapped sweeps (hsg_set_overlap): two halves of every group's samples on
    // two streams, each with its own device sweep counter (cohort 0: the
    // counter at the start of the state buffer, cohort 1: the next word).
    bool overlap = false;
    int32_t cohort = 0;  // the counter the launches being enqueued read
    hipStream_t stream2 = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // fork, half 0 HB, half 1 HB, join
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};         // 1 sweep, kGraphSweeps sweeps
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
};

namespace {

constexpr int kGraphSweeps = 8;

hipStream_t S(hsg_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

uint32_t *dev_counter(const hsg_lattice *h) { return reinterpret_cast<uint32_t *>(h->state) + h->cohort; }

void drop_graphs(hsg_lattice *h)
{
    for (int k = 0; k < 2; ++k) {
        if (h->graph_exec[k]) (void)hipGraphExecDestroy(h->graph_exec[k]);
        if (h->graph[k]) (void)hipGraphDestroy(h->graph[k]);
        h->graph_exec[k] = nullptr;
        h->graph[k] = nullptr;
    }
}

int chunk_for(const hsg_lattice *h, const Group &g)
{
    const int spp = g.O * g.T;
    int c = h->slots_per_item > 0 ? h->slots_per_item : 8;
    return c < spp ? c : spp;
}

hsg::SweepArgs sweep_args(const hsg_lattice *h, const Group &g, int parity, uint32_t rep)
{
    hsg::SweepArgs a{};
    a.spins = h->state + g.o_spins;
    a.J6 = reinterpret_cast<const float *>(h->coup + g.o_J6);
    a.Hp = g.field ? reinterpret_cast<const float *>(h->field + g.o_H) : nullptr;
    a.temp_of_slot = reinterpret_cast<const int32_t *>(h->state + g.o_tos);
    a.beta32 = reinterpret_cast<const float *>(h->coup + g.o_b32);
    a.e_partials = reinterpret_cast<double *>(h->scratch + g.o_scr);
    a.Nh = g.Nh;
    a.L = g.L;
    a.Lh = g.L / 2;
    a.slots_per_sample = g.O * g.T;
    a.T = g.T;
    a.chunk = chunk_for(h, g);
    a.n_chunks = (a.slots_per_sample + a.chunk - 1) / a.chunk;
    a.n_pb = g.n_pb_sweep;
    a.n_blocks = g.D * a.n_chunks * a.n_pb;
    a.tptr = dev_counter(h);
    a.rep = rep;
    a.parity = (uint32_t)parity;
    a.key0 = (uint32_t)(h->seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(h->seed >> 32);
    a.uid_base = g.uid_base;
    return a;
}

bool use_stream(const hsg_lattice *h, const Group &g)
{
    if (h->kernel_variant == 1) return false;
    return g.stream_ok;
}

// Both half-sweeps of a pair in one z-march: whole planes in LDS (TY = L).
bool use_pair(const hsg_lattice *h, const Group &g)
{
    if (h->kernel_variant == 1 || h->kernel_variant == 2) return false;
    return g.stream_ok && g.s_TY == g.L;
}

// LDS floats per replica of a fused z-march over whole planes: 6 planes for a
// pair, 11 for two over-relaxation pairs, each 3 components of L x L/2.
size_t fused_lds_bytes(const Group &g, int fuse)
{
    const size_t planes = fuse == 2 ? 11 : fuse == 1 ? 6 : 2;
    return planes * (size_t)g.s_RB * 3 * (size_t)g.s_rows * (size_t)(g.L / 2) * sizeof(float);
}

// Two over-relaxation pairs in one z-march, where the pair is fused and the
// eleven staged planes fit the work-group's LDS.
bool use_quad(const hsg_lattice *h, const Group &g)
{
    if (h->kernel_variant != 0 && h->kernel_variant != 4 && h->kernel_variant != 5) return false;
    // automatic choice: quantised angles are decoded and re-encoded at every
    // stage, which costs the two-pair launch more than the bytes it saves
    if (h->kernel_variant == 0 && h->storage == HSG_STORE_QANGLE) return false;
    return use_pair(h, g) && fused_lds_bytes(g, 2) <= h->max_lds;
}

hsg::StreamArgs stream_args(const hsg_lattice *h, const Group &g, int parity, uint32_t rep, int fuse,
                            int64_t r0 = 0, int64_t r1 = -1)
{
    if (r1 < 0) r1 = g.n_rep;
    hsg::StreamArgs a{};
    a.spins = h->state + g.o_spins;
    a.J6 = reinterpret_cast<const float *>(h->coup + g.o_J6);
    a.Jbits = g.ckind == 1 ? reinterpret_cast<const uint8_t *>(h->coup + g.o_Jbits) : nullptr;
    a.Hp = g.field ? reinterpret_cast<const float *>(h->field + g.o_H) : nullptr;
    a.temp_of_slot = reinterpret_cast<const int32_t *>(h->state + g.o_tos);
    a.beta32 = reinterpret_cast<const float *>(h->coup + g.o_b32);
    a.e_partials = reinterpret_cast<double *>(h->scratch + g.o_scr);
    a.Nh = g.Nh;
    a.n_rep = r1;
    a.r_base = r0;
    a.L = g.L;
    a.Lh = g.L / 2;
    a.P = g.L / 4;
    a.TY = g.s_TY;
    a.RB = g.s_RB;
    a.rows = g.s_rows;
    a.n_ytiles = g.s_ytiles;
    a.n_zslabs = fuse ? 1 : g.s_zslabs;
    a.zlen = g.L / a.n_zslabs;
    const int64_t nb = (r1 - r0 + g.s_RB - 1) / g.s_RB * g.s_ytiles * a.n_zslabs;
    a.n_blocks = nb > 0x7FFFFFFFll ? -1 : (int32_t)nb;
    a.slots_per_sample = g.O * g.T;
    a.T = g.T;
    a.tptr = dev_counter(h);
    a.rep = rep;
    a.parity = (uint32_t)parity;
    a.key0 = (uint32_t)(h->seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(h->seed >> 32);
    a.uid_base = g.uid_base;
    return a;
}

// Launches one half-sweep of parity `parity` (fuse = 0), one fused pair
// (fuse = 1) or two fused over-relaxation pairs (fuse = 2) for the groups
// `pick` selects, over replicas [r0, r1) of each (r1 < 0: all). The z-march
// groups go into as few launches as possible (up to kMaxStreamGroups per
// launch); the others use the gather kernel one group at a time. With energy,
// the partial sums are reduced into E unless reduce is false (the caller
// reduces once every replica range is done).
template <class Pick>
hsg_status run_groups(hsg_lattice *h, int kind, int parity, int rep, bool energy, int fuse, Pick pick,
                      hipStream_t s, int64_t r0 = 0, int64_t r1 = -1, bool reduce = true)
{
    if (kind == 0 && h->hw_math) kind = 2;
    hsg::MultiStreamArgs m{};
    unsigned threads = 0;
    size_t lds = 0;
    int64_t blocks = 0;
    auto flush = [&]() -> hsg_status {
        if (m.n_groups == 0) return HSG_OK;
        m.block_start[m.n_groups] = (int32_t)blocks;
        m.n_blocks = (int32_t)blocks;
        const hipError_t e = hsg::launch_half_sweep_stream(m, h->storage, kind, energy, fuse, threads, lds, s);
        m = hsg::MultiStreamArgs{};
        threads = 0;
        lds = 0;
        blocks = 0;
        if (e != hipSuccess) return hip_fail(e, "half-sweep launch");
        return HSG_OK;
    };
    for (const Group &g : h->lay.g) {
        if (!pick(g)) continue;
        if (fuse || use_stream(h, g)) {
            if (m.n_groups == hsg::kMaxStreamGroups) {
                hsg_status st = flush();
                if (st != HSG_OK) return st;
            }
            const hsg::StreamArgs a = stream_args(h, g, parity, (uint32_t)rep, fuse, r0, r1);
            const int64_t nb = (int64_t)a.n_blocks;
            if (nb < 0 || blocks + nb > 0x7FFFFFFFll) return fail(HSG_E_SIZE, "grid too large");
            m.block_start[m.n_groups] = (int32_t)blocks;
            m.g[m.n_groups++] = a;
            blocks += nb;
            const unsigned t = (unsigned)((a.RB * a.TY * a.P + 63) / 64 * 64);
            threads = t > threads ? t : threads;
            const size_t l = fused_lds_bytes(g, fuse);
            lds = l > lds ? l : lds;
        } else {
            if (r0 != 0 || (r1 >= 0 && r1 != g.n_rep)) return fail(HSG_E_STATE, "replica ranges need the z-march");
            const hsg::SweepArgs a = sweep_args(h, g, parity, (uint32_t)rep);
            if ((int64_t)g.D * a.n_chunks * a.n_pb > 0x7FFFFFFFll) return fail(HSG_E_SIZE, "grid too large");
            const hipError_t e = hsg::launch_half_sweep(a, h->storage, kind, g.field, energy, s);
            if (e != hipSuccess) return hip_fail(e, "half-sweep launch");
        }
    }
    hsg_status st = flush();
    if (st != HSG_OK) return st;
    if (energy && reduce) {
        for (const Group &g : h->lay.g) {
            if (!pick(g)) continue;
            const int n_pb = fuse ? 1 : use_stream(h, g) ? g.s_ytiles * g.s_zslabs : g.n_pb_sweep;
            const hipError_t e = hsg::launch_reduce_partials(reinterpret_cast<double *>(h->scratch + g.o_scr), n_pb,
                                                             g.n_rep, reinterpret_cast<double *>(h->state + g.o_E), s);
            if (e != hipSuccess) return hip_fail(e, "energy reduction launch");
        }
    }
    return HSG_OK;
}

hsg_status run_half_sweep(hsg_lattice *h, int kind, int parity, int rep, bool energy, hipStream_t s)
{
    return run_groups(h, kind, parity, rep, energy, 0, [](const Group &) { return true; }, s);
}

// A pair of half-sweeps (parity 0, then parity 1) of the groups `pick`
// selects: fused where the group holds whole planes, as two single passes
// otherwise. `energy`: the parity-1 pass computes the energies.
template <class Pick>
hsg_status run_pair_of(hsg_lattice *h, int kind, int rep, bool energy, hipStream_t s, Pick pick, int64_t r0,
                       int64_t r1, bool reduce)
{
    bool any_pair = false, any_single = false;
    for (const Group &g : h->lay.g) {
        if (!pick(g)) continue;
        any_pair = any_pair || use_pair(h, g);
        any_single = any_single || !use_pair(h, g);
    }
    if (any_pair) {
        auto fused = [h, &pick](const Group &g) { return pick(g) && use_pair(h, g); };
        hsg_status st = run_groups(h, kind, 0, rep, energy, 1, fused, s, r0, r1, reduce);
        if (st != HSG_OK) return st;
    }
    if (any_single) {
        auto single = [h, &pick](const Group &g) { return pick(g) && !use_pair(h, g); };
        hsg_status st = run_groups(h, kind, 0, rep, false, 0, single, s, r0, r1, reduce);
        if (st == HSG_OK) st = run_groups(h, kind, 1, rep, energy, 0, single, s, r0, r1, reduce);
        if (st != HSG_OK) return st;
    }
    return HSG_OK;
}

// One pair for every group (only == nullptr) or for group *only.
hsg_status run_pair(hsg_lattice *h, int kind, int rep, bool energy, hipStream_t s, const Group *only = nullptr,
                    int64_t r0 = 0, int64_t r1 = -1, bool reduce = true)
{
    auto pick = [only](const Group &g) { return only == nullptr || &g == only; };
    return run_pair_of(h, kind, rep, energy, s, pick, r0, r1, reduce);
}

// Two over-relaxation pairs: one z-march where use_quad allows it, two pairs
// elsewhere. `energy`: the last pass computes the energies.
hsg_status run_or_quad(hsg_lattice *h, bool energy, hipStream_t s, const Group *only = nullptr, int64_t r0 = 0,
                       int64_t r1 = -1, bool reduce = true)
{
    bool any_quad = false, any_other = false;
    for (const Group &g : h->lay.g) {
        if (only != nullptr && &g != only) continue;
        any_quad = any_quad || use_quad(h, g);
        any_other = any_other || !use_quad(h, g);
    }
    if (any_quad) {
        auto quad = [h, only](const Group &g) { return (only == nullptr || &g == only) && use_quad(h, g); };
        hsg_status st = run_groups(h, 1, 0, 0, energy, 2, quad, s, r0, r1, reduce);
        if (st != HSG_OK) return st;
    }
    if (any_other) {
        auto other = [h, only](const Group &g) { return (only == nullptr || &g == only) && !use_quad(h, g); };
        hsg_status st = run_pair_of(h, 1, 0, false, s, other, r0, r1, reduce);
        if (st == HSG_OK) st = run_pair_of(h, 1, 0, energy, s, other, r0, r1, reduce);
        if (st != HSG_OK) return st;
    }
    return HSG_OK;
}

// n_or over-relaxation pairs, two by two where possible; the last pass
// computes the energies when `energy` is set.
hsg_status run_or_rounds(hsg_lattice *h, int n_or, bool energy, hipStream_t s, const Group *only = nullptr,
                         int64_t r0 = 0, int64_t r1 = -1, bool reduce = true)
{
    bool any_quad = false;
    for (const Group &g : h->lay.g)
        if (only == nullptr || &g == only) any_quad = any_quad || use_quad(h, g);
    int r = 0;
    hsg_status st = HSG_OK;
    while (r < n_or && st == HSG_OK) {
        if (any_quad && r + 1 < n_or) {
            st = run_or_quad(h, energy && r + 2 == n_or, s, only, r0, r1, reduce);
            r += 2;
        } else {
            st = run_pair(h, 1, 0, energy && r + 1 == n_or, s, only, r0, r1, reduce);
            r += 1;
        }
    }
    return st;
}

// Replicas per batch of the sweep for group g (0: no batching). A batch's pairs
// run back to back, so the batch's spins stay in the last-level cache.
int64_t batch_of(const hsg_lattice *h, const Group &g)
{
    if (h->batch < 0 || !use_stream(h, g)) return 0;
    const int64_t per_rep = 2 * g.Nh * (int64_t)bytes_per_spin(h->storage);
    int64_t b = h->batch > 0 ? h->batch : (int64_t)(192ll << 20) / per_rep;
    if (b < 1) b = 1;
    return b < g.n_rep ? b : 0;
}


// Threads and replica groups of the resident launch for group g: G replica
// groups of Nh / 2 threads each, at most 512 threads; 0 when a sample does
// not fit.
unsigned resident_threads(const hsg_lattice *h, const Group &g, int32_t *groups)
{
    const int64_t Q = g.Nh / 2;
    const int R = g.O * g.T;
    if (Q < 1 || Q > 512) return 0;
    if (hsg::resident_lds_bytes(h->storage, g.Nh, R) > h->max_lds) return 0;
    const int G = (int)std::min<int64_t>(R, 512 / Q);
    if (groups) *groups = G;
    return (unsigned)((G * Q + 63) / 64 * 64);
}

// Whole sweeps a sample per work-group with the spins in LDS (kernel variant
// 5), where every lattice size allows it and no per-sweep series is recorded.
bool use_resident(const hsg_lattice *h)
{
    if (h->kernel_variant != 5 || h->chain != 0 || h->series != nullptr) return false;
    for (const Group &g : h->lay.g)
        if (resident_threads(h, g, nullptr) == 0) return false;
    return true;
}

// n sweeps of every group with the resident kernel, then the device counter.
hsg_status run_resident(hsg_lattice *h, int32_t n, hipStream_t s)
{
    for (const Group &g : h->lay.g) {
        hsg::ResidentArgs a{};
        int32_t G = 1;
        const unsigned threads = resident_threads(h, g, &G);
        a.spins = h->state + g.o_spins;
        a.J6 = reinterpret_cast<const float *>(h->coup + g.o_J6);
        a.Hp = g.field ? reinterpret_cast<const float *>(h->field + g.o_H) : nullptr;
        a.slot_at_temp = reinterpret_cast<int32_t *>(h->state + g.o_sat);
        a.temp_of_slot = reinterpret_cast<int32_t *>(h->state + g.o_tos);
        a.E = reinterpret_cast<double *>(h->state + g.o_E);
        a.beta32 = reinterpret_cast<const float *>(h->coup + g.o_b32);
        a.beta64 = reinterpret_cast<const double *>(h->coup + g.o_b64);
        a.accepts = reinterpret_cast<unsigned long long *>(h->state + g.o_acc);
        a.stat_sum = reinterpret_cast<double *>(h->state + g.o_ssum);
        a.stat_flag = reinterpret_cast<int32_t *>(h->state + g.o_sflag);
        a.stat_trips = reinterpret_cast<uint32_t *>(h->state + g.o_strips);
        a.tptr = dev_counter(h);
        a.Nh = g.Nh;
        a.L = g.L;
        a.Lh = g.L / 2;
        a.D = g.D;
        a.O = g.O;
        a.T = g.T;
        a.slots_per_sample = g.O * g.T;
        a.groups = G;
        a.n_sweeps = n;
        a.n_hb = h->n_hb;
        a.n_or = h->n_or;
        a.pt_every = h->pt_every;
        a.stats = h->stats ? 1 : 0;
        a.key0 = (uint32_t)(h->seed & 0xFFFFFFFFu);
        a.key1 = (uint32_t)(h->seed >> 32);
        a.uid_base = g.uid_base;
        const size_t lds = hsg::resident_lds_bytes(h->storage, g.Nh, g.O * g.T);
        const hipError_t e = hsg::launch_resident(a, h->storage, g.field, h->hw_math, threads, lds, s);
        if (e != hipSuccess) return hip_fail(e, "resident sweep launch");
    }
    const hipError_t e = hsg::launch_set_u32(dev_counter(h), (uint32_t)(h->t + (uint64_t)n), s);
    if (e != hipSuccess) return hip_fail(e, "counter launch");
    return HSG_OK;
}

// purpose 1: in-sweep pass, counter read from the device; 2: standalone pass.
hsg_status run_pt(hsg_lattice *h, uint32_t ctr1, uint32_t purpose, hipStream_t s)
{
    for (const Group &g : h->lay.g) {
        hsg::PtArgs a{};
        a.slot_at_temp = reinterpret_cast<int32_t *>(h->state + g.o_sat);
        a.temp_of_slot = reinterpret_cast<int32_t *>(h->state + g.o_tos);
        a.E = reinterpret_cast<const double *>(h->state + g.o_E);
        a.beta64 = reinterpret_cast<const double *>(h->coup + g.o_b64);
        a.accepts = reinterpret_cast<unsigned long long *>(h->state + g.o_acc);
        a.D = g.D;
        a.O = g.O;
        a.T = g.T;
        a.tptr = purpose == 1 ? dev_counter(h) : nullptr;
        a.ctr1 = ctr1;
        a.purpose = purpose;
        a.key0 = (uint32_t)(h->seed & 0xFFFFFFFFu);
        a.key1 = (uint32_t)(h->seed >> 32);
        a.uid_base = g.uid_base;
        const hipError_t e = hsg::launch_pt(a, s);
        if (e != hipSuccess) return hip_fail(e, "tempering launch");
    }
    return HSG_OK;
}

hsg::PackArgs pack_args(const hsg_lattice *h, const Group &g)
{
    hsg::PackArgs a{};
    a.spins_int = h->state + g.o_spins;
    a.J6 = reinterpret_cast<float *>(h->coup + g.o_J6);
    a.Hp = g.field ? reinterpret_cast<float *>(h->field + g.o_H) : nullptr;
    a.n_rep = g.n_rep;
    a.D = g.D;
    a.L = g.L;
    return a;
}

bool aligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) & (kAlign - 1)) == 0; }

// All launches of one sweep, kernels only (capturable): heat-bath pairs,
// over-relaxation pairs with the energy fused into the last pass, tempering,
// then the device sweep counter advances.
hsg::StatsArgs stats_args(const hsg_lattice *h, const Group &g)
{
    hsg::StatsArgs a{};
    a.slot_at_temp = reinterpret_cast<const int32_t *>(h->state + g.o_sat);
    a.E = reinterpret_cast<const double *>(h->state + g.o_E);
    a.sum = reinterpret_cast<double *>(h->state + g.o_ssum);
    a.flag = reinterpret_cast<int32_t *>(h->state + g.o_sflag);
    a.trips = reinterpret_cast<uint32_t *>(h->state + g.o_strips);
    a.D = g.D;
    a.O = g.O;
    a.T = g.T;
    return a;
}

hsg_status run_stats(hsg_lattice *h, bool clear, hipStream_t s)
{
    for (const Group &g : h->lay.g) {
        const hipError_t e = hsg::launch_stats(stats_args(h, g), clear, s);
        if (e != hipSuccess) return hip_fail(e, "statistics launch");
    }
    return HSG_OK;
}

// Doubles of one sweep's series record: per group the energies by rung
// [D][O][T], then q^2 [D][T] where the group has two copies or more.
int64_t series_record(const hsg_lattice *h)
{
    int64_t n = 0;
    for (const Group &g : h->lay.g) n += (int64_t)g.D * g.O * g.T + (g.O >= 2 ? (int64_t)g.D * g.T : 0);
    return n;
}

// Append this sweep's record to the series (after tempering; the device counter
// still holds the sweep's index).
hsg_status run_series(hsg_lattice *h, hipStream_t s)
{
    int64_t off = 0;
    for (const Group &g : h->lay.g) {
        hipError_t e = hipSuccess;
        double *q = nullptr;
        if (g.O >= 2) {
            hsg::OverlapArgs a{};
            a.spins = h->state + g.o_spins;
            a.slot_at_temp = reinterpret_cast<const int32_t *>(h->state + g.o_sat);
            a.partials = reinterpret_cast<double *>(h->scratch + g.o_scr);
            q = reinterpret_cast<double *>(h->scratch + g.o_scr_q);
            a.q = q;
            a.Nh = g.Nh;
            a.D = g.D;
            a.O = g.O;
            a.T = g.T;
            a.L = g.L;
            a.n_pb = (int32_t)hsg::march_partials(g.L, (int64_t)g.D * g.T, g.q_pb);
            a.chunk = g.q_chunk;
            e = hsg::launch_overlap(a, h->storage, s);
        }
        hsg::SeriesArgs r{};
        r.slot_at_temp = reinterpret_cast<const int32_t *>(h->state + g.o_sat);
        r.E = reinterpret_cast<const double *>(h->state + g.o_E);
        r.q = q;
        r.out = h->series + off;
        r.tptr = dev_counter(h);
        r.t0 = (uint32_t)h->series_t0;
        r.capacity = h->series_cap;
        r.stride = h->series_rec;
        r.D = g.D;
        r.O = g.O;
        r.T = g.T;
        if (e == hipSuccess) e = hsg::launch_series(r, s);
        if (e != hipSuccess) return hip_fail(e, "series launch");
        off += (int64_t)g.D * g.O * g.T + (g.O >= 2 ? (int64_t)g.D * g.T : 0);
    }
    return HSG_OK;
}

// Exact energies of every replica into E (full recomputation), all groups.
hsg_status run_energy(hsg_lattice *h, hipStream_t s)
{
    for (const Group &g : h->lay.g) {
        hsg::EnergyArgs a{};
        a.spins = h->state + g.o_spins;
        a.J6 = reinterpret_cast<const float *>(h->coup + g.o_J6);
        a.Hp = g.field ? reinterpret_cast<const float *>(h->field + g.o_H) : nullptr;
        a.partials = reinterpret_cast<double *>(h->scratch + g.o_scr);
        a.Nh = g.Nh;
        a.n_rep = g.n_rep;
        a.L = g.L;
        a.Lh = g.L / 2;
        a.slots_per_sample = g.O * g.T;
        a.n_pb = (int32_t)hsg::energy_partials(g.L, g.n_rep, g.n_pb_site);
        hipError_t e = hsg::launch_energy(a, h->storage, s);
        if (e == hipSuccess)
            e = hsg::launch_reduce_partials(a.partials, a.n_pb, g.n_rep, reinterpret_cast<double *>(h->state + g.o_E), s);
        if (e != hipSuccess) return hip_fail(e, "energy launch");
    }
    return HSG_OK;
}

int32_t tiles_in_phase(const Group &g, int phase)
{
    if (g.t_BX > 1) return g.t_BZ * g.t_BY * (g.t_BX / 2);
    if (g.t_BY > 1) return g.t_BZ * (g.t_BY / 2);
    if (g.t_BZ > 1) return g.t_BZ / 2;
    return phase == 0 ? 1 : 0;
}

// One sweep of the tile-local chain: the tiles of coarse parity 0, then 1.
hsg_status run_tile_sweep(hsg_lattice *h, hipStream_t s)
{
    for (int phase = 0; phase < 2; ++phase)
        for (const Group &g : h->lay.g) {
            const int32_t nt = tiles_in_phase(g, phase);
            if (nt == 0) continue;
            hsg::TileArgs a{};
            a.spins = h->state + g.o_spins;
            a.J6 = reinterpret_cast<const float *>(h->coup + g.o_J6);
            a.Jbits = g.ckind == 1 ? reinterpret_cast<const uint8_t *>(h->coup + g.o_Jbits) : nullptr;
            a.Hp = g.field ? reinterpret_cast<const float *>(h->field + g.o_H) : nullptr;
            a.temp_of_slot = reinterpret_cast<const int32_t *>(h->state + g.o_tos);
            a.beta32 = reinterpret_cast<const float *>(h->coup + g.o_b32);
            a.tptr = dev_counter(h);
            a.Nh = g.Nh;
            a.L = g.L;
            a.Lh = g.L / 2;
            a.TX = g.t_TX;
            a.TY = g.t_TY;
            a.TZ = g.t_TZ;
            a.BX = g.t_BX;
            a.BY = g.t_BY;
            a.BZ = g.t_BZ;
            a.hx = g.t_hx;
            a.hy = g.t_hy;
            a.hz = g.t_hz;
            a.RXh = g.t_RXh;
            a.RY = g.t_RY;
            a.RZ = g.t_RZ;
            a.P = g.t_P;
            a.RB = g.t_RB;
            a.n_chunks = g.t_chunks;
            a.phase = phase;
            a.n_tiles_phase = nt;
            const int64_t nb = (int64_t)g.D * nt * g.t_chunks;
            if (nb > 0x7FFFFFFFll) return fail(HSG_E_SIZE, "grid too large");
            a.n_blocks = (int32_t)nb;
            a.n_or = h->n_or;
            a.n_hb = h->n_hb;
            a.n_hit = h->n_hit;
            a.slots_per_sample = g.O * g.T;
            a.T = g.T;
            a.key0 = (uint32_t)(h->seed & 0xFFFFFFFFu);
            a.key1 = (uint32_t)(h->seed >> 32);
            a.uid_base = g.uid_base;
            const hipError_t e = hsg::launch_tile_visit(a, h->storage, g.field, g.ckind == 1, h->hw_math,
                                                        (unsigned)g.t_threads, g.t_lds, s);
            if (e != hipSuccess) return hip_fail(e, "tile launch");
        }
    return run_energy(h, s);
}

hsg_status enqueue_sweep(hsg_lattice *h, bool pt, hipStream_t s)
{
    if (h->chain == 1) {
        hsg_status st = run_tile_sweep(h, s);
        if (st == HSG_OK && pt) st = run_pt(h, 0u, 1u, s);
        if (st == HSG_OK && h->stats) st = run_stats(h, false, s);
        if (st == HSG_OK && h->series) st = run_series(h, s);
        if (st != HSG_OK) return st;
        const hipError_t e = hsg::launch_advance(dev_counter(h), s);
        if (e != hipSuccess) return hip_fail(e, "counter launch");
        return HSG_OK;
    }
    const int last_kind = h->n_or > 0 ? 1 : 0;
    bool batched = false;
    for (const Group &g : h->lay.g) batched = batched || batch_of(h, g) > 0;
    if (!batched) {
        for (int r = 0; r < h->n_hb; ++r) {
            hsg_status st = run_pair(h, 0, r, last_kind == 0 && r == h->n_hb - 1, s);
            if (st != HSG_OK) return st;
        }
        hsg_status st = run_or_rounds(h, h->n_or, true, s);
        if (st != HSG_OK) return st;
    } else {
        // Replicas never interact within the pairs of a sweep: all pairs of one
        // batch of replicas run back to back (the batch stays in the last-level
        // cache), then the next batch; the same updates in the same order per
        // replica, so the same bits.
        for (const Group &g : h->lay.g) {
            const int64_t b = batch_of(h, g);
            const int64_t step = b > 0 ? b : g.n_rep;
            for (int64_t r0 = 0; r0 < g.n_rep; r0 += step) {
                const int64_t r1 = std::min<int64_t>(g.n_rep, r0 + step);
                for (int r = 0; r < h->n_hb; ++r) {
                    hsg_status st = run_pair(h, 0, r, last_kind == 0 && r == h->n_hb - 1, s, &g, r0, r1, b == 0);
                    if (st != HSG_OK) return st;
                }
                hsg_status st = run_or_rounds(h, h->n_or, true, s, &g, r0, r1, b == 0);
                if (st != HSG_OK) return st;
            }
            if (b > 0) {  // one reduction over every batch's partial sums
                const int n_pb = use_pair(h, g) ? 1 : g.s_ytiles * g.s_zslabs;
                const hipError_t e = hsg::launch_reduce_partials(reinterpret_cast<double *>(h->scratch + g.o_scr),
                                                                 n_pb, g.n_rep,
                                                                 reinterpret_cast<double *>(h->state + g.o_E), s);
                if (e != hipSuccess) return hip_fail(e, "energy reduction launch");
            }
        }
    }
    if (pt) {
        hsg_status st = run_pt(h, 0u, 1u, s);
        if (st != HSG_OK) return st;
    }
    if (h->stats) {
        hsg_status st = run_stats(h, false, s);
        if (st != HSG_OK) return st;
    }
    if (h->series) {
        hsg_status st = run_series(h, s);
        if (st != HSG_OK) return st;
    }
    const hipError_t e = hsg::launch_advance(dev_counter(h), s);
    if (e != hipSuccess) return hip_fail(e, "counter launch");
    return HSG_OK;
}

// Graph k holds 1 (k = 0) or kGraphSweeps (k = 1) sweeps, each with tempering
// when pt_every == 1. Captured once on a private stream, replayed on the
// caller's stream.
hsg_status launch_graph(hsg_lattice *h, int k, hipStream_t s)
{
    if (h->graph_exec[k] == nullptr) {
        hipError_t e = hipSuccess;
        if (h->capture_stream == nullptr) e = hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "capture stream");
        e = hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "begin capture");
        const int n = k == 0 ? 1 : kGraphSweeps;
        hsg_status st = HSG_OK;
        for (int i = 0; i < n && st == HSG_OK; ++i) st = enqueue_sweep(h, h->pt_every == 1, h->capture_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(h->capture_stream, &g);
        if (st != HSG_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_fail(e, "graph instantiate");
        }
        h->graph[k] = g;
        h->graph_exec[k] = x;
    }
    const hipError_t e = hipGraphLaunch(h->graph_exec[k], s);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return HSG_OK;
}

}  // namespace

extern "C" {

const char *hsg_last_error(void) { return g_err.c_str(); }

#ifndef HSG_BUILD_ID
#define HSG_BUILD_ID "unknown"
#endif
const char *hsg_build_id(void) { return HSG_BUILD_ID; }

hsg_status hsg_query_sizes(const hsg_desc *desc, hsg_sizes *out)
{
    if (out == nullptr) return fail(HSG_E_INVALID, "out is NULL");
    Layout lay;
    const hsg_status st = build_layout(desc, lay);
    if (st != HSG_OK) return st;
    *out = lay.sz;
    return HSG_OK;
}

hsg_status hsg_init_lattice(const hsg_desc *desc, const float *d_spins0, const float *d_J, const float *d_H,
                            void *d_state, void *d_couplings, void *d_field, void *d_scratch, hsg_stream_t stream,
                            hsg_lattice **out)
{
    if (out == nullptr) return fail(HSG_E_INVALID, "out is NULL");
    *out = nullptr;
    Layout lay;
    hsg_status st = build_layout(desc, lay);
    if (st != HSG_OK) return st;
    bool any_field = false;
    for (const Group &g : lay.g) any_field = any_field || g.field;
    if (d_spins0 == nullptr || d_J == nullptr) return fail(HSG_E_INVALID, "d_spins0 and d_J are required");
    if (any_field && d_H == nullptr) return fail(HSG_E_INVALID, "a group has a field but d_H is NULL");
    if (d_state == nullptr || d_couplings == nullptr || d_scratch == nullptr)
        return fail(HSG_E_INVALID, "d_state, d_couplings and d_scratch are required");
    if (lay.sz.field_bytes > 0 && d_field == nullptr) return fail(HSG_E_INVALID, "d_field is required");
    if (!aligned(d_state) || !aligned(d_couplings) || !aligned(d_scratch) || (d_field && !aligned(d_field)))
        return fail(HSG_E_INVALID, "device buffers must be 256-byte aligned");

    hsg_lattice *h = new (std::nothrow) hsg_lattice();
    if (h == nullptr) return fail(HSG_E_INVALID, "out of host memory");
    h->lay = std::move(lay);
    h->storage = desc->storage;
    h->n_hb = desc->n_hb;
    h->n_or = desc->n_or;
    h->pt_every = desc->pt_every;
    h->seed = desc->seed;
    h->state = static_cast<char *>(d_state);
    h->coup = static_cast<char *>(d_couplings);
    h->field = static_cast<char *>(d_field);
    h->scratch = static_cast<char *>(d_scratch);
    {
        int dev = 0, v = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            h->max_lds = (size_t)v;
        h->device = dev;
        void *p = nullptr;
        if (e == hipSuccess) e = static_scratch_ptr(dev, &p);  // once per device, with the device current
        if (e != hipSuccess) {
            delete h;
            return hip_fail(e, "init: device scratch address");
        }
    }
    hipStream_t s = S(stream);
    {
        const hipError_t e = hipMemsetAsync(h->state, 0, kAlign, s);
        if (e != hipSuccess) {
            delete h;
            return hip_fail(e, "init");
        }
    }

    for (const Group &g : h->lay.g) {
        hsg::PackArgs a = pack_args(h, g);
        a.spins_can = const_cast<float *>(d_spins0) + g.can_spin0;
        a.J_can = d_J + g.can_site0;
        a.H_can = g.field ? d_H + g.can_site0 : nullptr;
        hipError_t e = hsg::launch_pack_spins(a, h->storage, s);
        if (e == hipSuccess) e = hsg::launch_pack_couplings(a, s);
        if (e == hipSuccess && g.ckind == 1) {
            int32_t *flag = reinterpret_cast<int32_t *>(h->scratch + g.o_scr);
            e = hsg::launch_check_pm1(a.J_can, (int64_t)g.D * 3 * g.N, flag, s);
            int32_t bad = 0;
            if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e == hipSuccess && bad != 0) {
                delete h;
                return fail(HSG_E_INVALID, "group with coupling_kind = 1 has couplings other than +-1");
            }
            if (e == hipSuccess)
                e = hsg::launch_pack_jbits(a.J_can, reinterpret_cast<uint8_t *>(h->coup + g.o_Jbits), g.D, g.L, s);
        }
        if (e == hipSuccess && g.field) e = hsg::launch_pack_field(a, s);
        // ladders: float64 and float32 inverse temperatures
        std::vector<double> b64(g.T);
        std::vector<float> b32(g.T);
        for (int k = 0; k < g.T; ++k) {
            b64[k] = 1.0 / g.temps[k];
            b32[k] = (float)b64[k];
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->coup + g.o_b64, b64.data(), g.T * 8, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->coup + g.o_b32, b32.data(), g.T * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hsg::launch_fill_identity_maps(reinterpret_cast<int32_t *>(h->state + g.o_sat),
                                               reinterpret_cast<int32_t *>(h->state + g.o_tos),
                                               (int64_t)g.D * g.O, g.T, s);
        if (e == hipSuccess)
            e = hipMemsetAsync(h->state + g.o_E, 0, (size_t)g.n_rep * 8, s);
        if (e == hipSuccess)
            e = hipMemsetAsync(h->state + g.o_acc, 0, (size_t)g.D * g.O * (g.T > 1 ? g.T - 1 : 1) * 8, s);
        if (e == hipSuccess) e = hsg::launch_stats(stats_args(h, g), true, s);
        if (e != hipSuccess) {
            delete h;
            return hip_fail(e, "init");
        }
        // the host copies above read stack vectors: wait before they go away
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            delete h;
            return hip_fail(e, "init");
        }
    }
    *out = h;
    return HSG_OK;
}

// ---------------------------------------------------------------- overlapped sweeps
// Samples never interact, so the two halves of every group's samples can run
// their sweeps on two streams, each half with its own device sweep counter.
// The second half's heat-bath pairs of a sweep wait for the first half's, and
// the first half's next heat-bath pairs for the second half's, so that each
// half's heat bath (bound by instruction issue) runs beside the other half's
// over-relaxation (bound by latency). Every replica gets the same updates with
// the same counters as in one stream, so the results are the same bits.
bool overlap_ok(const hsg_lattice *h)
{
    if (!h->overlap || h->chain != 0 || h->series != nullptr || use_resident(h)) return false;
    for (const Group &g : h->lay.g) {
        if (!use_stream(h, g) || g.D < 2 || batch_of(h, g) > 0) return false;
    }
    return true;
}

// Replica and sample range [r0, r1), [d0, d1) of half c of group g.
void half_range(const Group &g, int c, int64_t &d0, int64_t &d1, int64_t &r0, int64_t &r1)
{
    const int64_t half = g.D / 2, spp = (int64_t)g.O * g.T;
    d0 = c == 0 ? 0 : half;
    d1 = c == 0 ? half : g.D;
    r0 = d0 * spp;
    r1 = d1 * spp;
}

// One sweep of half c (heat-bath pairs, then the rest), on stream s; `hb_done`
// is recorded after the heat-bath pairs.
hsg_status enqueue_half_sweep(hsg_lattice *h, int c, bool pt, hipStream_t s, hipEvent_t hb_done)
{
    h->cohort = c;
    const int last_kind = h->n_or > 0 ? 1 : 0;
    hsg_status st = HSG_OK;
    for (const Group &g : h->lay.g) {
        int64_t d0, d1, r0, r1;
        half_range(g, c, d0, d1, r0, r1);
        for (int r = 0; r < h->n_hb && st == HSG_OK; ++r)
            st = run_pair(h, 0, r, last_kind == 0 && r == h->n_hb - 1, s, &g, r0, r1, false);
    }
    hipError_t e = st == HSG_OK ? hipEventRecord(hb_done, s) : hipSuccess;
    if (e != hipSuccess) st = hip_fail(e, "event record");
    for (const Group &g : h->lay.g) {
        if (st != HSG_OK) break;
        int64_t d0, d1, r0, r1;
        half_range(g, c, d0, d1, r0, r1);
        st = run_or_rounds(h, h->n_or, true, s, &g, r0, r1, false);
        if (st != HSG_OK) break;
        const int n_pb = use_pair(h, g) ? 1 : g.s_ytiles * g.s_zslabs;
        e = hsg::launch_reduce_partials(reinterpret_cast<double *>(h->scratch + g.o_scr) + r0 * n_pb, n_pb,
                                        r1 - r0, reinterpret_cast<double *>(h->state + g.o_E) + r0, s);
        if (e != hipSuccess) {
            st = hip_fail(e, "energy reduction launch");
            break;
        }
        const int64_t OT = (int64_t)g.O * g.T;
        if (pt) {
            hsg::PtArgs a{};
            a.slot_at_temp = reinterpret_cast<int32_t *>(h->state + g.o_sat) + d0 * OT;
            a.temp_of_slot = reinterpret_cast<int32_t *>(h->state + g.o_tos) + d0 * OT;
            a.E = reinterpret_cast<const double *>(h->state + g.o_E) + d0 * OT;
            a.beta64 = reinterpret_cast<const double *>(h->coup + g.o_b64);
            a.accepts = reinterpret_cast<unsigned long long *>(h->state + g.o_acc) + d0 * g.O * (g.T - 1);
            a.D = (int32_t)(d1 - d0);
            a.O = g.O;
            a.T = g.T;
            a.tptr = dev_counter(h);
            a.ctr1 = 0;
            a.purpose = 1;
            a.key0 = (uint32_t)(h->seed & 0xFFFFFFFFu);
            a.key1 = (uint32_t)(h->seed >> 32);
            a.uid_base = g.uid_base + (uint32_t)d0;
            e = hsg::launch_pt(a, s);
            if (e != hipSuccess) {
                st = hip_fail(e, "tempering launch");
                break;
            }
        }
        if (h->stats) {
            hsg::StatsArgs a = stats_args(h, g);
            a.slot_at_temp += d0 * OT;
            a.E += d0 * OT;
            a.sum += d0 * OT * 2;
            a.flag += d0 * OT;
            a.trips += d0 * OT;
            a.D = (int32_t)(d1 - d0);
            e = hsg::launch_stats(a, false, s);
            if (e != hipSuccess) {
                st = hip_fail(e, "statistics launch");
                break;
            }
        }
    }
    if (st == HSG_OK) {
        e = hsg::launch_advance(dev_counter(h), s);
        if (e != hipSuccess) st = hip_fail(e, "counter launch");
    }
    h->cohort = 0;
    return st;
}

hsg_status overlapped_sweeps(hsg_lattice *h, int32_t n_sweeps, hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (h->stream2 == nullptr) e = hipStreamCreateWithFlags(&h->stream2, hipStreamNonBlocking);
    for (auto &x : h->ev)
        if (e == hipSuccess && x == nullptr) e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "overlap stream or events");
    hipStream_t s2 = h->stream2;
    // Sweeps on one stream advance only the first counter: the second half starts from it.
    uint32_t *const ctr = reinterpret_cast<uint32_t *>(h->state);
    e = hsg::launch_copy_u32(ctr, ctr + 1, s);
    if (e == hipSuccess) e = hipEventRecord(h->ev[0], s);  // fork: the second stream starts after the caller's work
    if (e == hipSuccess) e = hipStreamWaitEvent(s2, h->ev[0], 0);
    if (e != hipSuccess) return hip_fail(e, "overlap fork");
    hsg_status st = HSG_OK;
    for (int k = 0; k < n_sweeps && st == HSG_OK; ++k) {
        const bool pt = h->pt_every > 0 && ((h->t + 1) % (uint64_t)h->pt_every) == 0;
        if (k > 0) e = hipStreamWaitEvent(s, h->ev[2], 0);  // half 0's heat bath after half 1's
        if (e != hipSuccess) {
            st = hip_fail(e, "overlap wait");
            break;
        }
        st = enqueue_half_sweep(h, 0, pt, s, h->ev[1]);
        if (st != HSG_OK) break;
        e = hipStreamWaitEvent(s2, h->ev[1], 0);  // half 1's heat bath after half 0's
        if (e != hipSuccess) {
            st = hip_fail(e, "overlap wait");
            break;
        }
        st = enqueue_half_sweep(h, 1, pt, s2, h->ev[2]);
        if (st == HSG_OK) h->t += 1;
    }
    // join, also after an error: the caller's stream continues after all that
    // the second stream was given
    e = hipEventRecord(h->ev[3], s2);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, h->ev[3], 0);
    if (e != hipSuccess && st == HSG_OK) st = hip_fail(e, "overlap join");
    return st;
}

hsg_status hsg_sweep(hsg_lattice *h, int32_t n_sweeps, hsg_stream_t stream)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (n_sweeps < 0) return fail(HSG_E_INVALID, "n_sweeps = %d < 0", n_sweeps);
    if (h->t + (uint64_t)n_sweeps > 0x100000000ull)
        return fail(HSG_E_SIZE, "the sweep counter would pass 2^32 (the counter map limit)");
    hipStream_t s = S(stream);
    const bool graphs = h->use_graphs && h->pt_every <= 1;
    int done = 0;
    if (n_sweeps > 0 && use_resident(h)) {
        constexpr int kMaxPerLaunch = 256;  // bounded launches for long runs
        while (done < n_sweeps) {
            const int n = std::min(kMaxPerLaunch, n_sweeps - done);
            hsg_status st = run_resident(h, n, s);
            if (st != HSG_OK) return st;
            done += n;
            h->t += (uint64_t)n;
        }
    } else if (n_sweeps > 0 && overlap_ok(h)) {
        hsg_status st = overlapped_sweeps(h, n_sweeps, s);
        if (st != HSG_OK) return st;
        done = n_sweeps;
    } else if (graphs) {
        while (n_sweeps - done >= kGraphSweeps) {
            hsg_status st = launch_graph(h, 1, s);
            if (st != HSG_OK) return st;
            done += kGraphSweeps;
            h->t += kGraphSweeps;
        }
        while (done < n_sweeps) {
            hsg_status st = launch_graph(h, 0, s);
            if (st != HSG_OK) return st;
            done += 1;
            h->t += 1;
        }
    } else {
        for (; done < n_sweeps; ++done) {
            const bool pt = h->pt_every > 0 && ((h->t + 1) % (uint64_t)h->pt_every) == 0;
            hsg_status st = enqueue_sweep(h, pt, s);
            if (st != HSG_OK) return st;
            h->t += 1;
        }
    }
    h->have_energies = n_sweeps > 0 || h->have_energies;
    if (h->stats) h->n_stats += (uint64_t)n_sweeps;
    return HSG_OK;
}

hsg_status hsg_half_sweep(hsg_lattice *h, int32_t kind, int32_t parity, int32_t rep, hsg_stream_t stream)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (kind != 0 && kind != 1) return fail(HSG_E_INVALID, "kind = %d, need 0 (HB) or 1 (OR)", kind);
    if (parity != 0 && parity != 1) return fail(HSG_E_INVALID, "parity = %d", parity);
    if (rep < 0 || rep > 15) return fail(HSG_E_SIZE, "rep = %d, need 0..15", rep);
    return run_half_sweep(h, kind, parity, rep, false, S(stream));
}

hsg_status hsg_pair_sweep(hsg_lattice *h, int32_t kind, int32_t rep, hsg_stream_t stream)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (kind != 0 && kind != 1) return fail(HSG_E_INVALID, "kind = %d, need 0 (HB) or 1 (OR)", kind);
    if (rep < 0 || rep > 15) return fail(HSG_E_SIZE, "rep = %d, need 0..15", rep);
    return run_pair(h, kind, rep, false, S(stream));
}

hsg_status hsg_or_pairs(hsg_lattice *h, int32_t n_pairs, hsg_stream_t stream)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (n_pairs < 1 || n_pairs > 1000) return fail(HSG_E_INVALID, "n_pairs = %d, need 1..1000", n_pairs);
    return run_or_rounds(h, n_pairs, false, S(stream));
}

hsg_status hsg_pt_exchange(hsg_lattice *h, hsg_stream_t stream)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (h->pt_calls >= 0x100000000ull) return fail(HSG_E_SIZE, "standalone tempering counter exhausted");
    const hsg_status st = run_pt(h, (uint32_t)h->pt_calls, 2u, S(stream));
    if (st == HSG_OK) h->pt_calls += 1;
    return st;
}

hsg_status hsg_measure_energy(hsg_lattice *h, double *d_E, hsg_stream_t stream)
{
    if (h == nullptr || d_E == nullptr) return fail(HSG_E_INVALID, "handle and d_E are required");
    hipStream_t s = S(stream);
    for (const Group &g : h->lay.g) {
        hsg::EnergyArgs a{};
        a.spins = h->state + g.o_spins;
        a.J6 = reinterpret_cast<const float *>(h->coup + g.o_J6);
        a.Hp = g.field ? reinterpret_cast<const float *>(h->field + g.o_H) : nullptr;
        a.partials = reinterpret_cast<double *>(h->scratch + g.o_scr);
        a.Nh = g.Nh;
        a.n_rep = g.n_rep;
        a.L = g.L;
        a.Lh = g.L / 2;
        a.slots_per_sample = g.O * g.T;
        a.n_pb = (int32_t)hsg::energy_partials(g.L, g.n_rep, g.n_pb_site);
        hipError_t e = hsg::launch_energy(a, h->storage, s);
        double *E = reinterpret_cast<double *>(h->state + g.o_E);
        if (e == hipSuccess) e = hsg::launch_reduce_partials(a.partials, a.n_pb, g.n_rep, E, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_E + g.rep0, E, (size_t)g.n_rep * 8, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "measure_energy");
    }
    h->have_energies = true;
    return HSG_OK;
}

hsg_status hsg_measure_energy_static(hsg_lattice *h, double *d_E, hsg_stream_t stream)
{
    if (h == nullptr || d_E == nullptr) return fail(HSG_E_INVALID, "handle and d_E are required");
    for (const Group &g : h->lay.g) {
        const uint64_t need = (uint64_t)g.n_rep * hsg::energy_partials(g.L, g.n_rep, g.n_pb_site) * sizeof(double);
        if (need > kStaticScratchBytes)
            return fail(HSG_E_SIZE, "group of L = %d needs %llu bytes of energy partials, the fixed scratch holds %zu",
                        g.L, (unsigned long long)need, kStaticScratchBytes);
    }
    void *p = nullptr;
    hipError_t e = static_scratch_ptr(h->device, &p);
    if (e != hipSuccess) return hip_fail(e, "measure_energy_static: device scratch address");
    hipStream_t s = S(stream);
    for (const Group &g : h->lay.g) {  // the groups run one after the other on the stream: one region suffices
        hsg::EnergyArgs a{};
        a.spins = h->state + g.o_spins;
        a.J6 = reinterpret_cast<const float *>(h->coup + g.o_J6);
        a.Hp = g.field ? reinterpret_cast<const float *>(h->field + g.o_H) : nullptr;
        a.partials = static_cast<double *>(p);
        a.Nh = g.Nh;
        a.n_rep = g.n_rep;
        a.L = g.L;
        a.Lh = g.L / 2;
        a.slots_per_sample = g.O * g.T;
        a.n_pb = (int32_t)hsg::energy_partials(g.L, g.n_rep, g.n_pb_site);
        e = hsg::launch_energy(a, h->storage, s);
        double *E = reinterpret_cast<double *>(h->state + g.o_E);
        if (e == hipSuccess) e = hsg::launch_reduce_partials(a.partials, a.n_pb, g.n_rep, E, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_E + g.rep0, E, (size_t)g.n_rep * 8, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "measure_energy_static");
    }
    h->have_energies = true;
    return HSG_OK;
}

hsg_status hsg_get_energies(const hsg_lattice *h, double *d_E, hsg_stream_t stream)
{
    if (h == nullptr || d_E == nullptr) return fail(HSG_E_INVALID, "handle and d_E are required");
    for (const Group &g : h->lay.g) {
        const hipError_t e = hipMemcpyAsync(d_E + g.rep0, h->state + g.o_E, (size_t)g.n_rep * 8,
                                            hipMemcpyDeviceToDevice, S(stream));
        if (e != hipSuccess) return hip_fail(e, "get_energies");
    }
    return HSG_OK;
}

hsg_status hsg_measure_overlap(hsg_lattice *h, double *d_q, hsg_stream_t stream)
{
    if (h == nullptr || d_q == nullptr) return fail(HSG_E_INVALID, "handle and d_q are required");
    for (const Group &g : h->lay.g)
        if (g.O < 2) return fail(HSG_E_INVALID, "the overlap needs n_copies >= 2 in every group");
    int64_t off = 0;
    for (const Group &g : h->lay.g) {
        hsg::OverlapArgs a{};
        a.spins = h->state + g.o_spins;
        a.slot_at_temp = reinterpret_cast<const int32_t *>(h->state + g.o_sat);
        a.partials = reinterpret_cast<double *>(h->scratch + g.o_scr);
        a.q = d_q + off;
        a.Nh = g.Nh;
        a.D = g.D;
        a.O = g.O;
        a.T = g.T;
        a.L = g.L;
        a.n_pb = (int32_t)hsg::march_partials(g.L, (int64_t)g.D * g.T, g.q_pb);
        a.chunk = g.q_chunk;
        const hipError_t e = hsg::launch_overlap(a, h->storage, S(stream));
        if (e != hipSuccess) return hip_fail(e, "measure_overlap");
        off += (int64_t)g.D * g.T * 10;
    }
    return HSG_OK;
}

hsg_status hsg_measure_kmodes(hsg_lattice *h, double *d_q, hsg_stream_t stream)
{
    if (h == nullptr || d_q == nullptr) return fail(HSG_E_INVALID, "handle and d_q are required");
    for (const Group &g : h->lay.g) {
        if (g.O < 2) return fail(HSG_E_INVALID, "the overlaps need n_copies >= 2 in every group");
        if (g.L > 1024) return fail(HSG_E_UNSUPPORTED, "k modes need L <= 1024");
    }
    int64_t off = 0;
    for (const Group &g : h->lay.g) {
        hsg::KmodeArgs a{};
        a.spins = h->state + g.o_spins;
        a.slot_at_temp = reinterpret_cast<const int32_t *>(h->state + g.o_sat);
        a.partials = reinterpret_cast<double *>(h->scratch + g.o_scr);
        a.q = d_q + off;
        a.Nh = g.Nh;
        a.L = g.L;
        a.D = g.D;
        a.O = g.O;
        a.T = g.T;
        a.n_pb = (int32_t)hsg::kmode_partials(g.L, g.q_pb);
        a.chunk = 2 * g.q_chunk;
        const hipError_t e = hsg::launch_kmodes(a, h->storage, S(stream));
        if (e != hipSuccess) return hip_fail(e, "measure_kmodes");
        off += (int64_t)g.D * g.T * 84;
    }
    return HSG_OK;
}

hsg_status hsg_measure_pair_overlaps(hsg_lattice *h, double *d_q, hsg_stream_t stream)
{
    if (h == nullptr || d_q == nullptr) return fail(HSG_E_INVALID, "handle and d_q are required");
    for (const Group &g : h->lay.g) {
        if (g.O < 2) return fail(HSG_E_INVALID, "pair overlaps need n_copies >= 2 in every group");
        if (g.L > 1024) return fail(HSG_E_UNSUPPORTED, "pair overlaps need L <= 1024");
    }
    int64_t off = 0;
    for (const Group &g : h->lay.g) {
        hsg::PairOvArgs a{};
        a.spins = h->state + g.o_spins;
        a.slot_at_temp = reinterpret_cast<const int32_t *>(h->state + g.o_sat);
        a.partials = reinterpret_cast<double *>(h->scratch + g.o_scr);
        a.q = d_q + off;
        a.Nh = g.Nh;
        a.L = g.L;
        a.D = g.D;
        a.O = g.O;
        a.T = g.T;
        a.n_pb = (int32_t)hsg::march_partials(g.L, (int64_t)g.D * g.T, g.q_pb);
        a.chunk = 2 * g.q_chunk;
        const hipError_t e = hsg::launch_pair_overlaps(a, h->storage, S(stream));
        if (e != hipSuccess) return hip_fail(e, "measure_pair_overlaps");
        off += (int64_t)g.D * g.T * 7 * (g.O * (g.O - 1) / 2);
    }
    return HSG_OK;
}

hsg_status hsg_measure_chi(hsg_lattice *h, double *d_chi, hsg_stream_t stream)
{
    if (h == nullptr || d_chi == nullptr) return fail(HSG_E_INVALID, "handle and d_chi are required");
    for (const Group &g : h->lay.g) {
        if (g.O < 4) return fail(HSG_E_INVALID, "the four-replica estimators need n_copies >= 4 in every group");
        if (g.L > 1024) return fail(HSG_E_UNSUPPORTED, "the four-replica estimators need L <= 1024");
    }
    int64_t off = 0;
    for (const Group &g : h->lay.g) {
        hsg::PairOvArgs a{};
        a.spins = h->state + g.o_spins;
        a.slot_at_temp = reinterpret_cast<const int32_t *>(h->state + g.o_sat);
        a.partials = reinterpret_cast<double *>(h->scratch + g.o_scr);
        a.q = nullptr;
        a.chi = d_chi + off;
        a.Nh = g.Nh;
        a.L = g.L;
        a.D = g.D;
        a.O = g.O;
        a.T = g.T;
        a.n_pb = (int32_t)hsg::march_partials(g.L, (int64_t)g.D * g.T, g.q_pb);
        a.chunk = 2 * g.q_chunk;
        const hipError_t e = hsg::launch_pair_overlaps(a, h->storage, S(stream));
        if (e != hipSuccess) return hip_fail(e, "measure_chi");
        off += (int64_t)g.D * g.T * 4 * 5;
    }
    return HSG_OK;
}

hsg_status hsg_set_series(hsg_lattice *h, double *d_series, int64_t capacity, int64_t *record_doubles)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if ((d_series == nullptr) != (capacity == 0) || capacity < 0)
        return fail(HSG_E_INVALID, "d_series and capacity must both be set (capacity > 0) or both be 0");
    if (capacity > 0x7FFFFFFFll) return fail(HSG_E_SIZE, "capacity = %lld exceeds 2^31 - 1", (long long)capacity);
    h->series = d_series;
    h->series_cap = capacity;
    h->series_rec = series_record(h);
    h->series_t0 = h->t;
    drop_graphs(h);
    if (record_doubles) *record_doubles = h->series_rec;
    return HSG_OK;
}

hsg_status hsg_get_series_count(const hsg_lattice *h, int64_t *n_records)
{
    if (h == nullptr || n_records == nullptr) return fail(HSG_E_INVALID, "handle and n_records are required");
    int64_t n = 0;
    if (h->series != nullptr && h->t > h->series_t0)
        n = (int64_t)std::min<uint64_t>(h->t - h->series_t0, (uint64_t)h->series_cap);
    *n_records = n;
    return HSG_OK;
}

hsg_status hsg_get_spins(const hsg_lattice *h, float *d_spins, hsg_stream_t stream)
{
    if (h == nullptr || d_spins == nullptr) return fail(HSG_E_INVALID, "handle and d_spins are required");
    for (const Group &g : h->lay.g) {
        hsg::PackArgs a = pack_args(h, g);
        a.spins_can = d_spins + g.can_spin0;
        const hipError_t e = hsg::launch_unpack_spins(a, h->storage, S(stream));
        if (e != hipSuccess) return hip_fail(e, "get_spins");
    }
    return HSG_OK;
}

hsg_status hsg_set_spins(hsg_lattice *h, const float *d_spins, hsg_stream_t stream)
{
    if (h == nullptr || d_spins == nullptr) return fail(HSG_E_INVALID, "handle and d_spins are required");
    for (const Group &g : h->lay.g) {
        hsg::PackArgs a = pack_args(h, g);
        a.spins_can = const_cast<float *>(d_spins) + g.can_spin0;
        const hipError_t e = hsg::launch_pack_spins(a, h->storage, S(stream));
        if (e != hipSuccess) return hip_fail(e, "set_spins");
    }
    return HSG_OK;
}

hsg_status hsg_get_temp_map(const hsg_lattice *h, int32_t *d_sat, hsg_stream_t stream)
{
    if (h == nullptr || d_sat == nullptr) return fail(HSG_E_INVALID, "handle and d_slot_at_temp are required");
    for (const Group &g : h->lay.g) {
        const hipError_t e = hipMemcpyAsync(d_sat + g.rep0, h->state + g.o_sat, (size_t)g.n_rep * 4,
                                            hipMemcpyDeviceToDevice, S(stream));
        if (e != hipSuccess) return hip_fail(e, "get_temp_map");
    }
    return HSG_OK;
}

hsg_status hsg_set_temp_map(hsg_lattice *h, const int32_t *d_sat, hsg_stream_t stream)
{
    if (h == nullptr || d_sat == nullptr) return fail(HSG_E_INVALID, "handle and d_slot_at_temp are required");
    for (const Group &g : h->lay.g) {
        int32_t *sat = reinterpret_cast<int32_t *>(h->state + g.o_sat);
        hipError_t e = hipMemcpyAsync(sat, d_sat + g.rep0, (size_t)g.n_rep * 4, hipMemcpyDeviceToDevice, S(stream));
        if (e == hipSuccess)
            e = hsg::launch_invert_maps(sat, reinterpret_cast<int32_t *>(h->state + g.o_tos), (int64_t)g.D * g.O,
                                        g.T, S(stream));
        if (e != hipSuccess) return hip_fail(e, "set_temp_map");
    }
    return HSG_OK;
}

hsg_status hsg_get_pt_accepts(const hsg_lattice *h, uint64_t *d_acc, hsg_stream_t stream)
{
    if (h == nullptr || d_acc == nullptr) return fail(HSG_E_INVALID, "handle and d_accepts are required");
    int64_t off = 0;
    for (const Group &g : h->lay.g) {
        const int64_t n = (int64_t)g.D * g.O * (g.T - 1);
        if (n > 0) {
            const hipError_t e =
                hipMemcpyAsync(d_acc + off, h->state + g.o_acc, (size_t)n * 8, hipMemcpyDeviceToDevice, S(stream));
            if (e != hipSuccess) return hip_fail(e, "get_pt_accepts");
        }
        off += n;
    }
    return HSG_OK;
}

hsg_status hsg_get_state(const hsg_lattice *h, uint64_t *sweep_counter, uint64_t *pt_calls, uint64_t *seed)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (sweep_counter) *sweep_counter = h->t;
    if (pt_calls) *pt_calls = h->pt_calls;
    if (seed) *seed = h->seed;
    return HSG_OK;
}

hsg_status hsg_set_state(hsg_lattice *h, uint64_t sweep_counter, uint64_t pt_calls, hsg_stream_t stream)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (sweep_counter > 0xFFFFFFFFull || pt_calls > 0xFFFFFFFFull)
        return fail(HSG_E_SIZE, "counters are limited to 32 bits");
    hipError_t e = hsg::launch_set_u32(reinterpret_cast<uint32_t *>(h->state), (uint32_t)sweep_counter, S(stream));
    if (e == hipSuccess)
        e = hsg::launch_set_u32(reinterpret_cast<uint32_t *>(h->state) + 1, (uint32_t)sweep_counter, S(stream));
    if (e != hipSuccess) return hip_fail(e, "set_state");
    h->t = sweep_counter;
    h->pt_calls = pt_calls;
    return HSG_OK;
}

hsg_status hsg_set_tuning(hsg_lattice *h, int32_t slots_per_item)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (slots_per_item < 0 || slots_per_item > 16 * 256)
        return fail(HSG_E_INVALID, "slots_per_item = %d", slots_per_item);
    h->slots_per_item = slots_per_item;
    drop_graphs(h);
    return HSG_OK;
}

hsg_status hsg_set_kernel(hsg_lattice *h, int32_t variant)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (variant < 0 || variant > 5) return fail(HSG_E_INVALID, "kernel variant = %d, need 0..5", variant);
    h->kernel_variant = variant;
    drop_graphs(h);
    return HSG_OK;
}

hsg_status hsg_set_overlap(hsg_lattice *h, int32_t enable)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (enable != 0 && enable != 1) return fail(HSG_E_INVALID, "overlap = %d, need 0 or 1", enable);
    h->overlap = enable == 1;
    return HSG_OK;
}

hsg_status hsg_get_tuning(const hsg_lattice *h, int32_t *variant, int32_t *slots_per_item, int32_t *overlap)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (variant) *variant = h->kernel_variant;
    if (slots_per_item) *slots_per_item = h->slots_per_item;
    if (overlap) *overlap = h->overlap ? 1 : 0;
    return HSG_OK;
}

hsg_status hsg_set_geometry(hsg_lattice *h, int32_t group, int32_t tile_y, int32_t z_slabs)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (group < 0 || group >= (int32_t)h->lay.g.size())
        return fail(HSG_E_INVALID, "group = %d, need 0..%zu", group, h->lay.g.size() - 1);
    Group &g = h->lay.g[group];
    if (!g.stream_ok) return fail(HSG_E_UNSUPPORTED, "group %d: L = %d runs no z-march (L %% 4 != 0)", group, g.L);
    if (tile_y == 0 && z_slabs == 0) {
        stream_geometry(g);
    } else {
        const std::pair<int, int> want(tile_y, z_slabs);
        const std::vector<std::pair<int, int>> gc = geometry_candidates(g);
        if (std::find(gc.begin(), gc.end(), want) == gc.end())
            return fail(HSG_E_INVALID, "group %d (L = %d): tile_y = %d, z_slabs = %d is not one of its z-march geometries",
                        group, g.L, tile_y, z_slabs);
        (void)apply_geometry(g, tile_y, z_slabs);
    }
    drop_graphs(h);
    return HSG_OK;
}

hsg_status hsg_get_geometry(const hsg_lattice *h, int32_t group, int32_t *tile_y, int32_t *z_slabs)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (group < 0 || group >= (int32_t)h->lay.g.size())
        return fail(HSG_E_INVALID, "group = %d, need 0..%zu", group, h->lay.g.size() - 1);
    const Group &g = h->lay.g[group];
    if (tile_y) *tile_y = g.stream_ok ? g.s_TY : 0;
    if (z_slabs) *z_slabs = g.stream_ok ? g.s_zslabs : 0;
    return HSG_OK;
}

hsg_status hsg_set_math(hsg_lattice *h, int32_t mode)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (mode != 0 && mode != 1) return fail(HSG_E_INVALID, "math mode = %d, need 0 or 1", mode);
    h->hw_math = mode == 1;
    drop_graphs(h);
    return HSG_OK;
}

hsg_status hsg_autotune(hsg_lattice *h, int32_t n_sweeps, void *d_backup, int32_t *variant_out,
                        int32_t *slots_out, hsg_stream_t stream)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (n_sweeps < 1 || n_sweeps > 1000) return fail(HSG_E_INVALID, "n_sweeps = %d, need 1..1000", n_sweeps);
    if (d_backup != nullptr && (reinterpret_cast<uintptr_t>(d_backup) % kAlign) != 0)
        return fail(HSG_E_INVALID, "backup buffer must be %d-byte aligned", (int)kAlign);
    const uint64_t need = (uint64_t)n_sweeps + kGraphSweeps + 2;  // trial sweeps per candidate and round
    struct Cand {
        int32_t variant, slots;
        bool overlap;
    };
    bool any_stream = false, any_pair = false, any_gather = false;
    int max_spp = 1;
    for (const Group &g : h->lay.g) {
        any_stream = any_stream || g.stream_ok;
        any_pair = any_pair || (g.stream_ok && g.s_TY == g.L);
        any_gather = any_gather || !g.stream_ok;
        max_spp = std::max(max_spp, g.O * g.T);
    }
    std::vector<int32_t> slot_opts;  // slots per work item of the gather kernel, distinct after clamping
    for (int c : {2, 4, 8, 16}) {
        const int v = std::min(c, max_spp);
        if (std::find(slot_opts.begin(), slot_opts.end(), v) == slot_opts.end()) slot_opts.push_back(v);
    }
    std::vector<Cand> cands;
    auto add = [&](int32_t v, bool gather_used) {
        if (gather_used)
            for (int32_t c : slot_opts) cands.push_back({v, c, false});
        else
            cands.push_back({v, 0, false});
        if (any_stream) cands.push_back({v, gather_used ? slot_opts.back() : 0, true});
    };
    {
        const int32_t v0 = h->kernel_variant;
        h->kernel_variant = 5;
        const bool resident = use_resident(h);
        h->kernel_variant = v0;
        if (resident) cands.push_back({5, 0, false});
    }
    if (any_pair) {
        const int32_t v0 = h->kernel_variant;
        h->kernel_variant = 4;
        bool any_quad = false;
        for (const Group &g : h->lay.g) any_quad = any_quad || use_quad(h, g);
        h->kernel_variant = v0;
        if (any_quad && h->n_or >= 2) add(4, any_gather);
        add(3, any_gather);
    }
    if (any_stream) add(2, any_gather);
    add(1, true);
    constexpr int kRounds = 2;  // every candidate is timed once per round; its best time counts
    if (h->t + need * cands.size() * kRounds > 0x100000000ull)
        return fail(HSG_E_SIZE, "the trial sweeps would pass the sweep counter limit 2^32");

    hipStream_t s = S(stream);
    const uint64_t t0 = h->t, pt0 = h->pt_calls, n_stats0 = h->n_stats;
    const bool have_e0 = h->have_energies;
    const int32_t var0 = h->kernel_variant, slots0 = h->slots_per_item;
    const bool ov0 = h->overlap;
    hipError_t e = hipSuccess;
    if (d_backup != nullptr)
        e = hipMemcpyAsync(d_backup, h->state, h->lay.sz.state_bytes, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "autotune: saving the state");
    hipEvent_t ev[2] = {nullptr, nullptr};
    for (auto &x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    hsg_status st = e == hipSuccess ? HSG_OK : hip_fail(e, "autotune: event");
    std::vector<float> best(cands.size(), -1.0f);  // -1: not timed (a choice that does not apply)
    for (size_t q = 0; q < kRounds * cands.size() && st == HSG_OK; ++q) {
        const size_t k = q % cands.size();
        h->kernel_variant = cands[k].variant;
        h->slots_per_item = cands[k].slots;
        h->overlap = cands[k].overlap;
        if (h->overlap && !overlap_ok(h)) continue;  // this choice would run as the one without overlap
        drop_graphs(h);
        // warm-up: captures and launches both sweep graphs (kGraphSweeps sweeps,
        // then one sweep, twice), since a fresh graph's first launch is slower
        // than the later ones
        st = hsg_sweep(h, kGraphSweeps + 2, stream);
        if (st != HSG_OK) break;
        e = hipEventRecord(ev[0], s);
        if (e == hipSuccess) st = hsg_sweep(h, n_sweeps, stream);
        if (st != HSG_OK) break;
        if (e == hipSuccess) e = hipEventRecord(ev[1], s);
        if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (e != hipSuccess) {
            st = hip_fail(e, "autotune: timing");
            break;
        }
        if (best[k] < 0.0f || ms < best[k]) best[k] = ms;
    }
    // The candidates come in order of preference (the default first); a later
    // one is taken only when it is at least 1 % faster, more than the trial
    // timings resolve.
    Cand pick{var0, slots0, ov0};
    float best_ms = -1.0f;
    for (size_t k = 0; k < cands.size(); ++k)
        if (best[k] >= 0.0f && (best_ms < 0.0f || best[k] < 0.99f * best_ms)) {
            best_ms = best[k];
            pick = cands[k];
        }
    h->kernel_variant = st == HSG_OK ? pick.variant : var0;
    h->slots_per_item = st == HSG_OK ? pick.slots : slots0;
    h->overlap = st == HSG_OK ? pick.overlap : ov0;
    // Second stage, with that choice in force: the z-march geometry (row-band
    // height and z-slabs) of each lattice size that runs single passes, one
    // size after the other, the current geometry first and kept unless another
    // is at least 1 % faster.
    std::vector<std::pair<int, int>> geo0;
    for (const Group &g : h->lay.g) geo0.emplace_back(g.s_TY, g.s_zslabs);
    for (size_t gi = 0; gi < h->lay.g.size() && st == HSG_OK; ++gi) {
        Group &g = h->lay.g[gi];
        if (!use_stream(h, g) || use_pair(h, g)) continue;
        std::vector<std::pair<int, int>> gc = geometry_candidates(g);
        const std::pair<int, int> cur(g.s_TY, g.s_zslabs);
        gc.erase(std::remove(gc.begin(), gc.end(), cur), gc.end());
        gc.insert(gc.begin(), cur);
        if (gc.size() < 2) continue;
        if (h->t + need * gc.size() * kRounds > 0x100000000ull) break;  // no room left in the counter map
        std::vector<float> gbest(gc.size(), -1.0f);
        for (size_t q = 0; q < kRounds * gc.size() && st == HSG_OK; ++q) {
            const size_t k = q % gc.size();
            (void)apply_geometry(g, gc[k].first, gc[k].second);
            drop_graphs(h);
            st = hsg_sweep(h, kGraphSweeps + 2, stream);
            if (st != HSG_OK) break;
            e = hipEventRecord(ev[0], s);
            if (e == hipSuccess) st = hsg_sweep(h, n_sweeps, stream);
            if (st != HSG_OK) break;
            if (e == hipSuccess) e = hipEventRecord(ev[1], s);
            if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
            if (e != hipSuccess) {
                st = hip_fail(e, "autotune: timing");
                break;
            }
            if (gbest[k] < 0.0f || ms < gbest[k]) gbest[k] = ms;
        }
        size_t kb = 0;
        for (size_t k = 1; k < gc.size(); ++k)
            if (gbest[k] >= 0.0f && gbest[k] < 0.99f * gbest[kb]) kb = k;
        (void)apply_geometry(g, gc[kb].first, gc[kb].second);
    }
    if (st != HSG_OK) {  // on error the previous tuning is kept
        h->kernel_variant = var0;
        h->slots_per_item = slots0;
        h->overlap = ov0;
        for (size_t gi = 0; gi < h->lay.g.size(); ++gi)
            (void)apply_geometry(h->lay.g[gi], geo0[gi].first, geo0[gi].second);
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    drop_graphs(h);
    if (d_backup != nullptr) {
        e = hipMemcpyAsync(h->state, d_backup, h->lay.sz.state_bytes, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess && st == HSG_OK) st = hip_fail(e, "autotune: restoring the state");
        h->t = t0;
        h->pt_calls = pt0;
        h->n_stats = n_stats0;
        h->have_energies = have_e0;
    }
    if (st != HSG_OK) return st;
    if (variant_out) *variant_out = h->kernel_variant;
    if (slots_out) *slots_out = h->slots_per_item;
    return HSG_OK;
}

hsg_status hsg_set_chain(hsg_lattice *h, int32_t chain, int32_t tile_x, int32_t tile_y, int32_t tile_z,
                         int32_t n_hit)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (chain != 0 && chain != 1) return fail(HSG_E_INVALID, "chain = %d, need 0 or 1", chain);
    if (chain == 0) {
        h->chain = 0;
        drop_graphs(h);
        return HSG_OK;
    }
    if (tile_x < 0 || tile_y < 0 || tile_z < 0) return fail(HSG_E_INVALID, "tile edges must be >= 0");
    if (n_hit < 1 || n_hit * h->n_hb > 16)
        return fail(HSG_E_INVALID, "n_hit = %d: need n_hit >= 1 and n_hit * n_hb <= 16", n_hit);
    std::vector<Group> gs = h->lay.g;
    for (size_t k = 0; k < gs.size(); ++k) {
        Group &g = gs[k];
        const int L = g.L;
        if (L % 4 != 0) return fail(HSG_E_UNSUPPORTED, "group %zu: the tile chain needs L %% 4 == 0 (L = %d)", k, L);
        const int tx = tile_x == 0 ? L : tile_x, ty = tile_y == 0 ? L : tile_y, tz = tile_z == 0 ? L : tile_z;
        if (tx > L || ty > L || tz > L || L % tx != 0 || L % ty != 0 || L % tz != 0)
            return fail(HSG_E_INVALID, "group %zu: tile edges %d, %d, %d must divide L = %d", k, tx, ty, tz, L);
        if (tx % 4 != 0)
            return fail(HSG_E_INVALID, "group %zu: the tile edge along x (%d) must be a multiple of 4", k, tx);
        const int bx = L / tx, by = L / ty, bz = L / tz;
        if ((bx != 1 && (bx & 1)) || (by != 1 && (by & 1)) || (bz != 1 && (bz & 1)))
            return fail(HSG_E_INVALID, "group %zu: L / tile edge must be 1 or even (L = %d, tiles %d, %d, %d)", k, L,
                        tx, ty, tz);
        g.t_TX = tx;
        g.t_TY = ty;
        g.t_TZ = tz;
        g.t_BX = bx;
        g.t_BY = by;
        g.t_BZ = bz;
        g.t_hx = bx > 1 ? 1 : 0;
        g.t_hy = by > 1 ? 1 : 0;
        g.t_hz = bz > 1 ? 1 : 0;
        g.t_RXh = tx / 2 + 4 * g.t_hx;
        g.t_RY = ty + 2 * g.t_hy;
        g.t_RZ = tz + 2 * g.t_hz;
        g.t_P = tz * ty * (tx / 4);
        const size_t per_rep = (size_t)2 * 3 * g.t_RZ * g.t_RY * g.t_RXh * sizeof(float);
        if (g.t_P > 1024 || per_rep > 64 * 1024)
            return fail(HSG_E_UNSUPPORTED, "group %zu: tile %d x %d x %d is too large for one work-group", k, tx, ty,
                        tz);
        // replicas per work-group: up to 1024 threads and 64 KiB of LDS
        int rb = std::min<int64_t>(1024 / g.t_P, (int64_t)(64 * 1024 / per_rep));
        rb = std::max(1, std::min(rb, g.O * g.T));
        g.t_RB = rb;
        g.t_chunks = (g.O * g.T + rb - 1) / rb;
        g.t_threads = (g.t_P * rb + 63) / 64 * 64;
        g.t_lds = per_rep * rb;
    }
    h->lay.g = gs;
    h->chain = 1;
    h->tile_x = tile_x;
    h->tile_y = tile_y;
    h->tile_z = tile_z;
    h->n_hit = n_hit;
    drop_graphs(h);
    return HSG_OK;
}

hsg_status hsg_set_stats(hsg_lattice *h, int32_t enable)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    h->stats = enable != 0;
    drop_graphs(h);
    return HSG_OK;
}

hsg_status hsg_reset_stats(hsg_lattice *h, hsg_stream_t stream)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    hsg_status st = run_stats(h, true, S(stream));
    if (st == HSG_OK) h->n_stats = 0;
    return st;
}

hsg_status hsg_get_stats(const hsg_lattice *h, double *d_sums, uint32_t *d_trips, uint64_t *n_sweeps,
                         hsg_stream_t stream)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    hipStream_t s = S(stream);
    for (const Group &g : h->lay.g) {
        hipError_t e = hipSuccess;
        if (d_sums)
            e = hipMemcpyAsync(d_sums + g.rep0 * 2, h->state + g.o_ssum, (size_t)g.n_rep * 16,
                               hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && d_trips)
            e = hipMemcpyAsync(d_trips + g.rep0, h->state + g.o_strips, (size_t)g.n_rep * 4,
                               hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "get_stats");
    }
    if (n_sweeps) *n_sweeps = h->n_stats;
    return HSG_OK;
}

hsg_status hsg_set_batch(hsg_lattice *h, int64_t replicas)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    if (replicas < -1) return fail(HSG_E_INVALID, "replicas per batch = %lld, need -1, 0 or > 0", (long long)replicas);
    h->batch = replicas;
    drop_graphs(h);
    return HSG_OK;
}

hsg_status hsg_set_graphs(hsg_lattice *h, int32_t enable)
{
    if (h == nullptr) return fail(HSG_E_INVALID, "handle is NULL");
    h->use_graphs = enable != 0;
    return HSG_OK;
}

hsg_status hsg_sync(hsg_lattice *h, hsg_stream_t stream)
{
    (void)h;
    hipError_t e = hipStreamSynchronize(S(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "sync");
    return HSG_OK;
}

void hsg_destroy(hsg_lattice *h)
{
    if (h == nullptr) return;
    drop_graphs(h);
    if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
    if (h->stream2) (void)hipStreamDestroy(h->stream2);
    for (auto &x : h->ev)
        if (x) (void)hipEventDestroy(x);
    delete h;
}

hsg_status hsg_debug_philox(const uint32_t *d_ctr, const uint32_t *d_key, uint32_t *d_out, int64_t n,
                            hsg_stream_t stream)
{
    if (n < 0 || (n > 0 && (d_ctr == nullptr || d_key == nullptr || d_out == nullptr)))
        return fail(HSG_E_INVALID, "bad philox arguments");
    const hipError_t e = hsg::launch_philox(d_ctr, d_key, d_out, n, S(stream));
    if (e != hipSuccess) return hip_fail(e, "philox");
    return HSG_OK;
}

hsg_status hsg_debug_hw_math(const float *d_x, float *d_out, int64_t n, hsg_stream_t stream)
{
    if (n < 0 || (n > 0 && (d_x == nullptr || d_out == nullptr))) return fail(HSG_E_INVALID, "bad arguments");
    const hipError_t e = hsg::launch_hw_math(d_x, d_out, n, S(stream));
    if (e != hipSuccess) return hip_fail(e, "hw_math");
    return HSG_OK;
}

}  // extern "C"
