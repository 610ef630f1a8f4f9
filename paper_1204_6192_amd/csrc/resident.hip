// resident.hip -- whole runs of small lattices in one launch, a sample per
// work-group, its spins held in LDS.
//
// When every replica of a disorder sample fits a work-group's LDS (the
// R_O R_T replicas of L = 8 at float32 take 96 KiB of the 160 KiB), one
// work-group can run any number of complete sweeps of that sample without
// touching HBM for spins: the heat-bath and over-relaxation half-sweeps
// (Eqs. (2), (3)), the float64 energy of Eq. (1) in the last pass, the
// tempering walk of Eq. (4) over the sample's ladders, and the run
// statistics. Samples never interact (tempering stays within a sample), so
// the work-groups need no grid-wide synchronisation: one launch is a
// persistent fused sweep + tempering run. LDS holds the spins in the same
// internal layout and storage codec as HBM ([replica][parity][plane][Nh]), read
// and written through the codec exactly as the other kernels read and write
// HBM, with the same per-site arithmetic and neighbour order: the spins and
// temperature maps equal those of the separate launches bit for bit, the
// energies to rounding (another summation order).
//
// Threads: thread (g, q) owns the site pair (2q, 2q + 1) of each parity for the
// replicas g, g + G, g + 2G, ... of the sample (G replica groups of Q = Nh / 2
// threads) and reads that pair's couplings and field (cache hits after the
// first sweep) once per half-sweep. A half-sweep is one pass over the owned
// sites and one barrier.
#include <type_traits>

#include "device.h"
#include "kernels.h"
#include "ladder.h"

namespace hsg {

// neighbours of the parity-p site with half-index j, order +x, -x, +y, -y, +z, -z
__device__ __forceinline__ void nb_of(uint32_t j, int L, int Lh, int p, uint32_t nb[6])
{
    const uint32_t r = j / (uint32_t)Lh;
    const uint32_t xh = j - r * (uint32_t)Lh;
    const uint32_t y = r % (uint32_t)L, z = r / (uint32_t)L;
    const int o = (int)((y + z + (uint32_t)p) & 1u);
    const uint32_t xp = o ? (xh + 1 == (uint32_t)Lh ? 0 : xh + 1) : xh;
    const uint32_t xm = o ? xh : (xh == 0 ? (uint32_t)Lh - 1 : xh - 1);
    const uint32_t yp = (y + 1 == (uint32_t)L) ? 0 : y + 1, ym = (y == 0) ? (uint32_t)L - 1 : y - 1;
    const uint32_t zp = (z + 1 == (uint32_t)L) ? 0 : z + 1, zm = (z == 0) ? (uint32_t)L - 1 : z - 1;
    const uint32_t row = r * (uint32_t)Lh;
    nb[0] = row + xp;
    nb[1] = row + xm;
    nb[2] = (z * (uint32_t)L + yp) * (uint32_t)Lh + xh;
    nb[3] = (z * (uint32_t)L + ym) * (uint32_t)Lh + xh;
    nb[4] = (zp * (uint32_t)L + y) * (uint32_t)Lh + xh;
    nb[5] = (zm * (uint32_t)L + y) * (uint32_t)Lh + xh;
}

template <int STORE, bool FIELD, bool HW>
__global__ __launch_bounds__(512) void k_resident_sweeps(ResidentArgs a)
{
    using C = Codec<STORE>;
    using T = typename C::T;
    extern __shared__ __align__(16) unsigned char smem[];
    // LDS: spins [R][2][kPlanes][Nh] T | energy partials [R][Q] | E [R] | sat, tos [R] int32
    const int R = a.slots_per_sample, Q = (int)(a.Nh >> 1), G = a.groups;
    const uint32_t Nh = (uint32_t)a.Nh;
    const size_t spin_bytes = ((size_t)R * 2 * C::kPlanes * Nh * sizeof(T) + 15) / 16 * 16;
    T *sp = reinterpret_cast<T *>(smem);
    double *ep = reinterpret_cast<double *>(smem + spin_bytes);
    double *E = ep + (size_t)R * Q;
    int32_t *sat = reinterpret_cast<int32_t *>(E + R);
    int32_t *tos = sat + R;

    const int d = (int)blockIdx.x;  // sample
    const int tid = (int)threadIdx.x;
    const int g = tid / Q, q = tid - g * Q;
    const bool active = g < G;
    const int64_t rep0 = (int64_t)d * R;  // first replica of the sample in the group
    const size_t per_rep = (size_t)2 * C::kPlanes * Nh;

    // the sample's spins, maps and energies into LDS (raw codes, byte for byte)
    {
        const uint32_t *src = reinterpret_cast<const uint32_t *>((const T *)a.spins + rep0 * per_rep);
        uint32_t *dst = reinterpret_cast<uint32_t *>(sp);
        const size_t words = (size_t)R * per_rep * sizeof(T) / 4;
        for (size_t w = tid; w < words; w += blockDim.x) dst[w] = src[w];
        for (int r = tid; r < R; r += blockDim.x) {
            sat[r] = a.slot_at_temp[rep0 + r];
            tos[r] = a.temp_of_slot[rep0 + r];
            E[r] = a.E[rep0 + r];
        }
    }
    const uint32_t t0 = *a.tptr;
    const uint32_t uid = a.uid_base + (uint32_t)d;
    __syncthreads();

    // one half-sweep of parity P; KIND 0 heat bath (repetition rep), 1 over-relaxation;
    // with ENERGY, every replica's float64 energy goes to E
    auto half = [&](auto kc, auto pc, auto ec, uint32_t rep, uint32_t t) __attribute__((always_inline)) {
        constexpr int kind = decltype(kc)::value, p = decltype(pc)::value;
        constexpr bool energy = decltype(ec)::value;
        if (active) {
            // the neighbour indices are recomputed for every half-sweep: an empty
            // asm statement hides that they never change, which keeps the
            // compiler from holding those of all eight half-sweep forms in
            // registers across the whole launch
            uint32_t qq = (uint32_t)q;
            asm volatile("" : "+v"(qq));
            uint32_t nb[2][6];
            nb_of(2 * qq, a.L, a.Lh, p, nb[0]);
            nb_of(2 * qq + 1, a.L, a.Lh, p, nb[1]);
            // my pair's couplings and field of this parity (and the other
            // parity's field for the energy), from the cache every half-sweep
            float Jc[2][6];
            v3 Hs[2] = {v3{0.f, 0.f, 0.f}, v3{0.f, 0.f, 0.f}}, He[2] = {v3{0.f, 0.f, 0.f}, v3{0.f, 0.f, 0.f}};
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const uint32_t j = 2 * qq + k;
                const float *Jb = a.J6 + ((int64_t)d * 2 + p) * 6 * (int64_t)Nh;
#pragma unroll
                for (int n = 0; n < 6; ++n) Jc[k][n] = Jb[(int64_t)n * Nh + j];
                if constexpr (FIELD) {
                    const float *Hb = a.Hp + ((int64_t)d * 2 + p) * 3 * (int64_t)Nh;
                    Hs[k] = v3{Hb[j], Hb[Nh + j], Hb[2 * Nh + j]};
                    if constexpr (energy) {
                        const float *Ho = a.Hp + ((int64_t)d * 2 + (1 - p)) * 3 * (int64_t)Nh;
                        He[k] = v3{Ho[j], Ho[Nh + j], Ho[2 * Nh + j]};
                    }
                }
            }
#pragma unroll 1
            for (int sis = g; sis < R; sis += G) {
                T *base = sp + (size_t)sis * per_rep;
                T *own = base + (size_t)p * C::kPlanes * Nh;
                const T *oth = base + (size_t)(1 - p) * C::kPlanes * Nh;
                const float beta = a.beta32[tos[sis]];
                u32x4 r{0u, 0u, 0u, 0u};
                if constexpr (kind == 0) {
                    const int o = sis / a.T, ts = sis - o * a.T;
                    const uint32_t c2 = (uint32_t)ts | ((uint32_t)o << 8) | (rep << 12) | ((uint32_t)p << 16);
                    r = philox4x32_10(u32x4{(uint32_t)q, t, c2, uid}, a.key0, a.key1);
                }
                double e = 0.0;
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const uint32_t j = 2 * (uint32_t)q + k;
                    v3 h = Hs[k];
                    double hx = Hs[k].x, hy = Hs[k].y, hz = Hs[k].z;
#pragma unroll
                    for (int n = 0; n < 6; ++n) {
                        const v3 sn = C::load(oth, Nh, nb[k][n]);
                        acc3(h, Jc[k][n], sn);
                        if constexpr (energy) {
                            hx = fma((double)Jc[k][n], (double)sn.x, hx);
                            hy = fma((double)Jc[k][n], (double)sn.y, hy);
                            hz = fma((double)Jc[k][n], (double)sn.z, hz);
                        }
                    }
                    v3 s1;
                    if constexpr (kind == 0) s1 = heat_bath<HW, STORE == 0>(h, beta, k ? r.z : r.x, k ? r.w : r.y);
                    else s1 = over_relax<STORE == 0>(C::load(own, Nh, j), h);
                    C::store(own, Nh, j, s1);
                    if constexpr (energy) {
                        // each bond has exactly one endpoint on this (odd) parity
                        const v3 sv = C::stored_value(s1);
                        e -= (double)sv.x * hx + (double)sv.y * hy + (double)sv.z * hz;
                        if (FIELD) {  // the field on the even site at the same half-index
                            const v3 so = C::load(oth, Nh, j);
                            e -= (double)He[k].x * so.x + (double)He[k].y * so.y + (double)He[k].z * so.z;
                        }
                    }
                }
                if constexpr (energy) ep[(size_t)sis * Q + q] = e;
            }
        }
        __syncthreads();
        if constexpr (energy) {
            for (int rr = tid; rr < R; rr += blockDim.x) {  // fixed order over the pairs
                double s = 0.0;
                for (int k = 0; k < Q; ++k) s += ep[(size_t)rr * Q + k];
                E[rr] = s;
            }
            __syncthreads();
        }
    };

    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using NoE = std::false_type;
    using WithE = std::true_type;
#pragma unroll 1
    for (int i = 0; i < a.n_sweeps; ++i) {
        const uint32_t t = t0 + (uint32_t)i;
#pragma unroll 1
        for (int r = 0; r < a.n_hb; ++r) {
            half(I0{}, I0{}, NoE{}, (uint32_t)r, t);
            if (a.n_or == 0 && r == a.n_hb - 1) half(I0{}, I1{}, WithE{}, (uint32_t)r, t);
            else half(I0{}, I1{}, NoE{}, (uint32_t)r, t);
        }
#pragma unroll 1
        for (int r = 0; r < a.n_or; ++r) {
            half(I1{}, I0{}, NoE{}, 0u, t);
            if (r == a.n_or - 1) half(I1{}, I1{}, WithE{}, 0u, t);
            else half(I1{}, I1{}, NoE{}, 0u, t);
        }
        if (a.pt_every > 0 && ((uint64_t)t + 1) % (uint64_t)a.pt_every == 0) {
            PtArgs pa{};
            pa.slot_at_temp = sat;
            pa.temp_of_slot = tos;
            pa.E = E;
            pa.beta64 = a.beta64;
            pa.accepts = a.accepts + (int64_t)d * a.O * (a.T > 1 ? a.T - 1 : 1);
            pa.D = 1;
            pa.O = a.O;
            pa.T = a.T;
            pa.purpose = 1;
            pa.key0 = a.key0;
            pa.key1 = a.key1;
            pa.uid_base = uid;
            if (a.T > 1)
                for (int lad = tid; lad < a.O; lad += blockDim.x) pt_ladder(pa, lad, t);
            __syncthreads();
        }
        if (a.stats) {
            StatsArgs st{};
            st.slot_at_temp = sat;
            st.E = E;
            st.sum = a.stat_sum + rep0 * 2;
            st.flag = a.stat_flag + rep0;
            st.trips = a.stat_trips + rep0;
            st.D = 1;
            st.O = a.O;
            st.T = a.T;
            for (int lad = tid; lad < a.O; lad += blockDim.x) stats_ladder(st, lad);
            __syncthreads();
        }
    }

    // back to HBM
    {
        uint32_t *dst = reinterpret_cast<uint32_t *>((T *)a.spins + rep0 * per_rep);
        const uint32_t *src = reinterpret_cast<const uint32_t *>(sp);
        const size_t words = (size_t)R * per_rep * sizeof(T) / 4;
        for (size_t w = tid; w < words; w += blockDim.x) dst[w] = src[w];
        for (int r = tid; r < R; r += blockDim.x) {
            a.slot_at_temp[rep0 + r] = sat[r];
            a.temp_of_slot[rep0 + r] = tos[r];
            a.E[rep0 + r] = E[r];
        }
    }
}

template <int STORE>
static size_t resident_lds_bytes_s(int64_t Nh, int32_t slots_per_sample)
{
    using C = Codec<STORE>;
    const size_t R = (size_t)slots_per_sample;
    const size_t spin = (R * 2 * C::kPlanes * (size_t)Nh * sizeof(typename C::T) + 15) / 16 * 16;
    return spin + R * (size_t)(Nh / 2) * 8 + R * 8 + 2 * R * 4;
}

size_t resident_lds_bytes(int storage, int64_t Nh, int32_t slots_per_sample)
{
    switch (storage) {
    case 0: return resident_lds_bytes_s<0>(Nh, slots_per_sample);
    case 1: return resident_lds_bytes_s<1>(Nh, slots_per_sample);
    case 2: return resident_lds_bytes_s<2>(Nh, slots_per_sample);
    default: return resident_lds_bytes_s<3>(Nh, slots_per_sample);
    }
}

template <int STORE>
static hipError_t launch_resident_s(const ResidentArgs &a, bool field, bool hw, unsigned threads, size_t lds,
                                    hipStream_t s)
{
    const dim3 grid((unsigned)a.D), block(threads);
#define HSG_R(F, H) hipLaunchKernelGGL((k_resident_sweeps<STORE, F, H>), grid, block, lds, s, a)
    if (field) {
        if (hw) HSG_R(true, true); else HSG_R(true, false);
    } else {
        if (hw) HSG_R(false, true); else HSG_R(false, false);
    }
#undef HSG_R
    return hipGetLastError();
}

hipError_t launch_resident(const ResidentArgs &a, int storage, bool field, bool hw, unsigned threads, size_t lds,
                           hipStream_t s)
{
    if (a.D < 1 || a.n_sweeps < 1 || threads == 0 || threads > 1024 || a.groups < 1 ||
        (int64_t)a.groups * (a.Nh / 2) > (int64_t)threads)
        return hipErrorInvalidValue;
    switch (storage) {
    case 0: return launch_resident_s<0>(a, field, hw, threads, lds, s);
    case 1: return launch_resident_s<1>(a, field, hw, threads, lds, s);
    case 2: return launch_resident_s<2>(a, field, hw, threads, lds, s);
    case 3: return launch_resident_s<3>(a, field, hw, threads, lds, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hsg
