// kernels.hip -- device kernels of libhsg.so (gfx950).
//
// Checkerboard half-sweeps (Sec. 3.1; Eqs. (2) and (3)) over the parity-split
// structure-of-arrays layout, with the couplings of a sample held in registers
// while a work item walks several replicas of that sample (the J/H recycling
// of Sec. 3.3); the exact float64 energy of Eq. (1) fused into the last pass;
// the tempering walk of Eq. (4); energy and overlap (Eq. (5)) reductions; and
// layout conversion between the canonical and internal arrays.
#include "device.h"
#include "kernels.h"
#include "ladder.h"

namespace hsg {

// ---------------------------------------------------------------- geometry
struct Site {
    int32_t x, y, z;
};

// Neighbours (in the other parity's half-index space) of the parity-p site
// with half-index j, in the order +x, -x, +y, -y, +z, -z.
__device__ __forceinline__ void neighbours(int64_t j, int32_t L, int32_t Lh, int p, int64_t nb[6])
{
    const int32_t r = (int32_t)(j / Lh);
    const int32_t xh = (int32_t)(j - (int64_t)r * Lh);
    const int32_t y = r % L, z = r / L;
    const int o = (y + z + p) & 1;  // x = 2 xh + o
    const int32_t xp = o ? (xh + 1 == Lh ? 0 : xh + 1) : xh;
    const int32_t xm = o ? xh : (xh == 0 ? Lh - 1 : xh - 1);
    const int32_t yp = (y + 1 == L) ? 0 : y + 1, ym = (y == 0) ? L - 1 : y - 1;
    const int32_t zp = (z + 1 == L) ? 0 : z + 1, zm = (z == 0) ? L - 1 : z - 1;
    const int64_t row = (int64_t)r * Lh;
    nb[0] = row + xp;
    nb[1] = row + xm;
    nb[2] = ((int64_t)z * L + yp) * Lh + xh;
    nb[3] = ((int64_t)z * L + ym) * Lh + xh;
    nb[4] = ((int64_t)zp * L + y) * Lh + xh;
    nb[5] = ((int64_t)zm * L + y) * Lh + xh;
}

// ---------------------------------------------------------------- half-sweep
// One thread owns the two parity-p sites with half-indices 2q and 2q + 1 (they
// share Philox block q) and walks `chunk` replicas of one sample, keeping the
// sample's couplings and field in registers. Grid: samples x replica chunks x
// blocks of 256 site pairs, remapped so each XCD gets contiguous work.
template <int STORE, int KIND, bool FIELD, bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_half_sweep(SweepArgs a)
{
    using C = Codec<STORE>;
    using T = typename C::T;
    __shared__ double red[4];

    const int lb = xcd_remap((int)blockIdx.x, a.n_blocks);
    const int pb = lb % a.n_pb;
    const int rest = lb / a.n_pb;
    const int ch = rest % a.n_chunks;
    const int d = rest / a.n_chunks;
    const int64_t Nh = a.Nh;
    const int64_t q = (int64_t)pb * kBlock + threadIdx.x;
    const bool active = q < (Nh >> 1);
    const int p = (int)a.parity;

    int64_t nb[2][6];
    float Jc[2][6];
    v3 Hs[2] = {v3{0.f, 0.f, 0.f}, v3{0.f, 0.f, 0.f}};
    v3 He[2] = {v3{0.f, 0.f, 0.f}, v3{0.f, 0.f, 0.f}};
    if (active) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int64_t j = 2 * q + k;
            neighbours(j, a.L, a.Lh, p, nb[k]);
            const float *Jb = a.J6 + ((int64_t)d * 2 + p) * 6 * Nh;
#pragma unroll
            for (int n = 0; n < 6; ++n) Jc[k][n] = Jb[n * Nh + j];
            if (FIELD) {
                const float *Hb = a.Hp + ((int64_t)d * 2 + p) * 3 * Nh;
                Hs[k] = v3{Hb[j], Hb[Nh + j], Hb[2 * Nh + j]};
                if (ENERGY) {  // the field on the other parity at the same half-index
                    const float *Ho = a.Hp + ((int64_t)d * 2 + (1 - p)) * 3 * Nh;
                    He[k] = v3{Ho[j], Ho[Nh + j], Ho[2 * Nh + j]};
                }
            }
        }
    }

    T *spins = (T *)a.spins;
    const uint32_t tsweep = *a.tptr;
    for (int cs = 0; cs < a.chunk; ++cs) {
        const int sis = ch * a.chunk + cs;  // replica index inside the sample: o * T + slot
        if (sis >= a.slots_per_sample) break;
        const int64_t rep = (int64_t)d * a.slots_per_sample + sis;
        double e = 0.0;
        if (active) {
            const float beta = a.beta32[a.temp_of_slot[rep]];
            T *base = spins + rep * 2 * C::kPlanes * Nh;
            T *own = base + (int64_t)p * C::kPlanes * Nh;
            const T *oth = base + (int64_t)(1 - p) * C::kPlanes * Nh;
            u32x4 r{0u, 0u, 0u, 0u};
            if (KIND != 1) {
                const int o = sis / a.T, ts = sis - o * a.T;
                const uint32_t c2 = (uint32_t)ts | ((uint32_t)o << 8) | (a.rep << 12) | ((uint32_t)p << 16);
                r = philox4x32_10(u32x4{(uint32_t)q, tsweep, c2, a.uid_base + (uint32_t)d}, a.key0, a.key1);
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int64_t j = 2 * q + k;
                v3 h = Hs[k];
                double hx = Hs[k].x, hy = Hs[k].y, hz = Hs[k].z;
#pragma unroll
                for (int n = 0; n < 6; ++n) {
                    const v3 sn = C::load(oth, Nh, nb[k][n]);
                    acc3(h, Jc[k][n], sn);
                    if (ENERGY) {
                        hx = fma((double)Jc[k][n], (double)sn.x, hx);
                        hy = fma((double)Jc[k][n], (double)sn.y, hy);
                        hz = fma((double)Jc[k][n], (double)sn.z, hz);
                    }
                }
                v3 s1;
                if (KIND != 1)
                    s1 = heat_bath<KIND == 2, STORE == 0>(h, beta, k ? r.z : r.x, k ? r.w : r.y);
                else
                    s1 = over_relax<STORE == 0>(C::load(own, Nh, j), h);
                C::store(own, Nh, j, s1);
                if (ENERGY) {
                    // each bond has exactly one endpoint on this parity (the odd one)
                    const v3 sv = C::stored_value(s1);
                    e -= (double)sv.x * hx + (double)sv.y * hy + (double)sv.z * hz;
                    if (FIELD) {
                        const v3 so = C::load(oth, Nh, j);
                        e -= (double)He[k].x * so.x + (double)He[k].y * so.y + (double)He[k].z * so.z;
                    }
                }
            }
        }
        if (ENERGY) {
            const double tot = block_sum(e, red);
            if (threadIdx.x == 0) a.e_partials[rep * a.n_pb + pb] = tot;
        }
    }
}

template <int STORE>
static hipError_t launch_half_sweep_s(const SweepArgs &a, int kind, bool field, bool energy, hipStream_t s)
{
    const dim3 grid((unsigned)a.n_blocks), block(kBlock);
#define HSG_L(K, F, E) hipLaunchKernelGGL((k_half_sweep<STORE, K, F, E>), grid, block, 0, s, a)
    if (kind == 0) {
        if (field) { if (energy) HSG_L(0, true, true); else HSG_L(0, true, false); }
        else { if (energy) HSG_L(0, false, true); else HSG_L(0, false, false); }
    } else if (kind == 2) {
        if (field) { if (energy) HSG_L(2, true, true); else HSG_L(2, true, false); }
        else { if (energy) HSG_L(2, false, true); else HSG_L(2, false, false); }
    } else {
        if (field) { if (energy) HSG_L(1, true, true); else HSG_L(1, true, false); }
        else { if (energy) HSG_L(1, false, true); else HSG_L(1, false, false); }
    }
#undef HSG_L
    return hipGetLastError();
}

hipError_t launch_half_sweep(const SweepArgs &a, int storage, int kind, bool field, bool energy, hipStream_t s)
{
    switch (storage) {
    case 0: return launch_half_sweep_s<0>(a, kind, field, energy, s);
    case 1: return launch_half_sweep_s<1>(a, kind, field, energy, s);
    case 2: return launch_half_sweep_s<2>(a, kind, field, energy, s);
    case 3: return launch_half_sweep_s<3>(a, kind, field, energy, s);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------- partial sums
// One wave per replica; lane l adds partials l, l + 64, ... in order, then a
// fixed butterfly: the result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_reduce_partials(const double *partials, int n_pb, int64_t n_rep, double *E)
{
    const int64_t rep = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    double v = 0.0;
    if (rep < n_rep)
        for (int i = lane; i < n_pb; i += 64) v += partials[rep * n_pb + i];
    v = wave_sum(v);
    if (rep < n_rep && lane == 0) E[rep] = v;
}

hipError_t launch_reduce_partials(const double *partials, int n_pb, int64_t n_rep, double *E, hipStream_t s)
{
    const unsigned blocks = (unsigned)((n_rep + 3) / 4);
    hipLaunchKernelGGL(k_reduce_partials, dim3(blocks), dim3(256), 0, s, partials, n_pb, n_rep, E);
    return hipGetLastError();
}

// ---------------------------------------------------------------- tempering
// One thread per (sample, copy) ladder (pt_ladder in ladder.h).
__global__ __launch_bounds__(64) void k_pt(PtArgs a)
{
    const int64_t lad = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lad >= (int64_t)a.D * a.O) return;
    pt_ladder(a, lad, a.tptr ? *a.tptr : a.ctr1);
}

hipError_t launch_pt(const PtArgs &a, hipStream_t s)
{
    const int64_t n = (int64_t)a.D * a.O;
    if (a.T < 2 || n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pt, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- run statistics
// One thread per ladder (stats_ladder in ladder.h).
__global__ __launch_bounds__(64) void k_stats(StatsArgs a)
{
    const int64_t lad = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lad >= (int64_t)a.D * a.O) return;
    stats_ladder(a, lad);
}

__global__ __launch_bounds__(256) void k_stats_clear(StatsArgs a)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)a.D * a.O * a.T;
    if (g >= n) return;
    a.sum[2 * g] = 0.0;
    a.sum[2 * g + 1] = 0.0;
    a.flag[g] = 0;
    a.trips[g] = 0u;
}

hipError_t launch_stats(const StatsArgs &a, bool clear, hipStream_t s)
{
    const int64_t n = (int64_t)a.D * a.O;
    if (n == 0) return hipSuccess;
    if (clear)
        hipLaunchKernelGGL(k_stats_clear, dim3((unsigned)((n * a.T + 255) / 256)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_stats, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- layouts
__device__ __forceinline__ Site site_of(int64_t i, int32_t L)
{
    Site c;
    c.x = (int32_t)(i % L);
    const int64_t r = i / L;
    c.y = (int32_t)(r % L);
    c.z = (int32_t)(r / L);
    return c;
}

__device__ __forceinline__ int64_t index_of(int32_t x, int32_t y, int32_t z, int32_t L)
{
    x = (x + L) % L;
    y = (y + L) % L;
    z = (z + L) % L;
    return (int64_t)x + (int64_t)L * ((int64_t)y + (int64_t)L * z);
}

template <int STORE>
__global__ __launch_bounds__(256) void k_pack_spins(PackArgs a)
{
    using C = Codec<STORE>;
    const int64_t N = (int64_t)a.L * a.L * a.L, Nh = N / 2;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= a.n_rep * N) return;
    const int64_t rep = gid / N, i = gid - rep * N;
    const Site c = site_of(i, a.L);
    const int p = (c.x + c.y + c.z) & 1;
    const float *src = a.spins_can + rep * 3 * N;
    typename C::T *dst = (typename C::T *)a.spins_int + (rep * 2 + p) * C::kPlanes * Nh;
    C::store(dst, Nh, i >> 1, v3{src[i], src[N + i], src[2 * N + i]});
}

template <int STORE>
__global__ __launch_bounds__(256) void k_unpack_spins(PackArgs a)
{
    using C = Codec<STORE>;
    const int64_t N = (int64_t)a.L * a.L * a.L, Nh = N / 2;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= a.n_rep * N) return;
    const int64_t rep = gid / N, i = gid - rep * N;
    const Site c = site_of(i, a.L);
    const int p = (c.x + c.y + c.z) & 1;
    const typename C::T *src = (const typename C::T *)a.spins_int + (rep * 2 + p) * C::kPlanes * Nh;
    const v3 s = C::load(src, Nh, i >> 1);
    float *dst = a.spins_can + rep * 3 * N;
    dst[i] = s.x;
    dst[N + i] = s.y;
    dst[2 * N + i] = s.z;
}

__global__ __launch_bounds__(256) void k_pack_couplings(PackArgs a)
{
    const int64_t N = (int64_t)a.L * a.L * a.L, Nh = N / 2;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= a.D * N) return;
    const int64_t d = gid / N, i = gid - d * N;
    const Site c = site_of(i, a.L);
    const int p = (c.x + c.y + c.z) & 1;
    const int64_t j = i >> 1;
    const float *Jc = a.J_can + d * 3 * N;
    float *J6 = a.J6 + (d * 2 + p) * 6 * Nh;
    J6[0 * Nh + j] = Jc[0 * N + i];
    J6[1 * Nh + j] = Jc[0 * N + index_of(c.x - 1, c.y, c.z, a.L)];
    J6[2 * Nh + j] = Jc[1 * N + i];
    J6[3 * Nh + j] = Jc[1 * N + index_of(c.x, c.y - 1, c.z, a.L)];
    J6[4 * Nh + j] = Jc[2 * N + i];
    J6[5 * Nh + j] = Jc[2 * N + index_of(c.x, c.y, c.z - 1, a.L)];
}

__global__ __launch_bounds__(256) void k_pack_field(PackArgs a)
{
    const int64_t N = (int64_t)a.L * a.L * a.L, Nh = N / 2;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= a.D * N) return;
    const int64_t d = gid / N, i = gid - d * N;
    const Site c = site_of(i, a.L);
    const int p = (c.x + c.y + c.z) & 1;
    const int64_t j = i >> 1;
    const float *Hc = a.H_can + d * 3 * N;
    float *Hp = a.Hp + (d * 2 + p) * 3 * Nh;
    for (int m = 0; m < 3; ++m) Hp[m * Nh + j] = Hc[m * N + i];
}

// Coupling sign bits: bit n of byte [d][p][j] is set when the n-th coupling of
// the site (order +x, -x, +y, -y, +z, -z) is negative.
__global__ __launch_bounds__(256) void k_pack_jbits(const float *J_can, uint8_t *Jbits, int64_t D, int32_t L)
{
    const int64_t N = (int64_t)L * L * L, Nh = N / 2;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= D * N) return;
    const int64_t d = gid / N, i = gid - d * N;
    const int32_t x = (int32_t)(i % L), y = (int32_t)((i / L) % L), z = (int32_t)(i / ((int64_t)L * L));
    const int p = (x + y + z) & 1;
    const float *Jc = J_can + d * 3 * N;
    const int64_t xm = (int64_t)((x + L - 1) % L) + (int64_t)L * (y + (int64_t)L * z);
    const int64_t ym = (int64_t)x + (int64_t)L * (((y + L - 1) % L) + (int64_t)L * z);
    const int64_t zm = (int64_t)x + (int64_t)L * (y + (int64_t)L * ((z + L - 1) % L));
    const float j6[6] = {Jc[i], Jc[xm], Jc[N + i], Jc[N + ym], Jc[2 * N + i], Jc[2 * N + zm]};
    uint32_t b = 0;
    for (int n = 0; n < 6; ++n) b |= (j6[n] < 0.0f ? 1u : 0u) << n;
    Jbits[(d * 2 + p) * Nh + (i >> 1)] = (uint8_t)b;
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

__global__ void k_clear_i32(int32_t *flag)
{
    if (threadIdx.x == 0) *flag = 0;
}

__global__ __launch_bounds__(256) void k_check_pm1(const float *v, int64_t n, int32_t *flag)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n && v[g] != 1.0f && v[g] != -1.0f) atomicOr(flag, 1);
}

hipError_t launch_check_pm1(const float *v, int64_t n, int32_t *flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_i32, dim3(1), dim3(64), 0, s, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n == 0) return e;
    hipLaunchKernelGGL(k_check_pm1, dim3(blocks_for(n)), dim3(256), 0, s, v, n, flag);
    return hipGetLastError();
}

hipError_t launch_pack_jbits(const float *J_can, uint8_t *Jbits, int64_t D, int32_t L, hipStream_t s)
{
    const int64_t n = D * (int64_t)L * L * L;
    hipLaunchKernelGGL(k_pack_jbits, dim3(blocks_for(n)), dim3(256), 0, s, J_can, Jbits, D, L);
    return hipGetLastError();
}

hipError_t launch_pack_spins(const PackArgs &a, int storage, hipStream_t s)
{
    const int64_t n = a.n_rep * (int64_t)a.L * a.L * a.L;
    if (n == 0) return hipSuccess;
    switch (storage) {
    case 0: hipLaunchKernelGGL(k_pack_spins<0>, dim3(blocks_for(n)), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_pack_spins<1>, dim3(blocks_for(n)), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_pack_spins<2>, dim3(blocks_for(n)), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_pack_spins<3>, dim3(blocks_for(n)), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_unpack_spins(const PackArgs &a, int storage, hipStream_t s)
{
    const int64_t n = a.n_rep * (int64_t)a.L * a.L * a.L;
    if (n == 0) return hipSuccess;
    switch (storage) {
    case 0: hipLaunchKernelGGL(k_unpack_spins<0>, dim3(blocks_for(n)), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_unpack_spins<1>, dim3(blocks_for(n)), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_unpack_spins<2>, dim3(blocks_for(n)), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_unpack_spins<3>, dim3(blocks_for(n)), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pack_couplings(const PackArgs &a, hipStream_t s)
{
    const int64_t n = a.D * (int64_t)a.L * a.L * a.L;
    hipLaunchKernelGGL(k_pack_couplings, dim3(blocks_for(n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pack_field(const PackArgs &a, hipStream_t s)
{
    const int64_t n = a.D * (int64_t)a.L * a.L * a.L;
    hipLaunchKernelGGL(k_pack_field, dim3(blocks_for(n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- energy
// Exact float64 energy of Eq. (1): every bond has one even endpoint, so the sum
// over even sites of s_i . sum_n J_n s_n counts each bond once; the field term
// runs over both parities at the same half-index.
template <int STORE>
__global__ __launch_bounds__(kBlock) void k_energy(EnergyArgs a)
{
    using C = Codec<STORE>;
    using T = typename C::T;
    __shared__ double red[4];
    const int64_t rep = blockIdx.x / a.n_pb;
    const int pb = (int)(blockIdx.x - rep * a.n_pb);
    const int64_t Nh = a.Nh;
    const int64_t j = (int64_t)pb * kBlock + threadIdx.x;
    const int64_t d = rep / a.slots_per_sample;
    double e = 0.0;
    if (j < Nh) {
        const T *base = (const T *)a.spins + rep * 2 * C::kPlanes * Nh;
        int64_t nb[6];
        neighbours(j, a.L, a.Lh, 0, nb);
        const v3 s0 = C::load(base, Nh, j);
        const float *J6 = a.J6 + (d * 2 + 0) * 6 * Nh;
        for (int n = 0; n < 6; ++n) {
            const v3 sn = C::load(base + C::kPlanes * Nh, Nh, nb[n]);
            const double sd = (double)s0.x * sn.x + (double)s0.y * sn.y + (double)s0.z * sn.z;
            e -= (double)J6[n * Nh + j] * sd;
        }
        if (a.Hp != nullptr) {
            const v3 s1 = C::load(base + C::kPlanes * Nh, Nh, j);
            const float *H0 = a.Hp + (d * 2 + 0) * 3 * Nh;
            const float *H1 = a.Hp + (d * 2 + 1) * 3 * Nh;
            e -= (double)H0[j] * s0.x + (double)H0[Nh + j] * s0.y + (double)H0[2 * Nh + j] * s0.z;
            e -= (double)H1[j] * s1.x + (double)H1[Nh + j] * s1.y + (double)H1[2 * Nh + j] * s1.z;
        }
    }
    const double tot = block_sum(e, red);
    if (threadIdx.x == 0) a.partials[rep * a.n_pb + pb] = tot;
}

// The same energies as a z-march where kmode_rows(L) > 0: one work-group per
// (replica, band of TY = kmode_rows(L) rows, z-slab of L / march_slabs(L, n_rep)
// planes), the thread of row y and quarter q
// holding the sites x = 4q .. 4q + 3 of plane z as z advances (planes z and
// z + 1 in registers, the next one loaded a step ahead), plane z staged in LDS
// with the row above the band. Every bond is counted once, as the +x, +y and +z
// bonds of each site: s(i) . s(i + a) in float64 from float32 components (exact
// products), times its coupling, as in k_energy; every spin is read once
// instead of seven times. The sums run in another order than k_energy's, so
// the two agree to float64 rounding. A work-group's sum goes to the partial of
// its band and slab.
template <int STORE>
__global__ __launch_bounds__(kBlock) void k_energy_stream(EnergyArgs a)
{
    using C = Codec<STORE>;
    using T = typename C::T;
    // [2 buffers][3 components][TY + 1 rows][L]: rows 0 .. TY - 1 the band,
    // row TY the row above it
    extern __shared__ __align__(16) float plane[];
    __shared__ double red[4];
    const int L = a.L, Lh = L >> 1, Q = L >> 2;
    const int TY = kmode_rows(L), n_bands = L / TY, RL = (TY + 1) * L;
    const int S = march_slabs(L, a.n_rep), Z = L / S;
    const int64_t rep = blockIdx.x / (n_bands * S);
    const int pb = (int)(blockIdx.x - rep * n_bands * S);  // band * S + slab
    const int band = pb / S, y0 = band * TY, z0 = (pb - band * S) * Z;
    const int64_t Nh = a.Nh;
    const int64_t d = rep / a.slots_per_sample;
    const T *base = (const T *)a.spins + rep * 2 * C::kPlanes * Nh;
    const float *J6 = a.J6 + d * 2 * 6 * Nh;
    const float *H = a.Hp != nullptr ? a.Hp + d * 2 * 3 * Nh : nullptr;
    const int tid = threadIdx.x;
    const bool active = tid < TY * Q;
    const int ly = active ? tid / Q : 0, x0 = active ? 4 * (tid - (tid / Q) * Q) : 0;
    const int y = y0 + ly;
    const int xp = x0 + 4 == L ? 0 : x0 + 4;
    // threads 0 .. Q - 1 stage the row above the band (LDS row TY)
    const bool halo = tid < Q;
    const int hy = y0 + TY == L ? 0 : y0 + TY, hx0 = halo ? 4 * tid : 0;
    // the four sites x .. x + 3 of row yy of plane zz: x and x + 2 on the parity
    // of yy + zz (half-indices x / 2, x / 2 + 1), x + 1 and x + 3 on the other
    auto load4 = [&](int zz, int yy, int xx, typename C::R &e, typename C::R &f) {
        const int p0 = (yy + zz) & 1;
        const uint32_t jj = (uint32_t)((zz * L + yy) * Lh + (xx >> 1));
        C::load_raw_pair(base + (int64_t)p0 * C::kPlanes * Nh, (uint32_t)Nh, jj, e);
        C::load_raw_pair(base + (int64_t)(1 - p0) * C::kPlanes * Nh, (uint32_t)Nh, jj, f);
    };
    auto decode4 = [&](const typename C::R &e, const typename C::R &f, v3 (&s)[4]) {
        C::decode_pair(e, s[0], s[2]);
        C::decode_pair(f, s[1], s[3]);
    };
    auto lp = [&](int b, int m) { return plane + (b * 3 + m) * RL; };
    auto put4 = [&](int b, int row, int xx, const v3 (&v)[4]) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const float4 q = m == 0 ? make_float4(v[0].x, v[1].x, v[2].x, v[3].x)
                           : m == 1 ? make_float4(v[0].y, v[1].y, v[2].y, v[3].y)
                                    : make_float4(v[0].z, v[1].z, v[2].z, v[3].z);
            *reinterpret_cast<float4 *>(lp(b, m) + row * L + xx) = q;
        }
    };
    auto bond = [](v3 s, v3 t) {
        return (double)s.x * t.x + (double)s.y * t.y + (double)s.z * t.z;
    };
    v3 cur[4], nxt[4];
    typename C::R ne, nf, he, hf;
    {
        typename C::R e, f;
        load4(z0, y, x0, e, f);
        decode4(e, f, cur);
        load4(z0 + 1 < L ? z0 + 1 : 0, y, x0, ne, nf);
        if (halo) load4(z0, hy, hx0, he, hf);
    }
    double e = 0.0;
    for (int z = z0; z < z0 + Z; ++z) {
        const int b = z & 1;
        decode4(ne, nf, nxt);
        const int zn = z + 2 < L ? z + 2 : z + 2 - L;
        load4(zn, y, x0, ne, nf);
        if (active) put4(b, ly, x0, cur);
        if (halo) {
            v3 hv[4];
            decode4(he, hf, hv);
            put4(b, TY, hx0, hv);
            load4(z + 1 < L ? z + 1 : 0, hy, hx0, he, hf);
        }
        // couplings (+x, +y, +z) and field of my sites: x0, x0 + 2 on parity
        // p0 at half-indices jj, jj + 1; x0 + 1, x0 + 3 on the other parity
        const int p0 = (y + z) & 1;
        const int64_t jj = (int64_t)(z * L + y) * Lh + (x0 >> 1);
        float2 jc[3][2];
#pragma unroll
        for (int a3 = 0; a3 < 3; ++a3) {
            jc[a3][0] = *reinterpret_cast<const float2 *>(J6 + ((int64_t)p0 * 6 + 2 * a3) * Nh + jj);
            jc[a3][1] = *reinterpret_cast<const float2 *>(J6 + ((int64_t)(1 - p0) * 6 + 2 * a3) * Nh + jj);
        }
        __syncthreads();
        if (active) {
            const int lyp = ly + 1;  // the row above: in the band, or the staged row TY
            const float4 a0 = *reinterpret_cast<const float4 *>(lp(b, 0) + lyp * L + x0);
            const float4 a1 = *reinterpret_cast<const float4 *>(lp(b, 1) + lyp * L + x0);
            const float4 a2 = *reinterpret_cast<const float4 *>(lp(b, 2) + lyp * L + x0);
            const v3 yn[4] = {v3{a0.x, a1.x, a2.x}, v3{a0.y, a1.y, a2.y}, v3{a0.z, a1.z, a2.z},
                              v3{a0.w, a1.w, a2.w}};
            const v3 xr{lp(b, 0)[ly * L + xp], lp(b, 1)[ly * L + xp], lp(b, 2)[ly * L + xp]};
            // coupling of site u along axis a3: parity plane u & 1, element u >> 1
            auto J = [&](int a3, int u) { return (u >> 1) ? jc[a3][u & 1].y : jc[a3][u & 1].x; };
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const v3 xn = u == 3 ? xr : cur[u == 3 ? 0 : u + 1];
                e -= (double)J(0, u) * bond(cur[u], xn);
                e -= (double)J(1, u) * bond(cur[u], yn[u]);
                e -= (double)J(2, u) * bond(cur[u], nxt[u]);
            }
            if (H != nullptr) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t hj = (int64_t)((u & 1) ? 1 - p0 : p0) * 3 * Nh + jj + (u >> 1);
                    e -= (double)H[hj] * cur[u].x + (double)H[Nh + hj] * cur[u].y + (double)H[2 * Nh + hj] * cur[u].z;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) cur[u] = nxt[u];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = (int)(blockDim.x >> 6);
    const double v = wave_sum(e);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < n_waves; ++w) t += red[w];
        a.partials[rep * a.n_pb + pb] = t;
    }
}

int64_t energy_partials(int L, int64_t n_rep, int64_t n_pb_site)
{
    const int rows = kmode_rows(L);
    return rows > 0 ? (int64_t)(L / rows) * march_slabs(L, n_rep) : n_pb_site;
}

hipError_t launch_energy(const EnergyArgs &a, int storage, hipStream_t s)
{
    const int rows = kmode_rows(a.L);
    if (rows > 0) {
        const int64_t parts = (int64_t)(a.L / rows) * march_slabs(a.L, a.n_rep);
        if (a.n_pb != parts) return hipErrorInvalidValue;  // one partial per band and slab
        const int64_t blocks = a.n_rep * parts;
        if (blocks == 0) return hipSuccess;
        if (blocks > 0x7FFFFFFFll) return hipErrorInvalidValue;
        const unsigned threads = (unsigned)((rows * (a.L / 4) + 63) / 64 * 64);
        const size_t lds = (size_t)2 * 3 * (rows + 1) * a.L * sizeof(float);
        switch (storage) {
        case 0: hipLaunchKernelGGL(k_energy_stream<0>, dim3((unsigned)blocks), dim3(threads), lds, s, a); break;
        case 1: hipLaunchKernelGGL(k_energy_stream<1>, dim3((unsigned)blocks), dim3(threads), lds, s, a); break;
        case 2: hipLaunchKernelGGL(k_energy_stream<2>, dim3((unsigned)blocks), dim3(threads), lds, s, a); break;
        case 3: hipLaunchKernelGGL(k_energy_stream<3>, dim3((unsigned)blocks), dim3(threads), lds, s, a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const int64_t blocks = a.n_rep * a.n_pb;
    if (blocks == 0) return hipSuccess;
    switch (storage) {
    case 0: hipLaunchKernelGGL(k_energy<0>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_energy<1>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_energy<2>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_energy<3>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- overlap
// Work-group (d * T + k, pb) sums s^mu(copy 0) s^nu(copy 1) over the sites
// [pb * chunk, (pb + 1) * chunk) of both parities of rung k; one wave per
// (d, k) then adds the n_pb partials in a fixed order and forms q^2.
template <int STORE>
__global__ __launch_bounds__(kBlock) void k_overlap(OverlapArgs a)
{
    using C = Codec<STORE>;
    using T = typename C::T;
    __shared__ double red[4][9];
    const int64_t dk = blockIdx.x / a.n_pb;  // d * T + k
    const int pb = (int)(blockIdx.x - dk * a.n_pb);
    const int d = (int)(dk / a.T), k = (int)(dk - (int64_t)d * a.T);
    const int64_t Nh = a.Nh;
    const int32_t sa = a.slot_at_temp[((int64_t)d * a.O + 0) * a.T + k];
    const int32_t sb = a.slot_at_temp[((int64_t)d * a.O + 1) * a.T + k];
    const T *A = (const T *)a.spins + (((int64_t)d * a.O + 0) * a.T + sa) * 2 * C::kPlanes * Nh;
    const T *B = (const T *)a.spins + (((int64_t)d * a.O + 1) * a.T + sb) * 2 * C::kPlanes * Nh;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t j_end = ((int64_t)(pb + 1) * a.chunk < Nh) ? (int64_t)(pb + 1) * a.chunk : Nh;
    // unrolled so that the loads of several iterations are in flight together
    // (the sums keep their order)
#pragma unroll 4
    for (int64_t j = (int64_t)pb * a.chunk + threadIdx.x; j < j_end; j += kBlock) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const v3 x = C::load(A + (int64_t)p * C::kPlanes * Nh, Nh, j);
            const v3 y = C::load(B + (int64_t)p * C::kPlanes * Nh, Nh, j);
            const double xa[3] = {x.x, x.y, x.z}, ya[3] = {y.x, y.y, y.z};
            for (int m = 0; m < 3; ++m)
                for (int n = 0; n < 3; ++n) acc[3 * m + n] += xa[m] * ya[n];
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int m = 0; m < 9; ++m) {
        const double v = wave_sum(acc[m]);
        if (lane == 0) red[wave][m] = v;
    }
    __syncthreads();
    if (threadIdx.x < 9)
        a.partials[(dk * a.n_pb + pb) * 9 + threadIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// The same sums as a z-march where kmode_rows(L) > 0: one work-group per
// (sample, rung, band of kmode_rows(L) rows, z-slab of L / march_slabs(L, D T)
// planes), the thread of row y and quarter q holding the sites x = 4q .. 4q + 3
// of plane z as z advances, the next plane's loads issued a step ahead; every
// spin is read once, with 32-bit offsets and no coordinate arithmetic per site.
// The sums run in another order than k_overlap's, so the two agree to float64
// rounding. A work-group's sums go to the partial of its band and slab.
template <int STORE>
__global__ __launch_bounds__(kBlock) void k_overlap_stream(OverlapArgs a)
{
    using C = Codec<STORE>;
    using T = typename C::T;
    __shared__ double red[4][9];
    const int L = a.L, Lh = L >> 1, Q = L >> 2;
    const int TY = kmode_rows(L), n_bands = L / TY;
    const int S = march_slabs(L, (int64_t)a.D * a.T), Z = L / S;
    const int64_t dk = blockIdx.x / (n_bands * S);  // d * T + k
    const int pb = (int)(blockIdx.x - dk * n_bands * S);  // band * S + slab
    const int band = pb / S, z0 = (pb - band * S) * Z;
    const int d = (int)(dk / a.T), k = (int)(dk - (int64_t)d * a.T);
    const int64_t Nh = a.Nh;
    const int32_t sa = a.slot_at_temp[((int64_t)d * a.O + 0) * a.T + k];
    const int32_t sb = a.slot_at_temp[((int64_t)d * a.O + 1) * a.T + k];
    const T *R[2] = {(const T *)a.spins + (((int64_t)d * a.O + 0) * a.T + sa) * 2 * C::kPlanes * Nh,
                     (const T *)a.spins + (((int64_t)d * a.O + 1) * a.T + sb) * 2 * C::kPlanes * Nh};
    const int tid = threadIdx.x;
    const bool active = tid < TY * Q;
    const int y = band * TY + (active ? tid / Q : 0), x0 = active ? 4 * (tid - (tid / Q) * Q) : 0;
    // the four sites of plane zz of copy c: x0 and x0 + 2 on the parity of
    // y + zz (half-indices x0 / 2, x0 / 2 + 1), x0 + 1 and x0 + 3 on the other
    auto load4 = [&](int c, int zz, typename C::R &e, typename C::R &f) {
        const int p0 = (y + zz) & 1;
        const uint32_t jj = (uint32_t)((zz * L + y) * Lh + (x0 >> 1));
        C::load_raw_pair(R[c] + (int64_t)p0 * C::kPlanes * Nh, (uint32_t)Nh, jj, e);
        C::load_raw_pair(R[c] + (int64_t)(1 - p0) * C::kPlanes * Nh, (uint32_t)Nh, jj, f);
    };
    typename C::R ne[2], nf[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) load4(c, z0, ne[c], nf[c]);
    double acc[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) acc[m] = 0.0;
    for (int z = z0; z < z0 + Z; ++z) {
        v3 s[2][4];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            C::decode_pair(ne[c], s[c][0], s[c][2]);
            C::decode_pair(nf[c], s[c][1], s[c][3]);
            if (z + 1 < z0 + Z) load4(c, z + 1, ne[c], nf[c]);
        }
        if (active) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double xa[3] = {s[0][u].x, s[0][u].y, s[0][u].z}, ya[3] = {s[1][u].x, s[1][u].y, s[1][u].z};
#pragma unroll
                for (int m = 0; m < 3; ++m)
#pragma unroll
                    for (int n = 0; n < 3; ++n) acc[3 * m + n] += xa[m] * ya[n];
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = (int)(blockDim.x >> 6);
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        const double v = wave_sum(acc[m]);
        if (lane == 0) red[wave][m] = v;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        double t = 0.0;
        for (int w = 0; w < n_waves; ++w) t += red[w][threadIdx.x];
        a.partials[(dk * a.n_pb + pb) * 9 + threadIdx.x] = t;
    }
}

__global__ __launch_bounds__(64) void k_overlap_finish(OverlapArgs a)
{
    const int64_t dk = blockIdx.x;
    const int lane = threadIdx.x;
    const double invN = 1.0 / (double)(2 * a.Nh);
    double q2 = 0.0;
    for (int m = 0; m < 9; ++m) {
        double v = 0.0;
        for (int pb = lane; pb < a.n_pb; pb += 64) v += a.partials[(dk * a.n_pb + pb) * 9 + m];
        v = wave_sum(v) * invN;
        if (lane == 0) a.q[dk * 10 + m] = v;
        q2 += v * v;
    }
    if (lane == 0) a.q[dk * 10 + 9] = q2;
}

hipError_t launch_overlap(const OverlapArgs &a, int storage, hipStream_t s)
{
    const int64_t blocks = (int64_t)a.D * a.T * a.n_pb;
    if (blocks == 0) return hipSuccess;
    const int rows = kmode_rows(a.L);
    if (rows > 0) {
        if (a.n_pb != march_partials(a.L, (int64_t)a.D * a.T, 0)) return hipErrorInvalidValue;
        if (blocks > 0x7FFFFFFFll) return hipErrorInvalidValue;
        const dim3 grid((unsigned)blocks), block((unsigned)((rows * (a.L / 4) + 63) / 64 * 64));
        switch (storage) {
        case 0: hipLaunchKernelGGL(k_overlap_stream<0>, grid, block, 0, s, a); break;
        case 1: hipLaunchKernelGGL(k_overlap_stream<1>, grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_overlap_stream<2>, grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL(k_overlap_stream<3>, grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (storage) {
        case 0: hipLaunchKernelGGL(k_overlap<0>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
        case 1: hipLaunchKernelGGL(k_overlap<1>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_overlap<2>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL(k_overlap<3>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_overlap_finish, dim3((unsigned)((int64_t)a.D * a.T)), dim3(64), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- k modes
// Wave-vector dependent overlap q^{mu nu}(k) and chiral overlap q_c^alpha(k)
// between copies 0 and 1 at each rung, for k = 0 and k = (2 pi / L) e_a. The
// 84 outputs per (sample, rung) are split into three groups of accumulators
// (G = 0: q(0) and q(k_x), 27 values; G = 1: q(k_y), q(k_z), 36; G = 2: the
// chiral overlaps, 21), one grid column each. The phases exp(i 2 pi R / L) come
// from a per-block table in float64. Products, chiralities and sums are float64.
// Lattices with kmode_rows(L) > 0 take the two z-marches further below instead
// of these gathering passes.
template <int G>
struct KGroup;
template <>
struct KGroup<0> {
    static constexpr int first = 0, count = 27;
};
template <>
struct KGroup<1> {
    static constexpr int first = 27, count = 36;
};
template <>
struct KGroup<2> {
    static constexpr int first = 63, count = 21;
};

// The spin at (x, y, z), every coordinate in 0 .. L - 1 (L <= 1024, so the
// half-index fits 32 bits). B32: the replica's spins span less than 4 GiB, so
// every access is the (uniform) replica base plus a 32-bit byte offset.
template <int STORE, bool B32>
__device__ __forceinline__ v3 load_site(const typename Codec<STORE>::T *rep, int64_t Nh, uint32_t L, uint32_t x,
                                        uint32_t y, uint32_t z)
{
    const uint32_t p = (x + y + z) & 1u;
    const uint32_t j = (z * L + y) * (L >> 1) + (x >> 1);
    if constexpr (B32)
        return Codec<STORE>::load32(rep, (uint32_t)Nh, (p ? (uint32_t)Codec<STORE>::kPlanes * (uint32_t)Nh : 0u) + j);
    else
        return Codec<STORE>::load(rep + (p ? (int64_t)Codec<STORE>::kPlanes * Nh : 0), Nh, (int64_t)j);
}

// u . (v x w) in float64: each product of two float32 components is exact, so
// every component of v x w is rounded once; the dot product uses fused
// multiply-adds.
__device__ __forceinline__ double chirality(v3 u, v3 v, v3 w)
{
    const double vx = v.x, vy = v.y, vz = v.z, wx = w.x, wy = w.y, wz = w.z;
    const double cx = fma(vy, wz, -(vz * wy)), cy = fma(vz, wx, -(vx * wz)), cz = fma(vx, wy, -(vy * wx));
    return fma((double)u.x, cx, fma((double)u.y, cy, (double)u.z * cz));
}

template <int STORE, int G, bool B32>
__global__ __launch_bounds__(kBlock) void k_kmodes(KmodeArgs a)
{
    using C = Codec<STORE>;
    using T = typename C::T;
    constexpr int K = KGroup<G>::count;
    __shared__ double red[4][K];
    __shared__ double cph[1024], sph[1024];
    const int L = a.L;
    for (int r = threadIdx.x; r < L; r += kBlock) {
        double sv, cv;
        sincospi(2.0 * (double)r / (double)L, &sv, &cv);
        cph[r] = cv;
        sph[r] = sv;
    }
    __syncthreads();
    const int64_t dk = blockIdx.x / a.n_pb;  // d * T + k
    const int pb = (int)(blockIdx.x - dk * a.n_pb);
    const int d = (int)(dk / a.T), k = (int)(dk - (int64_t)d * a.T);
    const int64_t Nh = a.Nh, N = 2 * Nh;
    const int32_t sa = a.slot_at_temp[((int64_t)d * a.O + 0) * a.T + k];
    const int32_t sb = a.slot_at_temp[((int64_t)d * a.O + 1) * a.T + k];
    const T *A = (const T *)a.spins + (((int64_t)d * a.O + 0) * a.T + sa) * 2 * C::kPlanes * Nh;
    const T *B = (const T *)a.spins + (((int64_t)d * a.O + 1) * a.T + sb) * 2 * C::kPlanes * Nh;
    double acc[K];
#pragma unroll
    for (int m = 0; m < K; ++m) acc[m] = 0.0;
    // N = L^3 <= 2^30: the site index and its coordinates fit 32 bits. The
    // coordinates of the thread's first site come from one division; then they
    // advance by kBlock sites per iteration with carries.
    const uint32_t Lu = (uint32_t)L, LL = Lu * Lu;
    const uint32_t i_end = (uint32_t)(((int64_t)(pb + 1) * a.chunk < N) ? (int64_t)(pb + 1) * a.chunk : N);
    const uint32_t i0 = (uint32_t)((int64_t)pb * a.chunk) + threadIdx.x;
    uint32_t x = i0 % Lu, y = (i0 / Lu) % Lu, z = i0 / LL;
    const uint32_t sx = (uint32_t)kBlock % Lu, sy = ((uint32_t)kBlock / Lu) % Lu, sz = (uint32_t)kBlock / LL;
    // U sites per iteration, their loads issued before any is used (several
    // sites' loads in flight per wave); the sums still take the sites in order.
    // A site past the end reads site 0 of the replica (valid memory) and is not
    // counted.
    constexpr int U = G < 2 ? 4 : 2;
    for (uint32_t i = i0; i < i_end; i += U * kBlock) {
        uint32_t cx[U], cy[U], cz[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ok[u] = i + (uint32_t)u * kBlock < i_end;
            cx[u] = ok[u] ? x : 0u;
            cy[u] = ok[u] ? y : 0u;
            cz[u] = ok[u] ? z : 0u;
            x += sx;
            uint32_t c = x >= Lu ? 1u : 0u;
            x -= c * Lu;
            y += sy + c;
            c = y >= Lu ? 1u : 0u;
            y -= c * Lu;
            z += sz + c;
        }
        v3 sa0[U], sb0[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            sa0[u] = load_site<STORE, B32>(A, Nh, Lu, cx[u], cy[u], cz[u]);
            sb0[u] = load_site<STORE, B32>(B, Nh, Lu, cx[u], cy[u], cz[u]);
        }
        if constexpr (G < 2) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!ok[u]) continue;
                const double xa[3] = {sa0[u].x, sa0[u].y, sa0[u].z}, ya[3] = {sb0[u].x, sb0[u].y, sb0[u].z};
                const uint32_t R0 = G == 0 ? cx[u] : cy[u], R1 = G == 0 ? cx[u] : cz[u];
                const double c0 = cph[R0], s0 = sph[R0], c1 = cph[R1], s1 = sph[R1];
#pragma unroll
                for (int m = 0; m < 3; ++m)
#pragma unroll
                    for (int n = 0; n < 3; ++n) {
                        const double f = xa[m] * ya[n];
                        const int mn = 3 * m + n;
                        if (G == 0) {
                            acc[mn] += f;
                            acc[9 + 2 * mn] += f * c0;
                            acc[9 + 2 * mn + 1] += f * s0;
                        } else {
                            acc[2 * mn] += f * c0;
                            acc[2 * mn + 1] += f * s0;
                            acc[18 + 2 * mn] += f * c1;
                            acc[18 + 2 * mn + 1] += f * s1;
                        }
                    }
            }
        } else {
            // the neighbours along each axis: (+, -) of replicas A and B
            v3 na[U][3][2], nb[U][3][2];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t X = cx[u], Y = cy[u], Z = cz[u];
                const uint32_t xp = X + 1 == Lu ? 0 : X + 1, xm = X == 0 ? Lu - 1 : X - 1;
                const uint32_t yp = Y + 1 == Lu ? 0 : Y + 1, ym = Y == 0 ? Lu - 1 : Y - 1;
                const uint32_t zp = Z + 1 == Lu ? 0 : Z + 1, zm = Z == 0 ? Lu - 1 : Z - 1;
                na[u][0][0] = load_site<STORE, B32>(A, Nh, Lu, xp, Y, Z);
                na[u][0][1] = load_site<STORE, B32>(A, Nh, Lu, xm, Y, Z);
                na[u][1][0] = load_site<STORE, B32>(A, Nh, Lu, X, yp, Z);
                na[u][1][1] = load_site<STORE, B32>(A, Nh, Lu, X, ym, Z);
                na[u][2][0] = load_site<STORE, B32>(A, Nh, Lu, X, Y, zp);
                na[u][2][1] = load_site<STORE, B32>(A, Nh, Lu, X, Y, zm);
                nb[u][0][0] = load_site<STORE, B32>(B, Nh, Lu, xp, Y, Z);
                nb[u][0][1] = load_site<STORE, B32>(B, Nh, Lu, xm, Y, Z);
                nb[u][1][0] = load_site<STORE, B32>(B, Nh, Lu, X, yp, Z);
                nb[u][1][1] = load_site<STORE, B32>(B, Nh, Lu, X, ym, Z);
                nb[u][2][0] = load_site<STORE, B32>(B, Nh, Lu, X, Y, zp);
                nb[u][2][1] = load_site<STORE, B32>(B, Nh, Lu, X, Y, zm);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!ok[u]) continue;
                const double cx0 = cph[cx[u]], snx = sph[cx[u]], cy0 = cph[cy[u]], sny = sph[cy[u]];
                const double cz0 = cph[cz[u]], snz = sph[cz[u]];
#pragma unroll
                for (int al = 0; al < 3; ++al) {
                    const double ka = chirality(na[u][al][0], sa0[u], na[u][al][1]);
                    const double kb = chirality(nb[u][al][0], sb0[u], nb[u][al][1]);
                    const double g = ka * kb;
                    acc[7 * al] += g;
                    acc[7 * al + 1] = fma(g, cx0, acc[7 * al + 1]);
                    acc[7 * al + 2] = fma(g, snx, acc[7 * al + 2]);
                    acc[7 * al + 3] = fma(g, cy0, acc[7 * al + 3]);
                    acc[7 * al + 4] = fma(g, sny, acc[7 * al + 4]);
                    acc[7 * al + 5] = fma(g, cz0, acc[7 * al + 5]);
                    acc[7 * al + 6] = fma(g, snz, acc[7 * al + 6]);
                }
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < K; ++m) {
        const double v = wave_sum(acc[m]);
        if (lane == 0) red[wave][m] = v;
    }
    __syncthreads();
    if (threadIdx.x < K)
        a.partials[(dk * a.n_pb + pb) * 84 + KGroup<G>::first + threadIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// One block per (sample, rung): output m adds the n_pb partials in order.
__global__ __launch_bounds__(128) void k_kmodes_finish(KmodeArgs a)
{
    const int64_t dk = blockIdx.x;
    const int m = threadIdx.x;
    if (m >= 84) return;
    double v = 0.0;
    for (int pb = 0; pb < a.n_pb; ++pb) v += a.partials[(dk * a.n_pb + pb) * 84 + m];
    a.q[dk * 84 + m] = v / (double)(2 * a.Nh);
}

// The spin-overlap groups (G = 0 and 1, outputs 0 .. 62) in one pass for the
// lattices the chiral z-march takes (kmode_rows(L) > 0): one work-group per
// (sample, rung, band of kmode_rows(L) rows), the thread of row y and quarter q
// holding the sites x = 4q .. 4q + 3 of plane z as z advances, the next
// plane's loads issued a step ahead. Since x and y stay fixed per thread, the phase factors split:
// per step the thread adds its four products s^mu(1) s^nu(2) with weights 1,
// cos kx and sin kx, and accumulates those three sums over z, the first also
// weighted by cos kz and sin kz; q(k_y) is cos ky and sin ky times the
// unweighted sum at the end. 45 float64 accumulators replace the 63 of the two
// gathering passes, and both copies are read once instead of twice. The sums
// run in another order than the gathering kernel's, so the two agree to
// float64 rounding. A work-group's sums go to the partial of its band. (Unlike
// the copy-pair and energy marches these take no z-slabs: their per-work-group
// start, the phase tables and the reduction of 63 or 21 sums, cost more than
// the extra work-groups gain, 593 against 631 us on the large workload.)
template <int STORE>
__global__ __launch_bounds__(kBlock) void k_qk_stream(KmodeArgs a)
{
    using C = Codec<STORE>;
    using T = typename C::T;
    constexpr int K = KGroup<0>::count + KGroup<1>::count;  // 63
    __shared__ double red[4][K];
    __shared__ double cph[224], sph[224];
    const int L = a.L, Lh = L >> 1, Q = L >> 2;
    const int TY = kmode_rows(L), n_bands = L / TY;
    constexpr int z0 = 0;
    const int Z = L;
    for (int r = threadIdx.x; r < L; r += blockDim.x) {
        double sv, cv;
        sincospi(2.0 * (double)r / (double)L, &sv, &cv);
        cph[r] = cv;
        sph[r] = sv;
    }
    const int64_t dk = blockIdx.x / n_bands;  // d * T + k
    const int pb = (int)(blockIdx.x - dk * n_bands), band = pb;
    const int d = (int)(dk / a.T), k = (int)(dk - (int64_t)d * a.T);
    const int64_t Nh = a.Nh;
    const int32_t sa = a.slot_at_temp[((int64_t)d * a.O + 0) * a.T + k];
    const int32_t sb = a.slot_at_temp[((int64_t)d * a.O + 1) * a.T + k];
    const T *R[2] = {(const T *)a.spins + (((int64_t)d * a.O + 0) * a.T + sa) * 2 * C::kPlanes * Nh,
                     (const T *)a.spins + (((int64_t)d * a.O + 1) * a.T + sb) * 2 * C::kPlanes * Nh};
    const int tid = threadIdx.x;
    const bool active = tid < TY * Q;
    const int y = band * TY + (active ? tid / Q : 0), x0 = active ? 4 * (tid - (tid / Q) * Q) : 0;
    // the four sites of plane zz of copy c: x0 and x0 + 2 on the parity of
    // y + zz (half-indices x0 / 2, x0 / 2 + 1), x0 + 1 and x0 + 3 on the other
    auto load4 = [&](int c, int zz, typename C::R &e, typename C::R &f) {
        const int p0 = (y + zz) & 1;
        const uint32_t jj = (uint32_t)((zz * L + y) * Lh + (x0 >> 1));
        C::load_raw_pair(R[c] + (int64_t)p0 * C::kPlanes * Nh, (uint32_t)Nh, jj, e);
        C::load_raw_pair(R[c] + (int64_t)(1 - p0) * C::kPlanes * Nh, (uint32_t)Nh, jj, f);
    };
    typename C::R ne[2], nf[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) load4(c, z0, ne[c], nf[c]);
    double A0[9], Ac[9], As[9], Zc[9], Zs[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) A0[m] = Ac[m] = As[m] = Zc[m] = Zs[m] = 0.0;
    __syncthreads();  // the phase tables
    double cx[4], sx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        cx[u] = cph[x0 + u];
        sx[u] = sph[x0 + u];
    }
    for (int z = z0; z < z0 + Z; ++z) {
        v3 s[2][4];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            C::decode_pair(ne[c], s[c][0], s[c][2]);
            C::decode_pair(nf[c], s[c][1], s[c][3]);
            if (z + 1 < z0 + Z) load4(c, z + 1, ne[c], nf[c]);
        }
        if (active) {
            const double cz = cph[z], sz = sph[z];
            double av[4][3], bv[4][3];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                av[u][0] = s[0][u].x; av[u][1] = s[0][u].y; av[u][2] = s[0][u].z;
                bv[u][0] = s[1][u].x; bv[u][1] = s[1][u].y; bv[u][2] = s[1][u].z;
            }
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
                for (int n = 0; n < 3; ++n) {
                    const int mn = 3 * m + n;
                    double t0 = 0.0, tc = 0.0, ts = 0.0;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const double f = av[u][m] * bv[u][n];
                        t0 += f;
                        tc = fma(f, cx[u], tc);
                        ts = fma(f, sx[u], ts);
                    }
                    A0[mn] += t0;
                    Ac[mn] += tc;
                    As[mn] += ts;
                    Zc[mn] = fma(t0, cz, Zc[mn]);
                    Zs[mn] = fma(t0, sz, Zs[mn]);
                }
        }
    }
    const double cy = cph[y], sy = sph[y];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = (int)(blockDim.x >> 6);
#pragma unroll
    for (int mn = 0; mn < 9; ++mn) {
        // the output layout of the gathering kernel: group 0 holds q(0) at mn and
        // q(k_x) at 9 + 2 mn (cos, sin); group 1 q(k_y) at 27 + 2 mn and q(k_z)
        // at 45 + 2 mn
        const double v0 = wave_sum(A0[mn]), v1 = wave_sum(Ac[mn]), v2 = wave_sum(As[mn]);
        const double v3c = wave_sum(cy * A0[mn]), v4 = wave_sum(sy * A0[mn]);
        const double v5 = wave_sum(Zc[mn]), v6 = wave_sum(Zs[mn]);
        if (lane == 0) {
            red[wave][mn] = v0;
            red[wave][9 + 2 * mn] = v1;
            red[wave][9 + 2 * mn + 1] = v2;
            red[wave][27 + 2 * mn] = v3c;
            red[wave][27 + 2 * mn + 1] = v4;
            red[wave][45 + 2 * mn] = v5;
            red[wave][45 + 2 * mn + 1] = v6;
        }
    }
    __syncthreads();
    for (int m = threadIdx.x; m < K; m += blockDim.x) {
        double v = 0.0;
        for (int w = 0; w < n_waves; ++w) v += red[w][m];
        a.partials[(dk * a.n_pb + pb) * 84 + m] = v;
    }
}

// The chiral group (G = 2) where kmode_rows(L) > 0: one work-group per
// (sample, rung, band of TY = kmode_rows(L) rows) marches over z with plane z
// of both copies staged in LDS and the planes z - 1, z and z + 1 at the
// thread's own sites in registers, so that every spin is read from memory once
// instead of seven times (the gathering kernel's own site and six neighbours).
// Where TY < L the rows just above and below the band (halo rows, read by the
// first 2 L / 4 threads) are staged too, so bands add 2 / TY to the reads.
// The thread of row y and quarter q owns the sites x = 4q .. 4q + 3. The
// chiralities are float64 as in the gathering kernel; along x, pairs of
// neighbouring sites share one cross product (kappa at x0 and x0 + 1 both use
// s(x0 + 1) x s(x0), by the cyclic symmetry of the triple product), and the
// phase factors split as in the overlap march (x and y fixed per thread): per
// step and axis the thread adds its four products kappa(1) kappa(2) with
// weights 1, cos kx and sin kx and accumulates those over z, the first also
// weighted by cos kz and sin kz; q_c(k_y) is cos ky and sin ky times the
// unweighted sum at the end. The sums run in another order than the gathering
// kernel's, so the two agree to float64 rounding. A work-group's sums go to
// the partial of its band.
template <int STORE, bool BANDED>
__global__ __launch_bounds__(kBlock, 2) void k_chiral_stream(KmodeArgs a)
{
    using C = Codec<STORE>;
    using T = typename C::T;
    constexpr int K = KGroup<2>::count;
    // [2 buffers][2 copies][3 components][TY + 2 rows][L]: row 0 the halo row
    // below the band, rows 1 .. TY the band, row TY + 1 the halo row above
    extern __shared__ __align__(16) float plane[];
    __shared__ double red[4][K];
    __shared__ double cph[224], sph[224];
    const int L = a.L, Lh = L >> 1, Q = L >> 2;
    const int TY = BANDED ? kmode_rows(L) : L, n_bands = L / TY, RL = (TY + 2) * L;
    constexpr int z0 = 0;
    const int Z = L;
    constexpr bool banded = BANDED;  // TY < L
    for (int r = threadIdx.x; r < L; r += blockDim.x) {
        double sv, cv;
        sincospi(2.0 * (double)r / (double)L, &sv, &cv);
        cph[r] = cv;
        sph[r] = sv;
    }
    const int64_t dk = blockIdx.x / n_bands;  // d * T + k
    const int pb = (int)(blockIdx.x - dk * n_bands), band = pb, y0 = band * TY;
    const int d = (int)(dk / a.T), k = (int)(dk - (int64_t)d * a.T);
    const int64_t Nh = a.Nh;
    const int32_t sa = a.slot_at_temp[((int64_t)d * a.O + 0) * a.T + k];
    const int32_t sb = a.slot_at_temp[((int64_t)d * a.O + 1) * a.T + k];
    const T *R[2] = {(const T *)a.spins + (((int64_t)d * a.O + 0) * a.T + sa) * 2 * C::kPlanes * Nh,
                     (const T *)a.spins + (((int64_t)d * a.O + 1) * a.T + sb) * 2 * C::kPlanes * Nh};
    const int tid = threadIdx.x;
    const bool active = tid < TY * Q;
    const int ly = active ? tid / Q : 0, x0 = active ? 4 * (tid - (tid / Q) * Q) : 0;
    const int y = y0 + ly;
    // LDS rows of the band row, the row above (y + 1) and the row below (y - 1)
    const int lr = ly + 1;
    const int lrp = banded ? lr + 1 : (ly + 1 == L ? 0 : ly + 1) + 1;
    const int lrm = banded ? lr - 1 : (ly == 0 ? L - 1 : ly - 1) + 1;
    const int xm = x0 == 0 ? L - 1 : x0 - 1, xp = x0 + 4 == L ? 0 : x0 + 4;
    // halo rows: threads 0 .. Q - 1 stage the row below the band (LDS row 0),
    // threads Q .. 2Q - 1 the row above it (LDS row TY + 1)
    const bool halo = banded && tid < 2 * Q;
    const bool hlow = tid < Q;
    const int hy = !halo ? 0 : hlow ? (y0 == 0 ? L - 1 : y0 - 1) : (y0 + TY == L ? 0 : y0 + TY);
    const int hx0 = !halo ? 0 : 4 * (hlow ? tid : tid - Q), hlr = hlow ? 0 : TY + 1;
    // the four sites x .. x + 3 (x % 4 == 0) of row yy of plane zz of copy c:
    // x and x + 2 lie on the parity of yy + zz, at half-indices x / 2 and
    // x / 2 + 1; x + 1 and x + 3 on the other
    auto load4r = [&](int c, int zz, int yy, int xx, typename C::R &e, typename C::R &f) {
        const int p0 = (yy + zz) & 1;
        const uint32_t jj = (uint32_t)((zz * L + yy) * Lh + (xx >> 1));
        C::load_raw_pair(R[c] + (int64_t)p0 * C::kPlanes * Nh, (uint32_t)Nh, jj, e);
        C::load_raw_pair(R[c] + (int64_t)(1 - p0) * C::kPlanes * Nh, (uint32_t)Nh, jj, f);
    };
    auto load4 = [&](int c, int zz, typename C::R &e, typename C::R &f) { load4r(c, zz, y, x0, e, f); };
    auto decode4 = [&](const typename C::R &e, const typename C::R &f, v3 (&s)[4]) {
        C::decode_pair(e, s[0], s[2]);
        C::decode_pair(f, s[1], s[3]);
    };
    v3 prv[2][4], cur[2][4], nxt[2][4];
    typename C::R ne[2], nf[2], he[2], hf[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        typename C::R e, f;
        load4(c, z0 == 0 ? L - 1 : z0 - 1, e, f);
        decode4(e, f, prv[c]);
        load4(c, z0, e, f);
        decode4(e, f, cur[c]);
        load4(c, z0 + 1 < L ? z0 + 1 : 0, ne[c], nf[c]);
        if (BANDED && halo) load4r(c, z0, hy, hx0, he[c], hf[c]);
    }
    double P0[3], Pc[3], Ps[3], Zc[3], Zs[3];
#pragma unroll
    for (int al = 0; al < 3; ++al) P0[al] = Pc[al] = Ps[al] = Zc[al] = Zs[al] = 0.0;
    auto lp = [&](int b, int c, int m) { return plane + ((b * 2 + c) * 3 + m) * RL; };
    auto put4 = [&](int b, int c, int row, int xx, const v3 (&v)[4]) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const float4 q = m == 0 ? make_float4(v[0].x, v[1].x, v[2].x, v[3].x)
                           : m == 1 ? make_float4(v[0].y, v[1].y, v[2].y, v[3].y)
                                    : make_float4(v[0].z, v[1].z, v[2].z, v[3].z);
            *reinterpret_cast<float4 *>(lp(b, c, m) + row * L + xx) = q;
        }
    };
    __syncthreads();  // the phase tables
    double cx[4], sx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        cx[u] = cph[x0 + u];
        sx[u] = sph[x0 + u];
    }
    for (int z = z0; z < z0 + Z; ++z) {
        const int b = z & 1;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            decode4(ne[c], nf[c], nxt[c]);
            const int zn = z + 2 < L ? z + 2 : z + 2 - L;  // the next step's plane z + 1 (wrapping)
            load4(c, zn, ne[c], nf[c]);
            if (active) put4(b, c, lr, x0, cur[c]);
            if (BANDED && halo) {  // this plane's halo row, then the next plane's load
                v3 hv[4];
                decode4(he[c], hf[c], hv);
                put4(b, c, hlr, hx0, hv);
                load4r(c, z + 1 < L ? z + 1 : 0, hy, hx0, he[c], hf[c]);
            }
        }
        __syncthreads();
        if (active) {
            double kap[2][4][3];  // chirality of copy c, site u, axis alpha
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                v3 ypl[4], ymi[4], xl, xr;
                {
                    const float4 a0 = *reinterpret_cast<const float4 *>(lp(b, c, 0) + lrp * L + x0);
                    const float4 a1 = *reinterpret_cast<const float4 *>(lp(b, c, 1) + lrp * L + x0);
                    const float4 a2 = *reinterpret_cast<const float4 *>(lp(b, c, 2) + lrp * L + x0);
                    ypl[0] = v3{a0.x, a1.x, a2.x}; ypl[1] = v3{a0.y, a1.y, a2.y};
                    ypl[2] = v3{a0.z, a1.z, a2.z}; ypl[3] = v3{a0.w, a1.w, a2.w};
                    const float4 b0 = *reinterpret_cast<const float4 *>(lp(b, c, 0) + lrm * L + x0);
                    const float4 b1 = *reinterpret_cast<const float4 *>(lp(b, c, 1) + lrm * L + x0);
                    const float4 b2 = *reinterpret_cast<const float4 *>(lp(b, c, 2) + lrm * L + x0);
                    ymi[0] = v3{b0.x, b1.x, b2.x}; ymi[1] = v3{b0.y, b1.y, b2.y};
                    ymi[2] = v3{b0.z, b1.z, b2.z}; ymi[3] = v3{b0.w, b1.w, b2.w};
                    xl = v3{lp(b, c, 0)[lr * L + xm], lp(b, c, 1)[lr * L + xm], lp(b, c, 2)[lr * L + xm]};
                    xr = v3{lp(b, c, 0)[lr * L + xp], lp(b, c, 1)[lr * L + xp], lp(b, c, 2)[lr * L + xp]};
                }
                const v3 (&w)[4] = cur[c];
                // kappa_x(u) = s(u+1) . (s(u) x s(u-1)); x0 and x0 + 1 share
                // s(x0+1) x s(x0), x0 + 2 and x0 + 3 share s(x0+3) x s(x0+2)
                kap[c][0][0] = chirality(xl, w[1], w[0]);
                kap[c][1][0] = chirality(w[2], w[1], w[0]);
                kap[c][2][0] = chirality(w[1], w[3], w[2]);
                kap[c][3][0] = chirality(xr, w[3], w[2]);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    kap[c][u][1] = chirality(ypl[u], w[u], ymi[u]);
                    kap[c][u][2] = chirality(nxt[c][u], w[u], prv[c][u]);
                }
            }
            const double cz = cph[z], sz = sph[z];
#pragma unroll
            for (int al = 0; al < 3; ++al) {
                double t0 = 0.0, tc = 0.0, ts = 0.0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double g = kap[0][u][al] * kap[1][u][al];
                    t0 += g;
                    tc = fma(g, cx[u], tc);
                    ts = fma(g, sx[u], ts);
                }
                P0[al] += t0;
                Pc[al] += tc;
                Ps[al] += ts;
                Zc[al] = fma(t0, cz, Zc[al]);
                Zs[al] = fma(t0, sz, Zs[al]);
            }
        }
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                prv[c][u] = cur[c][u];
                cur[c][u] = nxt[c][u];
            }
    }
    const double cy = cph[y], sy = sph[y];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = (int)(blockDim.x >> 6);
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        // the gathering kernel's layout: per axis, k = 0, then (cos, sin) of
        // k_x, k_y, k_z
        const double v0 = wave_sum(P0[al]), v1 = wave_sum(Pc[al]), v2 = wave_sum(Ps[al]);
        const double v3c = wave_sum(cy * P0[al]), v4 = wave_sum(sy * P0[al]);
        const double v5 = wave_sum(Zc[al]), v6 = wave_sum(Zs[al]);
        if (lane == 0) {
            red[wave][7 * al] = v0;
            red[wave][7 * al + 1] = v1;
            red[wave][7 * al + 2] = v2;
            red[wave][7 * al + 3] = v3c;
            red[wave][7 * al + 4] = v4;
            red[wave][7 * al + 5] = v5;
            red[wave][7 * al + 6] = v6;
        }
    }
    __syncthreads();
    for (int m = threadIdx.x; m < K; m += blockDim.x) {
        double v = 0.0;
        for (int w = 0; w < n_waves; ++w) v += red[w][m];
        a.partials[(dk * a.n_pb + pb) * 84 + KGroup<2>::first + m] = v;
    }
}

template <int STORE>
static hipError_t launch_kmodes_s(const KmodeArgs &a, hipStream_t s)
{
    const dim3 grid((unsigned)((int64_t)a.D * a.T * a.n_pb)), block(kBlock);
    // a replica's spins within 4 GiB: 32-bit offsets from its base
    const bool b32 = 2 * (uint64_t)Codec<STORE>::kPlanes * (uint64_t)a.Nh * sizeof(typename Codec<STORE>::T) <
                     (1ull << 32);
    // z-marches over bands of rows where kmode_rows(L) > 0: the overlap groups
    // in one pass, the chiral group in another
    const int rows = kmode_rows(a.L);
    if (rows > 0) {
        const int64_t parts = kmode_partials(a.L, 0);
        if (a.n_pb != parts) return hipErrorInvalidValue;  // one partial per band
        if ((int64_t)a.D * a.T * parts > 0x7FFFFFFFll) return hipErrorInvalidValue;
        const unsigned threads = (unsigned)((rows * (a.L / 4) + 63) / 64 * 64);
        const size_t lds = (size_t)2 * 2 * 3 * (rows + 2) * a.L * sizeof(float);
        const dim3 cols((unsigned)((int64_t)a.D * a.T * parts));
        hipLaunchKernelGGL((k_qk_stream<STORE>), cols, dim3(threads), 0, s, a);
        if (rows < a.L)
            hipLaunchKernelGGL((k_chiral_stream<STORE, true>), cols, dim3(threads), lds, s, a);
        else
            hipLaunchKernelGGL((k_chiral_stream<STORE, false>), cols, dim3(threads), lds, s, a);
    } else if (b32) {
        hipLaunchKernelGGL((k_kmodes<STORE, 0, true>), grid, block, 0, s, a);
        hipLaunchKernelGGL((k_kmodes<STORE, 1, true>), grid, block, 0, s, a);
        hipLaunchKernelGGL((k_kmodes<STORE, 2, true>), grid, block, 0, s, a);
    } else {
        hipLaunchKernelGGL((k_kmodes<STORE, 0, false>), grid, block, 0, s, a);
        hipLaunchKernelGGL((k_kmodes<STORE, 1, false>), grid, block, 0, s, a);
        hipLaunchKernelGGL((k_kmodes<STORE, 2, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_kmodes(const KmodeArgs &a, int storage, hipStream_t s)
{
    const int64_t blocks = (int64_t)a.D * a.T * a.n_pb;
    if (blocks == 0) return hipSuccess;
    if (a.L > 1024 || blocks > 0x7FFFFFFFll) return hipErrorInvalidValue;
    hipError_t e;
    switch (storage) {
    case 0: e = launch_kmodes_s<0>(a, s); break;
    case 1: e = launch_kmodes_s<1>(a, s); break;
    case 2: e = launch_kmodes_s<2>(a, s); break;
    case 3: e = launch_kmodes_s<3>(a, s); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_kmodes_finish, dim3((unsigned)((int64_t)a.D * a.T)), dim3(128), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- copy-pair overlaps
// A_ab(k) = (1/N) sum_i (s_i(a) . s_i(b)) exp(i k.R_i) for every copy pair a < b at
// each rung, k = 0 and (2 pi / L) e_a: the building blocks of the four-replica
// estimators. Grid column c takes pairs [4 c, 4 c + 4) (28 float64
// accumulators per thread).
template <int STORE>
__global__ __launch_bounds__(kBlock) void k_pair_overlaps(PairOvArgs a)
{
    using C = Codec<STORE>;
    using T = typename C::T;
    __shared__ double red[4][28];
    __shared__ double cph[1024], sph[1024];
    const int L = a.L;
    for (int r = threadIdx.x; r < L; r += kBlock) {
        double sv, cv;
        sincospi(2.0 * (double)r / (double)L, &sv, &cv);
        cph[r] = cv;
        sph[r] = sv;
    }
    __syncthreads();
    const int64_t dk = blockIdx.x / a.n_pb;
    const int pb = (int)(blockIdx.x - dk * a.n_pb);
    const int d = (int)(dk / a.T), k = (int)(dk - (int64_t)d * a.T);
    const int O = a.O, P = O * (O - 1) / 2;
    const int p0 = 4 * (int)blockIdx.y;
    const int np = P - p0 < 4 ? P - p0 : 4;
    const int64_t Nh = a.Nh, N = 2 * Nh;
    const T *U[4], *V[4];
    {
        int q = 0, p = 0;
        for (int ca = 0; ca < O; ++ca)
            for (int cb = ca + 1; cb < O; ++cb, ++p)
                if (p >= p0 && q < np) {
                    const int32_t sa = a.slot_at_temp[((int64_t)d * O + ca) * a.T + k];
                    const int32_t sb = a.slot_at_temp[((int64_t)d * O + cb) * a.T + k];
                    U[q] = (const T *)a.spins + (((int64_t)d * O + ca) * a.T + sa) * 2 * C::kPlanes * Nh;
                    V[q] = (const T *)a.spins + (((int64_t)d * O + cb) * a.T + sb) * 2 * C::kPlanes * Nh;
                    ++q;
                }
        for (; q < 4; ++q) U[q] = V[q] = nullptr;
    }
    double acc[28];
#pragma unroll
    for (int m = 0; m < 28; ++m) acc[m] = 0.0;
    const int64_t i_end = ((int64_t)(pb + 1) * a.chunk < N) ? (int64_t)(pb + 1) * a.chunk : N;
    for (int64_t i = (int64_t)pb * a.chunk + threadIdx.x; i < i_end; i += kBlock) {
        const int x = (int)(i % L), y = (int)((i / L) % L), z = (int)(i / ((int64_t)L * L));
        const int p = (x + y + z) & 1;
        const int64_t j = ((int64_t)z * L + y) * (L / 2) + (x >> 1);
        const double ph[7] = {1.0, cph[x], sph[x], cph[y], sph[y], cph[z], sph[z]};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q < np) {
                const v3 u = C::load(U[q] + (int64_t)p * C::kPlanes * Nh, Nh, j);
                const v3 v = C::load(V[q] + (int64_t)p * C::kPlanes * Nh, Nh, j);
                const double f = (double)u.x * v.x + (double)u.y * v.y + (double)u.z * v.z;
#pragma unroll
                for (int m = 0; m < 7; ++m) acc[7 * q + m] += f * ph[m];
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < 28; ++m) {
        const double v = wave_sum(acc[m]);
        if (lane == 0) red[wave][m] = v;
    }
    __syncthreads();
    if (threadIdx.x < 7 * np)
        a.partials[(dk * a.n_pb + pb) * (int64_t)(7 * P) + 7 * p0 + threadIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// One block per (sample, rung): output m adds the n_pb partials in order. With
// chi, four threads then form the four-replica estimators of Eq. (10) from the
// pair sums of copies 0..3: the double sum over (i, j) of each factorises into
// N A_ab(k) times N conj(A_cd(k)), so chi_1 = N^2 |A_01|^2, chi_2 = N^2 A_02
// conj(A_03), chi_3 = N^2 A_02 conj(A_13).
__global__ __launch_bounds__(256) void k_pair_overlaps_finish(PairOvArgs a)
{
    __shared__ double A[7 * 120];
    const int64_t dk = blockIdx.x;
    const int O = a.O;
    const int n = 7 * (O * (O - 1) / 2);
    for (int m = threadIdx.x; m < n; m += blockDim.x) {
        double v = 0.0;
        for (int pb = 0; pb < a.n_pb; ++pb) v += a.partials[(dk * a.n_pb + pb) * (int64_t)n + m];
        v = v / (double)(2 * a.Nh);
        if (a.q) a.q[dk * n + m] = v;
        A[m] = v;
    }
    if (a.chi == nullptr) return;
    __syncthreads();
    const int w = threadIdx.x;
    if (w >= 4) return;
    // pair (p, q), p < q, sits at p O - p (p + 1) / 2 + q - p - 1
    const int i01 = 0, i02 = 1, i03 = 2, i13 = O;
    auto re = [&](int pair) { return w == 0 ? A[7 * pair] : A[7 * pair + 1 + 2 * (w - 1)]; };
    auto im = [&](int pair) { return w == 0 ? 0.0 : A[7 * pair + 2 + 2 * (w - 1)]; };
    const double N = (double)(2 * a.Nh), N2 = N * N;
    const double r01 = re(i01), m01 = im(i01), r02 = re(i02), m02 = im(i02);
    const double r03 = re(i03), m03 = im(i03), r13 = re(i13), m13 = im(i13);
    double *out = a.chi + (dk * 4 + w) * 5;
    out[0] = N2 * (r01 * r01 + m01 * m01);
    out[1] = N2 * (r02 * r03 + m02 * m03);
    out[2] = N2 * (m02 * r03 - r02 * m03);
    out[3] = N2 * (r02 * r13 + m02 * m13);
    out[4] = N2 * (m02 * r13 - r02 * m13);
}

// The copy-pair sums as a z-march where kmode_rows(L) > 0: one work-group per
// (sample, rung, band of kmode_rows(L) rows, z-slab of L / march_slabs(L, D T)
// planes) and copy pair (grid column y),
// the thread of row y and quarter q holding the sites x = 4q .. 4q + 3 of
// plane z as z advances, the next plane's loads issued a step ahead. Per step
// the thread forms the local overlaps s(a) . s(b) of its four sites in float64
// and adds them with weights 1, cos kx and sin kx, the first also with cos kz
// and sin kz; the k_y terms are cos ky and sin ky times the unweighted sum at
// the end (x and y stay fixed per thread). Every spin is read once. The sums
// run in another order than k_pair_overlaps', so the two agree to float64
// rounding. A work-group's sums go to the partial of its band and slab.
template <int STORE>
__global__ __launch_bounds__(kBlock) void k_pair_overlaps_stream(PairOvArgs a)
{
    using C = Codec<STORE>;
    using T = typename C::T;
    __shared__ double red[4][7];
    __shared__ double cph[224], sph[224];
    const int L = a.L, Lh = L >> 1, Q = L >> 2;
    const int TY = kmode_rows(L), n_bands = L / TY;
    const int S = march_slabs(L, (int64_t)a.D * a.T), Z = L / S;
    for (int r = threadIdx.x; r < L; r += blockDim.x) {
        double sv, cv;
        sincospi(2.0 * (double)r / (double)L, &sv, &cv);
        cph[r] = cv;
        sph[r] = sv;
    }
    const int64_t dk = blockIdx.x / (n_bands * S);  // d * T + k
    const int pb = (int)(blockIdx.x - dk * n_bands * S);  // band * S + slab
    const int band = pb / S, z0 = (pb - band * S) * Z;
    const int d = (int)(dk / a.T), k = (int)(dk - (int64_t)d * a.T);
    const int O = a.O, P = O * (O - 1) / 2, pair = (int)blockIdx.y;
    int ca = 0, cb = 1;  // the copies of this pair, in the order (0, 1), (0, 2), ..., (1, 2), ...
    for (int i = 0, q = 0; i < O; ++i)
        for (int j = i + 1; j < O; ++j, ++q)
            if (q == pair) {
                ca = i;
                cb = j;
            }
    const int64_t Nh = a.Nh;
    const int32_t sa = a.slot_at_temp[((int64_t)d * O + ca) * a.T + k];
    const int32_t sb = a.slot_at_temp[((int64_t)d * O + cb) * a.T + k];
    const T *R[2] = {(const T *)a.spins + (((int64_t)d * O + ca) * a.T + sa) * 2 * C::kPlanes * Nh,
                     (const T *)a.spins + (((int64_t)d * O + cb) * a.T + sb) * 2 * C::kPlanes * Nh};
    const int tid = threadIdx.x;
    const bool active = tid < TY * Q;
    const int y = band * TY + (active ? tid / Q : 0), x0 = active ? 4 * (tid - (tid / Q) * Q) : 0;
    // the four sites of plane zz of copy c: x0 and x0 + 2 on the parity of
    // y + zz (half-indices x0 / 2, x0 / 2 + 1), x0 + 1 and x0 + 3 on the other
    auto load4 = [&](int c, int zz, typename C::R &e, typename C::R &f) {
        const int p0 = (y + zz) & 1;
        const uint32_t jj = (uint32_t)((zz * L + y) * Lh + (x0 >> 1));
        C::load_raw_pair(R[c] + (int64_t)p0 * C::kPlanes * Nh, (uint32_t)Nh, jj, e);
        C::load_raw_pair(R[c] + (int64_t)(1 - p0) * C::kPlanes * Nh, (uint32_t)Nh, jj, f);
    };
    typename C::R ne[2], nf[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) load4(c, z0, ne[c], nf[c]);
    double A0 = 0.0, Ac = 0.0, As = 0.0, Zc = 0.0, Zs = 0.0;
    __syncthreads();  // the phase tables
    double cx[4], sx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        cx[u] = cph[x0 + u];
        sx[u] = sph[x0 + u];
    }
    for (int z = z0; z < z0 + Z; ++z) {
        v3 s[2][4];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            C::decode_pair(ne[c], s[c][0], s[c][2]);
            C::decode_pair(nf[c], s[c][1], s[c][3]);
            if (z + 1 < z0 + Z) load4(c, z + 1, ne[c], nf[c]);
        }
        if (active) {
            double t0 = 0.0, tc = 0.0, ts = 0.0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double f = (double)s[0][u].x * s[1][u].x + (double)s[0][u].y * s[1][u].y +
                                 (double)s[0][u].z * s[1][u].z;
                t0 += f;
                tc = fma(f, cx[u], tc);
                ts = fma(f, sx[u], ts);
            }
            A0 += t0;
            Ac += tc;
            As += ts;
            Zc = fma(t0, cph[z], Zc);
            Zs = fma(t0, sph[z], Zs);
        }
    }
    const double cy = cph[y], sy = sph[y];
    // the layout of k_pair_overlaps: k = 0, then (cos, sin) of k_x, k_y, k_z
    const double v[7] = {A0, Ac, As, cy * A0, sy * A0, Zc, Zs};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = (int)(blockDim.x >> 6);
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        const double w = wave_sum(v[m]);
        if (lane == 0) red[wave][m] = w;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        double t = 0.0;
        for (int w = 0; w < n_waves; ++w) t += red[w][threadIdx.x];
        a.partials[(dk * a.n_pb + pb) * (int64_t)(7 * P) + 7 * pair + threadIdx.x] = t;
    }
}

int64_t march_partials(int L, int64_t n_items, int64_t q_pb)
{
    const int rows = kmode_rows(L);
    return rows > 0 ? (int64_t)(L / rows) * march_slabs(L, n_items) : q_pb;
}

int64_t kmode_partials(int L, int64_t q_pb)
{
    const int rows = kmode_rows(L);
    return rows > 0 ? L / rows : q_pb;
}

hipError_t launch_pair_overlaps(const PairOvArgs &a, int storage, hipStream_t s)
{
    const int P = a.O * (a.O - 1) / 2;
    const int rows = kmode_rows(a.L);
    if (rows > 0) {
        const int64_t parts = march_partials(a.L, (int64_t)a.D * a.T, 0);
        if (a.n_pb != parts) return hipErrorInvalidValue;  // one partial per band and slab
        const int64_t blocks = (int64_t)a.D * a.T * parts;
        if (blocks == 0 || P == 0) return hipSuccess;
        if (blocks > 0x7FFFFFFFll || P > 65535) return hipErrorInvalidValue;
        const dim3 grid((unsigned)blocks, (unsigned)P), block((unsigned)((rows * (a.L / 4) + 63) / 64 * 64));
        switch (storage) {
        case 0: hipLaunchKernelGGL(k_pair_overlaps_stream<0>, grid, block, 0, s, a); break;
        case 1: hipLaunchKernelGGL(k_pair_overlaps_stream<1>, grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_pair_overlaps_stream<2>, grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL(k_pair_overlaps_stream<3>, grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        const int64_t blocks = (int64_t)a.D * a.T * a.n_pb;
        if (blocks == 0 || P == 0) return hipSuccess;
        if (a.L > 1024 || blocks > 0x7FFFFFFFll) return hipErrorInvalidValue;
        const dim3 grid((unsigned)blocks, (unsigned)((P + 3) / 4)), block(kBlock);
        switch (storage) {
        case 0: hipLaunchKernelGGL(k_pair_overlaps<0>, grid, block, 0, s, a); break;
        case 1: hipLaunchKernelGGL(k_pair_overlaps<1>, grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_pair_overlaps<2>, grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL(k_pair_overlaps<3>, grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pair_overlaps_finish, dim3((unsigned)((int64_t)a.D * a.T)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- time series
__global__ __launch_bounds__(256) void k_series(SeriesArgs a)
{
    const uint32_t p = *a.tptr - a.t0;
    if ((int64_t)p >= a.capacity) return;
    const int64_t nE = (int64_t)a.D * a.O * a.T;
    const int64_t nq = a.q ? (int64_t)a.D * a.T : 0;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double *out = a.out + (int64_t)p * a.stride;
    if (g < nE) {
        const int64_t lad = g / a.T;  // (d, o); g - lad T is the rung
        out[g] = a.E[lad * a.T + a.slot_at_temp[g]];
    } else if (g < nE + nq) {
        out[g] = a.q[(g - nE) * 10 + 9];
    }
}

hipError_t launch_series(const SeriesArgs &a, hipStream_t s)
{
    const int64_t n = (int64_t)a.D * a.O * a.T + (a.q ? (int64_t)a.D * a.T : 0);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_series, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- maps
__global__ __launch_bounds__(256) void k_fill_identity(int32_t *sat, int32_t *tos, int64_t n_lad, int32_t T)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_lad * T) return;
    const int32_t k = (int32_t)(g % T);
    sat[g] = k;
    tos[g] = k;
}

__global__ __launch_bounds__(256) void k_invert(const int32_t *sat, int32_t *tos, int64_t n_lad, int32_t T)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_lad * T) return;
    const int64_t lad = g / T;
    const int32_t k = (int32_t)(g - lad * T);
    const int32_t s = sat[g];
    if (s >= 0 && s < T) tos[lad * T + s] = k;
}

hipError_t launch_fill_identity_maps(int32_t *sat, int32_t *tos, int64_t n_lad, int32_t T, hipStream_t s)
{
    const int64_t n = n_lad * T;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_identity, dim3(blocks_for(n)), dim3(256), 0, s, sat, tos, n_lad, T);
    return hipGetLastError();
}

hipError_t launch_invert_maps(const int32_t *sat, int32_t *tos, int64_t n_lad, int32_t T, hipStream_t s)
{
    const int64_t n = n_lad * T;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_invert, dim3(blocks_for(n)), dim3(256), 0, s, sat, tos, n_lad, T);
    return hipGetLastError();
}

__global__ void k_advance(uint32_t *tptr)
{
    if (threadIdx.x == 0) *tptr += 1u;
}

hipError_t launch_advance(uint32_t *tptr, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, tptr);
    return hipGetLastError();
}

__global__ void k_set_u32(uint32_t *ptr, uint32_t value)
{
    if (threadIdx.x == 0) *ptr = value;
}

hipError_t launch_set_u32(uint32_t *ptr, uint32_t value, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, s, ptr, value);
    return hipGetLastError();
}

__global__ void k_copy_u32(const uint32_t *src, uint32_t *dst)
{
    if (threadIdx.x == 0) *dst = *src;
}

hipError_t launch_copy_u32(const uint32_t *src, uint32_t *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(64), 0, s, src, dst);
    return hipGetLastError();
}

// ---------------------------------------------------------------- debug
__global__ __launch_bounds__(256) void k_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const u32x4 r = philox4x32_10(u32x4{ctr[4 * g], ctr[4 * g + 1], ctr[4 * g + 2], ctr[4 * g + 3]},
                                  key[2 * g], key[2 * g + 1]);
    out[4 * g] = r.x;
    out[4 * g + 1] = r.y;
    out[4 * g + 2] = r.z;
    out[4 * g + 3] = r.w;
}

// out[6 i + k] = hw_sin_rev, hw_cos_rev, hw_log, hw_exp(-x), hw_rcp, hw_rsq of x[i].
__global__ __launch_bounds__(256) void k_hw_math(const float *x, float *out, int64_t n)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const float v = x[g];
    float *o = out + 12 * g;
    o[0] = hw_sin_rev(v);
    o[1] = hw_cos_rev(v);
    o[2] = hw_log(v);
    o[3] = hw_exp(-v);
    o[4] = hw_rcp(v);
    o[5] = hw_rsq(v);
    sincos_2pi(v, o[6], o[7]);
    o[8] = v > 0.0f ? sqrt_rsqrt_nr(v, o[9]) : 0.0f;
    if (!(v > 0.0f)) o[9] = 0.0f;
    o[10] = v >= 0.0f ? exp_nonpos(-v) : 0.0f;
    o[11] = v >= 0x1p-126f ? log_normal(v) : 0.0f;
}

hipError_t launch_hw_math(const float *x, float *out, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hw_math, dim3(blocks_for(n)), dim3(256), 0, s, x, out, n);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3(blocks_for(n)), dim3(256), 0, s, ctr, key, out, n);
    return hipGetLastError();
}

}  // namespace hsg
