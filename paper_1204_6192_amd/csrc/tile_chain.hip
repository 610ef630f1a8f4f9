// tile_chain.hip -- the tile-local chain of the double checkerboard decomposition.
//
// The lattice is cut into tiles of TX x TY x TZ sites: whole rows along x
// (TX = L: every row of a tile is one contiguous run of each parity array) or
// cubes such as the paper's 8^3 (TX a multiple of 4). Tiles carry the coarse
// parity (X + Y + Z) mod 2 of their tile coordinates; with L / TX, L / TY and
// L / TZ each 1 or even, tiles of one coarse parity never share a face. One
// launch visits every tile of one coarse parity of every replica of a group.
// A work-group stages RB replicas of one sample's tile, with a one-site halo
// along every tiled axis, in LDS (both parities), then
// runs n_hit repetitions of n_or over-relaxation rounds and n_hb heat-bath
// rounds, a round being the even sites of the tile, then the odd sites (the
// numbered procedure of the paper's implementation section, with the tile
// loaded once per visit). The halo belongs to tiles of the other coarse parity,
// which no work-group of this launch changes. Finally the tile's own sites are
// written back. A thread owns one pair of neighbouring sites (x/2 = 2m, 2m + 1)
// of each parity in one replica and keeps their couplings (and field) in
// registers for the whole visit.
//
// What LDS holds: every spin as a load returns it (decoded and renormalised).
// The final store must write exactly the code of each site's last update:
// float32 spins are their own code; quantised angles are held decoded, and the
// octahedral projection divides by the L1 norm, so re-encoding gives the code
// back; for float16 / bfloat16 the renormalised value would not re-encode to
// its code, so each thread keeps the exact decoded components of its own four
// sites in registers and stores those.
#include "device.h"
#include "kernels.h"

namespace hsg {

// raw(s): the exact decoded value of the code an update stores (float16 /
// bfloat16: the representable components, not renormalised; the others: what a
// load returns). shared(raw): what LDS holds for every reader (decoded and
// renormalised, as a load returns it).
template <int STORE>
struct TileRep {
    static constexpr bool kRaw = STORE == 1 || STORE == 2;  // own sites' codes kept in registers
    __device__ static __forceinline__ v3 raw(v3 s)
    {
        if constexpr (STORE == 0) return s;
        else if constexpr (STORE == 1)
            return v3{__half2float(__float2half_rn(s.x)), __half2float(__float2half_rn(s.y)),
                      __half2float(__float2half_rn(s.z))};
        else if constexpr (STORE == 2)
            return v3{bf16_to_f32(f32_to_bf16_rne(s.x)), bf16_to_f32(f32_to_bf16_rne(s.y)),
                      bf16_to_f32(f32_to_bf16_rne(s.z))};
        else return oct_decode(oct_encode(s));
    }
    __device__ static __forceinline__ v3 shared(v3 r)
    {
        if constexpr (kRaw) return normalise_rsq(r);
        else return r;
    }
};

// The raw components of a float16 / bfloat16 pair as stored (no renormalisation).
template <int STORE>
__device__ __forceinline__ void load_raw_pair(const typename Codec<STORE>::T *p, uint32_t cs, uint32_t j0, v3 &a,
                                              v3 &b)
{
    if constexpr (STORE == 1) {
        const __half2 x = *reinterpret_cast<const __half2 *>(p + j0);
        const __half2 y = *reinterpret_cast<const __half2 *>(p + cs + j0);
        const __half2 z = *reinterpret_cast<const __half2 *>(p + 2 * cs + j0);
        a = v3{__low2float(x), __low2float(y), __low2float(z)};
        b = v3{__high2float(x), __high2float(y), __high2float(z)};
    } else if constexpr (STORE == 2) {
        const uint32_t x = *reinterpret_cast<const uint32_t *>(p + j0);
        const uint32_t y = *reinterpret_cast<const uint32_t *>(p + cs + j0);
        const uint32_t z = *reinterpret_cast<const uint32_t *>(p + 2 * cs + j0);
        a = v3{__uint_as_float(x << 16), __uint_as_float(y << 16), __uint_as_float(z << 16)};
        b = v3{__uint_as_float(x & 0xFFFF0000u), __uint_as_float(y & 0xFFFF0000u), __uint_as_float(z & 0xFFFF0000u)};
    } else {
        Codec<STORE>::load_pair(p, cs, j0, a, b);
    }
}

// Tile coordinates (X, Y, Z) of the q-th tile of coarse parity `phase`, in the
// order Z, then Y, then X. The first tiled axis (an even count of tiles) takes
// the parity; the axes before it hold one tile.
__device__ __forceinline__ void phase_tile(int q, int phase, int BX, int BY, int &X, int &Y, int &Z)
{
    if (BX > 1) {
        const int per = BX / 2;
        const int yz = q / per;
        Y = yz % BY;
        Z = yz / BY;
        X = 2 * (q - yz * per) + ((Y + Z + phase) & 1);
    } else if (BY > 1) {
        const int per = BY / 2;
        X = 0;
        Z = q / per;
        Y = 2 * (q - Z * per) + ((Z + phase) & 1);
    } else {
        X = 0;
        Y = 0;
        Z = 2 * q + phase;
    }
}

template <int STORE, int KIND>
__device__ __forceinline__ void pair_update(const v3 (&nb0)[6], const v3 (&nb1)[6], const float2 (&jc)[6], v3 hs0,
                                            v3 hs1, v3 old0, v3 old1, u32x4 rr, float beta, bool hw, v3 &s0,
                                            v3 &s1)
{
    v3 h0 = hs0, h1 = hs1;
#pragma unroll
    for (int n = 0; n < 6; ++n) {
        acc3(h0, jc[n].x, nb0[n]);
        acc3(h1, jc[n].y, nb1[n]);
    }
    if (KIND == 1) {
        s0 = over_relax<STORE == 0>(old0, h0);
        s1 = over_relax<STORE == 0>(old1, h1);
    } else if (hw) {
        s0 = heat_bath<true, STORE == 0>(h0, beta, rr.x, rr.y);
        s1 = heat_bath<true, STORE == 0>(h1, beta, rr.z, rr.w);
    } else {
        s0 = heat_bath<false, STORE == 0>(h0, beta, rr.x, rr.y);
        s1 = heat_bath<false, STORE == 0>(h1, beta, rr.z, rr.w);
    }
}

template <int STORE, bool FIELD, bool JB, bool HW>
__global__ __launch_bounds__(1024) void k_tile_visit(TileArgs a)
{
    extern __shared__ float lds[];  // [RB][parity][3][RZ][RY][Lh]
    using C = Codec<STORE>;
    using R = TileRep<STORE>;
    using T = typename C::T;
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int chunk = b % a.n_chunks;
    const int rest = b / a.n_chunks;
    const int q = rest % a.n_tiles_phase;
    const int d = rest / a.n_tiles_phase;  // sample
    int X, Y, Z;
    phase_tile(q, a.phase, a.BX, a.BY, X, Y, Z);
    const int y0 = Y * a.TY, z0 = Z * a.TZ;
    const int L = a.L, Lh = a.Lh, RXh = a.RXh, RY = a.RY, RZ = a.RZ;
    const int xs = a.hx ? (X * a.TX / 2 - 2 + Lh) % Lh : 0;  // half-index of LDS column 0
    const uint32_t Nh = (uint32_t)a.Nh;
    const int cs = RZ * RY * RXh;  // floats per component of one parity of one replica
    const int tid = threadIdx.x;
    const int P = a.P;  // site pairs per parity of the tile
    const int rb = tid / P;
    const int qp = tid - rb * P;
    const int sis = chunk * a.RB + rb;  // replica within the sample
    const bool active = rb < a.RB && sis < a.slots_per_sample;
    const int64_t r = (int64_t)d * a.slots_per_sample + (active ? sis : 0);
    T *base = (T *)a.spins + r * 2 * C::kPlanes * (int64_t)Nh;

    // stage the tile and its halo, both parities, of every replica of the block
    const int Lq = RXh / 2;  // staged site pairs per row and parity
    const int n_pairs = a.RB * 2 * RZ * RY * Lq;
    for (int e = tid; e < n_pairs; e += blockDim.x) {
        int k = e;
        const int xp = k % Lq;
        k /= Lq;
        const int ly = k % RY;
        k /= RY;
        const int lz = k % RZ;
        k /= RZ;
        const int par = k & 1;
        const int rr = k >> 1;
        if (chunk * a.RB + rr >= a.slots_per_sample) continue;
        int y = y0 - a.hy + ly, z = z0 - a.hz + lz;
        y = y < 0 ? y + L : (y >= L ? y - L : y);
        z = z < 0 ? z + L : (z >= L ? z - L : z);
        const int64_t rep = (int64_t)d * a.slots_per_sample + chunk * a.RB + rr;
        const T *src = (const T *)a.spins + (rep * 2 + par) * C::kPlanes * (int64_t)Nh;
        int xh = xs + 2 * xp;  // even, so the pair does not straddle the periodic wrap
        xh = xh >= Lh ? xh - Lh : xh;
        v3 s0, s1;
        C::load_pair(src, Nh, (uint32_t)((z * L + y) * Lh + xh), s0, s1);
        lds_put_pair(lds, ((rr * 2 + par) * 3 * RZ + lz) * RY * RXh + ly * RXh + 2 * xp, cs, s0, s1);
    }

    // my pair, its couplings and field (both parities)
    const int TXq = a.TX / 4;  // site pairs per tile row and parity
    const int lx0 = 2 * (qp % TXq) + 2 * a.hx;  // my first half-index in the LDS row
    const int xh0 = X * a.TX / 2 + 2 * (qp % TXq);
    const int lyi = (qp / TXq) % a.TY, lzi = qp / (TXq * a.TY);
    const int y = y0 + lyi, z = z0 + lzi;
    const int ly = lyi + a.hy, lz = lzi + a.hz;
    const int lym = ly == 0 ? RY - 1 : ly - 1, lyp = ly + 1 == RY ? 0 : ly + 1;  // wrap only without halo
    const int lzm = lz == 0 ? RZ - 1 : lz - 1, lzp = lz + 1 == RZ ? 0 : lz + 1;
    const uint32_t j0 = (uint32_t)((z * L + y) * Lh + xh0);
    float2 jc[2][6];
    v3 hs[2][2];
    float beta = 0.0f;
    uint32_t c2 = 0, uid = a.uid_base + (uint32_t)d;
    if (active) {
#pragma unroll
        for (int par = 0; par < 2; ++par) {
            const float *Jb = a.J6 + ((int64_t)d * 2 + par) * 6 * (int64_t)Nh;
            const uint8_t *Jbb = JB ? a.Jbits + ((int64_t)d * 2 + par) * (int64_t)Nh : nullptr;
            const float *Hb = FIELD ? a.Hp + ((int64_t)d * 2 + par) * 3 * (int64_t)Nh : nullptr;
            load_couplings<JB, FIELD>(Jb, Jbb, Hb, JB, FIELD, Nh, j0, jc[par], hs[par][0], hs[par][1]);
        }
        beta = a.beta32[a.temp_of_slot[r]];
        const int o = sis / a.T, ts = sis - o * a.T;
        c2 = (uint32_t)ts | ((uint32_t)o << 8);
    } else {
#pragma unroll
        for (int par = 0; par < 2; ++par) {
#pragma unroll
            for (int n = 0; n < 6; ++n) jc[par][n] = make_float2(0.f, 0.f);
            hs[par][0] = hs[par][1] = v3{0.f, 0.f, 0.f};
        }
    }
    v3 own_raw[2][2];  // float16 / bfloat16: exact components of my sites' current codes
    if (R::kRaw && active) {
#pragma unroll
        for (int par = 0; par < 2; ++par)
            load_raw_pair<STORE>(base + (int64_t)par * C::kPlanes * Nh, Nh, j0, own_raw[par][0], own_raw[par][1]);
    }
    const uint32_t tsweep = *a.tptr;
    __syncthreads();

    auto at = [&](int par, int pz, int py, int lx) { return ((rb * 2 + par) * 3 * RZ + pz) * RY * RXh + py * RXh + lx; };
    auto rd = [&](int w) { return v3{lds[w], lds[w + cs], lds[w + 2 * cs]}; };
    auto half_round = [&](int kind, int p, uint32_t rep) {
        if (active) {
            const int qo = 1 - p;
            const int o = (y + z + p) & 1;  // x = 2 x/2 + o on this row
            // the x-neighbour that is not one of my two positions (periodic only
            // when the row is whole; with a halo it lies inside the staged row)
            const int xe = o ? (lx0 + 2 == RXh ? 0 : lx0 + 2) : (lx0 == 0 ? RXh - 1 : lx0 - 1);
            const v3 c0 = rd(at(qo, lz, ly, lx0)), c1 = rd(at(qo, lz, ly, lx0 + 1)), ex = rd(at(qo, lz, ly, xe));
            const v3 ym0 = rd(at(qo, lz, lym, lx0)), ym1 = rd(at(qo, lz, lym, lx0 + 1));
            const v3 yp0 = rd(at(qo, lz, lyp, lx0)), yp1 = rd(at(qo, lz, lyp, lx0 + 1));
            const v3 zm0 = rd(at(qo, lzm, ly, lx0)), zm1 = rd(at(qo, lzm, ly, lx0 + 1));
            const v3 zp0 = rd(at(qo, lzp, ly, lx0)), zp1 = rd(at(qo, lzp, ly, lx0 + 1));
            v3 nb0[6], nb1[6];  // neighbours in the order +x, -x, +y, -y, +z, -z
            if (o) {
                nb0[0] = c1; nb0[1] = c0;
                nb1[0] = ex; nb1[1] = c1;
            } else {
                nb0[0] = c0; nb0[1] = ex;
                nb1[0] = c1; nb1[1] = c0;
            }
            nb0[2] = yp0; nb1[2] = yp1;
            nb0[3] = ym0; nb1[3] = ym1;
            nb0[4] = zp0; nb1[4] = zp1;
            nb0[5] = zm0; nb1[5] = zm1;
            const int w = at(p, lz, ly, lx0);
            v3 s0, s1;
            if (kind == 1) {
                const v3 old0 = rd(w), old1 = rd(w + 1);
                pair_update<STORE, 1>(nb0, nb1, jc[p], hs[p][0], hs[p][1], old0, old1, u32x4{0u, 0u, 0u, 0u}, beta,
                                      false, s0, s1);
            } else {
                const u32x4 rr = philox4x32_10(u32x4{j0 >> 1, tsweep, c2 | (rep << 12) | ((uint32_t)p << 16), uid},
                                               a.key0, a.key1);
                pair_update<STORE, 0>(nb0, nb1, jc[p], hs[p][0], hs[p][1], v3{}, v3{}, rr, beta, HW, s0, s1);
            }
            const v3 r0 = R::raw(s0), r1 = R::raw(s1);
            if (R::kRaw) {
                own_raw[p][0] = r0;
                own_raw[p][1] = r1;
            }
            lds_put_pair(lds, w, cs, R::shared(r0), R::shared(r1));
        }
        __syncthreads();
    };

    for (int h = 0; h < a.n_hit; ++h) {
        for (int m = 0; m < a.n_or; ++m) {
            half_round(1, 0, 0u);
            half_round(1, 1, 0u);
        }
        for (int bb = 0; bb < a.n_hb; ++bb) {
            const uint32_t rep = (uint32_t)(h * a.n_hb + bb);
            half_round(0, 0, rep);
            half_round(0, 1, rep);
        }
    }

    // write back my two sites of each parity
    if (active) {
#pragma unroll
        for (int par = 0; par < 2; ++par) {
            v3 s0, s1;
            if (R::kRaw) {
                s0 = own_raw[par][0];
                s1 = own_raw[par][1];
            } else {
                lds_get_pair(lds, at(par, lz, ly, lx0), cs, s0, s1);
            }
            C::store_pair(base + (int64_t)par * C::kPlanes * Nh, Nh, j0, s0, s1);
        }
    }
}

template <int STORE>
static hipError_t launch_tile_s(const TileArgs &a, bool field, bool jb, bool hw, unsigned threads, size_t lds,
                                hipStream_t s)
{
    const dim3 grid((unsigned)a.n_blocks), block(threads);
#define HSG_T(F, J, H) hipLaunchKernelGGL((k_tile_visit<STORE, F, J, H>), grid, block, lds, s, a)
    if (hw) {
        if (field) { if (jb) HSG_T(true, true, true); else HSG_T(true, false, true); }
        else { if (jb) HSG_T(false, true, true); else HSG_T(false, false, true); }
    } else {
        if (field) { if (jb) HSG_T(true, true, false); else HSG_T(true, false, false); }
        else { if (jb) HSG_T(false, true, false); else HSG_T(false, false, false); }
    }
#undef HSG_T
    return hipGetLastError();
}

hipError_t launch_tile_visit(const TileArgs &a, int storage, bool field, bool jb, bool hw, unsigned threads,
                             size_t lds, hipStream_t s)
{
    if (threads == 0 || threads > 1024 || a.n_blocks <= 0) return hipErrorInvalidValue;
    switch (storage) {
    case 0: return launch_tile_s<0>(a, field, jb, hw, threads, lds, s);
    case 1: return launch_tile_s<1>(a, field, jb, hw, threads, lds, s);
    case 2: return launch_tile_s<2>(a, field, jb, hw, threads, lds, s);
    case 3: return launch_tile_s<3>(a, field, jb, hw, threads, lds, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hsg
