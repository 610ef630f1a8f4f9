// sweep_stream.h -- checkerboard half-sweep as a z-march (L divisible by 4).
//
// One work-group owns RB replicas x TY rows (all of x) and walks the planes
// z0 .. z0 + zlen - 1 of one z-slab (the whole lattice, or a slab when a
// launch would otherwise have too few work-groups to keep HBM busy).
// At step z every thread updates the two parity-p sites (x/2 = 2m, 2m + 1) of
// its row in plane z (Eqs. (2) and (3)). Their six neighbours all lie on the
// other parity:
//   - plane z of the other parity is staged in LDS (decoded and renormalised
//     once per site), giving the +-x and +-y neighbours, with periodic wrap;
//   - planes z - 1 and z + 1 at the thread's own two positions stay in
//     registers and roll forward, giving the +-z neighbours.
// So each stored spin of a replica is read from HBM once per half-sweep (plus
// two halo rows per plane when the tile is narrower than the lattice). The
// sample's couplings stay in L2: the replicas of one sample run as consecutive
// work-groups on the same XCD. The arithmetic per site is the one of the
// generic kernel (same neighbour order, same functions), so both produce the
// same bits.
#pragma once
#include <type_traits>

#include "device.h"
#include "kernels.h"

namespace hsg {

// UNI: every wave holds a single replica (TY * P a multiple of 64) and L <= 512,
// so the replica's base addresses are wave-uniform and live in scalar
// registers, and every load and store takes such a base (one per coupling
// plane) plus the lane's 32-bit byte offset: no 64-bit address arithmetic.
// FIELD / JB: some group of the launch has a field / sign-bit couplings (each
// group is then checked at run time); UNI: every group of the launch is UNI.
template <int STORE, int KIND, bool FIELD, bool ENERGY, bool UNI, bool JB>
__device__ __forceinline__ void stream_body(const StreamArgs &a, const int lb, float *lds, double *red)
{
    using C = Codec<STORE>;
    using T = typename C::T;
    const int ytile = lb % a.n_ytiles;
    const int zrest = lb / a.n_ytiles;
    const int zslab = zrest % a.n_zslabs;
    const int rblk = zrest / a.n_zslabs;
    const int z0 = zslab * a.zlen, z1 = z0 + a.zlen;
    const int tid = threadIdx.x;
    const int per_rep = a.TY * a.P;
    const int rb = tid / per_rep;
    const int rem = tid - rb * per_rep;
    const int ty = rem / a.P, m = rem - ty * a.P;
    const int64_t r_lane = a.r_base + (int64_t)rblk * a.RB + rb;  // replica (canonical order within the group)
    const bool active = rb < a.RB && r_lane < a.n_rep;
    const int L = a.L, Lh = a.Lh;
    const uint32_t Nh = (uint32_t)a.Nh;
    const int p = (int)a.parity;
    const bool full = a.TY == L;
    const int y = ytile * a.TY + ty;
    const int lrow = full ? ty : ty + 1;                         // my row in the LDS plane
    const int lrm = full ? (ty == 0 ? L - 1 : ty - 1) : ty;      // row y - 1
    const int lrp = full ? (ty == L - 1 ? 0 : ty + 1) : ty + 2;  // row y + 1
    const int cstride = a.rows * Lh;                             // floats per component plane
    const int xh0 = 2 * m;
    const int rbc = active ? rb : 0;
    const int lbuf[2] = {rbc * 3 * cstride, (a.RB + rbc) * 3 * cstride};

    // Idle lanes read the group's first replica (valid memory) and discard it, so
    // that every global load is issued on every path: the hardware counts
    // outstanding memory operations in issue order, and a wait then names only
    // the loads it needs.
    const int64_t r_first = a.r_base + (int64_t)rblk * a.RB;
    int64_t r = active ? r_lane : r_first;
    if (UNI) r = ((int64_t)__builtin_amdgcn_readfirstlane((int)(r >> 32)) << 32) |
                 (uint32_t)__builtin_amdgcn_readfirstlane((int)(r & 0xFFFFFFFF));
    const int64_t d = r / a.slots_per_sample;
    const int sis = (int)(r - d * a.slots_per_sample);
    T *base = (T *)a.spins + r * 2 * C::kPlanes * (int64_t)Nh;
    T *own = base + (int64_t)p * C::kPlanes * Nh;
    const T *oth = base + (int64_t)(1 - p) * C::kPlanes * Nh;
    const float *Jb = a.J6 + (d * 2 + p) * 6 * (int64_t)Nh;
    const bool jbits = JB && a.Jbits != nullptr;
    const bool field = FIELD && a.Hp != nullptr;
    const uint8_t *Jbb = jbits ? a.Jbits + (d * 2 + p) * (int64_t)Nh : nullptr;
    const float *Hb = field ? a.Hp + (d * 2 + p) * 3 * (int64_t)Nh : nullptr;
    const float *Ho = field ? a.Hp + (d * 2 + (1 - p)) * 3 * (int64_t)Nh : nullptr;
    const float *Jp[6];  // one base per coupling plane (uniform with UNI)
#pragma unroll
    for (int n = 0; n < 6; ++n) Jp[n] = Jb + n * (int64_t)Nh;
    float beta = 0.0f;
    uint32_t c2 = 0, uid = 0;
    const uint32_t tsweep = *a.tptr + a.t_offset;
    if (active) {
        beta = a.beta32[a.temp_of_slot[r]];
        const int o = sis / a.T, ts = sis - o * a.T;
        c2 = (uint32_t)ts | ((uint32_t)o << 8) | (a.rep << 12) | ((uint32_t)p << 16);
        uid = a.uid_base + (uint32_t)d;
    }
    // The halo rows y0 - 1 and y0 + TY of the other parity are staged by the
    // first and last rows' threads; the others load their own row in their place
    // (a cache hit), so the load is issued by every lane.
    const bool halo = !full && (ty == 0 || ty == a.TY - 1);
    const int hy = !halo ? y : (ty == 0) ? (y == 0 ? L - 1 : y - 1) : (y + 1 == L ? 0 : y + 1);
    const int hw_row = (ty == 0) ? 0 : a.TY + 1;
    auto wrapz = [L](int v) { return v >= L ? v - L : v; };

    // Other parity at my two positions: planes z - 1, z, z + 1 decoded and
    // rolling; plane z + 2, the halo row of plane z + 1 and (over-relaxation)
    // my own old spins of plane z + 1 are loaded one step ahead, raw.
    v3 prv0{}, prv1{}, cur0{}, cur1{}, nxt0{}, nxt1{};
    typename C::R nraw, graw, oraw;
    {
        C::template load_pair<UNI>(oth, Nh, (uint32_t)((((z0 == 0 ? L : z0) - 1) * L + y) * Lh + xh0), prv0, prv1);
        C::template load_pair<UNI>(oth, Nh, (uint32_t)((z0 * L + y) * Lh + xh0), cur0, cur1);
        C::template load_raw_pair<UNI>(oth, Nh, (uint32_t)((wrapz(z0 + 1) * L + y) * Lh + xh0), nraw);
        C::template load_raw_pair<UNI>(oth, Nh, (uint32_t)((z0 * L + hy) * Lh + xh0), graw);
        C::template load_raw_pair<UNI>(own, Nh, (uint32_t)((z0 * L + y) * Lh + xh0), oraw);
    }
    double e = 0.0;

    for (int z = z0; z < z1; ++z) {
        const int lo = lbuf[z & 1];
        const uint32_t j0 = (uint32_t)((z * L + y) * Lh + xh0);  // my first site, half-index
        // values that arrived during the last step
        C::decode_pair(nraw, nxt0, nxt1);
        v3 old0{}, old1{};
        if (KIND == 1) C::decode_pair(oraw, old0, old1);
        if (active) {  // stage plane z (my two positions, and the halo rows) in LDS
            const int w = lo + lrow * Lh + xh0;
            *reinterpret_cast<float2 *>(&lds[w]) = make_float2(cur0.x, cur1.x);
            *reinterpret_cast<float2 *>(&lds[w + cstride]) = make_float2(cur0.y, cur1.y);
            *reinterpret_cast<float2 *>(&lds[w + 2 * cstride]) = make_float2(cur0.z, cur1.z);
            if (halo) {  // whole rows: a wave without halo rows skips the decoding
                v3 g0, g1;
                C::decode_pair(graw, g0, g1);
                const int hw = lo + hw_row * Lh + xh0;
                *reinterpret_cast<float2 *>(&lds[hw]) = make_float2(g0.x, g1.x);
                *reinterpret_cast<float2 *>(&lds[hw + cstride]) = make_float2(g0.y, g1.y);
                *reinterpret_cast<float2 *>(&lds[hw + 2 * cstride]) = make_float2(g0.z, g1.z);
            }
        }
        float2 jc[6];
        v3 hs0, hs1;  // +-1 couplings come from sign bits (exactly the float values)
        if constexpr (UNI) load_couplings_planes<JB, FIELD>(Jp, Jbb, Hb, jbits, field, Nh, j0, jc, hs0, hs1);
        else load_couplings<JB, FIELD>(Jb, Jbb, Hb, jbits, field, Nh, j0, jc, hs0, hs1);
        // Loads for the next step go out last, so that waiting for this step's
        // couplings leaves them in flight. At the end of the slab they repeat
        // planes already read (their values are never used).
        __builtin_amdgcn_sched_barrier(0);
        {
            const int zn = z + 1 < z1 ? z + 1 : z;
            C::template load_raw_pair<UNI>(oth, Nh, (uint32_t)((wrapz(z + 2 <= z1 ? z + 2 : z1) * L + y) * Lh + xh0), nraw);
            C::template load_raw_pair<UNI>(oth, Nh, (uint32_t)((zn * L + hy) * Lh + xh0), graw);
            C::template load_raw_pair<UNI>(own, Nh, (uint32_t)((zn * L + y) * Lh + xh0), oraw);
        }
        u32x4 rr{0u, 0u, 0u, 0u};
        if (KIND != 1 && active) rr = philox4x32_10(u32x4{j0 >> 1, tsweep, c2, uid}, a.key0, a.key1);
        __syncthreads();
        if (active) {
            const int o = (y + z + p) & 1;  // x = 2 x/2 + o on this row
            // the x-neighbour that is not one of my own two positions
            const int xe = o ? (xh0 + 2 == Lh ? 0 : xh0 + 2) : (xh0 == 0 ? Lh - 1 : xh0 - 1);
            const int we = lo + lrow * Lh + xe;
            const v3 ex{lds[we], lds[we + cstride], lds[we + 2 * cstride]};
            const int wm = lo + lrm * Lh + xh0, wp = lo + lrp * Lh + xh0;
            const float2 ym0 = *reinterpret_cast<const float2 *>(&lds[wm]);
            const float2 ym1 = *reinterpret_cast<const float2 *>(&lds[wm + cstride]);
            const float2 ym2 = *reinterpret_cast<const float2 *>(&lds[wm + 2 * cstride]);
            const float2 yp0 = *reinterpret_cast<const float2 *>(&lds[wp]);
            const float2 yp1 = *reinterpret_cast<const float2 *>(&lds[wp + cstride]);
            const float2 yp2 = *reinterpret_cast<const float2 *>(&lds[wp + 2 * cstride]);
            // neighbours in the order +x, -x, +y, -y, +z, -z
            v3 nb0[6], nb1[6];
            if (o) {  // site k at x = 2(xh0 + k) + 1: +x -> xh0 + k + 1, -x -> xh0 + k
                nb0[0] = cur1; nb0[1] = cur0;
                nb1[0] = ex;   nb1[1] = cur1;
            } else {  // x = 2(xh0 + k): +x -> xh0 + k, -x -> xh0 + k - 1
                nb0[0] = cur0; nb0[1] = ex;
                nb1[0] = cur1; nb1[1] = cur0;
            }
            nb0[2] = v3{yp0.x, yp1.x, yp2.x};
            nb1[2] = v3{yp0.y, yp1.y, yp2.y};
            nb0[3] = v3{ym0.x, ym1.x, ym2.x};
            nb1[3] = v3{ym0.y, ym1.y, ym2.y};
            nb0[4] = nxt0; nb1[4] = nxt1;
            nb0[5] = prv0; nb1[5] = prv1;
            v3 h0 = hs0, h1 = hs1;
            double hx0 = hs0.x, hy0 = hs0.y, hz0 = hs0.z, hx1 = hs1.x, hy1 = hs1.y, hz1 = hs1.z;
#pragma unroll
            for (int n = 0; n < 6; ++n) {
                acc3(h0, jc[n].x, nb0[n]);
                acc3(h1, jc[n].y, nb1[n]);
                if (ENERGY) {
                    hx0 = fma((double)jc[n].x, (double)nb0[n].x, hx0);
                    hy0 = fma((double)jc[n].x, (double)nb0[n].y, hy0);
                    hz0 = fma((double)jc[n].x, (double)nb0[n].z, hz0);
                    hx1 = fma((double)jc[n].y, (double)nb1[n].x, hx1);
                    hy1 = fma((double)jc[n].y, (double)nb1[n].y, hy1);
                    hz1 = fma((double)jc[n].y, (double)nb1[n].z, hz1);
                }
            }
            v3 s0, s1;
            if (KIND != 1) {
                s0 = heat_bath<KIND == 2, STORE == 0>(h0, beta, rr.x, rr.y);
                s1 = heat_bath<KIND == 2, STORE == 0>(h1, beta, rr.z, rr.w);
            } else {
                s0 = over_relax<STORE == 0>(old0, h0);
                s1 = over_relax<STORE == 0>(old1, h1);
            }
            const typename C::R code = C::encode_pair(s0, s1);
            C::template store_raw_pair<UNI>(own, Nh, j0, code);
            if (ENERGY) {
                // each bond has exactly one endpoint on this (odd) parity; the stored values
                v3 v0, v1;
                C::decode_pair(code, v0, v1);
                e -= (double)v0.x * hx0 + (double)v0.y * hy0 + (double)v0.z * hz0;
                e -= (double)v1.x * hx1 + (double)v1.y * hy1 + (double)v1.z * hz1;
                if (field) {  // field term of the even sites at my two half-indices
                    const float2 fx = *reinterpret_cast<const float2 *>(elem<UNI>(Ho, j0));
                    const float2 fy = *reinterpret_cast<const float2 *>(elem<UNI>(Ho, Nh + j0));
                    const float2 fz = *reinterpret_cast<const float2 *>(elem<UNI>(Ho, 2 * Nh + j0));
                    e -= (double)fx.x * cur0.x + (double)fy.x * cur0.y + (double)fz.x * cur0.z;
                    e -= (double)fx.y * cur1.x + (double)fy.y * cur1.y + (double)fz.y * cur1.z;
                }
            }
        }
        prv0 = cur0; prv1 = cur1;
        cur0 = nxt0; cur1 = nxt1;
    }

    if (ENERGY) {
        red[tid] = e;
        __syncthreads();
        if (tid < a.RB) {
            const int64_t r2 = a.r_base + (int64_t)rblk * a.RB + tid;
            if (r2 < a.n_rep) {
                double s = 0.0;
                for (int k = 0; k < per_rep; ++k) s += red[tid * per_rep + k];
                a.e_partials[(r2 * a.n_ytiles + ytile) * a.n_zslabs + zslab] = s;
            }
        }
    }
}

// ---------------------------------------------------------------- fused pair
// One site pair's update from its six neighbours: the x and y neighbours of
// the plane staged in LDS at offset lo (with the thread's own two positions of
// that plane in c0, c1 and the third x neighbour read from LDS), the z
// neighbours in registers. Same arithmetic and neighbour order as the
// single-pass kernels. Gives the codes of the two new spins and their stored
// values (the codes read back); returns the energy term of the two sites when
// ENERGY.
template <int STORE, int KIND, bool ENERGY>
__device__ __forceinline__ double update_pair(const float *lds, int lo, int cstride, int Lh, int lrow, int lrm,
                                              int lrp, int xh0, int o, v3 c0, v3 c1, v3 zp0, v3 zp1, v3 zm0,
                                              v3 zm1, const float2 (&jc)[6], v3 hs0, v3 hs1, v3 old0, v3 old1,
                                              u32x4 rr, float beta, typename Codec<STORE>::R &code, v3 &s0,
                                              v3 &s1)
{
    using C = Codec<STORE>;
    const int xe = o ? (xh0 + 2 == Lh ? 0 : xh0 + 2) : (xh0 == 0 ? Lh - 1 : xh0 - 1);
    const int we = lo + lrow * Lh + xe;
    const v3 ex{lds[we], lds[we + cstride], lds[we + 2 * cstride]};
    const int wm = lo + lrm * Lh + xh0, wp = lo + lrp * Lh + xh0;
    const float2 ym0 = *reinterpret_cast<const float2 *>(&lds[wm]);
    const float2 ym1 = *reinterpret_cast<const float2 *>(&lds[wm + cstride]);
    const float2 ym2 = *reinterpret_cast<const float2 *>(&lds[wm + 2 * cstride]);
    const float2 yp0 = *reinterpret_cast<const float2 *>(&lds[wp]);
    const float2 yp1 = *reinterpret_cast<const float2 *>(&lds[wp + cstride]);
    const float2 yp2 = *reinterpret_cast<const float2 *>(&lds[wp + 2 * cstride]);
    v3 nb0[6], nb1[6];
    if (o) {
        nb0[0] = c1; nb0[1] = c0;
        nb1[0] = ex; nb1[1] = c1;
    } else {
        nb0[0] = c0; nb0[1] = ex;
        nb1[0] = c1; nb1[1] = c0;
    }
    nb0[2] = v3{yp0.x, yp1.x, yp2.x};
    nb1[2] = v3{yp0.y, yp1.y, yp2.y};
    nb0[3] = v3{ym0.x, ym1.x, ym2.x};
    nb1[3] = v3{ym0.y, ym1.y, ym2.y};
    nb0[4] = zp0; nb1[4] = zp1;
    nb0[5] = zm0; nb1[5] = zm1;
    v3 h0 = hs0, h1 = hs1;
    double hx0 = hs0.x, hy0 = hs0.y, hz0 = hs0.z, hx1 = hs1.x, hy1 = hs1.y, hz1 = hs1.z;
#pragma unroll
    for (int n = 0; n < 6; ++n) {
        acc3(h0, jc[n].x, nb0[n]);
        acc3(h1, jc[n].y, nb1[n]);
        if (ENERGY) {
            hx0 = fma((double)jc[n].x, (double)nb0[n].x, hx0);
            hy0 = fma((double)jc[n].x, (double)nb0[n].y, hy0);
            hz0 = fma((double)jc[n].x, (double)nb0[n].z, hz0);
            hx1 = fma((double)jc[n].y, (double)nb1[n].x, hx1);
            hy1 = fma((double)jc[n].y, (double)nb1[n].y, hy1);
            hz1 = fma((double)jc[n].y, (double)nb1[n].z, hz1);
        }
    }
    v3 n0, n1;
    if (KIND != 1) {
        n0 = heat_bath<KIND == 2, STORE == 0>(h0, beta, rr.x, rr.y);
        n1 = heat_bath<KIND == 2, STORE == 0>(h1, beta, rr.z, rr.w);
    } else {
        n0 = over_relax<STORE == 0>(old0, h0);
        n1 = over_relax<STORE == 0>(old1, h1);
    }
    // the codes, and the values that reading them back gives (the stored values)
    code = C::encode_pair(n0, n1);
    C::decode_pair(code, s0, s1);
    double e = 0.0;
    if (ENERGY) {
        e -= (double)s0.x * hx0 + (double)s0.y * hy0 + (double)s0.z * hz0;
        e -= (double)s1.x * hx1 + (double)s1.y * hy1 + (double)s1.z * hz1;
    }
    return e;
}

// Both half-sweeps of a pair (parity 0, then parity 1, of the same kind) in one
// z-march over whole planes (TY = L). At step z, stage A updates the parity-0
// sites of plane z from the old parity-1 planes z - 1, z, z + 1; stage B then
// updates the parity-1 sites of plane z - 1 from the new parity-0 planes
// z - 2, z - 1, z. The periodic seam is closed after the march: the parity-1
// sites of planes L - 1 and 0 need new parity-0 planes 0 and 1, kept in LDS
// from the first two steps. The result equals the two single half-sweeps bit
// for bit; every stored spin is read and written once per pair. Whole planes
// in one work-group mean L <= 32, so every byte offset into a replica's spins,
// couplings and field fits 32 bits (the fused kernels address that way).
template <int STORE, int KIND, bool FIELD, bool ENERGY, bool UNI, bool JB>
__device__ __forceinline__ void pair_body(const StreamArgs &a, const int lb, float *lds, double *red)
{
    using C = Codec<STORE>;
    using T = typename C::T;
    const int tid = threadIdx.x;
    const int per_rep = a.TY * a.P;
    const int rb = tid / per_rep;
    const int rem = tid - rb * per_rep;
    const int ty = rem / a.P, m = rem - ty * a.P;
    const int64_t r_lane = a.r_base + (int64_t)lb * a.RB + rb;
    const bool active = rb < a.RB && r_lane < a.n_rep;
    const int L = a.L, Lh = a.Lh;
    const uint32_t Nh = (uint32_t)a.Nh;
    const int y = ty;
    const int lrm = ty == 0 ? L - 1 : ty - 1;
    const int lrp = ty == L - 1 ? 0 : ty + 1;
    const int cstride = L * Lh;
    const int xh0 = 2 * m;
    const int rbc = active ? rb : 0;
    const int base_l = rbc * 18 * cstride;  // [A0 A1 B0 B1 S0 S1] x 3 components
    const int lA[2] = {base_l, base_l + 3 * cstride};
    const int lB[2] = {base_l + 6 * cstride, base_l + 9 * cstride};
    const int lS[2] = {base_l + 12 * cstride, base_l + 15 * cstride};
    const int lrow_w = ty * Lh + xh0;

    int64_t r = r_lane;
    if (UNI) r = ((int64_t)__builtin_amdgcn_readfirstlane((int)(r_lane >> 32)) << 32) |
                 (uint32_t)__builtin_amdgcn_readfirstlane((int)(r_lane & 0xFFFFFFFF));
    const int64_t d = r / a.slots_per_sample;
    const int sis = (int)(r - d * a.slots_per_sample);
    T *sp0 = (T *)a.spins + r * 2 * C::kPlanes * (int64_t)Nh;
    T *sp1 = sp0 + (int64_t)C::kPlanes * Nh;
    const bool jbits = JB && a.Jbits != nullptr;
    const bool field = FIELD && a.Hp != nullptr;
    const float *J0 = a.J6 + (d * 2 + 0) * 6 * (int64_t)Nh;
    const float *J1 = a.J6 + (d * 2 + 1) * 6 * (int64_t)Nh;
    const uint8_t *Jb0 = jbits ? a.Jbits + (d * 2 + 0) * (int64_t)Nh : nullptr;
    const uint8_t *Jb1 = jbits ? a.Jbits + (d * 2 + 1) * (int64_t)Nh : nullptr;
    const float *H0 = field ? a.Hp + (d * 2 + 0) * 3 * (int64_t)Nh : nullptr;
    const float *H1 = field ? a.Hp + (d * 2 + 1) * 3 * (int64_t)Nh : nullptr;
    const float *Jp0[6], *Jp1[6];  // one uniform base per coupling plane
#pragma unroll
    for (int n = 0; n < 6; ++n) {
        Jp0[n] = J0 + n * Nh;
        Jp1[n] = J1 + n * Nh;
    }
    float beta = 0.0f;
    uint32_t c2A = 0, c2B = 0, uid = 0;
    const uint32_t tsweep = *a.tptr + a.t_offset;
    if (active) {
        beta = a.beta32[a.temp_of_slot[r]];
        const int o = sis / a.T, ts = sis - o * a.T;
        c2A = (uint32_t)ts | ((uint32_t)o << 8) | (a.rep << 12);
        c2B = c2A | (1u << 16);
        uid = a.uid_base + (uint32_t)d;
    }

    v3 o_prv0{}, o_prv1{}, o_cur0{}, o_cur1{}, o_nxt0{}, o_nxt1{};  // old parity 1, planes z-1, z, z+1
    v3 a_m10{}, a_m11{}, a_m20{}, a_m21{};                          // new parity 0, planes z-1, z-2
    // The spin loads run one step ahead: the old spins step z + 1 needs are
    // issued at the top of step z and land while step z computes. Couplings come
    // from L2 (shared by the sample's replicas) and are loaded within the step.
    v3 o_nn0{}, o_nn1{}, oldA0{}, oldA1{}, oldN0{}, oldN1{};
    float2 jcA[6], jcB[6];
    v3 hA0{}, hA1{}, hB0{}, hB1{};
#pragma unroll
    for (int n = 0; n < 6; ++n) jcB[n] = make_float2(0.f, 0.f);
    if (active) {
        C::template load_pair<true>(sp1, Nh, (uint32_t)(((L - 1) * L + y) * Lh + xh0), o_prv0, o_prv1);
        C::template load_pair<true>(sp1, Nh, (uint32_t)(y * Lh + xh0), o_cur0, o_cur1);
        C::template load_pair<true>(sp1, Nh, (uint32_t)((L + y) * Lh + xh0), o_nxt0, o_nxt1);
        if (KIND == 1) C::template load_pair<true>(sp0, Nh, (uint32_t)(y * Lh + xh0), oldA0, oldA1);
    }
    double e = 0.0;

    for (int z = 0; z < L; ++z) {
        const uint32_t jA = (uint32_t)((z * L + y) * Lh + xh0);
        const uint32_t jB = (uint32_t)(((z - 1) * L + y) * Lh + xh0);  // valid when z >= 1
        const bool doB = z >= 2;
        u32x4 rrA{0u, 0u, 0u, 0u}, rrB{0u, 0u, 0u, 0u};
        if (active) {
            if (z + 1 < L) {  // for step z + 1: old parity 1 of plane z + 2, old parity 0 of plane z + 1
                const int z2 = (z + 2 >= L) ? z + 2 - L : z + 2;
                const uint32_t jA1 = jA + (uint32_t)(L * Lh);
                C::template load_pair<true>(sp1, Nh, (uint32_t)((z2 * L + y) * Lh + xh0), o_nn0, o_nn1);
                if (KIND == 1) C::template load_pair<true>(sp0, Nh, jA1, oldN0, oldN1);
            }
            {
                if constexpr (UNI) load_couplings_planes<JB, FIELD>(Jp0, Jb0, H0, jbits, field, Nh, jA, jcA, hA0, hA1);
                else load_couplings<JB, FIELD, true>(J0, Jb0, H0, jbits, field, Nh, jA, jcA, hA0, hA1);
            }
            if (doB) {
                if constexpr (UNI) load_couplings_planes<JB, FIELD>(Jp1, Jb1, H1, jbits, field, Nh, jB, jcB, hB0, hB1);
                else load_couplings<JB, FIELD, true>(J1, Jb1, H1, jbits, field, Nh, jB, jcB, hB0, hB1);
            }
            lds_put_pair(lds, lA[z & 1] + lrow_w, cstride, o_cur0, o_cur1);
            if (KIND != 1) {
                rrA = philox4x32_10(u32x4{jA >> 1, tsweep, c2A, uid}, a.key0, a.key1);
                if (doB) rrB = philox4x32_10(u32x4{jB >> 1, tsweep, c2B, uid}, a.key0, a.key1);
            }
        }
        __syncthreads();
        if (active) {
            v3 sA0, sA1;  // later stages read the stored (rounded) values, as the single passes do
            typename C::R cA;
            update_pair<STORE, KIND, false>(lds, lA[z & 1], cstride, Lh, ty, lrm, lrp, xh0, (y + z) & 1, o_cur0,
                                            o_cur1, o_nxt0, o_nxt1, o_prv0, o_prv1, jcA, hA0, hA1, oldA0, oldA1, rrA,
                                            beta, cA, sA0, sA1);
            C::template store_raw_pair<true>(sp0, Nh, jA, cA);
            lds_put_pair(lds, lB[z & 1] + lrow_w, cstride, sA0, sA1);
            if (z < 2) lds_put_pair(lds, lS[z] + lrow_w, cstride, sA0, sA1);
            if (doB) {
                v3 sB0, sB1;
                typename C::R cB;
                e += update_pair<STORE, KIND, ENERGY>(lds, lB[(z - 1) & 1], cstride, Lh, ty, lrm, lrp, xh0,
                                                      (y + z) & 1, a_m10, a_m11, sA0, sA1, a_m20, a_m21, jcB, hB0,
                                                      hB1, o_prv0, o_prv1, rrB, beta, cB, sB0, sB1);
                C::template store_raw_pair<true>(sp1, Nh, jB, cB);
                if (ENERGY && field) {  // field on the parity-0 sites at the same half-indices
                    const float2 fx = *reinterpret_cast<const float2 *>(elem<true>(H0, jB));
                    const float2 fy = *reinterpret_cast<const float2 *>(elem<true>(H0, Nh + jB));
                    const float2 fz = *reinterpret_cast<const float2 *>(elem<true>(H0, 2 * Nh + jB));
                    e -= (double)fx.x * a_m10.x + (double)fy.x * a_m10.y + (double)fz.x * a_m10.z;
                    e -= (double)fx.y * a_m11.x + (double)fy.y * a_m11.y + (double)fz.y * a_m11.z;
                }
            }
            a_m20 = a_m10; a_m21 = a_m11;
            a_m10 = sA0; a_m11 = sA1;
        }
        o_prv0 = o_cur0; o_prv1 = o_cur1;
        o_cur0 = o_nxt0; o_cur1 = o_nxt1;
        o_nxt0 = o_nn0; o_nxt1 = o_nn1;
        oldA0 = oldN0; oldA1 = oldN1;
    }

    // seam: parity-1 sites of planes L - 1 and 0
    {
        const uint32_t jL = (uint32_t)(((L - 1) * L + y) * Lh + xh0);
        const uint32_t j0 = (uint32_t)(y * Lh + xh0);
        float2 jcL[6], jc0[6];
        v3 hL0, hL1, hZ0, hZ1;
        u32x4 rrL{0u, 0u, 0u, 0u}, rr0{0u, 0u, 0u, 0u};
        if (active) {
            {
                if constexpr (UNI) load_couplings_planes<JB, FIELD>(Jp1, Jb1, H1, jbits, field, Nh, jL, jcL, hL0, hL1);
                else load_couplings<JB, FIELD, true>(J1, Jb1, H1, jbits, field, Nh, jL, jcL, hL0, hL1);
            }
            {
                if constexpr (UNI) load_couplings_planes<JB, FIELD>(Jp1, Jb1, H1, jbits, field, Nh, j0, jc0, hZ0, hZ1);
                else load_couplings<JB, FIELD, true>(J1, Jb1, H1, jbits, field, Nh, j0, jc0, hZ0, hZ1);
            }
            if (KIND != 1) {
                rrL = philox4x32_10(u32x4{jL >> 1, tsweep, c2B, uid}, a.key0, a.key1);
                rr0 = philox4x32_10(u32x4{j0 >> 1, tsweep, c2B, uid}, a.key0, a.key1);
            }
        }
        __syncthreads();  // the parity-0 plane L - 1 written at the last step
        if (active) {
            v3 n00, n01, n10, n11;  // new parity 0, planes 0 and 1, my positions
            lds_get_pair(lds, lS[0] + lrow_w, cstride, n00, n01);
            lds_get_pair(lds, lS[1] + lrow_w, cstride, n10, n11);
            v3 sL0, sL1, sZ0, sZ1;
            typename C::R cL, cZ;
            // plane L - 1: parity-0 neighbours L - 2 (a_m2), L - 1 (a_m1, LDS B), 0 (saved)
            e += update_pair<STORE, KIND, ENERGY>(lds, lB[(L - 1) & 1], cstride, Lh, ty, lrm, lrp, xh0,
                                                  (y + L) & 1, a_m10, a_m11, n00, n01, a_m20, a_m21, jcL, hL0, hL1,
                                                  o_prv0, o_prv1, rrL, beta, cL, sL0, sL1);
            // plane 0: parity-0 neighbours L - 1 (a_m1), 0 (saved, LDS S0), 1 (saved)
            e += update_pair<STORE, KIND, ENERGY>(lds, lS[0], cstride, Lh, ty, lrm, lrp, xh0, (y + 1) & 1, n00,
                                                  n01, n10, n11, a_m10, a_m11, jc0, hZ0, hZ1, o_cur0, o_cur1, rr0,
                                                  beta, cZ, sZ0, sZ1);
            C::template store_raw_pair<true>(sp1, Nh, jL, cL);
            C::template store_raw_pair<true>(sp1, Nh, j0, cZ);
            if (ENERGY && field) {
                const float2 fx = *reinterpret_cast<const float2 *>(elem<true>(H0, jL));
                const float2 fy = *reinterpret_cast<const float2 *>(elem<true>(H0, Nh + jL));
                const float2 fz = *reinterpret_cast<const float2 *>(elem<true>(H0, 2 * Nh + jL));
                e -= (double)fx.x * a_m10.x + (double)fy.x * a_m10.y + (double)fz.x * a_m10.z;
                e -= (double)fx.y * a_m11.x + (double)fy.y * a_m11.y + (double)fz.y * a_m11.z;
                const float2 gx = *reinterpret_cast<const float2 *>(elem<true>(H0, j0));
                const float2 gy = *reinterpret_cast<const float2 *>(elem<true>(H0, Nh + j0));
                const float2 gz = *reinterpret_cast<const float2 *>(elem<true>(H0, 2 * Nh + j0));
                e -= (double)gx.x * n00.x + (double)gy.x * n00.y + (double)gz.x * n00.z;
                e -= (double)gx.y * n01.x + (double)gy.y * n01.y + (double)gz.y * n01.z;
            }
        }
    }

    if (ENERGY) {
        red[tid] = e;
        __syncthreads();
        if (tid < a.RB) {
            const int64_t r2 = a.r_base + (int64_t)lb * a.RB + tid;
            if (r2 < a.n_rep) {
                double sum = 0.0;
                for (int k = 0; k < per_rep; ++k) sum += red[tid * per_rep + k];
                a.e_partials[r2 * a.n_ytiles] = sum;
            }
        }
    }
}

// Two over-relaxation pairs (four half-sweeps: parity 0, 1, 0, 1) in one z-march
// over whole planes (TY = L). Stage s = 0 .. 3 updates parity s & 1; at step z
// it works on plane w = z - s (mod L), for the steps 2s .. 2s + L - 1, so it
// visits the planes s, s + 1, ..., L - 1, 0, ..., s - 1. Its inputs come from
// stage s - 1 (stage 0: the old parity-1 planes): plane w + 1 made earlier in
// the same step, plane w made one step before (staged in LDS for the in-plane
// neighbours) and plane w - 1 made two steps before; over-relaxation also needs
// the site's own value from stage s - 2 (stages 0 and 1: the old spins). The
// last two planes of a stage need the first two planes of the stages before
// it, made at the start of the march: the first is kept in LDS, the second at
// the thread's own positions in registers. Only stages 2 and 3 store, so every
// stored spin is read and written once per four half-sweeps; every stage
// rounds its output through the storage codec as a stored and reloaded
// half-sweep would, and the result equals four single half-sweeps bit for bit.
__device__ __forceinline__ v3 pick(bool c, v3 a, v3 b)
{
    return v3{c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z};
}

template <int STORE, bool FIELD, bool ENERGY, bool UNI, bool JB>
__device__ __forceinline__ void quad_body(const StreamArgs &a, const int lb, float *lds, double *red)
{
    constexpr int D = 4;  // half-sweeps per march
    using C = Codec<STORE>;
    using T = typename C::T;
    const int tid = threadIdx.x;
    const int per_rep = a.TY * a.P;
    const int rb = tid / per_rep;
    const int rem = tid - rb * per_rep;
    const int ty = rem / a.P, m = rem - ty * a.P;
    const int64_t r_first = a.r_base + (int64_t)lb * a.RB;  // the group's first replica (always present)
    const int64_t r_lane = r_first + rb;
    const bool active = rb < a.RB && r_lane < a.n_rep;
    const int L = a.L, Lh = a.Lh;
    const uint32_t Nh = (uint32_t)a.Nh;
    const int y = ty;
    const int lrm = ty == 0 ? L - 1 : ty - 1;
    const int lrp = ty == L - 1 ? 0 : ty + 1;
    const int cstride = L * Lh;
    const int xh0 = 2 * m;
    const int rbc = active ? rb : 0;
    const int pl = 3 * cstride;  // floats per staged plane
    // per replica: IN[2] (old parity 1), RING[s][2] and SAVED[s] for s < D - 1
    const int base_l = rbc * (3 * D - 1) * pl;
    const int lrow_w = ty * Lh + xh0;
    auto l_in = [&](int k) { return base_l + k * pl; };
    auto l_ring = [&](int s, int k) { return base_l + (2 + 2 * s + k) * pl; };
    auto l_saved = [&](int s) { return base_l + (2 * D + s) * pl; };

    // Idle lanes read the group's first replica (valid memory) and discard it:
    // every global load is issued on every path, so the hardware's in-order
    // count of outstanding memory operations lets each wait below name exactly
    // the loads it needs.
    int64_t r = active ? r_lane : r_first;
    if (UNI) r = ((int64_t)__builtin_amdgcn_readfirstlane((int)(r >> 32)) << 32) |
                 (uint32_t)__builtin_amdgcn_readfirstlane((int)(r & 0xFFFFFFFF));
    const int64_t d = r / a.slots_per_sample;
    T *sp0 = (T *)a.spins + r * 2 * C::kPlanes * (int64_t)Nh;
    T *sp1 = sp0 + (int64_t)C::kPlanes * Nh;
    const bool jbits = JB && a.Jbits != nullptr;
    const bool field = FIELD && a.Hp != nullptr;
    const float *J0 = a.J6 + (d * 2 + 0) * 6 * (int64_t)Nh;
    const float *J1 = a.J6 + (d * 2 + 1) * 6 * (int64_t)Nh;
    const uint8_t *Jb0 = jbits ? a.Jbits + (d * 2 + 0) * (int64_t)Nh : nullptr;
    const uint8_t *Jb1 = jbits ? a.Jbits + (d * 2 + 1) * (int64_t)Nh : nullptr;
    const float *H0 = field ? a.Hp + (d * 2 + 0) * 3 * (int64_t)Nh : nullptr;
    const float *H1 = field ? a.Hp + (d * 2 + 1) * 3 * (int64_t)Nh : nullptr;
    // one base per coupling plane: uniform, so each load is that base plus the
    // lane's byte offset, with no per-load address arithmetic
    const float *Jp[2][6];
#pragma unroll
    for (int n = 0; n < 6; ++n) {
        Jp[0][n] = J0 + n * Nh;
        Jp[1][n] = J1 + n * Nh;
    }

    // The loaded spins are addressed by the step modulo 4 (the march is
    // unrolled by four, so the indices are constants and a load lands where it
    // is used): old parity-1 spins at my positions, slot (z' mod 4) for planes
    // z' = z - 1 .. z + 2 of the march; old parity-0 spins, slot (z' mod 2) for
    // z' = z, z + 1. Stage outputs at my positions roll forward: slot 0 this
    // step, 1 and 2 one and two steps before. Then the second plane of each
    // stage but the last.
    v3 ia[4], ib[4], oa[2], ob[2];
    v3 qa[D - 1][3], qb[D - 1][3];
    v3 fa[D - 1], fb[D - 1];
#pragma unroll
    for (int k = 0; k < 4; ++k) ia[k] = ib[k] = v3{0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < D - 1; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k) qa[s][k] = qb[s][k] = v3{0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < D - 1; ++s) fa[s] = fb[s] = v3{0.f, 0.f, 0.f};
    oa[1] = ob[1] = v3{0.f, 0.f, 0.f};
    C::template load_pair<true>(sp1, Nh, (uint32_t)(((L - 1) * L + y) * Lh + xh0), ia[3], ib[3]);
    C::template load_pair<true>(sp1, Nh, (uint32_t)(y * Lh + xh0), ia[0], ib[0]);
    C::template load_pair<true>(sp1, Nh, (uint32_t)((L + y) * Lh + xh0), ia[1], ib[1]);
    C::template load_pair<true>(sp0, Nh, (uint32_t)(y * Lh + xh0), oa[0], ob[0]);
    double e = 0.0;
    const int n_steps = L + 2 * (D - 1);
    auto wrap = [L](int v) {
        while (v >= L) v -= L;
        return v;
    };

    // F: a step of the steady state (8 <= z, z + 3 < L), where every stage is
    // active and takes all its inputs from registers and the LDS ring.
    auto step = [&](auto kc, auto fc, const int z) __attribute__((always_inline)) {
        constexpr int K = decltype(kc)::value;  // z mod 4
        constexpr bool F = decltype(fc)::value;
        float2 jc[D][6];
        v3 hs0[D], hs1[D];
        if (active && (F || z < L)) lds_put_pair(lds, l_in(K & 1) + lrow_w, cstride, ia[K], ib[K]);
#pragma unroll
        for (int s = 0; s < D; ++s) {  // every stage's couplings, also for the steps it idles
            const uint32_t jw = (uint32_t)((wrap(z + L - s) * L + y) * Lh + xh0);
            // per-plane bases pay off where they are uniform (scalar registers);
            // per lane they would cost 24 vector registers
            if constexpr (UNI) {
                if (s & 1) load_couplings_planes<JB, FIELD>(Jp[1], Jb1, H1, jbits, field, Nh, jw, jc[s], hs0[s], hs1[s]);
                else load_couplings_planes<JB, FIELD>(Jp[0], Jb0, H0, jbits, field, Nh, jw, jc[s], hs0[s], hs1[s]);
            } else {
                if (s & 1) load_couplings<JB, FIELD, true>(J1, Jb1, H1, jbits, field, Nh, jw, jc[s], hs0[s], hs1[s]);
                else load_couplings<JB, FIELD, true>(J0, Jb0, H0, jbits, field, Nh, jw, jc[s], hs0[s], hs1[s]);
            }
        }
        // The spin loads for the next step go out last, so that the waits for
        // this step's couplings leave them in flight. Past the end of the march
        // their values are never used: they repeat the last loads (cache hits).
        __builtin_amdgcn_sched_barrier(0);
        const int zi = z + 1 < L ? wrap(z + 2) : 0, zo = z + 1 < L ? z + 1 : L - 1;
        C::template load_pair<true>(sp1, Nh, (uint32_t)((zi * L + y) * Lh + xh0), ia[(K + 2) & 3], ib[(K + 2) & 3]);
        C::template load_pair<true>(sp0, Nh, (uint32_t)((zo * L + y) * Lh + xh0), oa[(K + 1) & 1], ob[(K + 1) & 1]);
        __syncthreads();
        // one stage; written as a function of a constant so that every register
        // index is known before the compiler places the arrays
        auto stage = [&](auto sc) __attribute__((always_inline)) {
            constexpr int s = decltype(sc)::value;
            const int i = z - 2 * s;
            if constexpr (!F)
                if (i < 0 || i >= L) return;
            const int w = wrap(z + L - s);
            const uint32_t jw = (uint32_t)((w * L + y) * Lh + xh0);
            const int o = (y + w + (s & 1)) & 1;
            int lo;
            v3 c0, c1, zp0, zp1, zm0, zm1, od0, od1;
            if constexpr (s == 0) {
                lo = l_in(K & 1);
                c0 = ia[K]; c1 = ib[K];
                zp0 = ia[(K + 1) & 3]; zp1 = ib[(K + 1) & 3];
                zm0 = ia[(K + 3) & 3]; zm1 = ib[(K + 3) & 3];
                od0 = oa[K & 1]; od1 = ob[K & 1];
            } else if constexpr (F) {
                lo = l_ring(s - 1, (K + 1) & 1);
                c0 = qa[s - 1][1]; c1 = qb[s - 1][1];
                zp0 = qa[s - 1][0]; zp1 = qb[s - 1][0];
                zm0 = qa[s - 1][2]; zm1 = qb[s - 1][2];
                if constexpr (s == 1) {
                    od0 = ia[(K + 3) & 3]; od1 = ib[(K + 3) & 3];
                } else {
                    od0 = qa[s - 2][2]; od1 = qb[s - 2][2];
                }
            } else {
                // The first plane of stage s - 1 (and of s - 2) at my positions is
                // read from LDS every time and picked by value: a branch between a
                // register and an LDS read would make the compiler address the
                // registers through memory.
                v3 g0, g1, h0, h1;
                lds_get_pair(lds, l_saved(s - 1) + lrow_w, cstride, g0, g1);
                if constexpr (s >= 2) lds_get_pair(lds, l_saved(s - 2) + lrow_w, cstride, h0, h1);
                else h0 = h1 = v3{0.f, 0.f, 0.f};
                const bool c_ring = i <= L - 2;  // plane w of stage s - 1, made one step before, else its first
                lo = c_ring ? l_ring(s - 1, (K + 1) & 1) : l_saved(s - 1);
                c0 = pick(c_ring, qa[s - 1][1], g0);
                c1 = pick(c_ring, qb[s - 1][1], g1);
                // plane w + 1 of stage s - 1: made earlier in this step, else its first or second plane
                zp0 = pick(i <= L - 3, qa[s - 1][0], pick(i == L - 2, g0, fa[s - 1]));
                zp1 = pick(i <= L - 3, qb[s - 1][0], pick(i == L - 2, g1, fb[s - 1]));
                zm0 = qa[s - 1][2]; zm1 = qb[s - 1][2];
                if constexpr (s == 1) {  // the old parity-1 spin of plane w = z - 1
                    od0 = ia[(K + 3) & 3]; od1 = ib[(K + 3) & 3];
                } else {
                    od0 = pick(i <= L - 3, qa[s - 2][2], pick(i == L - 2, h0, fa[s - 2]));
                    od1 = pick(i <= L - 3, qb[s - 2][2], pick(i == L - 2, h1, fb[s - 2]));
                }
            }
            v3 r0, r1;  // the stored values of the new spins
            typename C::R code;
            if constexpr (s == D - 1) {
                e += update_pair<STORE, 1, ENERGY>(lds, lo, cstride, Lh, ty, lrm, lrp, xh0, o, c0, c1, zp0, zp1, zm0,
                                                   zm1, jc[s], hs0[s], hs1[s], od0, od1, u32x4{0u, 0u, 0u, 0u}, 0.0f,
                                                   code, r0, r1);
                if (ENERGY && field) {  // field on the parity-0 sites at the same half-indices: stage D - 2
                    const float2 fx = *reinterpret_cast<const float2 *>(elem<true>(H0, jw));
                    const float2 fy = *reinterpret_cast<const float2 *>(elem<true>(H0, Nh + jw));
                    const float2 fz = *reinterpret_cast<const float2 *>(elem<true>(H0, 2 * Nh + jw));
                    e -= (double)fx.x * c0.x + (double)fy.x * c0.y + (double)fz.x * c0.z;
                    e -= (double)fx.y * c1.x + (double)fy.y * c1.y + (double)fz.y * c1.z;
                }
            } else {
                (void)update_pair<STORE, 1, false>(lds, lo, cstride, Lh, ty, lrm, lrp, xh0, o, c0, c1, zp0, zp1, zm0,
                                                   zm1, jc[s], hs0[s], hs1[s], od0, od1, u32x4{0u, 0u, 0u, 0u}, 0.0f,
                                                   code, r0, r1);
            }
            if (s >= D - 2) C::template store_raw_pair<true>((s & 1) ? sp1 : sp0, Nh, jw, code);
            if constexpr (s < D - 1) {
                lds_put_pair(lds, l_ring(s, K & 1) + lrow_w, cstride, r0, r1);
                if constexpr (!F) {
                    if (i == 0) lds_put_pair(lds, l_saved(s) + lrow_w, cstride, r0, r1);
                    if (i == 1) { fa[s] = r0; fb[s] = r1; }
                }
                qa[s][0] = r0; qb[s][0] = r1;
            }
        };
        if (active) {
            stage(std::integral_constant<int, 0>{});
            stage(std::integral_constant<int, 1>{});
            stage(std::integral_constant<int, 2>{});
            stage(std::integral_constant<int, 3>{});
        }
        static_assert(D == 4, "the stages are listed by hand");
#pragma unroll
        for (int s = 0; s < D - 1; ++s) {
            qa[s][2] = qa[s][1]; qb[s][2] = qb[s][1];
            qa[s][1] = qa[s][0]; qb[s][1] = qb[s][0];
        }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using G = std::false_type;
    using S = std::true_type;
    // n_steps = L + 6 >= 10, so the first two groups of four are whole. The
    // last group stops at n_steps (the test is uniform over the work-group, so
    // every thread meets the same barriers); the spin loads that the last step
    // issued for the next one are dropped.
    int z = 0;
    for (; z < 8 && z < n_steps; z += 4) {
        step(I0{}, G{}, z);
        step(I1{}, G{}, z + 1);
        step(I2{}, G{}, z + 2);
        step(I3{}, G{}, z + 3);
    }
    for (; z + 4 <= L; z += 4) {
        step(I0{}, S{}, z);
        step(I1{}, S{}, z + 1);
        step(I2{}, S{}, z + 2);
        step(I3{}, S{}, z + 3);
    }
    for (; z < n_steps; z += 4) {
        step(I0{}, G{}, z);
        if (z + 1 >= n_steps) break;
        step(I1{}, G{}, z + 1);
        if (z + 2 >= n_steps) break;
        step(I2{}, G{}, z + 2);
        if (z + 3 >= n_steps) break;
        step(I3{}, G{}, z + 3);
    }

    if (ENERGY) {
        red[tid] = e;
        __syncthreads();
        if (tid < a.RB) {
            const int64_t r2 = a.r_base + (int64_t)lb * a.RB + tid;
            if (r2 < a.n_rep) {
                double sum = 0.0;
                for (int k = 0; k < per_rep; ++k) sum += red[tid * per_rep + k];
                a.e_partials[r2 * a.n_ytiles] = sum;
            }
        }
    }
}

template <int STORE, bool ENERGY, bool FIELD, bool UNI, bool JB>
__global__ __launch_bounds__(kBlock) void k_or_quad_stream(MultiStreamArgs m)
{
    extern __shared__ float lds[];  // [RB][IN0 IN1 R00 R01 R10 R11 R20 R21 S0 S1 S2][3][L][L/2] floats
    __shared__ double red[kBlock];
    const int b = xcd_remap((int)blockIdx.x, m.n_blocks);
    int k = 0;
    while (k + 1 < m.n_groups && b >= m.block_start[k + 1]) ++k;
    quad_body<STORE, FIELD, ENERGY, UNI, JB>(m.g[k], b - m.block_start[k], lds, red);
}

template <int STORE, int KIND, bool ENERGY, bool FIELD, bool UNI, bool JB>
__global__ __launch_bounds__(kBlock) void k_pair_stream(MultiStreamArgs m)
{
    extern __shared__ float lds[];  // [RB][A0 A1 B0 B1 S0 S1][3][L][L/2] floats of the group
    __shared__ double red[kBlock];
    const int b = xcd_remap((int)blockIdx.x, m.n_blocks);
    int k = 0;
    while (k + 1 < m.n_groups && b >= m.block_start[k + 1]) ++k;
    pair_body<STORE, KIND, FIELD, ENERGY, UNI, JB>(m.g[k], b - m.block_start[k], lds, red);
}

// One launch for every group of the table.
template <int STORE, int KIND, bool ENERGY, bool FIELD, bool UNI, bool JB>
__global__ __launch_bounds__(kBlock) void k_half_sweep_stream(MultiStreamArgs m)
{
    extern __shared__ float lds[];  // two buffers of [RB][3][rows][Lh] floats of the group
    __shared__ double red[kBlock];
    const int b = xcd_remap((int)blockIdx.x, m.n_blocks);
    int k = 0;
    while (k + 1 < m.n_groups && b >= m.block_start[k + 1]) ++k;
    stream_body<STORE, KIND, FIELD, ENERGY, UNI, JB>(m.g[k], b - m.block_start[k], lds, red);
}

// fuse: 0 one half-sweep, 1 a pair, 2 two over-relaxation pairs.
template <int STORE, int KIND, bool ENERGY>
static hipError_t launch_stream_e(const MultiStreamArgs &m, int fuse, bool field, bool uni, bool jb, dim3 grid,
                                  dim3 block, size_t lds_bytes, hipStream_t s)
{
    if (fuse == 2 && KIND != 1) return hipErrorInvalidValue;
#define HSG_L(F, U, J)                                                                                        \
    do {                                                                                                      \
        if constexpr (KIND == 1) {                                                                            \
            if (fuse == 2) {                                                                                  \
                hipLaunchKernelGGL((k_or_quad_stream<STORE, ENERGY, F, U, J>), grid, block, lds_bytes, s, m); \
                break;                                                                                        \
            }                                                                                                 \
        }                                                                                                     \
        if (fuse == 1) hipLaunchKernelGGL((k_pair_stream<STORE, KIND, ENERGY, F, U, J>), grid, block, lds_bytes, s, m); \
        else hipLaunchKernelGGL((k_half_sweep_stream<STORE, KIND, ENERGY, F, U, J>), grid, block, lds_bytes, s, m); \
    } while (0)
    if (field) {
        if (uni) { if (jb) HSG_L(true, true, true); else HSG_L(true, true, false); }
        else { if (jb) HSG_L(true, false, true); else HSG_L(true, false, false); }
    } else {
        if (uni) { if (jb) HSG_L(false, true, true); else HSG_L(false, true, false); }
        else { if (jb) HSG_L(false, false, true); else HSG_L(false, false, false); }
    }
#undef HSG_L
    return hipGetLastError();
}

template <int STORE>
hipError_t launch_stream_s(const MultiStreamArgs &m, int kind, bool energy, int fuse, unsigned threads,
                           size_t lds_bytes, hipStream_t s)
{
    bool field = false, uni = true, jb = false;
    for (int k = 0; k < m.n_groups; ++k) {
        field = field || m.g[k].Hp != nullptr;
        // 32-bit byte offsets within a replica's spins and a sample's couplings: 6 Nh 4 B < 2^32
        uni = uni && (m.g[k].TY * m.g[k].P) % 64 == 0 && m.g[k].L <= 512;
        jb = jb || m.g[k].Jbits != nullptr;
    }
    const dim3 grid((unsigned)m.n_blocks), block(threads);
    if (kind == 0) {
        if (energy) return launch_stream_e<STORE, 0, true>(m, fuse, field, uni, jb, grid, block, lds_bytes, s);
        return launch_stream_e<STORE, 0, false>(m, fuse, field, uni, jb, grid, block, lds_bytes, s);
    }
    if (kind == 2) {
        if (energy) return launch_stream_e<STORE, 2, true>(m, fuse, field, uni, jb, grid, block, lds_bytes, s);
        return launch_stream_e<STORE, 2, false>(m, fuse, field, uni, jb, grid, block, lds_bytes, s);
    }
    if (energy) return launch_stream_e<STORE, 1, true>(m, fuse, field, uni, jb, grid, block, lds_bytes, s);
    return launch_stream_e<STORE, 1, false>(m, fuse, field, uni, jb, grid, block, lds_bytes, s);
}

}  // namespace hsg
