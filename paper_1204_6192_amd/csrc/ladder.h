// ladder.h -- per-ladder steps after the updates of a sweep, shared by the
// separate kernels and the persistent launch: the tempering walk of Eq. (4)
// and the run statistics.
#pragma once
#include "device.h"
#include "kernels.h"

namespace hsg {

// One (sample, copy) ladder walks k = 0 .. T-2 from the lowest temperature;
// float64 acceptance exponent (Eq. (4)); temperatures move, spins stay.
// ctr1 is the counter word of the draws (the sweep, or the standalone call).
__device__ __forceinline__ void pt_ladder(const PtArgs &a, int64_t lad, uint32_t ctr1)
{
    const int d = (int)(lad / a.O), o = (int)(lad - (int64_t)d * a.O);
    int32_t *sat = a.slot_at_temp + lad * a.T;
    int32_t *tos = a.temp_of_slot + lad * a.T;
    const double *E = a.E + lad * a.T;
    for (int k = 0; k + 1 < a.T; ++k) {
        const int32_t sa = sat[k], sb = sat[k + 1];
        const double delta = (a.beta64[k + 1] - a.beta64[k]) * (E[sb] - E[sa]);
        const u32x4 r = philox4x32_10(
            u32x4{(uint32_t)k, ctr1, ((uint32_t)o << 8) | (a.purpose << 20), a.uid_base + (uint32_t)d}, a.key0,
            a.key1);
        const double u = u53(r.x, r.y);
        if (delta >= 0.0 || u <= exp(delta)) {
            sat[k] = sb;
            sat[k + 1] = sa;
            tos[sb] = k;
            tos[sa] = k + 1;
            a.accepts[lad * (a.T - 1) + k] += 1ull;
        }
    }
}

// After a sweep: the energy of the configuration at each rung is added to
// float64 sums of E and E^2 (for U_L and C_L), and a replica that reaches the
// lowest rung after visiting the highest since its last visit to the lowest
// completes a round trip. flag per slot: 0 none yet, 1 at the lowest rung
// since, 2 reached the highest rung after that.
__device__ __forceinline__ void stats_ladder(const StatsArgs &a, int64_t lad)
{
    const int32_t *sat = a.slot_at_temp + lad * a.T;
    const double *E = a.E + lad * a.T;
    double *sum = a.sum + lad * a.T * 2;
    for (int k = 0; k < a.T; ++k) {
        const double e = E[sat[k]];
        sum[2 * k] += e;
        sum[2 * k + 1] += e * e;
    }
    if (a.T < 2) return;
    int32_t *flag = a.flag + lad * a.T;
    uint32_t *trips = a.trips + lad * a.T;
    const int32_t lo = sat[0], hi = sat[a.T - 1];
    if (flag[lo] == 2) trips[lo] += 1u;
    flag[lo] = 1;
    if (flag[hi] == 1) flag[hi] = 2;
}

}  // namespace hsg
