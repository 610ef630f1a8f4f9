/*
 * hsg_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, serial, double-precision CPU model of the Monte-Carlo sweep of the
 * three-dimensional Edwards-Anderson Heisenberg spin glass of
 * T. Yavors'kii and M. Weigel, "Optimized GPU simulation of continuous-spin
 * glass models", arXiv:1204.6192. Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it. It shares no code, header, table or
 * helper with the HIP library; the only thing the two have in common is the
 * seeded input generator that feeds both.
 *
 * Everything here is written for readability, not speed: one site at a time,
 * in canonical order, in float64. Inputs arrive as float64 arrays (the float32
 * instance promoted exactly).
 *
 * Conventions (fixed once, used by both implementations):
 *   site index        i = x + L (y + L z), periodic in all three directions;
 *   parity            (x + y + z) mod 2; "even" (parity 0) is updated first;
 *   spins             [sample d][copy o][slot s][component mu][site i];
 *   couplings         J[d][a][i] couples site i to i + e_a, a = x, y, z;
 *   field             H[d][mu][i], or NULL for H = 0;
 *   temperature map   slot_at_temp[d][o][k]: slot currently at rung k;
 *                     rung k has inverse temperature beta[k], beta decreasing.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key =
 * the 64-bit seed, counter = (c0, c1, c2, c3) with
 *   heat bath:  c0 = i >> 2, c1 = sweep t, c3 = sample uid,
 *               c2 = slot | copy << 8 | hb-repetition << 12 | parity << 16;
 *               the parity-p site with (i >> 1) even uses words (x0, x1), the
 *               other one sharing the block uses (x2, x3).
 *   tempering:  c0 = rung pair k, c1 = sweep t (or call count), c3 = sample uid,
 *               c2 = copy << 8 | purpose << 20, purpose 1 in-sweep, 2 standalone.
 *
 * Parity status of each function is listed with it; see the tests for the pins.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define HSGO_PI 3.14159265358979323846
#define HSGO_HB 0
#define HSGO_OR 1

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: ten rounds of the Philox S-box with the published           */
/* multipliers and Weyl key increments (Salmon et al., SC'11, Sec. 5).        */
/* Pinned against rocRAND's independent implementation.                       */
/* ------------------------------------------------------------------------ */
void hsgo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0, 1] from the top 24 bits of a word; exact in float and double. */
double hsgo_u24(uint32_t x) { return ((double)(x >> 8) + 1.0) * 0x1p-24; }

/* Uniform in (0, 1] with 53 bits from two words; exact in double. */
double hsgo_u53(uint32_t a, uint32_t b)
{
    uint64_t m = ((uint64_t)a << 21) ^ (uint64_t)(b >> 11);
    return ((double)m + 1.0) * 0x1p-53;
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void normalise3(double v[3])
{
    double n = sqrt(dot3(v, v));
    v[0] /= n; v[1] /= n; v[2] /= n;
}

/* Orthonormal frame (e1, e2) with e1 x e2 = n for a unit vector n, after
 * J. R. Frisvad, "Building an orthonormal basis from a 3D unit vector without
 * normalization", J. Graphics Tools 16(3), 2012:
 *   e1 = (1 - nx^2 a, -nx ny a, -nx),  e2 = (-nx ny a, 1 - ny^2 a, -ny),
 *   a = 1 / (1 + nz).
 * For nz < 0 the same 1 + nz is formed as (nx^2 + ny^2) / (1 - nz), which does
 * not cancel. The frame is continuous on the sphere except at nz = -1, where it
 * takes its limit along nx > 0, ny = 0: e1 = (-1, 0, 0), e2 = (0, 1, 0). */
void hsgo_frame(const double n[3], double e1[3], double e2[3])
{
    double a;
    if (n[2] >= 0.0) {
        a = 1.0 / (1.0 + n[2]);
    } else {
        double rxy = n[0] * n[0] + n[1] * n[1];
        if (rxy == 0.0) {
            e1[0] = -1.0; e1[1] = 0.0; e1[2] = 0.0;
            e2[0] = 0.0;  e2[1] = 1.0; e2[2] = 0.0;
            return;
        }
        a = (1.0 - n[2]) / rxy;
    }
    double b = -n[0] * n[1] * a;
    e1[0] = 1.0 - n[0] * n[0] * a;
    e1[1] = b;
    e1[2] = -n[0];
    e2[0] = b;
    e2[1] = 1.0 - n[1] * n[1] * a;
    e2[2] = -n[1];
}

/* Heat-bath draw, Eq. (2): the new spin has density proportional to
 * exp(beta h . s) on the unit sphere. With kappa = beta |h| and c = cos of the
 * angle to h, p(c) ~ exp(kappa c) on [-1, 1]; its CDF
 *   F(c) = (exp(kappa c) - exp(-kappa)) / (exp(kappa) - exp(-kappa))
 * inverts to c = 1 + ln(u + (1 - u) exp(-2 kappa)) / kappa, written with
 * log1p/expm1. The azimuth is phi = 2 pi u2 about h. For h = 0 the draw is
 * uniform (c = 2 u1 - 1) in the frame of the z axis. */
void hsgo_hb_draw(const double h[3], double beta, uint32_t x0, uint32_t x1, double out[3])
{
    double u1 = hsgo_u24(x0);
    double u2 = hsgo_u24(x1);
    double hn = sqrt(dot3(h, h));
    double n[3], e1[3], e2[3], c;
    double kappa = beta * hn;
    if (hn == 0.0 || kappa == 0.0) {
        n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
        c = 2.0 * u1 - 1.0;
    } else {
        n[0] = h[0] / hn; n[1] = h[1] / hn; n[2] = h[2] / hn;
        c = 1.0 + log1p((1.0 - u1) * expm1(-2.0 * kappa)) / kappa;
        if (c > 1.0) c = 1.0;
        if (c < -1.0) c = -1.0;
    }
    hsgo_frame(n, e1, e2);
    double st = sqrt((1.0 - c) * (1.0 + c));
    double phi = 2.0 * HSGO_PI * u2;
    double cp = cos(phi), sp = sin(phi);
    for (int m = 0; m < 3; ++m) out[m] = c * n[m] + st * (cp * e1[m] + sp * e2[m]);
    normalise3(out);
}

/* Over-relaxation, Eq. (3): reflect s about the local field h. A zero field
 * leaves the spin unchanged (Eq. (3) is undefined there). */
void hsgo_or_reflect(const double s[3], const double h[3], double out[3])
{
    double hh = dot3(h, h);
    if (hh == 0.0) {
        out[0] = s[0]; out[1] = s[1]; out[2] = s[2];
        return;
    }
    double f = 2.0 * dot3(s, h) / hh;
    double r[3];
    for (int m = 0; m < 3; ++m) r[m] = f * h[m] - s[m];
    normalise3(r);
    out[0] = r[0]; out[1] = r[1]; out[2] = r[2];
}

/* ------------------------------------------------------------------------ */
/* Lattice helpers.                                                          */
/* ------------------------------------------------------------------------ */
static int64_t site(int L, int x, int y, int z)
{
    x = (x % L + L) % L;
    y = (y % L + L) % L;
    z = (z % L + L) % L;
    return (int64_t)x + (int64_t)L * ((int64_t)y + (int64_t)L * (int64_t)z);
}

/* Local molecular field of Eq. (2): H_eff(i) = sum_j J_ij s_j + H_i over the six
 * nearest neighbours. J, H, s point at one sample's / one slot's arrays. */
static void local_field(int L, const double *J, const double *H, const double *s,
                        int x, int y, int z, double h[3])
{
    const int64_t N = (int64_t)L * L * L;
    int64_t i = site(L, x, y, z);
    int64_t up[3] = {site(L, x + 1, y, z), site(L, x, y + 1, z), site(L, x, y, z + 1)};
    int64_t dn[3] = {site(L, x - 1, y, z), site(L, x, y - 1, z), site(L, x, y, z - 1)};
    for (int m = 0; m < 3; ++m) h[m] = 0.0;
    for (int a = 0; a < 3; ++a) {
        double jf = J[a * N + i];      /* bond i -- i + e_a */
        double jb = J[a * N + dn[a]];  /* bond i - e_a -- i */
        for (int m = 0; m < 3; ++m)
            h[m] += jf * s[m * N + up[a]] + jb * s[m * N + dn[a]];
    }
    if (H != NULL)
        for (int m = 0; m < 3; ++m) h[m] += H[m * N + i];
}

/* Energy of one replica, Eq. (1): every nearest-neighbour bond counted once. */
double hsgo_energy(int L, const double *J, const double *H, const double *s)
{
    const int64_t N = (int64_t)L * L * L;
    double e = 0.0;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                int64_t i = site(L, x, y, z);
                int64_t up[3] = {site(L, x + 1, y, z), site(L, x, y + 1, z),
                                 site(L, x, y, z + 1)};
                for (int a = 0; a < 3; ++a) {
                    double sd = 0.0;
                    for (int m = 0; m < 3; ++m) sd += s[m * N + i] * s[m * N + up[a]];
                    e -= J[a * N + i] * sd;
                }
                if (H != NULL)
                    for (int m = 0; m < 3; ++m) e -= H[m * N + i] * s[m * N + i];
            }
    return e;
}

/* ------------------------------------------------------------------------ */
/* Group description and the sweep.                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t L, n_samples, n_copies, n_temps;
    int32_t n_hb, n_or, pt_every;
    uint32_t sample_uid_base;
    uint64_t seed;
} hsgo_cfg;

static void key_of(const hsgo_cfg *c, uint32_t key[2])
{
    key[0] = (uint32_t)(c->seed & 0xffffffffu);
    key[1] = (uint32_t)(c->seed >> 32);
}

/* The two words a parity-p site draws in heat-bath repetition `rep` of sweep t. */
void hsgo_hb_words(const hsgo_cfg *c, int d, int o, int slot, int rep, int parity,
                   uint32_t t, int64_t i, uint32_t w[2])
{
    uint32_t key[2], ctr[4], r[4];
    key_of(c, key);
    ctr[0] = (uint32_t)(i >> 2);
    ctr[1] = t;
    ctr[2] = (uint32_t)slot | ((uint32_t)o << 8) | ((uint32_t)rep << 12) |
             ((uint32_t)parity << 16);
    ctr[3] = c->sample_uid_base + (uint32_t)d;
    hsgo_philox4x32_10(ctr, key, r);
    if (((i >> 1) & 1) == 0) { w[0] = r[0]; w[1] = r[1]; }
    else                     { w[0] = r[2]; w[1] = r[3]; }
}

/* Storage emulation: after every update the spin is passed through this hook.
 * Mode 0 keeps float64. Modes 1..3 round each component (float16, bfloat16)
 * or the encoded angle to the stored precision and renormalise, mirroring
 * compressed spin storage. */
static int g_storage_mode = 0;
void hsgo_set_storage_mode(int mode) { g_storage_mode = mode; }
void hsgo_store_roundtrip(int mode, double s[3]);

/* Sensitivity probe (tests only): with eps > 0, every updated component is
 * multiplied by (1 + eps r), r uniform in [-1, 1) from a SplitMix64 stream,
 * before the storage rounding. eps = 2^-24 mimics float32 rounding of every
 * stored spin; runs with different noise seeds show how far two correct
 * trajectories drift apart. eps = 0 (the default) leaves the chain exact. */
static double g_noise_eps = 0.0;
static uint64_t g_noise_state = 0;
void hsgo_set_noise(double eps, uint64_t seed) { g_noise_eps = eps; g_noise_state = seed; }
static double noise_uniform(void)
{
    uint64_t z = (g_noise_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1p-52 - 1.0;
}

/* One half-sweep of one slot: every site of parity `parity` gets a heat-bath
 * draw (kind 0) or an over-relaxation reflection (kind 1). Sites of one parity
 * only see the other parity through H_eff, so the in-place update is exact.
 * `order`, if not NULL, lists the visiting order of the N/2 sites of this parity
 * as indices into the canonical enumeration of that parity (for the test that
 * the result does not depend on the order). */
/* One site's update in place: a heat-bath draw (kind 0) or an over-relaxation
 * reflection (kind 1) from the current neighbours, then the storage hook. */
static void update_site(const hsgo_cfg *c, const double *J, const double *H, double *s,
                        int d, int o, int slot, double beta, int kind, int rep, int parity,
                        uint32_t t, int64_t i)
{
    const int L = c->L;
    const int64_t N = (int64_t)L * L * L;
    int x = (int)(i % L), y = (int)((i / L) % L), z = (int)(i / ((int64_t)L * L));
    double h[3], sn[3], so[3];
    local_field(L, J, H, s, x, y, z, h);
    if (kind == HSGO_HB) {
        uint32_t w[2];
        hsgo_hb_words(c, d, o, slot, rep, parity, t, i, w);
        hsgo_hb_draw(h, beta, w[0], w[1], sn);
    } else {
        for (int m = 0; m < 3; ++m) so[m] = s[m * N + i];
        hsgo_or_reflect(so, h, sn);
    }
    if (g_noise_eps > 0.0)
        for (int m = 0; m < 3; ++m) sn[m] *= 1.0 + g_noise_eps * noise_uniform();
    hsgo_store_roundtrip(g_storage_mode, sn);
    for (int m = 0; m < 3; ++m) s[m * N + i] = sn[m];
}

/* One half-sweep of one slot: every site of parity `parity` gets a heat-bath
 * draw (kind 0) or an over-relaxation reflection (kind 1). Sites of one parity
 * only see the other parity through H_eff, so the in-place update is exact.
 * `order`, if not NULL, lists the visiting order of the N/2 sites of this parity
 * as indices into the canonical enumeration of that parity (for the test that
 * the result does not depend on the order). */
static void half_sweep_slot(const hsgo_cfg *c, const double *J, const double *H,
                            double *s, int d, int o, int slot, double beta,
                            int kind, int rep, int parity, uint32_t t,
                            const int64_t *order)
{
    const int L = c->L;
    const int64_t N = (int64_t)L * L * L;
    /* canonical list of the sites of this parity */
    int64_t *sites = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N / 2));
    int64_t n = 0;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x)
                if (((x + y + z) & 1) == parity) sites[n++] = site(L, x, y, z);
    for (int64_t q = 0; q < n; ++q)
        update_site(c, J, H, s, d, o, slot, beta, kind, rep, parity, t, sites[order ? order[q] : q]);
    free(sites);
}

static int rung_of_slot(const hsgo_cfg *c, const int32_t *sat, int d, int o, int slot)
{
    const int32_t *row = sat + ((int64_t)d * c->n_copies + o) * c->n_temps;
    for (int k = 0; k < c->n_temps; ++k)
        if (row[k] == slot) return k;
    return -1;
}

static double *slot_ptr(const hsgo_cfg *c, double *spins, int d, int o, int s)
{
    const int64_t N = (int64_t)c->L * c->L * c->L;
    return spins + (((int64_t)d * c->n_copies + o) * c->n_temps + s) * 3 * N;
}

/* One half-sweep of the whole group (every sample, copy and slot). */
int hsgo_half_sweep(const hsgo_cfg *c, const double *J, const double *H, double *spins,
                    const int32_t *slot_at_temp, const double *beta, int kind, int rep,
                    int parity, uint32_t t, const int64_t *order)
{
    const int64_t N = (int64_t)c->L * c->L * c->L;
    for (int d = 0; d < c->n_samples; ++d)
        for (int o = 0; o < c->n_copies; ++o)
            for (int s = 0; s < c->n_temps; ++s) {
                int k = rung_of_slot(c, slot_at_temp, d, o, s);
                if (k < 0) return -1;
                half_sweep_slot(c, J + (int64_t)d * 3 * N, H ? H + (int64_t)d * 3 * N : NULL,
                                slot_ptr(c, spins, d, o, s), d, o, s, beta[k], kind, rep,
                                parity, t, order);
            }
    return 0;
}

/* Parallel tempering, Eq. (4): for each (sample, copy) ladder, attempt swaps of
 * rungs k and k+1 for k = 0 .. R_T - 2 in order, starting at the lowest
 * temperature, with acceptance min[1, exp((beta_{k+1} - beta_k)(E_{k+1} - E_k))].
 * Temperatures move, spins stay in their slots. */
int hsgo_pt_pass(const hsgo_cfg *c, const double *E, int32_t *slot_at_temp,
                 const double *beta, uint32_t ctr1, uint32_t purpose, uint64_t *accepts)
{
    uint32_t key[2];
    key_of(c, key);
    for (int d = 0; d < c->n_samples; ++d)
        for (int o = 0; o < c->n_copies; ++o) {
            int32_t *row = slot_at_temp + ((int64_t)d * c->n_copies + o) * c->n_temps;
            const double *Eo = E + ((int64_t)d * c->n_copies + o) * c->n_temps;
            for (int k = 0; k + 1 < c->n_temps; ++k) {
                int a = row[k], b = row[k + 1];
                double delta = (beta[k + 1] - beta[k]) * (Eo[b] - Eo[a]);
                uint32_t ctr[4] = {(uint32_t)k, ctr1, ((uint32_t)o << 8) | (purpose << 20),
                                   c->sample_uid_base + (uint32_t)d};
                uint32_t r[4];
                hsgo_philox4x32_10(ctr, key, r);
                double u = hsgo_u53(r[0], r[1]);
                if (delta >= 0.0 || u <= exp(delta)) {
                    row[k] = b;
                    row[k + 1] = a;
                    if (accepts)
                        accepts[((int64_t)d * c->n_copies + o) * (c->n_temps - 1) + k] += 1;
                }
            }
        }
    return 0;
}

/* Energies of every slot, E[d][o][s]. */
void hsgo_energies(const hsgo_cfg *c, const double *J, const double *H, const double *spins,
                   double *E)
{
    const int64_t N = (int64_t)c->L * c->L * c->L;
    for (int d = 0; d < c->n_samples; ++d)
        for (int o = 0; o < c->n_copies; ++o)
            for (int s = 0; s < c->n_temps; ++s)
                E[((int64_t)d * c->n_copies + o) * c->n_temps + s] =
                    hsgo_energy(c->L, J + (int64_t)d * 3 * N,
                                H ? H + (int64_t)d * 3 * N : NULL,
                                slot_ptr(c, (double *)spins, d, o, s));
}

/* `n_sweeps` full sweeps starting at sweep counter *t. One sweep: n_hb heat-bath
 * half-sweep pairs (even, odd), then n_or over-relaxation pairs, then the exact
 * energy of each slot, then a tempering pass if (t + 1) is a multiple of
 * pt_every. On return *t has advanced by n_sweeps. E must hold R energies. */
int hsgo_sweep(const hsgo_cfg *c, const double *J, const double *H, double *spins,
               int32_t *slot_at_temp, const double *beta, double *E, uint64_t *t,
               int n_sweeps, uint64_t *accepts)
{
    for (int it = 0; it < n_sweeps; ++it) {
        uint32_t tt = (uint32_t)(*t);
        for (int rep = 0; rep < c->n_hb; ++rep)
            for (int p = 0; p < 2; ++p)
                if (hsgo_half_sweep(c, J, H, spins, slot_at_temp, beta, HSGO_HB, rep, p, tt,
                                    NULL))
                    return -1;
        for (int r = 0; r < c->n_or; ++r)
            for (int p = 0; p < 2; ++p)
                if (hsgo_half_sweep(c, J, H, spins, slot_at_temp, beta, HSGO_OR, 0, p, tt,
                                    NULL))
                    return -1;
        hsgo_energies(c, J, H, spins, E);
        if (c->pt_every > 0 && ((*t + 1) % (uint64_t)c->pt_every) == 0)
            hsgo_pt_pass(c, E, slot_at_temp, beta, tt, 1u, accepts);
        *t += 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The tile-local chain of the double checkerboard decomposition (§3.1 and    */
/* the numbered Monte Carlo procedure of §3.2).                               */
/* ------------------------------------------------------------------------ */
/* The lattice is cut into tiles of tx x ty x tz sites. Every edge divides L,
 * and the number of tiles along each axis is 1 (the tile wraps around that
 * axis) or even, so tiles of equal coarse parity (X + Y + Z) mod 2 of their
 * tile coordinates never share a face. One sweep visits every tile of coarse
 * parity 0, then every tile of coarse parity 1. On a visit, the tile's spins
 * get n_hit repetitions of: n_or over-relaxation rounds, then n_hb heat-bath
 * rounds, where a round updates all even sites of the tile and then all odd
 * sites (global parity). Spins outside the tile (its halo) belong to tiles of
 * the other coarse parity and stay fixed during the visit, so the visits of
 * one coarse parity are independent of each other. Heat-bath round b of
 * repetition r draws with repetition index r n_hb + b of the counter map.
 * Then the exact energies and a tempering pass, as in hsgo_sweep.
 * `tile_order`, if not NULL, gives the order in which the tiles of each coarse
 * parity are visited (indices into the canonical enumeration of that parity's
 * tiles; for the test that the order does not matter). */
typedef struct {
    int32_t tx, ty, tz, n_hit;
} hsgo_tiles;

int hsgo_tiles_valid(int L, const hsgo_tiles *tl, int n_hb)
{
    const int e[3] = {tl->tx, tl->ty, tl->tz};
    for (int a = 0; a < 3; ++a) {
        if (e[a] < 1 || L % e[a] != 0) return 0;
        int b = L / e[a];
        if (b != 1 && (b & 1)) return 0;
    }
    if (tl->n_hit < 1 || tl->n_hit * n_hb > 16) return 0;
    return 1;
}

static void tile_round(const hsgo_cfg *c, const double *J, const double *H, double *s, int d,
                       int o, int slot, double beta, int kind, int rep, uint32_t t, int x0,
                       int y0, int z0, const hsgo_tiles *tl)
{
    for (int p = 0; p < 2; ++p)
        for (int z = z0; z < z0 + tl->tz; ++z)
            for (int y = y0; y < y0 + tl->ty; ++y)
                for (int x = x0; x < x0 + tl->tx; ++x)
                    if (((x + y + z) & 1) == p)
                        update_site(c, J, H, s, d, o, slot, beta, kind, rep, p, t,
                                    site(c->L, x, y, z));
}

int hsgo_tile_sweep(const hsgo_cfg *c, const hsgo_tiles *tl, const double *J, const double *H,
                    double *spins, int32_t *slot_at_temp, const double *beta, double *E,
                    uint64_t *t, int n_sweeps, uint64_t *accepts, const int64_t *tile_order)
{
    const int L = c->L;
    const int64_t N = (int64_t)L * L * L;
    if (!hsgo_tiles_valid(L, tl, c->n_hb)) return -2;
    const int bx = L / tl->tx, by = L / tl->ty, bz = L / tl->tz;
    const int64_t nt = (int64_t)bx * by * bz;
    int64_t *tiles = (int64_t *)malloc(sizeof(int64_t) * (size_t)nt);
    for (int it = 0; it < n_sweeps; ++it) {
        uint32_t tt = (uint32_t)(*t);
        for (int cp = 0; cp < 2; ++cp) {
            /* canonical list of the tiles of coarse parity cp */
            int64_t n = 0;
            for (int Z = 0; Z < bz; ++Z)
                for (int Y = 0; Y < by; ++Y)
                    for (int X = 0; X < bx; ++X)
                        if (((X + Y + Z) & 1) == cp) tiles[n++] = X + (int64_t)bx * (Y + (int64_t)by * Z);
            for (int64_t q = 0; q < n; ++q) {
                int64_t T = tiles[tile_order ? tile_order[q] : q];
                int X = (int)(T % bx), Y = (int)((T / bx) % by), Z = (int)(T / ((int64_t)bx * by));
                for (int d = 0; d < c->n_samples; ++d)
                    for (int o = 0; o < c->n_copies; ++o)
                        for (int sl = 0; sl < c->n_temps; ++sl) {
                            int k = rung_of_slot(c, slot_at_temp, d, o, sl);
                            if (k < 0) { free(tiles); return -1; }
                            const double *Jd = J + (int64_t)d * 3 * N;
                            const double *Hd = H ? H + (int64_t)d * 3 * N : NULL;
                            double *sp = slot_ptr(c, spins, d, o, sl);
                            for (int r = 0; r < tl->n_hit; ++r) {
                                for (int m = 0; m < c->n_or; ++m)
                                    tile_round(c, Jd, Hd, sp, d, o, sl, beta[k], HSGO_OR, 0, tt,
                                               X * tl->tx, Y * tl->ty, Z * tl->tz, tl);
                                for (int b = 0; b < c->n_hb; ++b)
                                    tile_round(c, Jd, Hd, sp, d, o, sl, beta[k], HSGO_HB,
                                               r * c->n_hb + b, tt, X * tl->tx, Y * tl->ty,
                                               Z * tl->tz, tl);
                            }
                        }
            }
        }
        hsgo_energies(c, J, H, spins, E);
        if (c->pt_every > 0 && ((*t + 1) % (uint64_t)c->pt_every) == 0)
            hsgo_pt_pass(c, E, slot_at_temp, beta, tt, 1u, accepts);
        *t += 1;
    }
    free(tiles);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Wave-vector dependent and chiral overlaps (the analysis quantities of §2).  */
/* ------------------------------------------------------------------------ */
/* For every sample d and rung k, between copy 0 (1) and copy 1 (2) at that rung:
 *   q^{mu nu}(k) = (1/N) sum_i s_i^mu(1) s_i^nu(2) exp(i k.R_i) for k = 0 and
 *   k = (2 pi / L) e_a, a = x, y, z (the wave-vector dependent overlap of §2);
 *   kappa_i^alpha = s_{i+alpha} . (s_i x s_{i-alpha}) for alpha = x, y, z, each
 *   copy (the local chirality of three spins on a line), and
 *   q_c^alpha(k) = (1/N) sum_i kappa_i^alpha(1) kappa_i^alpha(2) exp(i k.R_i)
 *   (the chiral overlap, Eq. (12)) at the same four wave vectors.
 * out[(d T + k) 84 + m]:
 *   m = 0..8: q^{mu nu}(0), index 3 mu + nu;
 *   m = 9 + 18 a + 2 (3 mu + nu) + {0, 1}: Re, Im q^{mu nu}(k_a), a = 0, 1, 2 (x, y, z);
 *   m = 63 + 7 alpha: q_c^alpha(0);
 *   m = 63 + 7 alpha + 1 + 2 a + {0, 1}: Re, Im q_c^alpha(k_a).
 * Sums in float64 in the canonical site order. */
#define HSGO_KMODES 84
#define HSGO_TWO_PI 6.283185307179586476925286766559

void hsgo_kmodes(const hsgo_cfg *c, const double *spins, const int32_t *slot_at_temp,
                 double *out)
{
    const int L = c->L;
    const int64_t N = (int64_t)L * L * L;
    const double w0 = HSGO_TWO_PI / (double)L;
    for (int d = 0; d < c->n_samples; ++d)
        for (int k = 0; k < c->n_temps; ++k) {
            const int32_t s1 = slot_at_temp[((int64_t)d * c->n_copies + 0) * c->n_temps + k];
            const int32_t s2 = slot_at_temp[((int64_t)d * c->n_copies + 1) * c->n_temps + k];
            const double *a = slot_ptr(c, (double *)spins, d, 0, s1);
            const double *b = slot_ptr(c, (double *)spins, d, 1, s2);
            double acc[HSGO_KMODES];
            for (int m = 0; m < HSGO_KMODES; ++m) acc[m] = 0.0;
            for (int z = 0; z < L; ++z)
                for (int y = 0; y < L; ++y)
                    for (int x = 0; x < L; ++x) {
                        const int64_t i = site(L, x, y, z);
                        const int R[3] = {x, y, z};
                        double cph[3], sph[3];
                        for (int ax = 0; ax < 3; ++ax) {
                            cph[ax] = cos(w0 * R[ax]);
                            sph[ax] = sin(w0 * R[ax]);
                        }
                        for (int mu = 0; mu < 3; ++mu)
                            for (int nu = 0; nu < 3; ++nu) {
                                const double f = a[mu * N + i] * b[nu * N + i];
                                acc[3 * mu + nu] += f;
                                for (int ax = 0; ax < 3; ++ax) {
                                    acc[9 + 18 * ax + 2 * (3 * mu + nu)] += f * cph[ax];
                                    acc[9 + 18 * ax + 2 * (3 * mu + nu) + 1] += f * sph[ax];
                                }
                            }
                        for (int al = 0; al < 3; ++al) {
                            const int dx = al == 0, dy = al == 1, dz = al == 2;
                            const int64_t ip = site(L, x + dx, y + dy, z + dz);
                            const int64_t im = site(L, x - dx, y - dy, z - dz);
                            double kap[2];
                            for (int cp = 0; cp < 2; ++cp) {
                                const double *s = cp ? b : a;
                                const double u[3] = {s[ip], s[N + ip], s[2 * N + ip]};
                                const double v[3] = {s[i], s[N + i], s[2 * N + i]};
                                const double w[3] = {s[im], s[N + im], s[2 * N + im]};
                                const double cr[3] = {v[1] * w[2] - v[2] * w[1], v[2] * w[0] - v[0] * w[2],
                                                      v[0] * w[1] - v[1] * w[0]};
                                kap[cp] = u[0] * cr[0] + u[1] * cr[1] + u[2] * cr[2];
                            }
                            const double g = kap[0] * kap[1];
                            acc[63 + 7 * al] += g;
                            for (int ax = 0; ax < 3; ++ax) {
                                acc[63 + 7 * al + 1 + 2 * ax] += g * cph[ax];
                                acc[63 + 7 * al + 1 + 2 * ax + 1] += g * sph[ax];
                            }
                        }
                    }
            double *o = out + ((int64_t)d * c->n_temps + k) * HSGO_KMODES;
            for (int m = 0; m < HSGO_KMODES; ++m) o[m] = acc[m] / (double)N;
        }
}

/* Local-overlap Fourier sums for the connected susceptibility with more than two
 * copies (the four-replica estimators, Eqs. (9)-(11)): summing the estimators'
 * integrands over mu and nu leaves products of local overlaps s_i(a) . s_i(b),
 * so every chi_1, chi_2, chi_3 of Eq. (9) is a product of
 *   A_ab(k) = (1/N) sum_i (s_i(a) . s_i(b)) exp(i k.R_i)
 * over copy pairs (a, b) at the same rung: chi_1 = N^2 |A_12|^2, chi_2 =
 * N^2 A_13 conj(A_14), chi_3 = N^2 A_13 conj(A_24) (copies numbered from 1).
 * For every sample d, rung k and pair a < b (in the order (0,1), (0,2), ...,
 * (0,O-1), (1,2), ...), out[((d T + k) P + pair) 7 + m] with P = O (O - 1) / 2:
 *   m = 0: A_ab(0); m = 1 + 2 ax + {0, 1}: Re, Im A_ab(k_ax), ax = x, y, z. */
void hsgo_pair_overlaps(const hsgo_cfg *c, const double *spins, const int32_t *slot_at_temp,
                        double *out)
{
    const int L = c->L, O = c->n_copies;
    const int64_t N = (int64_t)L * L * L;
    const int P = O * (O - 1) / 2;
    const double w0 = HSGO_TWO_PI / (double)L;
    for (int d = 0; d < c->n_samples; ++d)
        for (int k = 0; k < c->n_temps; ++k) {
            int pair = 0;
            for (int a = 0; a < O; ++a)
                for (int b = a + 1; b < O; ++b, ++pair) {
                    const int32_t sa = slot_at_temp[((int64_t)d * O + a) * c->n_temps + k];
                    const int32_t sb = slot_at_temp[((int64_t)d * O + b) * c->n_temps + k];
                    const double *u = slot_ptr(c, (double *)spins, d, a, sa);
                    const double *v = slot_ptr(c, (double *)spins, d, b, sb);
                    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
                    for (int z = 0; z < L; ++z)
                        for (int y = 0; y < L; ++y)
                            for (int x = 0; x < L; ++x) {
                                const int64_t i = site(L, x, y, z);
                                const double f = u[i] * v[i] + u[N + i] * v[N + i] + u[2 * N + i] * v[2 * N + i];
                                const int R[3] = {x, y, z};
                                acc[0] += f;
                                for (int ax = 0; ax < 3; ++ax) {
                                    acc[1 + 2 * ax] += f * cos(w0 * R[ax]);
                                    acc[2 + 2 * ax] += f * sin(w0 * R[ax]);
                                }
                            }
                    double *o = out + (((int64_t)d * c->n_temps + k) * P + pair) * 7;
                    for (int m = 0; m < 7; ++m) o[m] = acc[m] / (double)N;
                }
        }
}

/* Edwards-Anderson overlap, Eq. (5), between copies 0 and 1 at every rung:
 * q[d][k][3 mu + nu] = (1/N) sum_i s_i^mu(copy 0) s_i^nu(copy 1), q[d][k][9] =
 * sum over mu, nu of q^2. */
void hsgo_overlap(const hsgo_cfg *c, const double *spins, const int32_t *slot_at_temp,
                  double *q)
{
    const int64_t N = (int64_t)c->L * c->L * c->L;
    for (int d = 0; d < c->n_samples; ++d)
        for (int k = 0; k < c->n_temps; ++k) {
            int sa = slot_at_temp[((int64_t)d * c->n_copies + 0) * c->n_temps + k];
            int sb = slot_at_temp[((int64_t)d * c->n_copies + 1) * c->n_temps + k];
            const double *A = slot_ptr(c, (double *)spins, d, 0, sa);
            const double *B = slot_ptr(c, (double *)spins, d, 1, sb);
            double *out = q + ((int64_t)d * c->n_temps + k) * 10;
            double q2 = 0.0;
            for (int mu = 0; mu < 3; ++mu)
                for (int nu = 0; nu < 3; ++nu) {
                    double acc = 0.0;
                    for (int64_t i = 0; i < N; ++i) acc += A[mu * N + i] * B[nu * N + i];
                    out[3 * mu + nu] = acc / (double)N;
                    q2 += out[3 * mu + nu] * out[3 * mu + nu];
                }
            out[9] = q2;
        }
}

/* ------------------------------------------------------------------------ */
/* Compressed-storage emulation (parity of the compressed storage modes).    */
/* ------------------------------------------------------------------------ */

/* Round a double to the nearest IEEE binary16 value (ties to even), returned
 * as a double. Overflow saturates to +-65504 is not needed: |v| <= 1. */
double hsgo_round_f16(double v)
{
    if (v == 0.0 || !isfinite(v)) return v;
    double a = fabs(v);
    int e;
    frexp(a, &e);              /* a = m 2^e, m in [0.5, 1) */
    int exp_unb = e - 1;       /* a in [2^exp_unb, 2^(exp_unb+1)) */
    if (exp_unb < -14) exp_unb = -14;  /* subnormal range: fixed quantum 2^-24 */
    double quantum = ldexp(1.0, exp_unb - 10);
    double r = nearbyint(a / quantum) * quantum;  /* default rounding: ties to even */
    return copysign(r, v);
}

/* Round a double to the nearest bfloat16 value (8 significant bits, ties to even). */
double hsgo_round_bf16(double v)
{
    if (v == 0.0 || !isfinite(v)) return v;
    double a = fabs(v);
    int e;
    frexp(a, &e);
    int exp_unb = e - 1;
    if (exp_unb < -126) exp_unb = -126;
    double quantum = ldexp(1.0, exp_unb - 7);
    double r = nearbyint(a / quantum) * quantum;
    return copysign(r, v);
}

/* Quantised-angle storage: the octahedral map of a unit vector (Cigolle,
 * Donow, Evangelakos, Mara, McGuire, Meyer, "A Survey of Efficient
 * Representations for Independent Unit Vectors", JCGT 3(2), 2014). v is
 * projected onto the octahedron |x| + |y| + |z| = 1; the lower half (z < 0) is
 * folded over the diagonals; the two coordinates in [-1, 1] are stored as 16-bit
 * signed normalised integers q = round_to_nearest_even(c * 32767). sgn(0) = +1. */
static double sgn_nz(double a) { return a >= 0.0 ? 1.0 : -1.0; }

void hsgo_oct_encode(const double v[3], int32_t q[2])
{
    double l1 = fabs(v[0]) + fabs(v[1]) + fabs(v[2]);
    double px = v[0] / l1, py = v[1] / l1;
    if (v[2] < 0.0) {
        double fx = (1.0 - fabs(py)) * sgn_nz(px);
        double fy = (1.0 - fabs(px)) * sgn_nz(py);
        px = fx;
        py = fy;
    }
    if (px > 1.0) px = 1.0;
    if (px < -1.0) px = -1.0;
    if (py > 1.0) py = 1.0;
    if (py < -1.0) py = -1.0;
    q[0] = (int32_t)nearbyint(px * 32767.0);
    q[1] = (int32_t)nearbyint(py * 32767.0);
}

void hsgo_oct_decode(const int32_t q[2], double v[3])
{
    double fx = (double)q[0] / 32767.0, fy = (double)q[1] / 32767.0;
    double vz = 1.0 - fabs(fx) - fabs(fy);
    if (vz < 0.0) {
        double ax = (1.0 - fabs(fy)) * sgn_nz(fx);
        double ay = (1.0 - fabs(fx)) * sgn_nz(fy);
        fx = ax;
        fy = ay;
    }
    v[0] = fx;
    v[1] = fy;
    v[2] = vz;
    normalise3(v);
}

void hsgo_store_roundtrip(int mode, double s[3])
{
    if (mode == 0) return;
    if (mode == 1) {
        for (int m = 0; m < 3; ++m) s[m] = hsgo_round_f16(s[m]);
    } else if (mode == 2) {
        for (int m = 0; m < 3; ++m) s[m] = hsgo_round_bf16(s[m]);
    } else if (mode == 3) {
        int32_t q[2];
        hsgo_oct_encode(s, q);
        hsgo_oct_decode(q, s);
        return;
    }
    normalise3(s);
}

/* Test convenience: n heat-bath draws about one fixed field h, the q-th draw
 * using words (x0, x1) of Philox block (q, 0, 0, 0) under `key`. */
void hsgo_hb_draw_many(const double h[3], double beta, const uint32_t key[2], int64_t n,
                       double *out)
{
    for (int64_t q = 0; q < n; ++q) {
        uint32_t ctr[4] = {(uint32_t)q, 0u, 0u, 0u}, r[4];
        hsgo_philox4x32_10(ctr, key, r);
        hsgo_hb_draw(h, beta, r[0], r[1], out + 3 * q);
    }
}

/* ------------------------------------------------------------------------ */
/* Run statistics (§2: U_L and C_L; §4: tunnelling events of the tempering).  */
/* ------------------------------------------------------------------------ */
/* Called once after every sweep (after its tempering pass). For every ladder
 * (sample d, copy o) and rung k, the energy of the configuration now at rung k
 * is added to sum_e[(d O + o) T + k] and its square to sum_e2[...]; the
 * internal energy U_L(T_k) is then sum_e / n and the specific heat
 * C_L(T_k) = (sum_e2 / n - U_L^2) / T_k^2 over the n sweeps recorded.
 *
 * A tunnelling event (a round trip) is a closed loop of one replica between
 * the end points of the ladder: lowest rung, highest rung, lowest rung again.
 * Per replica (slot) the oracle keeps which end it visited last, end[...] in
 * {-1 (none yet), 0 (lowest), 1 (highest)}, and whether it has ever been at
 * the lowest rung, seen_low[...]. Arriving at the lowest rung with the highest
 * as the last end visited, after an earlier visit to the lowest, closes one
 * loop. A ladder with one rung has no loops. */
void hsgo_stats_record(const hsgo_cfg *c, const double *E, const int32_t *slot_at_temp,
                       double *sum_e, double *sum_e2, int32_t *end, int32_t *seen_low,
                       uint32_t *trips)
{
    const int T = c->n_temps;
    for (int d = 0; d < c->n_samples; ++d)
        for (int o = 0; o < c->n_copies; ++o) {
            const int64_t lad = (int64_t)d * c->n_copies + o;
            const int32_t *row = slot_at_temp + lad * T;
            for (int k = 0; k < T; ++k) {
                const double e = E[lad * T + row[k]];
                sum_e[lad * T + k] += e;
                sum_e2[lad * T + k] += e * e;
            }
            if (T < 2) continue;
            for (int s = 0; s < T; ++s) {
                const int64_t r = lad * T + s;
                if (row[0] == s) {
                    if (end[r] == 1 && seen_low[r]) trips[r] += 1u;
                    end[r] = 0;
                    seen_low[r] = 1;
                } else if (row[T - 1] == s) {
                    end[r] = 1;
                }
            }
        }
}

/* U_L(T_k) and C_L(T_k) of every ladder from the sums of n recorded sweeps. */
void hsgo_stats_finish(const hsgo_cfg *c, const double *temps, const double *sum_e,
                       const double *sum_e2, uint64_t n, double *U, double *C)
{
    const int T = c->n_temps;
    const int64_t n_lad = (int64_t)c->n_samples * c->n_copies;
    for (int64_t lad = 0; lad < n_lad; ++lad)
        for (int k = 0; k < T; ++k) {
            const int64_t r = lad * T + k;
            const double u = sum_e[r] / (double)n;
            U[r] = u;
            C[r] = (sum_e2[r] / (double)n - u * u) / (temps[k] * temps[k]);
        }
}

/* ------------------------------------------------------------------------ */
/* Four-replica estimators of the connected spin-glass susceptibility in a    */
/* field, Eqs. (9)-(11).                                                      */
/* ------------------------------------------------------------------------ */
/* For every sample d and rung k, with copies 0, 1, 2, 3 at that rung as the
 * replicas (1), (2), (3), (4), the three double sums of Eq. (10) over all
 * ordered site pairs (i, j) and spin components (mu, nu), written out term by
 * term:
 *   chi_1(k) = sum_{i,j} sum_{mu,nu} s_i^mu(1) s_j^nu(1) s_i^mu(2) s_j^nu(2) e^{i k.(R_i - R_j)}
 *   chi_2(k) = sum_{i,j} sum_{mu,nu} s_i^mu(1) s_j^nu(1) s_i^mu(3) s_j^nu(4) e^{i k.(R_i - R_j)}
 *   chi_3(k) = sum_{i,j} sum_{mu,nu} s_i^mu(1) s_j^nu(2) s_i^mu(3) s_j^nu(4) e^{i k.(R_i - R_j)}
 * for k = 0 and k = (2 pi / L) e_a, a = x, y, z. Eq. (11) assembles
 * chi_SG(k) = [chi_1 - 2 chi_2 + chi_3] / N from their thermal and disorder
 * averages. O(N^2) per rung: for small lattices only.
 * out[((d T + k) 4 + w) 5 + m], w = 0 (k = 0), 1, 2, 3 (k_x, k_y, k_z):
 *   m = 0: Re chi_1; m = 1, 2: Re, Im chi_2; m = 3, 4: Re, Im chi_3.
 * (chi_1 is real; its imaginary part is not stored.) Needs n_copies >= 4. */
void hsgo_chi4(const hsgo_cfg *c, const double *spins, const int32_t *slot_at_temp,
               double *out)
{
    const int L = c->L, O = c->n_copies, T = c->n_temps;
    const int64_t N = (int64_t)L * L * L;
    const double w0 = HSGO_TWO_PI / (double)L;
    for (int d = 0; d < c->n_samples; ++d)
        for (int k = 0; k < T; ++k) {
            const double *r[4];
            for (int a = 0; a < 4; ++a)
                r[a] = slot_ptr(c, (double *)spins, d, a,
                                slot_at_temp[((int64_t)d * O + a) * T + k]);
            for (int w = 0; w < 4; ++w) {
                double re1 = 0.0, re2 = 0.0, im2 = 0.0, re3 = 0.0, im3 = 0.0;
                for (int64_t i = 0; i < N; ++i)
                    for (int64_t j = 0; j < N; ++j) {
                        double phase = 0.0;
                        if (w > 0) {
                            const int64_t ri = w == 1 ? i % L : w == 2 ? (i / L) % L : i / ((int64_t)L * L);
                            const int64_t rj = w == 1 ? j % L : w == 2 ? (j / L) % L : j / ((int64_t)L * L);
                            phase = w0 * (double)(ri - rj);
                        }
                        const double cs = cos(phase), sn = sin(phase);
                        double t1 = 0.0, t2 = 0.0, t3 = 0.0;
                        for (int mu = 0; mu < 3; ++mu)
                            for (int nu = 0; nu < 3; ++nu) {
                                t1 += r[0][mu * N + i] * r[0][nu * N + j] * r[1][mu * N + i] * r[1][nu * N + j];
                                t2 += r[0][mu * N + i] * r[0][nu * N + j] * r[2][mu * N + i] * r[3][nu * N + j];
                                t3 += r[0][mu * N + i] * r[1][nu * N + j] * r[2][mu * N + i] * r[3][nu * N + j];
                            }
                        re1 += t1 * cs;
                        re2 += t2 * cs;
                        im2 += t2 * sn;
                        re3 += t3 * cs;
                        im3 += t3 * sn;
                    }
                double *o = out + (((int64_t)d * T + k) * 4 + w) * 5;
                o[0] = re1;
                o[1] = re2;
                o[2] = im2;
                o[3] = re3;
                o[4] = im3;
            }
        }
}
