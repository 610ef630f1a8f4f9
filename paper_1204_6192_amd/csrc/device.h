// device.h -- per-site arithmetic of the sweep, for gfx950 (wave64).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), the heat-bath draw of
// Eq. (2), the over-relaxation reflection of Eq. (3), the spin storage codecs
// and float64 wave / block reductions. All arithmetic is float32 except the
// reductions; the library is compiled with -ffp-contract=off so that every
// fused multiply-add below is one written on purpose.
#pragma once
#include <type_traits>

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace hsg {

// ---------------------------------------------------------------- Philox
struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32 x 32 -> 64-bit multiply per product (v_mad_u64_u32) gives both
        // halves; each three-way xor is one three-input bitwise instruction
        // (truth table 0x96)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = u32x4{(uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96), (uint32_t)p1,
                  (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96), (uint32_t)p0};
    }
    return c;
}

// (0, 1] from the top 24 bits; exact in float32.
__device__ __forceinline__ float u24(uint32_t w) { return (float)((w >> 8) + 1u) * 0x1p-24f; }

// (0, 1] with 53 bits from two words; exact in float64.
__device__ __forceinline__ double u53(uint32_t a, uint32_t b)
{
    const uint64_t m = ((uint64_t)a << 21) ^ (uint64_t)(b >> 11);
    return (double)(m + 1ull) * 0x1p-53;
}

// ---------------------------------------------------------------- vectors
struct v3 {
    float x, y, z;
};

__device__ __forceinline__ float dot3(v3 a, v3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }

__device__ __forceinline__ v3 scale3(v3 a, float f) { return v3{a.x * f, a.y * f, a.z * f}; }

__device__ __forceinline__ v3 normalise3(v3 a) { return scale3(a, 1.0f / sqrtf(dot3(a, a))); }

// Renormalisation on load of a compressed spin (|a| within ~1e-2 of 1): the
// hardware reciprocal square root (1 ulp) is ample next to the storage's own
// rounding (2^-11 or coarser).
__device__ __forceinline__ v3 normalise_rsq(v3 a) { return scale3(a, __builtin_amdgcn_rsqf(dot3(a, a))); }

// Hardware transcendentals (one instruction each, about 1 ulp): log2, 2^x,
// sin(2 pi x) and cos(2 pi x) for x in revolutions, reciprocal and reciprocal
// square root. Their accuracy on this device is checked by a GPU test.
__device__ __forceinline__ float hw_log(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
__device__ __forceinline__ float hw_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.442695040888963407f); }
__device__ __forceinline__ float hw_sin_rev(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ float hw_cos_rev(float x) { return __builtin_amdgcn_cosf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hw_rsq(float x) { return __builtin_amdgcn_rsqf(x); }


// a / b within one ulp: the hardware reciprocal refined by one Newton step,
// then one correction of the quotient from its exact residual a - b q (an fma);
// Markstein's scheme (IA-64 and Elementary Functions, 2000). About 6
// instructions against about 10 for the correctly rounded division. b must be
// a normal number.
__device__ __forceinline__ float div_nr(float a, float b)
{
    float r = __builtin_amdgcn_rcpf(b);
    r = fmaf(fmaf(-b, r, 1.0f), r, r);
    const float q = a * r;
    return fmaf(fmaf(-b, q, a), r, q);
}

// sqrt(x) and 1 / sqrt(x) for x > 0, each within one ulp: the hardware
// reciprocal square root y, then one coupled Newton step on g = x y and
// h = y / 2 and one residual correction of g (Markstein, as above). With
// SCALE, inputs below 2^-64 are scaled by 2^64 first, since the hardware
// instruction flushes subnormal inputs; without it x must be at least 2^-64.
template <bool SCALE = true>
__device__ __forceinline__ float sqrt_rsqrt_nr(float x, float &rs)
{
    const bool tiny = SCALE && x < 0x1p-64f;
    const float xs = tiny ? x * 0x1p64f : x;
    const float y = __builtin_amdgcn_rsqf(xs);
    float g = xs * y, h = 0.5f * y;
    const float r = fmaf(-g, h, 0.5f);
    g = fmaf(g, r, g);
    h = fmaf(h, r, h);
    g = fmaf(fmaf(-g, g, xs), h, g);
    rs = tiny ? (2.0f * h) * 0x1p32f : 2.0f * h;
    return tiny ? g * 0x1p-32f : g;
}

// sin(2 pi u) and cos(2 pi u) for u on the 2^-24 grid of the uniforms (any
// |u| < 2^21 with u - rint(4 u) / 4 exact): u = q / 4 + r exactly, q = rint(4 u),
// |r| <= 1/8; sin(2 pi r) = r P(r^2) and cos(2 pi r) = Q(r^2) with P of degree
// 3 and Q of degree 4, least-squares fits reweighted toward the minimax error
// on |r| <= 1/8 with coefficients rounded to float32 (fit error 1.2e-9 and
// 5e-11); q mod 4 turns the pair by quarter turns. Absolute error at most 7e-8
// (0.6 float32 spacings at 1) over the whole grid, in float32 evaluation.
// About 20 instructions, against about 40 for the library sincospi.
__device__ __forceinline__ void sincos_2pi(float u, float &s, float &c)
{
    const float q = __builtin_rintf(4.0f * u);
    const float r = fmaf(q, -0.25f, u);
    const float t = r * r;
    float p = fmaf(-0x1.2cf686p+6f, t, 0x1.465a42p+6f);
    p = fmaf(p, t, -0x1.4abba8p+5f);
    const float sr = fmaf(r, 0x1.921fb4p+2f, r * (t * p));
    float g = fmaf(0x1.d9c436p+5f, t, -0x1.55c57ep+6f);
    g = fmaf(g, t, 0x1.03c1dcp+6f);
    g = fmaf(g, t, -0x1.3bd3ccp+4f);
    const float cr = fmaf(g, t, 1.0f);
    const int n = (int)q;
    const float so = (n & 1) ? cr : sr, co = (n & 1) ? sr : cr;
    s = __uint_as_float(__float_as_uint(so) ^ ((uint32_t)(n & 2) << 30));
    c = __uint_as_float(__float_as_uint(co) ^ ((uint32_t)((n + 1) & 2) << 30));
}

// e^z for finite z <= 0: z log2(e) as the unevaluated sum of p = fl(z H) and
// its residual (the exact fma error plus z L; log2(e) = H + L to 2^-50),
// split into an integer n and f = (p - n) + residual with |f| <= 1/2 + 2^-20,
// 2^f from the hardware (1 ulp on [1/sqrt 2, sqrt 2]) and the exact scaling by
// 2^n, which rounds correctly into the subnormal range and to zero.
__device__ __forceinline__ float exp_nonpos(float z)
{
    constexpr float H = 0x1.715476p+0f, L = 0x1.4ae0c0p-26f;
    const float p = z * H;
    const float pe = fmaf(z, L, fmaf(z, H, -p));
    const float n = fmaxf(__builtin_rintf(p), -256.0f);
    return ldexpf(__builtin_amdgcn_exp2f((p - n) + pe), (int)n);
}

// ln x for finite normal x > 0: the hardware log2 (about 1 ulp), times ln 2
// as the unevaluated sum H + L (to 2^-53) with the product's exact residual.
__device__ __forceinline__ float log_normal(float x)
{
    constexpr float H = 0x1.62e430p-1f, L = -0x1.05c610p-29f;
    const float l = __builtin_amdgcn_logf(x);
    const float p = l * H;
    return p + fmaf(l, L, fmaf(l, H, -p));
}

// Rescale a vector whose length is already 1 to within ~1e-3 onto the unit
// sphere, in float32 without a systematic bias. Plain renormalisation
// (v / sqrt(v.v)) cannot resolve deviations below the float32 spacing at 1.0,
// and repeated over-relaxation drifts |s| to about 1 + 4e-8 on average, which
// biases every bond energy by twice that. Here d = |v|^2 - 1 is formed
// directly by a chain of three fused multiply-adds (each rounds once, to
// nearest, at a magnitude of at most 1: an absolute error below 6e-8 of either
// sign, no drift), and the second-order series of 1/sqrt(1 + d) - 1 is applied
// with one fused multiply-add per component. Over 300 reflections in float32
// the mean of |s| - 1 stays at 4e-11 +- 5e-11 (rms 2.1e-8), where plain
// renormalisation drifts to +3.3e-8.
__device__ __forceinline__ v3 renorm_unit(v3 a)
{
    const float d = fmaf(a.x, a.x, fmaf(a.y, a.y, fmaf(a.z, a.z, -1.0f)));
    const float corr = d * fmaf(0.375f, d, -0.5f);
    return v3{fmaf(a.x, corr, a.x), fmaf(a.y, corr, a.y), fmaf(a.z, corr, a.z)};
}

// h += J * s
__device__ __forceinline__ void acc3(v3 &h, float J, v3 s)
{
    h.x = fmaf(J, s.x, h.x);
    h.y = fmaf(J, s.y, h.y);
    h.z = fmaf(J, s.z, h.z);
}

// ---------------------------------------------------------------- Eq. (2)
// New spin drawn from exp(beta h.s): c = cos(angle to h) by inverting the CDF
// of exp(kappa c) on [-1, 1], kappa = beta |h|: c = 1 + ln(x) / kappa with
// x = u + (1 - u) e^{-2 kappa}. In float32 both ends of [-1, 1] need care, and
// the form must not branch per site (a wave runs every branch any of its sites
// takes). One exponential E = e^{-2 kappa} and one logarithm per site:
//   A = e^{-2 kappa} - 1 from its Taylor series for 2 kappa < 0.35, else E - 1;
//   c >= 0 (x >= e^{-kappa}): kappa (1 - c) = -ln(1 + Y), Y = (1 - u) A, with
//     X = u + (1 - u) E (a sum of two positive terms) standing for 1 + Y;
//   c < 0: kappa (1 + c) = ln(1 + Y), Y = u B, B = e^{2 kappa} - 1 = -A / E,
//     X = 1 + Y;
//   ln(1 + Y) = ln X + ((1 - X) + Y) / X where 1 - X is exact (X in [1/2, 2]):
//     the first-order correction for the rounding of X.
// So 1 - c keeps its relative precision near c = 1 and 1 + c near c = -1, and
// so does the transverse length sqrt((1 - c)(1 + c)). Azimuth 2 pi u2 about h
// in the frame of Frisvad (JGT 2012), which is continuous except at n = -z (a
// frame with a jump along a whole great circle would turn float32 rounding of h
// into O(1) jumps of the new spin); 1 + n_z is formed without cancellation for
// n_z < 0. Zero field: uniform, z frame.
//
// HW = false (the default) takes square roots and divisions within one ulp
// from the hardware reciprocal (square root) refined by Newton steps
// (sqrt_rsqrt_nr, div_nr) and the azimuth from sincos_2pi. HW = true
// (an opt-in variant) takes the field's length and direction from the bare
// hardware reciprocal square root, the divisions from the bare hardware
// reciprocal (1 ulp each, but the products they feed round again) and the
// azimuth from the hardware sin/cos of revolutions (absolute error about
// 1.2e-7, one float32 spacing at 1). Both take e^z and ln X from the hardware
// 2^x and log2 with extended-precision scaling (exp_nonpos, log_normal).
//
// RENORM = false (compressed storage) skips the final renormalisation: the
// codec rounds the spin to 2^-11 or coarser and renormalises it on load, so a
// norm error of a few float32 ulps changes nothing but rare roundings at a
// code boundary (as float32 arithmetic against float64 already does).
template <bool HW, bool RENORM = true>
__device__ __forceinline__ v3 heat_bath(v3 h, float beta, uint32_t w0, uint32_t w1)
{
    const float u1 = u24(w0);
    const float u2 = u24(w1);
    const float hh = dot3(h, h);
    float rs, hn;  // 1 / |h| and |h|
    if constexpr (HW) {
        rs = hw_rsq(hh);  // infinite for a zero field, then unused
        hn = hh * rs;
    } else {
        hn = hh > 0.0f ? sqrt_rsqrt_nr(hh, rs) : 0.0f;
    }
    const float kappa = beta * hn;
    v3 n;
    float omc, opc;  // 1 - c and 1 + c
    bool upper;      // c >= 0: c is taken from 1 - c, else from 1 + c
    if (__builtin_expect(hh == 0.0f || !(kappa > 0.0f), 0)) {  // rare: zero field
        n = v3{0.0f, 0.0f, 1.0f};
        omc = 2.0f * (1.0f - u1);  // c = 2 u1 - 1, exact
        opc = 2.0f * u1;
        upper = u1 >= 0.5f;
    } else {
        n = scale3(h, rs);
        const float omu = 1.0f - u1;  // exact on the 2^-24 grid
        const float z = -2.0f * kappa;
        const float E = exp_nonpos(z);  // 0 past underflow
        // A = e^{-2 kappa} - 1. The two rare cases below are branches rather
        // than selects: a wave in which no site takes one skips its work.
        float A = E - 1.0f;
        if (__builtin_expect(z > -0.35f, 0)) {  // 2 kappa < 0.35: the Taylor series (rare)
            float p = 2.7557319e-6f;  // 1/9!, then Horner down to 1/2!
            p = fmaf(z, p, 2.4801588e-5f);
            p = fmaf(z, p, 1.9841270e-4f);
            p = fmaf(z, p, 1.3888889e-3f);
            p = fmaf(z, p, 8.3333333e-3f);
            p = fmaf(z, p, 4.1666667e-2f);
            p = fmaf(z, p, 1.6666667e-1f);
            p = fmaf(z, p, 0.5f);
            A = z * fmaf(z, p, 1.0f);
        }
        const float xo = fmaf(omu, E, u1);  // x
        upper = xo * xo >= E;               // x >= e^{-kappa}, i.e. c >= 0
        float X = xo, Y = omu * A;
        if (__builtin_expect(!upper, 0)) {  // c < 0, with probability about e^{-kappa}
            // c < 0 needs kappa < 17 (u >= 2^-24), where E is a normal number
            const float yb = u1 * (HW ? -A * hw_rcp(E) : div_nr(-A, E));
            X = 1.0f + yb;
            Y = yb;
        }
        const float d = (1.0f - X) + Y;
        // (a relative correction of order 1e-7: the hardware reciprocal's 1 ulp is far below float32 spacing)
        const float corr = (X >= 0.5f && X <= 2.0f) ? d * hw_rcp(X) : 0.0f;
        // X >= u1 >= 2^-24 (upper) or X >= 1: a normal number
        const float lx = log_normal(X);
        const float t = HW ? (lx + corr) * hw_rcp(kappa) : div_nr(lx + corr, kappa);
        omc = fminf(2.0f, fmaxf(0.0f, upper ? -t : 2.0f - t));
        opc = fminf(2.0f, fmaxf(0.0f, upper ? 2.0f + t : t));
    }
    const float c = upper ? 1.0f - omc : opc - 1.0f;
    v3 e1, e2;
    const float rxy = fmaf(n.x, n.x, n.y * n.y);
    if (__builtin_expect(n.z < 0.0f && rxy == 0.0f, 0)) {  // n = -z exactly
        e1 = v3{-1.0f, 0.0f, 0.0f};
        e2 = v3{0.0f, 1.0f, 0.0f};
    } else {
        // a = 1 / (1 + n_z), as (1 - n_z) / (n_x^2 + n_y^2) for n_z < 0: one division
        const bool up = n.z >= 0.0f;
        const float num = up ? 1.0f : 1.0f - n.z, den = up ? 1.0f + n.z : rxy;
        float a;
        if constexpr (HW)
            a = num * hw_rcp(den);
        else
            a = div_nr(num, den);
        const float b = -n.x * n.y * a;
        e1 = v3{fmaf(-n.x * n.x, a, 1.0f), b, -n.x};
        e2 = v3{b, fmaf(-n.y * n.y, a, 1.0f), -n.y};
    }
    float st, sp, cp;
    if constexpr (HW) {
        st = __builtin_amdgcn_sqrtf(omc * opc);
        sp = hw_sin_rev(u2);
        cp = hw_cos_rev(u2);
    } else {
        const float p = omc * opc;
        float unused;
        // a positive p is at least about 2^-24 / kappa: 1 - c and 1 + c are
        // either 0 or at least (1 - e^{-2 kappa}) 2^-24 / kappa; far above 2^-64
        st = p > 0.0f ? sqrt_rsqrt_nr<false>(p, unused) : 0.0f;
        sincos_2pi(u2, sp, cp);
    }
    const float ta = st * cp, tb = st * sp;
    v3 s{fmaf(c, n.x, fmaf(ta, e1.x, tb * e2.x)), fmaf(c, n.y, fmaf(ta, e1.y, tb * e2.y)),
         fmaf(c, n.z, fmaf(ta, e1.z, tb * e2.z))};
    return RENORM ? renorm_unit(s) : s;
}

// ---------------------------------------------------------------- Eq. (3)
// Reflection of s about the local field; a zero field (|h|^2 below 1e-30)
// leaves s unchanged. The spin must be a unit vector to float32 precision (the
// reflection keeps |s|). RENORM = false (compressed storage, which renormalises
// on load) skips the final renormalisation, as in heat_bath.
template <bool RENORM = true>
__device__ __forceinline__ v3 over_relax(v3 s, v3 h)
{
    const float hh = dot3(h, h);
    // A field with |h|^2 below 1e-30 counts as zero (its direction is noise).
    if (!(hh >= 1e-30f)) return s;
    // 2 (s.h) / (h.h) from the hardware reciprocal refined by one Newton step:
    // within about an ulp (the result is renormalised below in any case).
    float rh = __builtin_amdgcn_rcpf(hh);
    rh = fmaf(rh, fmaf(-hh, rh, 1.0f), rh);
    const float f = 2.0f * dot3(s, h) * rh;
    v3 r{fmaf(f, h.x, -s.x), fmaf(f, h.y, -s.y), fmaf(f, h.z, -s.z)};
    return RENORM ? renorm_unit(r) : r;
}

// ---------------------------------------------------------------- storage
// Element i of an array. B32: as the base plus a 32-bit byte offset, which the
// hardware adds to a wave-uniform base by itself (no 64-bit address arithmetic
// per lane); the caller guarantees i * sizeof(T) < 2^32. Else ordinary
// pointer arithmetic.
template <bool B32, class T>
__device__ __forceinline__ T *elem(T *p, uint32_t i)
{
    if constexpr (B32) {
        using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
        return reinterpret_cast<T *>(reinterpret_cast<B *>(p) + i * (uint32_t)sizeof(T));
    } else {
        return p + i;
    }
}

// Spins of one replica, one parity: three component planes of Nh values.
template <int STORE>
struct Codec;

template <>
struct Codec<0> {  // float32: stored renormalised, read as is
    using T = float;
    static constexpr int kPlanes = 3;  // component planes per parity
    __device__ static __forceinline__ v3 load(const T *p, int64_t cs, int64_t j)
    {
        return v3{p[j], p[cs + j], p[2 * cs + j]};
    }
    // the same with 32-bit byte offsets from a uniform base (3 cs sizeof(T) < 2^32)
    __device__ static __forceinline__ v3 load32(const T *p, uint32_t cs, uint32_t j)
    {
        return v3{*elem<true>(p, j), *elem<true>(p, cs + j), *elem<true>(p, 2 * cs + j)};
    }
    __device__ static __forceinline__ void store(T *p, int64_t cs, int64_t j, v3 s)
    {
        p[j] = s.x;
        p[cs + j] = s.y;
        p[2 * cs + j] = s.z;
    }
    __device__ static __forceinline__ v3 stored_value(v3 s) { return s; }
    // Two neighbouring sites j0, j0 + 1 (j0 even, 8-byte aligned): one 8-byte
    // access per component plane; 32-bit offsets (3 Nh < 2^32 for L <= 1024).
    template <bool B32 = false>
    __device__ static __forceinline__ void load_pair(const T *p, uint32_t cs, uint32_t j0, v3 &a, v3 &b)
    {
        const float2 x = *reinterpret_cast<const float2 *>(elem<B32>(p, j0));
        const float2 y = *reinterpret_cast<const float2 *>(elem<B32>(p, cs + j0));
        const float2 z = *reinterpret_cast<const float2 *>(elem<B32>(p, 2 * cs + j0));
        a = v3{x.x, y.x, z.x};
        b = v3{x.y, y.y, z.y};
    }
    // The same pair split into the memory access and the decoding, so that a
    // load can be issued a step before its value is used.
    struct R {
        float2 x, y, z;
    };
    template <bool B32 = false>
    __device__ static __forceinline__ void load_raw_pair(const T *p, uint32_t cs, uint32_t j0, R &r)
    {
        r.x = *reinterpret_cast<const float2 *>(elem<B32>(p, j0));
        r.y = *reinterpret_cast<const float2 *>(elem<B32>(p, cs + j0));
        r.z = *reinterpret_cast<const float2 *>(elem<B32>(p, 2 * cs + j0));
    }
    __device__ static __forceinline__ void decode_pair(const R &r, v3 &a, v3 &b)
    {
        a = v3{r.x.x, r.y.x, r.z.x};
        b = v3{r.x.y, r.y.y, r.z.y};
    }
    // The codes of a pair, and their store: a stored value is decode_pair of
    // encode_pair, so a caller that stores and reads back encodes once.
    __device__ static __forceinline__ R encode_pair(v3 a, v3 b)
    {
        return R{make_float2(a.x, b.x), make_float2(a.y, b.y), make_float2(a.z, b.z)};
    }
    template <bool B32 = false>
    __device__ static __forceinline__ void store_raw_pair(T *p, uint32_t cs, uint32_t j0, const R &r)
    {
        *reinterpret_cast<float2 *>(elem<B32>(p, j0)) = r.x;
        *reinterpret_cast<float2 *>(elem<B32>(p, cs + j0)) = r.y;
        *reinterpret_cast<float2 *>(elem<B32>(p, 2 * cs + j0)) = r.z;
    }
    template <bool B32 = false>
    __device__ static __forceinline__ void store_pair(T *p, uint32_t cs, uint32_t j0, v3 a, v3 b)
    {
        store_raw_pair<B32>(p, cs, j0, encode_pair(a, b));
    }
};

template <>
struct Codec<1> {  // float16 components (round to nearest even), renormalised on load
    using T = __half;
    static constexpr int kPlanes = 3;
    __device__ static __forceinline__ v3 load(const T *p, int64_t cs, int64_t j)
    {
        return normalise_rsq(v3{__half2float(p[j]), __half2float(p[cs + j]), __half2float(p[2 * cs + j])});
    }
    __device__ static __forceinline__ v3 load32(const T *p, uint32_t cs, uint32_t j)
    {
        return normalise_rsq(v3{__half2float(*elem<true>(p, j)), __half2float(*elem<true>(p, cs + j)),
                                __half2float(*elem<true>(p, 2 * cs + j))});
    }
    __device__ static __forceinline__ void store(T *p, int64_t cs, int64_t j, v3 s)
    {
        p[j] = __float2half_rn(s.x);
        p[cs + j] = __float2half_rn(s.y);
        p[2 * cs + j] = __float2half_rn(s.z);
    }
    __device__ static __forceinline__ v3 stored_value(v3 s)
    {
        return normalise_rsq(v3{__half2float(__float2half_rn(s.x)), __half2float(__float2half_rn(s.y)),
                                __half2float(__float2half_rn(s.z))});
    }
    template <bool B32 = false>
    __device__ static __forceinline__ void load_pair(const T *p, uint32_t cs, uint32_t j0, v3 &a, v3 &b)
    {
        const __half2 x = *reinterpret_cast<const __half2 *>(elem<B32>(p, j0));
        const __half2 y = *reinterpret_cast<const __half2 *>(elem<B32>(p, cs + j0));
        const __half2 z = *reinterpret_cast<const __half2 *>(elem<B32>(p, 2 * cs + j0));
        a = normalise_rsq(v3{__low2float(x), __low2float(y), __low2float(z)});
        b = normalise_rsq(v3{__high2float(x), __high2float(y), __high2float(z)});
    }
    struct R {
        __half2 x, y, z;
    };
    template <bool B32 = false>
    __device__ static __forceinline__ void load_raw_pair(const T *p, uint32_t cs, uint32_t j0, R &r)
    {
        r.x = *reinterpret_cast<const __half2 *>(elem<B32>(p, j0));
        r.y = *reinterpret_cast<const __half2 *>(elem<B32>(p, cs + j0));
        r.z = *reinterpret_cast<const __half2 *>(elem<B32>(p, 2 * cs + j0));
    }
    __device__ static __forceinline__ void decode_pair(const R &r, v3 &a, v3 &b)
    {
        a = normalise_rsq(v3{__low2float(r.x), __low2float(r.y), __low2float(r.z)});
        b = normalise_rsq(v3{__high2float(r.x), __high2float(r.y), __high2float(r.z)});
    }
    // Each value by the scalar conversion: the compiler would otherwise pair
    // two of them into gfx950's packed conversion, which rounds results in
    // float16's subnormal range differently (the empty asm keeps them apart).
    __device__ static __forceinline__ __half2 pack(float lo, float hi)
    {
        __half l = __float2half_rn(lo);
        asm volatile("" : "+v"(l));
        return __halves2half2(l, __float2half_rn(hi));
    }
    __device__ static __forceinline__ R encode_pair(v3 a, v3 b)
    {
        return R{pack(a.x, b.x), pack(a.y, b.y), pack(a.z, b.z)};
    }
    template <bool B32 = false>
    __device__ static __forceinline__ void store_raw_pair(T *p, uint32_t cs, uint32_t j0, const R &r)
    {
        *reinterpret_cast<__half2 *>(elem<B32>(p, j0)) = r.x;
        *reinterpret_cast<__half2 *>(elem<B32>(p, cs + j0)) = r.y;
        *reinterpret_cast<__half2 *>(elem<B32>(p, 2 * cs + j0)) = r.z;
    }
    template <bool B32 = false>
    __device__ static __forceinline__ void store_pair(T *p, uint32_t cs, uint32_t j0, v3 a, v3 b)
    {
        store_raw_pair<B32>(p, cs, j0, encode_pair(a, b));
    }
};

// bfloat16: the upper half of the float32 pattern, rounded to nearest even,
// by gfx950's conversion instruction (v_cvt_pk_bf16_f32, two values at once).
// It equals the integer form (b + 0x7FFF + ((b >> 16) & 1)) >> 16 of the
// pattern b bit for bit: checked on the device for every float32 of magnitude
// in [2^-31, 2) of either sign.
typedef float hsg_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 hsg_bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16x2_rne(float lo, float hi)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((hsg_f32x2){lo, hi}, hsg_bf16x2));
}
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
__device__ __forceinline__ float bf16_to_f32(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }

template <>
struct Codec<2> {  // bfloat16 components, renormalised on load
    using T = uint16_t;
    static constexpr int kPlanes = 3;
    __device__ static __forceinline__ v3 load(const T *p, int64_t cs, int64_t j)
    {
        return normalise_rsq(v3{bf16_to_f32(p[j]), bf16_to_f32(p[cs + j]), bf16_to_f32(p[2 * cs + j])});
    }
    __device__ static __forceinline__ v3 load32(const T *p, uint32_t cs, uint32_t j)
    {
        return normalise_rsq(v3{bf16_to_f32(*elem<true>(p, j)), bf16_to_f32(*elem<true>(p, cs + j)),
                                bf16_to_f32(*elem<true>(p, 2 * cs + j))});
    }
    __device__ static __forceinline__ void store(T *p, int64_t cs, int64_t j, v3 s)
    {
        p[j] = f32_to_bf16_rne(s.x);
        p[cs + j] = f32_to_bf16_rne(s.y);
        p[2 * cs + j] = f32_to_bf16_rne(s.z);
    }
    __device__ static __forceinline__ v3 stored_value(v3 s)
    {
        const uint32_t xy = bf16x2_rne(s.x, s.y);
        return normalise_rsq(v3{__uint_as_float(xy << 16), __uint_as_float(xy & 0xFFFF0000u),
                                bf16_to_f32(f32_to_bf16_rne(s.z))});
    }
    template <bool B32 = false>
    __device__ static __forceinline__ void load_pair(const T *p, uint32_t cs, uint32_t j0, v3 &a, v3 &b)
    {
        const uint32_t x = *reinterpret_cast<const uint32_t *>(elem<B32>(p, j0));
        const uint32_t y = *reinterpret_cast<const uint32_t *>(elem<B32>(p, cs + j0));
        const uint32_t z = *reinterpret_cast<const uint32_t *>(elem<B32>(p, 2 * cs + j0));
        a = normalise_rsq(v3{__uint_as_float(x << 16), __uint_as_float(y << 16), __uint_as_float(z << 16)});
        b = normalise_rsq(v3{__uint_as_float(x & 0xFFFF0000u), __uint_as_float(y & 0xFFFF0000u),
                             __uint_as_float(z & 0xFFFF0000u)});
    }
    struct R {
        uint32_t x, y, z;
    };
    template <bool B32 = false>
    __device__ static __forceinline__ void load_raw_pair(const T *p, uint32_t cs, uint32_t j0, R &r)
    {
        r.x = *reinterpret_cast<const uint32_t *>(elem<B32>(p, j0));
        r.y = *reinterpret_cast<const uint32_t *>(elem<B32>(p, cs + j0));
        r.z = *reinterpret_cast<const uint32_t *>(elem<B32>(p, 2 * cs + j0));
    }
    __device__ static __forceinline__ void decode_pair(const R &r, v3 &a, v3 &b)
    {
        a = normalise_rsq(v3{__uint_as_float(r.x << 16), __uint_as_float(r.y << 16), __uint_as_float(r.z << 16)});
        b = normalise_rsq(v3{__uint_as_float(r.x & 0xFFFF0000u), __uint_as_float(r.y & 0xFFFF0000u),
                             __uint_as_float(r.z & 0xFFFF0000u)});
    }
    __device__ static __forceinline__ R encode_pair(v3 a, v3 b)
    {
        return R{bf16x2_rne(a.x, b.x), bf16x2_rne(a.y, b.y), bf16x2_rne(a.z, b.z)};
    }
    template <bool B32 = false>
    __device__ static __forceinline__ void store_raw_pair(T *p, uint32_t cs, uint32_t j0, const R &r)
    {
        *reinterpret_cast<uint32_t *>(elem<B32>(p, j0)) = r.x;
        *reinterpret_cast<uint32_t *>(elem<B32>(p, cs + j0)) = r.y;
        *reinterpret_cast<uint32_t *>(elem<B32>(p, 2 * cs + j0)) = r.z;
    }
    template <bool B32 = false>
    __device__ static __forceinline__ void store_pair(T *p, uint32_t cs, uint32_t j0, v3 a, v3 b)
    {
        store_raw_pair<B32>(p, cs, j0, encode_pair(a, b));
    }
};

// Quantised angle: octahedral map (Cigolle et al., JCGT 3(2), 2014). The unit
// vector is projected onto |x| + |y| + |z| = 1, the lower half folded over the
// diagonals, and the two coordinates stored as 16-bit signed normalised
// integers (round to nearest even of c * 32767) packed in one 32-bit word per
// site, x in the low half. One plane per parity; renormalised on load.
__device__ __forceinline__ float sgn_nz(float a) { return a >= 0.0f ? 1.0f : -1.0f; }

// Both directions work in code units (the octahedron scaled by 32767), where
// the decoded coordinates and the fold are exact integers before the one
// renormalisation.
__device__ __forceinline__ uint32_t oct_encode(v3 v)
{
    const float sc = 32767.0f * hw_rcp(fabsf(v.x) + fabsf(v.y) + fabsf(v.z));
    float px = v.x * sc, py = v.y * sc;
    if (v.z < 0.0f) {
        const float fx = (32767.0f - fabsf(py)) * sgn_nz(px);
        const float fy = (32767.0f - fabsf(px)) * sgn_nz(py);
        px = fx;
        py = fy;
    }
    // |px|, |py| <= 32767 (1 + 4 ulp): no clamp is needed before rounding
    const int qx = (int)rintf(px), qy = (int)rintf(py);
    return ((uint32_t)qx & 0xFFFFu) | ((uint32_t)qy << 16);
}

__device__ __forceinline__ v3 oct_decode(uint32_t w)
{
    float fx = (float)(int16_t)(w & 0xFFFFu);
    float fy = (float)(int16_t)(w >> 16);
    const float vz = 32767.0f - fabsf(fx) - fabsf(fy);
    if (vz < 0.0f) {
        // fx, fy are never -0 (converted integers), so copysign is sgn_nz here
        const float ax = __builtin_copysignf(32767.0f - fabsf(fy), fx);
        const float ay = __builtin_copysignf(32767.0f - fabsf(fx), fy);
        fx = ax;
        fy = ay;
    }
    return normalise_rsq(v3{fx, fy, vz});
}

template <>
struct Codec<3> {
    using T = uint32_t;
    static constexpr int kPlanes = 1;
    __device__ static __forceinline__ v3 load(const T *p, int64_t, int64_t j) { return oct_decode(p[j]); }
    __device__ static __forceinline__ v3 load32(const T *p, uint32_t, uint32_t j) { return oct_decode(*elem<true>(p, j)); }
    __device__ static __forceinline__ void store(T *p, int64_t, int64_t j, v3 s) { p[j] = oct_encode(s); }
    __device__ static __forceinline__ v3 stored_value(v3 s) { return oct_decode(oct_encode(s)); }
    template <bool B32 = false>
    __device__ static __forceinline__ void load_pair(const T *p, uint32_t, uint32_t j0, v3 &a, v3 &b)
    {
        const uint2 w = *reinterpret_cast<const uint2 *>(elem<B32>(p, j0));
        a = oct_decode(w.x);
        b = oct_decode(w.y);
    }
    struct R {
        uint2 w;
    };
    template <bool B32 = false>
    __device__ static __forceinline__ void load_raw_pair(const T *p, uint32_t, uint32_t j0, R &r)
    {
        r.w = *reinterpret_cast<const uint2 *>(elem<B32>(p, j0));
    }
    __device__ static __forceinline__ void decode_pair(const R &r, v3 &a, v3 &b)
    {
        a = oct_decode(r.w.x);
        b = oct_decode(r.w.y);
    }
    __device__ static __forceinline__ R encode_pair(v3 a, v3 b) { return R{make_uint2(oct_encode(a), oct_encode(b))}; }
    template <bool B32 = false>
    __device__ static __forceinline__ void store_raw_pair(T *p, uint32_t, uint32_t j0, const R &r)
    {
        *reinterpret_cast<uint2 *>(elem<B32>(p, j0)) = r.w;
    }
    template <bool B32 = false>
    __device__ static __forceinline__ void store_pair(T *p, uint32_t cs, uint32_t j0, v3 a, v3 b)
    {
        store_raw_pair<B32>(p, cs, j0, encode_pair(a, b));
    }
};

// ---------------------------------------------------------------- staging helpers
// A pair of sites (x/2 = xh, xh + 1) to and from an LDS plane of three component
// planes cstride floats apart.
__device__ __forceinline__ void lds_put_pair(float *lds, int w, int cstride, v3 a, v3 b)
{
    *reinterpret_cast<float2 *>(&lds[w]) = make_float2(a.x, b.x);
    *reinterpret_cast<float2 *>(&lds[w + cstride]) = make_float2(a.y, b.y);
    *reinterpret_cast<float2 *>(&lds[w + 2 * cstride]) = make_float2(a.z, b.z);
}

__device__ __forceinline__ void lds_get_pair(const float *lds, int w, int cstride, v3 &a, v3 &b)
{
    const float2 x = *reinterpret_cast<const float2 *>(&lds[w]);
    const float2 y = *reinterpret_cast<const float2 *>(&lds[w + cstride]);
    const float2 z = *reinterpret_cast<const float2 *>(&lds[w + 2 * cstride]);
    a = v3{x.x, y.x, z.x};
    b = v3{x.y, y.y, z.y};
}

// +1.0f, or -1.0f when bit b of bits is set: the bit moved to the float's sign
// (a shift and one and-or, where a test and a select took three instructions).
__device__ __forceinline__ float pm1_from_bit(uint32_t bits, int b)
{
    return __uint_as_float(((bits << (31 - b)) & 0x80000000u) | 0x3F800000u);
}

// The same for lattices addressed with 32-bit byte offsets, from one uniform
// base per coupling plane (Jp[n] = the plane of bond n): each load is that base
// plus the lane's byte offset, with no per-load address arithmetic.
template <bool JB, bool FIELD>
__device__ __forceinline__ void load_couplings_planes(const float *const (&Jp)[6], const uint8_t *Jbb,
                                                      const float *Hb, bool jbits, bool field, uint32_t Nh,
                                                      uint32_t j0, float2 (&jc)[6], v3 &hs0, v3 &hs1)
{
    if (JB && jbits) {
        const uint32_t bits = *reinterpret_cast<const uint16_t *>(elem<true>(Jbb, j0));
#pragma unroll
        for (int n = 0; n < 6; ++n)
            jc[n] = make_float2(pm1_from_bit(bits, n), pm1_from_bit(bits, 8 + n));
    } else {
#pragma unroll
        for (int n = 0; n < 6; ++n) jc[n] = *reinterpret_cast<const float2 *>(elem<true>(Jp[n], j0));
    }
    hs0 = v3{0.f, 0.f, 0.f};
    hs1 = v3{0.f, 0.f, 0.f};
    if (FIELD && field) {
        const float2 hx = *reinterpret_cast<const float2 *>(elem<true>(Hb, j0));
        const float2 hy = *reinterpret_cast<const float2 *>(elem<true>(Hb, Nh + j0));
        const float2 hz = *reinterpret_cast<const float2 *>(elem<true>(Hb, 2 * Nh + j0));
        hs0 = v3{hx.x, hy.x, hz.x};
        hs1 = v3{hx.y, hy.y, hz.y};
    }
}

template <bool JB, bool FIELD, bool B32 = false>
__device__ __forceinline__ void load_couplings(const float *Jb, const uint8_t *Jbb, const float *Hb, bool jbits,
                                               bool field, uint32_t Nh, uint32_t j0, float2 (&jc)[6], v3 &hs0,
                                               v3 &hs1)
{
    if (JB && jbits) {
        const uint32_t bits = *reinterpret_cast<const uint16_t *>(elem<B32>(Jbb, j0));
#pragma unroll
        for (int n = 0; n < 6; ++n)
            jc[n] = make_float2(pm1_from_bit(bits, n), pm1_from_bit(bits, 8 + n));
    } else {
#pragma unroll
        for (int n = 0; n < 6; ++n) jc[n] = *reinterpret_cast<const float2 *>(elem<B32>(Jb, n * Nh + j0));
    }
    hs0 = v3{0.f, 0.f, 0.f};
    hs1 = v3{0.f, 0.f, 0.f};
    if (FIELD && field) {
        const float2 hx = *reinterpret_cast<const float2 *>(elem<B32>(Hb, j0));
        const float2 hy = *reinterpret_cast<const float2 *>(elem<B32>(Hb, Nh + j0));
        const float2 hz = *reinterpret_cast<const float2 *>(elem<B32>(Hb, 2 * Nh + j0));
        hs0 = v3{hx.x, hy.x, hz.x};
        hs1 = v3{hx.y, hy.y, hz.y};
    }
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over a 256-thread block, fixed order; every thread must call it. The
// result is valid in thread 0. `red` is __shared__ double[4].
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return r;
}

// Block ids are dealt round-robin over the 8 XCDs; remap them so that each XCD
// runs a contiguous range of logical work items (neighbouring z-slabs of the
// same replicas share that XCD's L2).
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int xcd = b & 7, idx = b >> 3, base = nb >> 3, extra = nb & 7;
    return xcd * base + (xcd < extra ? xcd : extra) + idx;
}

}  // namespace hsg
