// Device-side building blocks of libosc shared by the plain and the batched
// kernels: the per-event probability (FP64 and FP32-mixed tiers), the bin
// index, the per-wave LDS histograms and the tile body.  Both kernels
// run the same code, so a batched (set, sample) histogram equals the plain
// one bit for bit.
#pragma once

#include <type_traits>

#include "osc_internal.h"

namespace osc {
namespace dev {


// Events of one lane computed together in one straight-line block (and
// loaded one block ahead).  One event per block keeps the register count
// low enough for six waves per SIMD, which hides latency better than
// interleaving events within a wave.
constexpr int kGroup = 1;
static_assert(kLaneEvents % kGroup == 0, "the group size divides the events per lane");

// ---------------------------------------------------------------------------
// FP64 sine and cosine - 1 of a phase given in units of pi/32 as the
// product a b (|a b| < 2^50).  The nearest integer n to the exact product
// comes out of one FMA against 1.5 * 2^52 (n lands in the low mantissa
// bits), u = a b - n (|u| <= 1/2) out of a second one, so the reduction is
// exact up to the final rounding of u.  With r = u pi/32 (|r| <= pi/64):
//   sin r      = u (pi/32 + u^2 (P3 + P5 u^2 + P7 u^4))   (Taylor, scaled
//                to u; truncation below 7e-18),
//   cos r - 1  = u^2 (Q2 + Q4 u^2 + Q6 u^4)        (least-maximum absolute
//                error fit on |u| <= 1/2, error below 8e-18),
// and the angle-addition formulas with the anchor k = n mod 64 from LDS:
//   sin = s_k + s_k (cos r - 1) + c_k sin r,
//   cos - 1 = (c_k - 1) + c_k (cos r - 1) - s_k sin r.
// ---------------------------------------------------------------------------
constexpr double kRoundMagic = 6755399441055744.0;        // 1.5 * 2^52
constexpr double kStep = 0.09817477042468103;             // fl(pi / 32)
constexpr double kP3 = -0.0001577060784927359;            // -(pi/32)^3 / 3!
constexpr double kP5 = 7.600081085793214e-08;             //  (pi/32)^5 / 5!
constexpr double kP7 = -1.7440893260086657e-11;           // -(pi/32)^7 / 7!
constexpr double kQ2 = -0.0048191427739688;
constexpr double kQ4 = 3.870689497756199e-06;
constexpr double kQ6 = -1.2434575820615234e-09;

__device__ __forceinline__ double flip_sign(double v, uint32_t sign_bit)
{
    return __hiloint2double(__double2hiint(v) ^ int(sign_bit), __double2loint(v));
}

// p7 and q6 are kP7 and kQ6; a caller that evaluates many phases passes
// them from VGPRs (see PolyRegs), so that each polynomial step reads at most
// one constant from an SGPR pair (the VALU reads one per instruction).
__device__ __forceinline__ void phase_sincos(double a, double b, const SinCosL* __restrict__ table,
                                             double& sn, double& cm1, double p7 = kP7,
                                             double q6 = kQ6)
{
    const double t = __builtin_fma(a, b, kRoundMagic);
    const double n = t - kRoundMagic;
    const double u = __builtin_fma(a, b, -n);
    const SinCosL k = table[__double2loint(t) & 63];
    const double z = u * u;
    const double s = u * __builtin_fma(z, __builtin_fma(z, __builtin_fma(z, p7, kP5), kP3), kStep);
    const double cm = z * __builtin_fma(z, __builtin_fma(z, q6, kQ4), kQ2);
    sn = __builtin_fma(k.s, cm, __builtin_fma(k.c, s, k.s));
    cm1 = __builtin_fma(k.c, cm, __builtin_fma(-k.s, s, k.cm1));
}

// Copy the sin/cos anchors into LDS (the 64 lanes of a wave, one each);
// c - 1 is exact for c >= 1/2 and within half an ulp of 1 below.
__device__ __forceinline__ void load_sincos(const SinCosTable& t, TileTables& T, int lane)
{
    if (lane < 64) {
        const SinCos e = t.e[lane];
        T.sct[lane] = SinCosL{e.s, e.c, e.c - 1.0};
    }
}

// Mixed tier: the phase (a b in units of pi/32, so a b / 64 in revolutions)
// is reduced to |rev| <= 1/2 in FP64 as above, rounded to FP32, and the FP32
// hardware sine and cosine (argument in revolutions) finish the job.
__device__ __forceinline__ void phase_sincos_mixed(double a, double b_rev, float& sn, float& cs)
{
    const double t = __builtin_fma(a, b_rev, kRoundMagic);
    const double n = t - kRoundMagic;
    const float rev = float(__builtin_fma(a, b_rev, -n));
    sn = __builtin_amdgcn_sinf(rev);
    cs = __builtin_amdgcn_cosf(rev);
}

// 1/y to within a few ulp: hardware reciprocal estimate r (relative error
// e ~ 3e-7) and one third-order correction r (1 + e + e^2), e = 1 - y r,
// which leaves ~e^3 (y normal, not huge).
__device__ __forceinline__ double recip(double y)
{
    const double r = __builtin_amdgcn_rcp(y);
    const double e = fma(-y, r, 1.0);
    return fma(r, fma(e, e, e), r);
}

// 1/y with one Newton-Raphson correction (relative error ~1e-13): enough
// where the quotient is a small correction to a root.
__device__ __forceinline__ double recip_coarse(double y)
{
    const double r = __builtin_amdgcn_rcp(y);
    return fma(r, fma(-y, r, 1.0), r);
}

// arccos(x) / (6 pi) on [-1, 1] in FP32 (the seed angle theta/3 in
// revolutions for the hardware cosine): Abramowitz & Stegun 4.4.45 on |x|
// (error <= 6.7e-5 rad; the FP64 refinement below absorbs seed errors far
// larger than that) with its coefficients scaled by 1 / (6 pi), and
// acos(-x) = pi - acos(x).
__device__ __forceinline__ float acos_seed_rev(float x)
{
    constexpr float c = 0.053051647697298445f;   // 1 / (6 pi)
    const float ax = __builtin_fabsf(x);
    float p = -0.0187293f * c;
    p = __builtin_fmaf(p, ax, 0.0742610f * c);
    p = __builtin_fmaf(p, ax, -0.2121144f * c);
    p = __builtin_fmaf(p, ax, 1.5707288f * c);
    const float r = __builtin_amdgcn_sqrtf(1.0f - ax) * p;
    return x < 0.0f ? (1.0f / 6.0f) - r : r;
}

// A value the compiler cannot see through, kept in an SGPR pair.  3.0 is
// not an inline constant of the FP64 VALU; as a literal it only fits the
// two-address v_fmac form, which costs a register copy whenever the
// addend stays live.  From an SGPR the three-address v_fma takes it.
__device__ __forceinline__ double sgpr_value(double v)
{
    asm("" : "+s"(v));
    return v;
}

// The same, kept in a VGPR: loop-invariant operands that would otherwise
// be the second SGPR operand of an instruction (and be copied into a VGPR
// on every use).
__device__ __forceinline__ double vgpr_value(double v)
{
    asm("" : "+v"(v));
    return v;
}

// The innermost sine and cosine coefficients of phase_sincos, which a
// kernel that evaluates many phases loads into VGPRs once.
struct PolyRegs {
    double p7 = kP7, q6 = kQ6;
    static __device__ __forceinline__ PolyRegs in_vgprs()
    {
        return PolyRegs{vgpr_value(kP7), vgpr_value(kQ6)};
    }
};

// Roots of f(x) = x^3 - tr x^2 + c1 x - det (three real roots: the matrix
// is Hermitian).  Two roots are seeded in FP32 from the trigonometric
// solution x = tr/3 + (2/3) sqrt(p) cos(theta - 2 pi k / 3),
// theta = acos(q / (2 p^1.5)) / 3 (p = tr^2 - 3 c1; qh = q / 2 with
// q = 2 tr^3 - 9 tr c1 + 27 det is passed in), each refined in FP64 by one
// Halley step on f with its third-order error term added back; the third
// root follows from the trace.  The two roots' divisions of each step
// share one reciprocal: 1/a = b / (a b), 1/b = a / (a b).
// The seeds err by about 1e-4 of the roots' spread, so relative to the
// smallest root distance they worsen as two roots close in.  With
// r = q / (2 p^1.5) = cos 3 theta, that distance over the spread is about
// sqrt((1 - |r|) / 3.4), and a wave where some lane has 1 - |r| below
// kNearDegenerate (distance under ~0.85 % of the spread: near a level
// crossing, or a matter term far above the vacuum splittings) adds one
// Newton step.  Elsewhere the corrected Halley step leaves the roots within
// ~1e-14 of their smallest distance, as Halley and Newton together do.
// HALLEY_ONLY (the FP32-mixed tier): a wave skips the Newton step when
// every lane's Halley corrections were at most 2^-12 of its smallest root
// distance.  Halley converges cubically, so the roots are then within about
// (2^-12)^3 ~ 1.5e-11 of that distance, far below what the FP32 amplitude
// assembly resolves, and the phases stay within ~1e-8 rad up to 1e3 rad.
constexpr double kHalleyOnly = 0x1p-12;
constexpr float kNearDegenerate = 0x1p-12f;
// Two roots closer than about 7e-4 of the spread (1 - |r| below this, near
// an exact level crossing, which needs a zero mixing angle) round r to
// within a few ulp of +-1 in FP32: both seeds then start from the pair's
// midpoint, where f' vanishes, and no refinement separates them.  Such a
// lane's P is undefined and comes out NaN (every such lane takes the
// Newton step, where this is applied).
constexpr float kUnresolved = 0x1p-19f;
// FP32-mixed tier: waves with a matter term above this (eV^2, about 4
// times the largest vacuum splitting) assemble the amplitude in FP64.
constexpr double kMixedWideA = 0.01;

template <bool HALLEY_ONLY = false>
__device__ __forceinline__ void cubic_roots(double tr, double c1, double det, double qh,
                                            double& l0, double& l1, double& l2)
{
    const double p = fma(tr, tr, -3.0 * c1);
    const float pf = float(p), qf = float(qh);
    const float rs = __builtin_amdgcn_rsqf(pf);                 // p^-1/2
    float rf = qf * (rs * rs * rs);                             // q / (2 p^3/2)
    rf = __builtin_fminf(1.0f, __builtin_fmaxf(-1.0f, rf));
    // theta in revolutions for the hardware cosine: acos(r) / (3 * 2 pi)
    const float th = acos_seed_rev(rf);
    // the seeds in FP32 (their FP32 rounding, ~6e-8 of |x|, is far below
    // their error of ~1e-4 of the roots' spread)
    const float kf = (2.0f / 3.0f) * (pf * rs);
    const float t3f = float(tr) * (1.0f / 3.0f);
    double x0 = double(__builtin_fmaf(kf, __builtin_amdgcn_cosf(th), t3f));
    double x1 = double(__builtin_fmaf(kf, __builtin_amdgcn_cosf(th - 0.33333333f), t3f));
    const double three = sgpr_value(3.0);
    // Halley: x -= 2 f f' / (2 f'^2 - f f'')
    {
        const double f0 = fma(fma(x0 - tr, x0, c1), x0, -det);
        const double f1 = fma(fma(x1 - tr, x1, c1), x1, -det);
        // m = tr - 3x = -f''/2, and f' = x (3x - 2 tr) + c1 = c1 - x (m + tr)
        const double m0 = fma(-three, x0, tr), m1 = fma(-three, x1, tr);
        const double g0 = fma(-x0, m0 + tr, c1);
        const double g1 = fma(-x1, m1 + tr, c1);
        const double d0 = fma(g0, g0, f0 * m0);
        const double d1 = fma(g1, g1, f1 * m1);
        const double r = recip_coarse(d0 * d1);
        if constexpr (!HALLEY_ONLY) {
            // the Halley step h and its leading error term: for this cubic
            // the root lies C h^3 beyond x - h, C = (f' - (3x - tr)^2) / f'^2
            // (to leading order; h is then the seed's error), so that term
            // is added; 1/f'^2 comes from the shared reciprocal, since
            // d = f'^2 (1 + O(h)).
            const double q0 = d1 * r, q1 = d0 * r;
            const double h0 = (f0 * g0) * q0, h1 = (f1 * g1) * q1;
            const double e0 = fma(-m0, m0, g0) * q0, e1 = fma(-m1, m1, g1) * q1;
            // x - h + e h^3 = x - h (1 - e h^2)
            x0 = fma(-h0, fma(-(e0 * h0), h0, 1.0), x0);
            x1 = fma(-h1, fma(-(e1 * h1), h1, 1.0), x1);
            if (!__any(__builtin_fabsf(rf) > 1.0f - kNearDegenerate)) {
                l0 = x0;
                l1 = x1;
                l2 = (tr - l0) - l1;
                return;
            }
        } else {
            const double h0 = (f0 * g0) * (d1 * r), h1 = (f1 * g1) * (d0 * r);
            x0 -= h0;
            x1 -= h1;
            // x0 > x1 > x2 = tr - x0 - x1: the smallest root distance is
            // x0 - x1 or x1 - x2 = 2 x1 + x0 - tr
            const double dmin = __builtin_fmin(__builtin_fabs(x0 - x1),
                                               __builtin_fabs(fma(2.0, x1, x0) - tr));
            const bool done = __builtin_fmax(__builtin_fabs(h0), __builtin_fabs(h1)) <=
                              kHalleyOnly * dmin;
            if (__all(done)) {
                l0 = x0;
                l1 = x1;
                l2 = (tr - l0) - l1;
                return;
            }
        }
    }
    // Newton: x -= f / f'
    {
        const double tr2 = 2.0 * tr;
        const double f0 = fma(fma(x0 - tr, x0, c1), x0, -det);
        const double f1 = fma(fma(x1 - tr, x1, c1), x1, -det);
        const double g0 = fma(x0, fma(three, x0, -tr2), c1);
        const double g1 = fma(x1, fma(three, x1, -tr2), c1);
        const double r = recip_coarse(g0 * g1);
        x0 -= f0 * (g1 * r);
        x1 -= f1 * (g0 * r);
        if (__builtin_fabsf(rf) > 1.0f - kUnresolved) x0 = __builtin_nan("");
    }
    l0 = x0;
    l1 = x1;
    l2 = (tr - l0) - l1;
}

// P(alpha -> beta) of one event.  The evolution operator over L is
// sum_k exp(-i phi_k) X_k with the spectral projectors
// X_k = (M - l_j)(M - l_l) / ((l_k - l_j)(l_k - l_l)); the common phase
// exp(-i phi_0) drops out of |.|^2, so only the differences phi_k - phi_0
// are formed.
template <bool MIXED>
__device__ __forceinline__ double event_prob(const SetConsts& sc, const Tables<MIXED>& T,
                                             double kA, double kL, double E, uint32_t f,
                                             const PolyRegs& pr = PolyRegs{})
{
    using Entry = std::conditional_t<MIXED, ChanF, ChanL>;
    using Real = std::conditional_t<MIXED, float, double>;
    // flag byte (alpha bits 0-1, beta bits 2-3, antineutrino bit 4) -> the
    // channel entry (conjugated for antineutrinos) and the sign of A
    const FlagInfo fl = T.flag[min(f, uint32_t(kFlagEntries - 1))];
    const Entry c = *reinterpret_cast<const Entry*>(
        reinterpret_cast<const unsigned char*>(T.ch) + fl.ch_off);
    const double A = flip_sign(kA * E, fl.sign);
    const Real dba = c.dba;   // [alpha = beta]; NaN for an invalid flag byte

    // amplitude inputs: M_ba and (M^2)_ba (FP32 in the mixed tier)
    const auto mad = [](Real a, Real b, Real d) -> Real {
        if constexpr (MIXED)
            return __builtin_fmaf(a, b, d);
        else
            return __builtin_fma(a, b, d);
    };
    const Real Ar = Real(A);
    const Real mre = mad(Ar, c.dee, c.m_re);
    const Real mim = c.m_im;
    const Real m2re = mad(Ar, mad(Ar, c.dee, c.g_re), c.m2_re);
    const Real m2im = mad(Ar, c.g_im, c.m2_im);

    // matter eigenvalues (FP64 in every tier)
    double l0, l1, l2;
    cubic_roots<MIXED>(sc.T0 + A, fma(A, sc.CA, sc.C0), A * sc.DA,
                       fma(fma(A + sc.QH2, A, sc.QH1), A, sc.QH0), l0, l1, l2);

    const double d01 = l0 - l1, d02 = l0 - l2, d12 = l1 - l2;
    const double Q = d01 * d02 * d12;
    const double R = recip(E * Q);
    const double invE = Q * R, invQ = E * R;
    // phase per eV^2 in units of pi/32 (FP64 tier) or of 2 pi (mixed tier)
    const double ph = (MIXED ? kL * (1.0 / 64.0) : kL) * invE;
    // numerator coefficients: N_k = (M^2)_ba - (l_j + l_l) M_ba + l_j l_l [a = b]
    // for k = 1, 2.  The projectors sum to the identity, so X0 = [a = b] -
    // X1 - X2 and S' = [a = b] + (exp(-i dphi1) - 1) X1 + (exp(-i dphi2) - 1) X2;
    // the projectors of a Hermitian matrix have entries of modulus <= 1, so
    // forming cos - 1 costs nothing in absolute accuracy.
    const double u1 = l0 + l2, v1 = l0 * l2;
    const double u2 = l0 + l1, v2 = l0 * l1;
    const double iD1 = -d02 * invQ, iD2 = d01 * invQ;

    double P;
    if constexpr (!MIXED) {
        double s1, e1, s2, e2;                        // sin and cos - 1
        phase_sincos(-d01, ph, T.sct, s1, e1, pr.p7, pr.q6);   // phi_1 - phi_0
        phase_sincos(-d02, ph, T.sct, s2, e2, pr.p7, pr.q6);   // phi_2 - phi_0
        const double x1r = fma(v1, dba, fma(-u1, mre, m2re)) * iD1;
        const double x1i = fma(-u1, mim, m2im) * iD1;
        const double x2r = fma(v2, dba, fma(-u2, mre, m2re)) * iD2;
        const double x2i = fma(-u2, mim, m2im) * iD2;
        const double sr = dba + e1 * x1r + s1 * x1i + e2 * x2r + s2 * x2i;
        const double si = e1 * x1i - s1 * x1r + e2 * x2i - s2 * x2r;
        P = sr * sr + si * si;
    } else {
        float s1, c1, s2, c2;
        phase_sincos_mixed(-d01, ph, s1, c1);
        phase_sincos_mixed(-d02, ph, s2, c2);
        if (__any(__builtin_fabs(A) > kMixedWideA)) {
            // Matter terms well above the vacuum splittings: the projector
            // numerators cancel over about |A| / dm^2_31, beyond what FP32
            // resolves, so such waves form them and the sum in FP64 (from
            // the same FP32 channel entries and FP32 phases).
            const double d_dee = c.dee, d_dba = c.dba;
            const double d_mre = fma(A, d_dee, double(c.m_re));
            const double d_mim = c.m_im;
            const double d_m2re = fma(A, fma(A, d_dee, double(c.g_re)), double(c.m2_re));
            const double d_m2im = fma(A, double(c.g_im), double(c.m2_im));
            const double x1r = fma(v1, d_dba, fma(-u1, d_mre, d_m2re)) * iD1;
            const double x1i = fma(-u1, d_mim, d_m2im) * iD1;
            const double x2r = fma(v2, d_dba, fma(-u2, d_mre, d_m2re)) * iD2;
            const double x2i = fma(-u2, d_mim, d_m2im) * iD2;
            const double e1 = double(c1) - 1.0, e2 = double(c2) - 1.0;
            const double ds1 = s1, ds2 = s2;
            const double sr = d_dba + e1 * x1r + ds1 * x1i + e2 * x2r + ds2 * x2i;
            const double si = e1 * x1i - ds1 * x1r + e2 * x2i - ds2 * x2r;
            return sr * sr + si * si;
        }
        // amplitude assembly in FP32 from FP32-rounded inputs
        const float fmre = mre, fmim = mim, fm2re = m2re, fm2im = m2im;
        const float fdba = dba;
        const float fu1 = float(u1), fu2 = float(u2);
        const float fv1 = float(v1), fv2 = float(v2);
        const float fi1 = float(iD1), fi2 = float(iD2);
        const float x1r = __builtin_fmaf(fv1, fdba, __builtin_fmaf(-fu1, fmre, fm2re)) * fi1;
        const float x1i = __builtin_fmaf(-fu1, fmim, fm2im) * fi1;
        const float x2r = __builtin_fmaf(fv2, fdba, __builtin_fmaf(-fu2, fmre, fm2re)) * fi2;
        const float x2i = __builtin_fmaf(-fu2, fmim, fm2im) * fi2;
        const float e1 = c1 - 1.0f, e2 = c2 - 1.0f;
        const float sr = fdba + e1 * x1r + s1 * x1i + e2 * x2r + s2 * x2i;
        const float si = e1 * x1i - s1 * x1r + e2 * x2i - s2 * x2r;
        P = double(sr * sr + si * si);
    }
    return P;
}

// P of one event through one constant-density layer: the policy the tile
// body calls (MIXED selects the FP32-mixed amplitude assembly).
template <bool MIXED>
struct ConstDensityProb {
    const SetConsts* sc;
    const Tables<MIXED>* tabs;
    double kA, kL;
    PolyRegs pr;
    __device__ __forceinline__ double operator()(double E, uint32_t f) const
    {
        return event_prob<MIXED>(*sc, *tabs, kA, kL, E, f, pr);
    }
};

// P(alpha -> beta) of one event through layers of constant density.  The
// evolution operator of the path is the product of the layers' operators,
// so only column alpha of it is needed: v = e_alpha is propagated layer by
// layer.  Within a layer, exp(-i M L / 2E) (common phase dropped) is the
// polynomial a2 M^2 + a1 M + a0 of its Lagrange form over the eigenvalues,
//   sum_k c_k (M - l_j)(M - l_l),  c_k = exp(-i dphi_k) / D_k,
// so v becomes a2 (M M v) + a1 (M v) + a0 v.  M is the flavour-basis mass
// matrix of the layer (H0 + A e_e e_e^T, conjugated with A -> -A for
// antineutrinos); its entries come from the channel table.  In the first
// layer v = e_alpha, so M v is column alpha of M; in the last layer only
// component beta of the new v is formed.  Both give the same roundings as
// the full products.
__device__ __forceinline__ double pick3(uint32_t k, double x0, double x1, double x2)
{
    return k == 0u ? x0 : (k == 1u ? x1 : x2);
}

__device__ __forceinline__ double event_prob_layered(const SetConsts& sc, const TileTables& T,
                                                     const LayerPath& lp, double E, uint32_t f)
{
    const bool valid = (f < 32u) && ((kValidFlags >> (f & 31u)) & 1u);
    const uint32_t a = min(f & 3u, 2u), b = min((f >> 2) & 3u, 2u);
    const uint32_t anti = (f << 27) & 0x80000000u;
    // H0 (conjugated for antineutrinos), row-major; the diagonal is real
    double hr[3][3], hi[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            hr[i][j] = T.ch[3 * i + j].m_re;
            hi[i][j] = flip_sign(T.ch[3 * i + j].m_im, anti);
        }
    double vr[3] = {a == 0u ? 1.0 : 0.0, a == 1u ? 1.0 : 0.0, a == 2u ? 1.0 : 0.0};
    double vi[3] = {0.0, 0.0, 0.0};
    const double invE = recip(E);
    for (int layer = 0; layer < lp.n; ++layer) {
        const PathConsts pc = lp.layer[layer];
        const double A = flip_sign(pc.kA * E, anti);
        double l0, l1, l2;
        cubic_roots(sc.T0 + A, fma(A, sc.CA, sc.C0), A * sc.DA,
                    fma(fma(A + sc.QH2, A, sc.QH1), A, sc.QH0), l0, l1, l2);
        const double d01 = l0 - l1, d02 = l0 - l2, d12 = l1 - l2;
        const double invQ = recip(d01 * d02 * d12);
        const double ph = pc.kL * invE;
        double s1, c1, s2, c2;
        phase_sincos(-d01, ph, T.sct, s1, c1);   // phi_1 - phi_0: sin, cos - 1
        phase_sincos(-d02, ph, T.sct, s2, c2);   // phi_2 - phi_0
        c1 += 1.0;
        c2 += 1.0;
        // c_k = exp(-i dphi_k) / D_k (c_0 real)
        const double iD0 = d12 * invQ, iD1 = -d02 * invQ, iD2 = d01 * invQ;
        const double k1r = c1 * iD1, k1i = -s1 * iD1;
        const double k2r = c2 * iD2, k2i = -s2 * iD2;
        const double u0 = l1 + l2, u1 = l0 + l2, u2 = l0 + l1;
        const double w0 = l1 * l2, w1 = l0 * l2, w2 = l0 * l1;
        const double a2r = iD0 + k1r + k2r, a2i = k1i + k2i;
        const double a1r = -(iD0 * u0 + k1r * u1 + k2r * u2), a1i = -(k1i * u1 + k2i * u2);
        const double a0r = iD0 * w0 + k1r * w1 + k2r * w2, a0i = k1i * w1 + k2i * w2;
        // y = M v
        double yr[3], yi[3], zr[3], zi[3];
        if (layer == 0) {
            // v = e_alpha: column alpha of H0, plus A on the (e, e) entry
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                yr[i] = pick3(a, hr[i][0], hr[i][1], hr[i][2]);
                yi[i] = pick3(a, hi[i][0], hi[i][1], hi[i][2]);
            }
            yr[0] = fma(A, vr[0], yr[0]);
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                double sr = (i == 0) ? A * vr[0] : 0.0, si = (i == 0) ? A * vi[0] : 0.0;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    sr = fma(hr[i][j], vr[j], fma(-hi[i][j], vi[j], sr));
                    si = fma(hr[i][j], vi[j], fma(hi[i][j], vr[j], si));
                }
                yr[i] = sr;
                yi[i] = si;
            }
        }
        if (layer == lp.n - 1) {
            // component beta of a2 (M y) + a1 y + a0 v: row beta of M
            double sr = (b == 0u) ? A * yr[0] : 0.0, si = (b == 0u) ? A * yi[0] : 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double mr = pick3(b, hr[0][j], hr[1][j], hr[2][j]);
                const double mi = pick3(b, hi[0][j], hi[1][j], hi[2][j]);
                sr = fma(mr, yr[j], fma(-mi, yi[j], sr));
                si = fma(mr, yi[j], fma(mi, yr[j], si));
            }
            const double ybr = pick3(b, yr[0], yr[1], yr[2]), ybi = pick3(b, yi[0], yi[1], yi[2]);
            const double vbr = pick3(b, vr[0], vr[1], vr[2]), vbi = pick3(b, vi[0], vi[1], vi[2]);
            const double nr = a2r * sr - a2i * si + a1r * ybr - a1i * ybi + a0r * vbr - a0i * vbi;
            const double ni = a2r * si + a2i * sr + a1r * ybi + a1i * ybr + a0r * vbi + a0i * vbr;
            vr[0] = nr;
            vi[0] = ni;
            break;
        }
        // z = M y
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double sr = (i == 0) ? A * yr[0] : 0.0, si = (i == 0) ? A * yi[0] : 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                sr = fma(hr[i][j], yr[j], fma(-hi[i][j], yi[j], sr));
                si = fma(hr[i][j], yi[j], fma(hi[i][j], yr[j], si));
            }
            zr[i] = sr;
            zi[i] = si;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double nr = a2r * zr[i] - a2i * zi[i] + a1r * yr[i] - a1i * yi[i] +
                              a0r * vr[i] - a0i * vi[i];
            const double ni = a2r * zi[i] + a2i * zr[i] + a1r * yi[i] + a1i * yr[i] +
                              a0r * vi[i] + a0i * vr[i];
            vr[i] = nr;
            vi[i] = ni;
        }
    }
    // the last layer left component beta in vr[0], vi[0]
    const double P = vr[0] * vr[0] + vi[0] * vi[0];
    return __hiloint2double(valid ? __double2hiint(P) : 0x7ff80000, __double2loint(P));
}

// P of one event through a layered path (FP64).
struct LayeredProb {
    const SetConsts* sc;
    const TileTables* tabs;
    const LayerPath* lp;
    __device__ __forceinline__ double operator()(double E, uint32_t f) const
    {
        return event_prob_layered(*sc, *tabs, *lp, E, f);
    }
};

// Bin of x: floor(fl(fl(x * scale - lo) / wb)) with under/overflow.  The
// quotient is first formed as fl(x * scale - lo) * fl(1 / wb); that is
// within 3 u |q| (u = 2^-53) of the correctly rounded quotient q, so the
// floors agree unless an integer lies within that distance.  Below
// kFastBinLimit = 2^12 in magnitude the distance is under 1.5 * 2^-40;
// lanes within 2^-38 of an integer are flagged and redone with the
// correctly rounded division.  Beyond 2^12 the bin is overflow (or
// underflow) either way, since no binning has that many bins.
__device__ __forceinline__ double bin_floor_fast(double x, const BinConsts& bc, bool& edge)
{
#pragma clang fp contract(off)
    const double d = x * bc.scale - bc.lo;   // scaled energy, then the offset: two roundings
    const double q = d * bc.inv_wb;
    const double k = __builtin_floor(q);
    edge = (__builtin_fabs((q - k) - 0.5) > 0.5 - 0x1p-38) && (__builtin_fabs(q) < kFastBinLimit);
    return k;
}

__device__ __forceinline__ double bin_floor_exact(double x, const BinConsts& bc)
{
#pragma clang fp contract(off)
    return __builtin_floor((x * bc.scale - bc.lo) / bc.wb);
}

// Row of floor value k in the LDS histograms: 0 underflow, 1 + k regular,
// nb + 1 overflow (NaN included: fmin returns the non-NaN operand).
__device__ __forceinline__ int lds_bin(double k, const BinConsts& bc)
{
    return int(__builtin_fmax(__builtin_fmin(k, double(bc.nb)), -1.0)) + 1;
}

// LDS row of output bin r (output order: nb regular bins, underflow, overflow).
__device__ __forceinline__ int lds_row_of_output(int r, int nb)
{
    return r < nb ? r + 1 : (r == nb ? 0 : nb + 1);
}

// Histogram accumulator slot: bin-major rows of kHistLanes accumulators,
// the accumulator index XOR-swizzled by the row so that both the per-lane
// accumulation and the per-bin transposed reads spread over the LDS banks.
// The swizzle uses row - 1 (the floor value k of the row), so that the
// row's +1 becomes a constant offset of the LDS instruction.
__device__ __forceinline__ int hslot(int row, int acc)
{
    return row * kHistLanes + (acc ^ ((row - 1) & (kHistLanes - 1)));
}

// complete binary tree over the kHistLanes accumulators of one bin
template <int N, int J0>
__device__ __forceinline__ double lane_tree(const double* h, int bin)
{
    if constexpr (N == 1) {
        return h[hslot(bin, J0)];
    } else {
        const double left = lane_tree<N / 2, J0>(h, bin);
        const double right = lane_tree<N / 2, J0 + N / 2>(h, bin);
        return left + right;
    }
}

// kPdfBinned: kPdf with the events' histogram slots read from a cached
// per-sample array (one 16-bit LDS slot index per event, see bin_slot)
// instead of computed from the reco energy.
enum Mode { kReweight = 0, kPdf = 1, kHist = 2, kPdfBinned = 3 };

constexpr bool reads_bins(int mode) { return mode == kPdfBinned; }
constexpr bool has_hist(int mode) { return mode != kReweight; }

struct EventIn {
    double e;       // true energy (or the given value in kHist mode)
    double w;
    double x;       // reco energy (kPdf, kHist)
    uint32_t f;
    uint32_t slot;  // cached histogram slot (kPdfBinned)
};

// The arrays of one tile as raw buffer resources (base in SGPRs, size in
// bytes as the bound): an event's loads and its P store then take the form
// buffer_load v, lane_offset, rsrc, group_offset -- the lane offset is
// loop-invariant, the group offset lives in an SGPR, and no per-event
// address arithmetic runs on the VALU.  Accesses past the bound read 0 and
// write nothing (the tail guards below still decide what is used).
constexpr int kBufDword3 = 0x00020000;   // gfx9 family: raw buffer, 32-bit data format
constexpr int kBufNonTemporal = 2;        // cache-policy operand: the nt bit
typedef unsigned int BufU2 __attribute__((ext_vector_type(2)));

struct TileBufs {
    __amdgpu_buffer_rsrc_t e, f, w, x, p;
};

template <int MODE>
__device__ __forceinline__ TileBufs tile_bufs(uint32_t n, const double* e_true,
                                              const uint8_t* flags, const double* weight,
                                              const double* e_reco, const uint16_t* bins,
                                              const double* value, double* p_out)
{
    const int nb = int(n * sizeof(double));
    TileBufs b;
    b.e = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double*>(MODE == kHist ? value : e_true), 0, nb, kBufDword3);
    b.f = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(flags), 0, int(n), kBufDword3);
    b.w = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(weight), 0, nb, kBufDword3);
    if constexpr (reads_bins(MODE))
        b.x = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(bins), 0,
                                                int(n * sizeof(uint16_t)), kBufDword3);
    else
        b.x = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(e_reco), 0, nb, kBufDword3);
    b.p = __builtin_amdgcn_make_buffer_rsrc(p_out, 0, nb, kBufDword3);
    return b;
}

__device__ __forceinline__ double buf_load_f64(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// The same arrays as plain pointers (global loads with 64-bit addresses):
// the batched kernel keeps this form, where the resources' SGPRs cost more
// than the address arithmetic they save.
struct TilePtrs {
    const double* e;
    const uint8_t* f;
    const double* w;
    const double* x;
    const uint16_t* s;
    double* p;
};

template <int MODE>
__device__ __forceinline__ TilePtrs tile_ptrs(const double* e_true, const uint8_t* flags,
                                              const double* weight, const double* e_reco,
                                              const uint16_t* bins, const double* value,
                                              double* p_out)
{
    return TilePtrs{MODE == kHist ? value : e_true, flags, weight, e_reco, bins, p_out};
}

template <int MODE, bool FULL>
__device__ __forceinline__ EventIn load_event(const TilePtrs& b, uint32_t l, uint32_t g0,
                                              uint32_t n)
{
    EventIn v;
    const uint32_t i = l + g0;
    const bool in = FULL || i < n;
    v.e = in ? b.e[i] : 1.0;
    v.f = (MODE != kHist && in) ? uint32_t(b.f[i]) : 0u;
    v.w = (has_hist(MODE) && in) ? b.w[i] : 0.0;
    v.x = (has_hist(MODE) && !reads_bins(MODE) && in) ? b.x[i] : 0.0;
    v.slot = (reads_bins(MODE) && in) ? uint32_t(b.s[i]) : 0u;
    return v;
}

__device__ __forceinline__ void store_p(const TilePtrs& b, uint32_t l, uint32_t g0, double P)
{
    __builtin_nontemporal_store(P, &b.p[l + g0]);
}

// Event g0 + l of a tile (0 <= g0 + l < kTileEvents); n = the tile's events
// (kTileEvents when FULL).  g0 is the same for the whole wave.
template <int MODE, bool FULL>
__device__ __forceinline__ EventIn load_event(const TileBufs& b, uint32_t l, uint32_t g0,
                                              uint32_t n)
{
    EventIn v;
    const bool in = FULL || l + g0 < n;
    const uint32_t l8 = l * 8u, g8 = g0 * 8u;
    v.e = in ? buf_load_f64(b.e, l8, g8) : 1.0;
    v.f = (MODE != kHist && in) ? uint32_t(__builtin_amdgcn_raw_buffer_load_b8(b.f, l, g0, 0))
                                : 0u;
    v.w = (has_hist(MODE) && in) ? buf_load_f64(b.w, l8, g8) : 0.0;
    v.x = (has_hist(MODE) && !reads_bins(MODE) && in) ? buf_load_f64(b.x, l8, g8) : 0.0;
    v.slot = (reads_bins(MODE) && in)
                 ? uint32_t(__builtin_amdgcn_raw_buffer_load_b16(b.x, l * 2u, g0 * 2u, 0))
                 : 0u;
    return v;
}

__device__ __forceinline__ void store_p(const TileBufs& b, uint32_t l, uint32_t g0, double P)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(BufU2, P), b.p, l * 8u, g0 * 8u,
                                          kBufNonTemporal);
}

// One group of kGroup events of a lane: the probabilities are computed in
// one straight-line block (no guards: lanes past the end of the sample hold
// dummy inputs), then stored, binned and accumulated in ascending m.
template <int MODE, bool WRITE_P, bool FULL, class PROB, class ARR>
__device__ __forceinline__ void tile_group(const PROB& prob, const BinConsts& bc, double* hist,
                                           int lane, uint32_t l, uint32_t g0, uint32_t n,
                                           const EventIn (&ev)[kGroup], const ARR& arr)
{
    constexpr bool kComputeBins = has_hist(MODE) && !reads_bins(MODE);
    double P[kGroup], k[kGroup];
    bool edge[kGroup];
#pragma unroll
    for (int j = 0; j < kGroup; ++j) {
        P[j] = (MODE != kHist) ? prob(ev[j].e, ev[j].f) : ev[j].e;
        edge[j] = false;
        k[j] = kComputeBins ? bin_floor_fast(ev[j].x, bc, edge[j]) : 0.0;
    }
    if (WRITE_P) {
#pragma unroll
        for (int j = 0; j < kGroup; ++j) {
            const uint32_t gj = g0 + j * kTileLanes;
            // streaming store (nt): P is not read again by this kernel, and
            // letting it allocate in L2 cost ~10 % of the kernel's time
            if (FULL || l + gj < n) store_p(arr, l, gj, P[j]);
        }
    }
    if (MODE == kReweight) return;
    bool any_edge = false;
#pragma unroll
    for (int j = 0; j < kGroup; ++j) any_edge |= edge[j];
    if (kComputeBins && __builtin_expect(any_edge, 0)) {
#pragma unroll
        for (int j = 0; j < kGroup; ++j)
            if (edge[j]) k[j] = bin_floor_exact(ev[j].x, bc);
    }
#pragma unroll
    for (int j = 0; j < kGroup; ++j) {
        if (FULL || l + g0 + j * kTileLanes < n) {
#pragma clang fp contract(off)
            const double cval = ev[j].w * P[j];            // rounded, never fused
            const int slot = reads_bins(MODE) ? int(ev[j].slot)
                                              : hslot(lds_bin(k[j], bc), lane & (kHistLanes - 1));
            // The lanes sharing an accumulator add in ascending lane order:
            // one masked LDS atomic add per lane group, group after group.
            // Within a group the lanes hit distinct accumulators, and the
            // DS instructions of a wave execute in issue order, so every
            // accumulator receives its additions in the contract's order
            // (the LDS adder rounds like v_add_f64: round to nearest even).
            // The empty asm with a memory clobber keeps the compiler from
            // merging or reordering the groups.
#pragma unroll
            for (int p = 0; p < kLaneShare; ++p) {
                if (lane / kHistLanes == p)
                    __hip_atomic_fetch_add(hist + slot, cval, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                asm volatile("" ::: "memory");
            }
        }
    }
}

// The kLaneEvents events of one lane of the tile whose arrays start at the
// tile's first event (n = the tile's events); the loads of group g + 1 are
// issued before group g is computed.  With ROLL the events run in a loop
// that is not unrolled (the last group reloads itself): about 6 KB of code
// instead of 60 KB and fewer live registers.  The callers choose it per
// kernel from measurements: rolled for the kernels that write P (both
// tiers) and for the batched kernel, fully unrolled for the kernels that
// write no P.
template <int MODE, bool WRITE_P, bool FULL, bool ROLL, bool BUF = true, class PROB>
__device__ __forceinline__ void tile_events(const PROB& prob, const BinConsts& bc, double* hist,
                                            int lane, uint32_t n, const double* e_true,
                                            const uint8_t* flags, const double* weight,
                                            const double* e_reco, const uint16_t* bins,
                                            const double* value, double* p_out)
{
    constexpr int kGroups = kLaneEvents / kGroup;
    const uint32_t l = uint32_t(lane);
    const auto bufs = [&] {
        if constexpr (BUF)
            return tile_bufs<MODE>(n, e_true, flags, weight, e_reco, bins, value, p_out);
        else
            return tile_ptrs<MODE>(e_true, flags, weight, e_reco, bins, value, p_out);
    }();
    if constexpr (ROLL) {
        EventIn cur[kGroup], nxt[kGroup];
#pragma unroll
        for (int j = 0; j < kGroup; ++j)
            cur[j] = load_event<MODE, FULL>(bufs, l, j * kTileLanes, n);
#pragma unroll 1
        for (int g = 0; g < kGroups; ++g) {
            const int gn = g + 1 < kGroups ? g + 1 : g;   // the last group reloads itself
#pragma unroll
            for (int j = 0; j < kGroup; ++j)
                nxt[j] = load_event<MODE, FULL>(bufs, l, (gn * kGroup + j) * kTileLanes, n);
            tile_group<MODE, WRITE_P, FULL>(prob, bc, hist, lane, l, g * kGroup * kTileLanes, n,
                                            cur, bufs);
#pragma unroll
            for (int j = 0; j < kGroup; ++j) cur[j] = nxt[j];
        }
    } else {
        EventIn ev[kGroups][kGroup];
#pragma unroll
        for (int j = 0; j < kGroup; ++j)
            ev[0][j] = load_event<MODE, FULL>(bufs, l, j * kTileLanes, n);
#pragma unroll
        for (int g = 0; g < kGroups; ++g) {
            if (g + 1 < kGroups) {
#pragma unroll
                for (int j = 0; j < kGroup; ++j)
                    ev[g + 1][j] = load_event<MODE, FULL>(bufs, l, ((g + 1) * kGroup + j) * kTileLanes,
                                                          n);
            }
            tile_group<MODE, WRITE_P, FULL>(prob, bc, hist, lane, l, g * kGroup * kTileLanes,
                                            n, ev[g], bufs);
        }
    }
}

// Tile of workgroup b of nb: workgroups are dispatched round-robin over the
// 8 XCDs (each with its own L2), so XCD x = b mod 8 is given the contiguous
// tile range that starts at x q + min(x, r) (q = nb / 8, r = nb mod 8); a
// bijection of [0, nb).  Neighbouring tiles then write their per-bin
// results into the same cache lines from one L2.
constexpr int64_t kXcds = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb)
{
    const int64_t q = nb / kXcds, r = nb % kXcds, x = b % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

// The arrays of one tile: the sample's arrays advanced to the tile's first
// event (absent arrays stay null) and the tile's event count.
struct TileArrays {
    const double* e_true;
    const uint8_t* flags;
    const double* weight;
    const double* e_reco;
    const uint16_t* bins;
    const double* value;
    double* p_out;
    uint32_t n;
};

__device__ __forceinline__ TileArrays tile_arrays(int64_t tile, int64_t n, const double* e_true,
                                                  const uint8_t* flags, const double* weight,
                                                  const double* e_reco, const uint16_t* bins,
                                                  const double* value, double* p_out)
{
    const int64_t t0 = tile * kTileEvents;
    TileArrays a;
    a.e_true = e_true ? e_true + t0 : nullptr;
    a.flags = flags ? flags + t0 : nullptr;
    a.weight = weight ? weight + t0 : nullptr;
    a.e_reco = e_reco ? e_reco + t0 : nullptr;
    a.bins = bins ? bins + t0 : nullptr;
    a.value = value ? value + t0 : nullptr;
    a.p_out = p_out ? p_out + t0 : nullptr;
    a.n = uint32_t(min(n - t0, int64_t(kTileEvents)));
    return a;
}

// Build the channel and flag tables of a parameter set in LDS (lanes 0-31
// of the block's first wave; the caller's barrier publishes them).  The
// mixed tier's tables hold the entries rounded to FP32.
template <bool MIXED = false>
__device__ __forceinline__ void load_tab(const SetConsts& sc, Tables<MIXED>& T, int lane)
{
    using Entry = std::conditional_t<MIXED, ChanF, ChanL>;
    if (lane < kLdsChannels) {
        ChanL e;
        if (lane < kInvalidChannel) {
            const int k = lane % kChannels;
            const Chan c = sc.ch[k];
            const bool conj = lane >= kChannels;
            e.m_re = c.m_re;
            e.m_im = conj ? -c.m_im : c.m_im;
            e.m2_re = c.m2_re;
            e.m2_im = conj ? -c.m2_im : c.m2_im;
            e.g_re = c.g_re;
            e.g_im = conj ? -c.g_im : c.g_im;
            e.dee = c.dee;
            e.dba = (k % 3 == k / 3) ? 1.0 : 0.0;
        } else {
            e.m_re = e.m_im = e.m2_re = e.m2_im = e.g_re = e.g_im = e.dee = 0.0;
            e.dba = __builtin_nan("");
        }
        if constexpr (MIXED)
            T.ch[lane] = ChanF{float(e.m_re), float(e.m_im), float(e.m2_re), float(e.m2_im),
                               float(e.g_re), float(e.g_im), float(e.dee), float(e.dba)};
        else
            T.ch[lane] = e;
    }
    if (lane < kFlagEntries) {
        const uint32_t f = uint32_t(lane);
        const bool valid = (kValidFlags >> f) & 1u;
        const uint32_t anti = (f >> 4) & 1u;
        const uint32_t entry =
            valid ? (f & 3u) + 3u * ((f >> 2) & 3u) + anti * uint32_t(kChannels)
                  : uint32_t(kInvalidChannel);
        T.flag[lane] = FlagInfo{entry * uint32_t(sizeof(Entry)), valid && anti ? 0x80000000u : 0u};
    }
}

__device__ __forceinline__ void hist_zero(double* hist, int lane, int nbt)
{
    for (int i = lane; i < nbt * kHistLanes; i += kTileLanes) hist[i] = 0.0;
}

// Tree over the 64 lanes of every bin of a finished tile, written as row
// `row` of the tile results at `out` (chunked bin-major layout).
__device__ __forceinline__ void tile_write(const double* hist, int lane, int nbt, int64_t row,
                                           double* out)
{
    for (int bin = lane; bin < nbt; bin += kTileLanes)
        out[partial_index(row, bin, nbt)] =
            lane_tree<kHistLanes, 0>(hist, lds_row_of_output(bin, nbt - 2));
}

// Adjacent-pair tree across the 64 lanes of a wave (xor butterfly: both
// partners of a pair form the same sum), result in every lane.
__device__ __forceinline__ double wave_tree(double v)
{
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) v = v + __shfl_xor(v, s, 64);
    return v;
}

// One merge level (see MergeLevel): block (gc, bin, set) reduces chunk gc
// of the set's input rows for one bin.  Thread t adds its kMergeThreadRows
// contiguous rows (+0.0 beyond the sample's rows) as a binary tree in
// registers; the 64 lanes of a wave meet in the butterfly tree and the
// block's waves in a last binary tree.
template <bool FINAL>
__device__ __forceinline__ void merge_level_block(const MergeLevel& L, const double* __restrict__ in,
                                                  double* __restrict__ out)
{
    __shared__ double wave_sum[kMergeWaves];
    const int nbt = L.nbt;
    const int bin = int(blockIdx.y);
    const int64_t gc = blockIdx.x, set = blockIdx.z;
    int s = 0;
    while (s + 1 < L.n_samples && gc >= L.chunk0[s + 1]) ++s;
    const int64_t c = gc - L.chunk0[s];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t first = c * kMergeChunkRows + int64_t(t) * kMergeThreadRows;
    const int64_t count = L.rows[s] - first;
    const double* src = in + set * L.set_stride_in + partial_index(L.in_row0[s] + first, bin, nbt);
    double v[kMergeThreadRows];
    if (count >= kMergeThreadRows) {
#pragma unroll
        for (int i = 0; i < kMergeThreadRows; ++i) v[i] = src[i];
    } else {
#pragma unroll
        for (int i = 0; i < kMergeThreadRows; ++i) v[i] = i < count ? src[i] : 0.0;
    }
#pragma unroll
    for (int w = kMergeThreadRows / 2; w >= 1; w >>= 1)
#pragma unroll
        for (int i = 0; i < w; ++i) v[i] = v[2 * i] + v[2 * i + 1];
    const double r = wave_tree(v[0]);
    if (lane == 0) wave_sum[wave] = r;
    __syncthreads();
    if (t == 0) {
        // binary tree over the waves' sums, in wave order
        double w[kMergeWaves];
#pragma unroll
        for (int i = 0; i < kMergeWaves; ++i) w[i] = wave_sum[i];
#pragma unroll
        for (int h = kMergeWaves / 2; h >= 1; h >>= 1)
#pragma unroll
            for (int i = 0; i < h; ++i) w[i] = w[2 * i] + w[2 * i + 1];
        const double total = w[0];
        if (FINAL)
            out[(set * L.n_samples + s) * nbt + bin] = total;
        else
            out[set * L.set_stride_out + partial_index(L.out_row0[s] + c, bin, nbt)] = total;
    }
}

}  // namespace dev
}  // namespace osc
