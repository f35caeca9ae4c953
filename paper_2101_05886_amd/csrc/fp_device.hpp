// fp_device.hpp -- device-side arithmetic of the free-stream-preserving face
// flux for gfx950 (CDNA4, wave64).  Included by the kernel headers only.
//
// One face i+1/2 of one grid line is evaluated by one lane.  The lane reads
// the stencil nodes through a loader (slot r = 0..7 <-> node i-3+r) phase by
// phase, so that only the values of the current phase are live in registers:
//   A. cell-face 1/J, metrics and Q~ = Q/J by the central interpolation of
//      the metric order Y; reference state Q* = Q~_f/(1/J)_f and reference
//      face flux F~*_f = F(Q*) s_f                                    [FP64]
//   B. Roe average of nodes i, i+1, unit normal, eigen-structure       [T]
//   C. per stencil node m = i-2..i+3: reference-subtracted dQ~_m, dF~_m
//      [FP64], local Lax-Friedrichs speeds, characteristic projections [T]
//   D. WENO5-JS (or WENO7-JS on slots 0..7) of both split parts of every
//      field, or (linear upwind) the closed form
//      central6(dF~) + (1/60) R Lambda L Delta^5(dQ~)                  [T]
//   E. back-projection and add-back of F~*_f                   [T, FP64 add]
// T is double for the FP64 path and float for the mixed path.
#pragma once
#include <hip/hip_runtime.h>

namespace fpk {

struct SchemeK {
    double gamma;
    double eps;
    int reform;  // 1: reference state subtracted (the paper); 0: standard scheme
    // floor of the Lax-Friedrichs speeds of the sweep direction (u_n - c,
    // u_n, u_n + c): the face takes max(local speed, floor).  With global
    // speeds the floor is the block's largest local speed, so the face takes
    // the global one (at the face that attains it, the larger of the two
    // roundings); with local speeds it points at zeros.  Never null.
    const double* glf;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// 1/x from the hardware approximation refined by two Newton steps
// (y <- y + y(1 - x y)); within a couple of ulps for normal x.
__device__ __forceinline__ double drcp(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

template <typename T>
__device__ __forceinline__ T rcp(T x);
template <>
__device__ __forceinline__ double rcp<double>(double x) { return drcp(x); }
template <>
__device__ __forceinline__ float rcp<float>(float x) { return fast_rcp(x); }

// Reduced-precision forms for the characteristic basis only (normal,
// tangents, Roe weights, sound speeds, eigenvalue scale): one Newton step
// on the hardware estimate leaves a relative error near 2^-46, far below
// the 1e-12 the flux is held to, and these quantities multiply
// reference-subtracted differences, so the free stream does not see them.
// (Newton's iteration for 1/x and for 1/sqrt(x).)  The reference state keeps
// the two-step drcp.
__device__ __forceinline__ double drcp1(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}
__device__ __forceinline__ double drsq1(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

template <typename T>
__device__ __forceinline__ T rcp1(T x);
template <>
__device__ __forceinline__ double rcp1<double>(double x) { return drcp1(x); }
template <>
__device__ __forceinline__ float rcp1<float>(float x) { return fast_rcp(x); }

template <typename T>
__device__ __forceinline__ T rsq1(T x);
template <>
__device__ __forceinline__ double rsq1<double>(double x) { return drsq1(x); }
template <>
__device__ __forceinline__ float rsq1<float>(float x) { return __builtin_amdgcn_rsqf(x); }

template <typename T>
__device__ __forceinline__ T vsqrt(T x);
template <>
__device__ __forceinline__ double vsqrt<double>(double x) { return sqrt(x); }
template <>
__device__ __forceinline__ float vsqrt<float>(float x) { return fast_sqrt(x); }

// central face interpolation weights of order Y on slot r (node i in slot 3)
template <int Y>
__device__ __forceinline__ constexpr double iw(int r) {
    if constexpr (Y == 2) {
        return (r == 3 || r == 4) ? 0.5 : 0.0;
    } else if constexpr (Y == 4) {
        return (r == 3 || r == 4) ? 7.0 / 12.0 : ((r == 2 || r == 5) ? -1.0 / 12.0 : 0.0);
    } else if constexpr (Y == 6) {
        return (r == 3 || r == 4) ? 37.0 / 60.0
             : ((r == 2 || r == 5) ? -8.0 / 60.0 : ((r == 1 || r == 6) ? 1.0 / 60.0 : 0.0));
    } else {
        return (r == 3 || r == 4) ? 533.0 / 840.0
             : (r == 2 || r == 5) ? -139.0 / 840.0
             : (r == 1 || r == 6) ? 29.0 / 840.0 : -3.0 / 840.0;
    }
}

// WENO5-JS of a 5-point window a..e (face between c and d, upwind side a),
// in a scaled form.  The window holds twice the split values and eps16 is
// 16 eps: the indicators are evaluated as 4 beta_k = 13/3 t^2 + s^2 of the
// doubled window, i.e. 16 beta_k of the split values, so with 16 eps every
// weight is that of the split values (powers of two: exact), and the
// result is twice their reconstruction.  (The flux splitting's 1/2 is
// applied once, after the back-projection.)  The optimal weights
// C = (1/10, 3/5, 3/10) are folded into the candidates' constants:
// c_k = C_k (6 q_k), and the denominator carries 6 C_k.
// FP64: weights C_k/(beta_k+eps)^2 normalised over one common denominator
// (products of the squared indicators), one reciprocal per reconstruction.
__device__ __forceinline__ double weno5(double a, double b, double c, double d, double e,
                                        double eps16) {
    const double c0 = 0.2 * a - 0.7 * b + 1.1 * c;
    const double c1 = -0.6 * b + 3.0 * c + 1.2 * d;
    const double c2 = 0.6 * c + 1.5 * d - 0.3 * e;
    const double t0 = a - 2.0 * b + c, s0 = a - 4.0 * b + 3.0 * c;
    const double t1 = b - 2.0 * c + d, s1 = d - b;
    const double t2 = c - 2.0 * d + e, s2 = 3.0 * c - 4.0 * d + e;
    const double k = 13.0 / 3.0;
    double d0 = fma(k * t0, t0, fma(s0, s0, eps16));
    double d1 = fma(k * t1, t1, fma(s1, s1, eps16));
    double d2 = fma(k * t2, t2, fma(s2, s2, eps16));
    d0 *= d0;
    d1 *= d1;
    d2 *= d2;
    const double p0 = d1 * d2, p1 = d0 * d2, p2 = d0 * d1;
    const double num = fma(p0, c0, fma(p1, c1, p2 * c2));
    const double den = fma(p0, 0.6, fma(p1, 3.6, p2 * 1.8));
    return num * drcp1(den);
}

// FP32 form: reciprocal weights (no overflow of the products for large beta)
__device__ __forceinline__ float weno5(float a, float b, float c, float d, float e, float eps16) {
    const float c0 = 0.2f * a - 0.7f * b + 1.1f * c;
    const float c1 = -0.6f * b + 3.0f * c + 1.2f * d;
    const float c2 = 0.6f * c + 1.5f * d - 0.3f * e;
    const float t0 = a - 2.0f * b + c, s0 = a - 4.0f * b + 3.0f * c;
    const float t1 = b - 2.0f * c + d, s1 = d - b;
    const float t2 = c - 2.0f * d + e, s2 = 3.0f * c - 4.0f * d + e;
    const float k = 13.0f / 3.0f;
    const float d0 = fmaf(k * t0, t0, fmaf(s0, s0, eps16));
    const float d1 = fmaf(k * t1, t1, fmaf(s1, s1, eps16));
    const float d2 = fmaf(k * t2, t2, fmaf(s2, s2, eps16));
    const float r0 = fast_rcp(d0 * d0), r1 = fast_rcp(d1 * d1), r2 = fast_rcp(d2 * d2);
    const float num = fmaf(r0, c0, fmaf(r1, c1, r2 * c2));
    const float den = fmaf(r0, 0.6f, fmaf(r1, 3.6f, r2 * 1.8f));
    return num * fast_rcp(den);
}

// WENO7-JS of a 7-point window v[0..6] (face between v[3] and v[4], upwind
// side v[0]): four cubic candidates, optimal weights (1, 12, 18, 4)/35,
// smoothness indicators as the integer quadratic forms (240 x the Jiang-Shu
// measure), weights C_k/(beta_k+eps)^2 from reciprocals (the indicators can
// be large, so no common-denominator products).  Called on twice the split
// values with 4 eps, it returns twice their reconstruction (the indicators
// are quadratic: exact).
template <typename T>
__device__ __forceinline__ T weno7(const T (&v)[7], T eps) {
    const T a = v[0], b = v[1], c = v[2], d = v[3], e = v[4], f = v[5], g = v[6];
    const T q0 = T(-3) * a + T(13) * b - T(23) * c + T(25) * d;
    const T q1 = b - T(5) * c + T(13) * d + T(3) * e;
    const T q2 = -c + T(7) * d + T(7) * e - f;
    const T q3 = T(3) * d + T(13) * e - T(5) * f + g;
    T b0 = a * (T(547) * a - T(3882) * b + T(4642) * c - T(1854) * d) +
           b * (T(7043) * b - T(17246) * c + T(7042) * d) + c * (T(11003) * c - T(9402) * d) +
           T(2107) * d * d;
    T b1 = b * (T(267) * b - T(1642) * c + T(1602) * d - T(494) * e) +
           c * (T(2843) * c - T(5966) * d + T(1922) * e) + d * (T(3443) * d - T(2522) * e) +
           T(547) * e * e;
    T b2 = c * (T(547) * c - T(2522) * d + T(1922) * e - T(494) * f) +
           d * (T(3443) * d - T(5966) * e + T(1602) * f) + e * (T(2843) * e - T(1642) * f) +
           T(267) * f * f;
    T b3 = d * (T(2107) * d - T(9402) * e + T(7042) * f - T(1854) * g) +
           e * (T(11003) * e - T(17246) * f + T(4642) * g) + f * (T(7043) * f - T(3882) * g) +
           T(547) * g * g;
    b0 += eps;
    b1 += eps;
    b2 += eps;
    b3 += eps;
    const T a0 = T(1) * rcp<T>(b0 * b0), a1 = T(12) * rcp<T>(b1 * b1);
    const T a2 = T(18) * rcp<T>(b2 * b2), a3 = T(4) * rcp<T>(b3 * b3);
    return (a0 * q0 + a1 * q1 + a2 * q2 + a3 * q3) * rcp<T>(T(12) * (a0 + a1 + a2 + a3));
}

// WENOCU6 (the adaptive central-upwind sixth-order WENO of Hu, Wang and Adams,
// Remark 2) of a 6-point window v[0..5] = f_{i-2} .. f_{i+3}, the face between
// v[2] and v[3].  Candidates: the three upwind quadratics of WENO5 and the
// downwind one on {i+1, i+2, i+3}; optimal weights (1, 9, 9, 1)/20 (the
// sixth-order central interpolation).  The downwind slot's indicator is beta6,
// the Jiang-Shu measure (derivative orders 1..5 over cell i) of the quintic
// through all six cell averages, evaluated from the quintic's Taylor
// coefficients D_l = p^(l) at the centre of cell i: each D_l is a difference
// stencil (its coefficients sum to zero), so beta6 keeps its accuracy in FP32,
// where the expanded integer quadratic form of the six values cancels to
// noise.  Weights alpha_k = d_k (C + tau6/(beta_k + eps))^2, C = 20,
// tau6 = beta6 - (beta_0 + 4 beta_1 + beta_2)/6, evaluated as
// ((C m + tau6 m/(beta_k+eps)) / (m + |tau6|))^2 with m = min_k (beta_k+eps):
// the same ratios, every factor in [-C, C], so no overflow for any eps.
// Called on twice the split values with 4 eps, it returns twice their
// reconstruction (indicators and tau6 are quadratic: exact).
template <typename T>
__device__ __forceinline__ T wenocu6(const T (&v)[6], T eps) {
    const T a = v[0], b = v[1], c = v[2], d = v[3], e = v[4], f = v[5];
    const T q0 = T(2) * a - T(7) * b + T(11) * c;
    const T q1 = -b + T(5) * c + T(2) * d;
    const T q2 = T(2) * c + T(5) * d - e;
    const T q3 = T(11) * d - T(7) * e + T(2) * f;
    const T t0 = a - T(2) * b + c, s0 = a - T(4) * b + T(3) * c;
    const T t1 = b - T(2) * c + d, s1 = d - b;
    const T t2 = c - T(2) * d + e, s2 = T(3) * c - T(4) * d + e;
    const T k13 = T(13.0 / 12.0);
    const T b0 = k13 * t0 * t0 + T(0.25) * s0 * s0;
    const T b1 = k13 * t1 * t1 + T(0.25) * s1 * s1;
    const T b2 = k13 * t2 * t2 + T(0.25) * s2 * s2;
    const T D1 = (T(341) * a - T(2785) * b - T(2590) * c + T(6670) * d - T(1895) * e + T(259) * f) *
                 T(1.0 / 5760.0);
    const T D2 = (-a + T(12) * b - T(22) * c + T(12) * d - e) * T(0.125);
    const T D3 = (T(-5) * a - T(11) * b + T(70) * c - T(94) * d + T(47) * e - T(7) * f) * T(1.0 / 24.0);
    const T D4 = a - T(4) * b + T(6) * c - T(4) * d + e;
    const T D5 = -a + T(5) * b - T(10) * c + T(10) * d - T(5) * e + f;
    const T b6 = D1 * (D1 + D3 * T(1.0 / 12.0) + D5 * T(1.0 / 960.0)) +
                 D2 * (D2 * T(13.0 / 12.0) + D4 * T(7.0 / 80.0)) +
                 D3 * (D3 * T(1043.0 / 960.0) + D5 * T(4709.0 / 53760.0)) +
                 D4 * D4 * T(87617.0 / 80640.0) + D5 * D5 * T(50467427.0 / 46448640.0);
    const T tau = b6 - (b0 + T(4) * b1 + b2) * T(1.0 / 6.0);
    const T e0 = b0 + eps, e1 = b1 + eps, e2 = b2 + eps, e3 = b6 + eps;
    const T m = fmin(fmin(e0, e1), fmin(e2, e3));
    const T ig = rcp<T>(m + fabs(tau));
    const T sC = T(20) * (m * ig), st = tau * ig;
    const T w0 = sC + st * (m * rcp<T>(e0)), w1 = sC + st * (m * rcp<T>(e1));
    const T w2 = sC + st * (m * rcp<T>(e2)), w3 = sC + st * (m * rcp<T>(e3));
    const T a0 = w0 * w0, a1 = T(9) * (w1 * w1), a2 = T(9) * (w2 * w2), a3 = w3 * w3;
    return (a0 * q0 + a1 * q1 + a2 * q2 + a3 * q3) * rcp<T>(T(6) * (a0 + a1 + a2 + a3));
}

// ---------------------------------------------------------------------------
// phase A: cell-face reference state
// ---------------------------------------------------------------------------

template <int DIM>
struct FaceRef {
    double Vf;
    double sf[DIM];
    double Qs[DIM + 2];  // Q* (zero for the standard scheme)
    double us[DIM];      // u*
    double ps;           // p*
    double Fts[DIM + 2]; // F(Q*) . s_f
    double s2;           // |s_f|^2
};

template <int DIM, int Y, class LD>
__device__ __forceinline__ void face_ref(const LD& ld, const SchemeK& sk, FaceRef<DIM>& R) {
    constexpr int NV = DIM + 2, E = NV - 1;
    constexpr int r0 = 4 - Y / 2, r1 = 4 + Y / 2;  // interpolation slots [r0, r1)
    double Vf = 0.0, sf[DIM], Qt[NV];
#pragma unroll
    for (int c = 0; c < DIM; ++c) sf[c] = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) Qt[v] = 0.0;
#pragma unroll
    for (int r = r0; r < r1; ++r) {
        double q[NV], V, s[DIM];
        ld.slot(r, q, V, s);
        const double w = iw<Y>(r);
        Vf += w * V;
#pragma unroll
        for (int c = 0; c < DIM; ++c) sf[c] += w * s[c];
#pragma unroll
        for (int v = 0; v < NV; ++v) Qt[v] += w * (q[v] * V);
    }
    R.Vf = Vf;
#pragma unroll
    for (int c = 0; c < DIM; ++c) R.sf[c] = sf[c];
    R.ps = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) R.Qs[v] = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) R.us[c] = 0.0;
    if (sk.reform) {
        const double iVf = drcp(Vf);
#pragma unroll
        for (int v = 0; v < NV; ++v) R.Qs[v] = Qt[v] * iVf;
        const double irs = drcp(R.Qs[0]);
        double m2 = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            R.us[c] = R.Qs[1 + c] * irs;
            m2 += R.Qs[1 + c] * R.us[c];
        }
        R.ps = (sk.gamma - 1.0) * (R.Qs[E] - 0.5 * m2);
    }
    double U = 0.0, s2 = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        U += R.us[c] * sf[c];
        s2 += sf[c] * sf[c];
    }
    R.Fts[0] = R.Qs[0] * U;
#pragma unroll
    for (int c = 0; c < DIM; ++c) R.Fts[1 + c] = R.Qs[1 + c] * U + R.ps * sf[c];
    R.Fts[E] = (R.Qs[E] + R.ps) * U;
    R.s2 = s2;
}

// ---------------------------------------------------------------------------
// phase B: Roe average and characteristic basis
// ---------------------------------------------------------------------------

template <int DIM, typename T>
struct Eig {
    T n[DIM], uh[DIM], t1[DIM], t2[3];
    T un, Hh, ch, hq2, ut1, ut2, sigma;
    // the projection's scales, halved: with b2 = (gamma-1)/c^2 and ic = 1/c,
    // pB = b2/2 and pI = ic/2
    T pB, pI;
};

template <int DIM, typename T, class LD>
__device__ __forceinline__ void roe(const LD& ld, const SchemeK& sk, const FaceRef<DIM>& R,
                                    Eig<DIM, T>& S) {
    constexpr int NV = DIM + 2, E = NV - 1;
    const double gm1 = sk.gamma - 1.0;
    const double isn = drsq1(R.s2);  // 1/|s_f|
#pragma unroll
    for (int c = 0; c < DIM; ++c) S.n[c] = T(R.sf[c] * isn);
    S.sigma = T(R.s2 * isn * drcp1(R.Vf));
    double uL[DIM], uR[DIM], HL, HR, rL, rR;
    {
        double q[NV], V, s[DIM];
        ld.slot(3, q, V, s);
        const double ir = drcp(q[0]);
        double m2 = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            uL[c] = q[1 + c] * ir;
            m2 += q[1 + c] * uL[c];
        }
        HL = (q[E] + gm1 * (q[E] - 0.5 * m2)) * ir;
        rL = q[0];
    }
    {
        double q[NV], V, s[DIM];
        ld.slot(4, q, V, s);
        const double ir = drcp(q[0]);
        double m2 = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            uR[c] = q[1 + c] * ir;
            m2 += q[1 + c] * uR[c];
        }
        HR = (q[E] + gm1 * (q[E] - 0.5 * m2)) * ir;
        rR = q[0];
    }
    const T wL = T(rL) * rsq1<T>(T(rL)), wR = T(rR) * rsq1<T>(T(rR));
    const T iwr = rcp1<T>(wL + wR);
    T q2 = T(0), un = T(0);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        S.uh[c] = (wL * T(uL[c]) + wR * T(uR[c])) * iwr;
        q2 += S.uh[c] * S.uh[c];
        un += S.uh[c] * S.n[c];
    }
    S.un = un;
    S.Hh = (wL * T(HL) + wR * T(HR)) * iwr;
    const T c2 = T(gm1) * (S.Hh - T(0.5) * q2);
    const T ic = rsq1<T>(c2);
    S.ch = c2 * ic;
    S.hq2 = T(0.5) * q2;
    S.pB = T(0.5 * gm1) * (ic * ic);
    S.pI = T(0.5) * ic;
    if constexpr (DIM == 2) {
        S.t1[0] = -S.n[1];
        S.t1[1] = S.n[0];
        S.ut1 = S.uh[0] * S.t1[0] + S.uh[1] * S.t1[1];
        S.ut2 = T(0);
    } else {
        // a = argmin |n_k|, components within 1e-10 count as tied and the
        // lowest k wins; t1 = normalize(n x e_a), t2 = n x t1
        const T tie = T(1e-10);
        const T a0 = fabs(S.n[0]), a1 = fabs(S.n[1]), a2 = fabs(S.n[2]);
        int a = 0;
        T am = a0;
        if (a1 < am - tie) { a = 1; am = a1; }
        if (a2 < am - tie) { a = 2; }
        T x0, x1, x2;
        if (a == 0) { x0 = T(0); x1 = S.n[2]; x2 = -S.n[1]; }
        else if (a == 1) { x0 = -S.n[2]; x1 = T(0); x2 = S.n[0]; }
        else { x0 = S.n[1]; x1 = -S.n[0]; x2 = T(0); }
        const T ix = rsq1<T>(x0 * x0 + x1 * x1 + x2 * x2);
        S.t1[0] = x0 * ix;
        S.t1[1] = x1 * ix;
        S.t1[2] = x2 * ix;
        S.t2[0] = S.n[1] * S.t1[2] - S.n[2] * S.t1[1];
        S.t2[1] = S.n[2] * S.t1[0] - S.n[0] * S.t1[2];
        S.t2[2] = S.n[0] * S.t1[1] - S.n[1] * S.t1[0];
        S.ut1 = S.uh[0] * S.t1[0] + S.uh[1] * S.t1[1] + S.uh[2] * S.t1[2];
        S.ut2 = S.uh[0] * S.t2[0] + S.uh[1] * S.t2[1] + S.uh[2] * S.t2[2];
    }
}

// ---------------------------------------------------------------------------
// phase C helper: reference-subtracted values and LF speeds at one node
// ---------------------------------------------------------------------------

template <int DIM, typename T>
struct NodeDiff {
    double dQ[DIM + 2], dF[DIM + 2];
    T un, cs;
};

template <int DIM, typename T, class LD>
__device__ __forceinline__ void node_diff(const LD& ld, int r, const SchemeK& sk,
                                          const FaceRef<DIM>& R, const Eig<DIM, T>& S,
                                          NodeDiff<DIM, T>& N) {
    constexpr int NV = DIM + 2, E = NV - 1;
    const double gm1 = sk.gamma - 1.0;
    double q[NV], V, s[DIM];
    ld.slot(r, q, V, s);
    const double ir = drcp(q[0]);
    double u[DIM], m2 = 0.0, U = 0.0, Us = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        u[c] = q[1 + c] * ir;
        m2 += q[1 + c] * u[c];
        U += u[c] * s[c];
        Us += R.us[c] * s[c];
    }
    const double p = gm1 * (q[E] - 0.5 * m2);
    const double dp = p - R.ps;
    N.dF[0] = q[0] * U - R.Qs[0] * Us;
#pragma unroll
    for (int c = 0; c < DIM; ++c) N.dF[1 + c] = q[1 + c] * U - R.Qs[1 + c] * Us + dp * s[c];
    N.dF[E] = (q[E] + p) * U - (R.Qs[E] + R.ps) * Us;
#pragma unroll
    for (int v = 0; v < NV; ++v) N.dQ[v] = (q[v] - R.Qs[v]) * V;
    T un = T(0);
#pragma unroll
    for (int c = 0; c < DIM; ++c) un += S.n[c] * T(u[c]);
    N.un = un;
    const T c2 = T(sk.gamma * p * ir);
    N.cs = c2 > T(0) ? c2 * rsq1<T>(c2) : T(0);
}

// l_s . w for the five (four in 2D) fields, using the structure of the Euler
// eigenvectors: l_0 w = (phi - psi)/2, l_1 w = w_0 - phi, l_t w = t.w_m -
// (u.t) w_0, l_E w = (phi + psi)/2 with phi = b2 (|u|^2/2 w_0 - u.w_m + w_E)
// and psi = (n.w_m - u_n w_0)/c; evaluated as phi/2 and psi/2 with the
// halved scales of Eig.
template <int DIM, typename T>
__device__ __forceinline__ void project(const Eig<DIM, T>& S, const T (&w)[DIM + 2],
                                        T (&a)[DIM + 2]) {
    constexpr int E = DIM + 1;
    T uw = T(0), nw = T(0), t1w = T(0), t2w = T(0);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        uw += S.uh[c] * w[1 + c];
        nw += S.n[c] * w[1 + c];
        t1w += S.t1[c] * w[1 + c];
        if constexpr (DIM == 3) t2w += S.t2[c] * w[1 + c];
    }
    const T phi = S.pB * (S.hq2 * w[0] - uw + w[E]);
    const T psi = (nw - S.un * w[0]) * S.pI;
    a[0] = phi - psi;
    a[1] = w[0] - T(2) * phi;
    a[2] = t1w - S.ut1 * w[0];
    if constexpr (DIM == 3) a[3] = t2w - S.ut2 * w[0];
    a[E] = phi + psi;
}

// R h: back to conservative components
template <int DIM, typename T>
__device__ __forceinline__ void backproject(const Eig<DIM, T>& S, const T (&h)[DIM + 2],
                                            T (&o)[DIM + 2]) {
    constexpr int E = DIM + 1;
    const T h0 = h[0], h1 = h[1], hE = h[E];
    const T hsum = h0 + h1 + hE, hdif = hE - h0;
    o[0] = hsum;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        T m = S.uh[c] * hsum + S.ch * S.n[c] * hdif + S.t1[c] * h[2];
        if constexpr (DIM == 3) m += S.t2[c] * h[3];
        o[1 + c] = m;
    }
    T en = S.Hh * (h0 + hE) + S.ch * S.un * hdif + S.hq2 * h1 + S.ut1 * h[2];
    if constexpr (DIM == 3) en += S.ut2 * h[3];
    o[E] = en;
}

// ---------------------------------------------------------------------------
// the face flux: WENO5-JS and WENOCU6 (stencil nodes i-2 .. i+3, slots 1..6)
// ---------------------------------------------------------------------------

template <int DIM, int Y, typename T, bool CU6, class LD>
__device__ __forceinline__ void face_flux_weno(const LD& ld, const SchemeK& sk,
                                               double (&Fo)[DIM + 2]) {
    constexpr int NV = DIM + 2, E = NV - 1;
    FaceRef<DIM> R;
    face_ref<DIM, Y>(ld, sk, R);
    Eig<DIM, T> S;
    roe<DIM, T>(ld.after(R.Vf), sk, R, S);
    // per stencil node: projections of dF~ (a) and dQ~ (b) on every field
    T a[NV][6], b[NV][6];
    T mxm = T(0), mx0 = T(0), mxp = T(0);
    double chain = double(S.pI);
#pragma unroll
    for (int r = 1; r <= 6; ++r) {
        NodeDiff<DIM, T> N;
        node_diff<DIM, T>(ld.after(chain), r, sk, R, S, N);
        chain = N.dQ[0];
        mxm = fmax(mxm, fabs(N.un - N.cs));
        mx0 = fmax(mx0, fabs(N.un));
        mxp = fmax(mxp, fabs(N.un + N.cs));
        T w[NV], pa[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) w[v] = T(N.dF[v]);
        project<DIM, T>(S, w, pa);
#pragma unroll
        for (int v = 0; v < NV; ++v) a[v][r - 1] = pa[v];
#pragma unroll
        for (int v = 0; v < NV; ++v) w[v] = T(N.dQ[v]);
        project<DIM, T>(S, w, pa);
#pragma unroll
        for (int v = 0; v < NV; ++v) b[v][r - 1] = pa[v];
    }
    // LF speeds: fields (u_n - c), (u_n) x (DIM - 1), (u_n + c)
    T lam[NV];
    lam[0] = fmax(S.sigma * mxm, T(sk.glf[0]));
    const T l1 = fmax(S.sigma * mx0, T(sk.glf[1]));
#pragma unroll
    for (int v = 1; v < E; ++v) lam[v] = l1;
    lam[E] = fmax(S.sigma * mxp, T(sk.glf[2]));
    // WENOCU6's eps may be far below the FP32 normal range (1e-40 in the
    // published scheme): the FP32 path floors it at 1e-30.  The
    // reconstructions take twice the split values a +- lambda b (the split's
    // 1/2 goes on the back-projected sum), so WENOCU6 takes 4 eps and WENO5,
    // whose indicators are also scaled by 4, 16 eps.
    const T eps = (CU6 && sizeof(T) == 4) ? fmax(T(sk.eps), T(1e-30)) : T(sk.eps);
    const T epsw = CU6 ? T(4) * eps : T(16) * eps;
    T h[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        T vp[6], vm[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            vp[r] = a[v][r] + lam[v] * b[v][r];
            vm[r] = a[v][5 - r] - lam[v] * b[v][5 - r];
        }
        if constexpr (CU6)
            h[v] = wenocu6<T>(vp, epsw) + wenocu6<T>(vm, epsw);
        else
            h[v] = weno5(vp[0], vp[1], vp[2], vp[3], vp[4], epsw) +
                   weno5(vm[0], vm[1], vm[2], vm[3], vm[4], epsw);
    }
    T o[NV];
    backproject<DIM, T>(S, h, o);
#pragma unroll
    for (int v = 0; v < NV; ++v) Fo[v] = fma(0.5, double(o[v]), R.Fts[v]);
}

// ---------------------------------------------------------------------------
// the face flux: WENO7-JS (Remark 2), stencil nodes i-3 .. i+4 (slots 0..7)
// ---------------------------------------------------------------------------

template <int DIM, int Y, typename T, class LD>
__device__ __forceinline__ void face_flux_weno7(const LD& ld, const SchemeK& sk,
                                                double (&Fo)[DIM + 2]) {
    constexpr int NV = DIM + 2, E = NV - 1;
    FaceRef<DIM> R;
    face_ref<DIM, Y>(ld, sk, R);
    Eig<DIM, T> S;
    roe<DIM, T>(ld.after(R.Vf), sk, R, S);
    T a[NV][8], b[NV][8];
    T mxm = T(0), mx0 = T(0), mxp = T(0);
    double chain = double(S.pI);
#pragma unroll
    for (int r = 0; r <= 7; ++r) {
        NodeDiff<DIM, T> N;
        node_diff<DIM, T>(ld.after(chain), r, sk, R, S, N);
        chain = N.dQ[0];
        mxm = fmax(mxm, fabs(N.un - N.cs));
        mx0 = fmax(mx0, fabs(N.un));
        mxp = fmax(mxp, fabs(N.un + N.cs));
        T w[NV], pa[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) w[v] = T(N.dF[v]);
        project<DIM, T>(S, w, pa);
#pragma unroll
        for (int v = 0; v < NV; ++v) a[v][r] = pa[v];
#pragma unroll
        for (int v = 0; v < NV; ++v) w[v] = T(N.dQ[v]);
        project<DIM, T>(S, w, pa);
#pragma unroll
        for (int v = 0; v < NV; ++v) b[v][r] = pa[v];
    }
    T lam[NV];
    lam[0] = fmax(S.sigma * mxm, T(sk.glf[0]));
    const T l1 = fmax(S.sigma * mx0, T(sk.glf[1]));
#pragma unroll
    for (int v = 1; v < E; ++v) lam[v] = l1;
    lam[E] = fmax(S.sigma * mxp, T(sk.glf[2]));
    // twice the split values, 4 eps; the split's 1/2 on the back-projected sum
    const T eps4 = T(4) * T(sk.eps);
    T h[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        T vp[7], vm[7];
#pragma unroll
        for (int r = 0; r < 7; ++r) {
            vp[r] = a[v][r] + lam[v] * b[v][r];
            vm[r] = a[v][7 - r] - lam[v] * b[v][7 - r];
        }
        h[v] = weno7<T>(vp, eps4) + weno7<T>(vm, eps4);
    }
    T o[NV];
    backproject<DIM, T>(S, h, o);
#pragma unroll
    for (int v = 0; v < NV; ++v) Fo[v] = fma(0.5, double(o[v]), R.Fts[v]);
}

// ---------------------------------------------------------------------------
// the face flux: fifth-order linear upwind
// ---------------------------------------------------------------------------
// With the optimal weights the two split parts reconstruct linearly, and
// since (LU5+ + LU5-)/2 is the sixth-order central interpolation and
// (LU5+ - LU5-)/2 the fifth difference (1,-5,10,-10,5,-1)/60,
//   sum_s r_s (h+_s + h-_s) = central6(dF~) + (1/60) R Lambda L Delta^5(dQ~),
// which is the linear-upwind member of eq. new_form_linear_upwind.

template <int DIM, int Y, typename T, class LD>
__device__ __forceinline__ void face_flux_lu5(const LD& ld, const SchemeK& sk,
                                              double (&Fo)[DIM + 2]) {
    constexpr int NV = DIM + 2, E = NV - 1;
    constexpr double c6[6] = {1.0 / 60, -8.0 / 60, 37.0 / 60, 37.0 / 60, -8.0 / 60, 1.0 / 60};
    constexpr double d5[6] = {1.0, -5.0, 10.0, -10.0, 5.0, -1.0};
    FaceRef<DIM> R;
    face_ref<DIM, Y>(ld, sk, R);
    Eig<DIM, T> S;
    roe<DIM, T>(ld.after(R.Vf), sk, R, S);
    double cen[NV], del[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) cen[v] = del[v] = 0.0;
    T mxm = T(0), mx0 = T(0), mxp = T(0);
    double chain = double(S.pI);
#pragma unroll
    for (int r = 1; r <= 6; ++r) {
        NodeDiff<DIM, T> N;
        node_diff<DIM, T>(ld.after(chain), r, sk, R, S, N);
        chain = N.dQ[0];
        mxm = fmax(mxm, fabs(N.un - N.cs));
        mx0 = fmax(mx0, fabs(N.un));
        mxp = fmax(mxp, fabs(N.un + N.cs));
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            cen[v] += c6[r - 1] * N.dF[v];
            del[v] += d5[r - 1] * N.dQ[v];
        }
    }
    T w[NV], pa[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v] = T(del[v]);
    project<DIM, T>(S, w, pa);
    const T l0 = fmax(S.sigma * mxm, T(sk.glf[0]));
    const T l1 = fmax(S.sigma * mx0, T(sk.glf[1]));
    const T l2 = fmax(S.sigma * mxp, T(sk.glf[2]));
    pa[0] *= l0;
#pragma unroll
    for (int v = 1; v < E; ++v) pa[v] *= l1;
    pa[E] *= l2;
    T o[NV];
    backproject<DIM, T>(S, pa, o);
#pragma unroll
    for (int v = 0; v < NV; ++v) Fo[v] = R.Fts[v] + cen[v] + double(o[v]) * (1.0 / 60.0);
}

template <int DIM, int RECON, int Y, typename T, class LD>
__device__ __forceinline__ void face_flux(const LD& ld, const SchemeK& sk, double (&Fo)[DIM + 2]) {
    if constexpr (RECON == 1)
        face_flux_lu5<DIM, Y, T>(ld, sk, Fo);
    else if constexpr (RECON == 2)
        face_flux_weno7<DIM, Y, T>(ld, sk, Fo);
    else
        face_flux_weno<DIM, Y, T, RECON == 3>(ld, sk, Fo);
}

}  // namespace fpk
