// fp_device.hpp -- device-side arithmetic of the free-stream-preserving face
// flux for gfx950 (CDNA4, wave64).  Included by fp_kernels.hip only.
//
// One face i+1/2 of one grid line is evaluated by one lane.  The stencil
// (state, 1/J and the metric vector of the sweep direction at nodes i-3..i+4)
// lives in registers; nothing of the per-face pipeline touches memory.
//
// Steps (Sec. 3 of the paper, with the readings listed in the design notes):
//   1. cell-face 1/J, Q~ = Q/J and metrics by the central interpolation of the
//      metric order Y; reference state Q* = Q~_f / (1/J)_f        [FP64]
//   2. reference face flux F~*_f = F(Q*) s_f                      [FP64]
//   3. reference-subtracted stencil values dQ~_m, dF~_m           [FP64]
//   4. Roe average of nodes i, i+1; unit normal; eigenvectors      [T]
//   5. local Lax-Friedrichs speed per field (stencil maximum)      [T]
//   6. characteristic projection and splitting                     [T]
//   7. WENO5-JS or linear-upwind reconstruction of both parts      [T]
//   8. back-projection, then the reference flux is added back      [T, FP64 add]
// T is double for the FP64 path and float for the mixed path.
#pragma once
#include <hip/hip_runtime.h>

namespace fpk {

struct SchemeK {
    double gamma;
    double eps;
    int reform;  // 1: reference state subtracted (the paper); 0: standard scheme
};

// Stencil slots r = 0..7 hold nodes i-3 .. i+4 of the face i+1/2.
template <int DIM>
struct Stencil {
    double q[8][DIM + 2];
    double V[8];
    double s[8][DIM];
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

template <typename T>
__device__ __forceinline__ T rcp(T x);
template <>
__device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }
template <>
__device__ __forceinline__ float rcp<float>(float x) { return fast_rcp(x); }

template <typename T>
__device__ __forceinline__ T vsqrt(T x);
template <>
__device__ __forceinline__ double vsqrt<double>(double x) { return sqrt(x); }
template <>
__device__ __forceinline__ float vsqrt<float>(float x) { return fast_sqrt(x); }

// central face interpolation of order Y from stencil slots (node i in slot 3)
template <int Y>
__device__ __forceinline__ double face_interp(const double (&w)[8]) {
    if constexpr (Y == 2) {
        return (w[3] + w[4]) * 0.5;
    } else if constexpr (Y == 4) {
        return (7.0 * (w[3] + w[4]) - (w[2] + w[5])) * (1.0 / 12.0);
    } else if constexpr (Y == 6) {
        return (37.0 * (w[3] + w[4]) - 8.0 * (w[2] + w[5]) + (w[1] + w[6])) * (1.0 / 60.0);
    } else {
        return (533.0 * (w[3] + w[4]) - 139.0 * (w[2] + w[5]) + 29.0 * (w[1] + w[6])
                - 3.0 * (w[0] + w[7])) * (1.0 / 840.0);
    }
}

// WENO5-JS of a 5-point window a..e (face between c and d, upwind side a).
// Weights C_k/(beta_k+eps)^2 normalised over one common denominator.
__device__ __forceinline__ double weno5(double a, double b, double c, double d, double e,
                                        double eps) {
    const double q0 = 2.0 * a - 7.0 * b + 11.0 * c;
    const double q1 = -b + 5.0 * c + 2.0 * d;
    const double q2 = 2.0 * c + 5.0 * d - e;
    const double t0 = a - 2.0 * b + c, s0 = a - 4.0 * b + 3.0 * c;
    const double t1 = b - 2.0 * c + d, s1 = d - b;
    const double t2 = c - 2.0 * d + e, s2 = 3.0 * c - 4.0 * d + e;
    const double k13 = 13.0 / 12.0;
    double d0 = k13 * t0 * t0 + 0.25 * s0 * s0 + eps;
    double d1 = k13 * t1 * t1 + 0.25 * s1 * s1 + eps;
    double d2 = k13 * t2 * t2 + 0.25 * s2 * s2 + eps;
    d0 *= d0;
    d1 *= d1;
    d2 *= d2;
    const double a0 = 0.1 * (d1 * d2), a1 = 0.6 * (d0 * d2), a2 = 0.3 * (d0 * d1);
    return (a0 * q0 + a1 * q1 + a2 * q2) / (6.0 * (a0 + a1 + a2));
}

// FP32 form: reciprocal weights (no overflow of the products for large beta)
__device__ __forceinline__ float weno5(float a, float b, float c, float d, float e, float eps) {
    const float q0 = 2.0f * a - 7.0f * b + 11.0f * c;
    const float q1 = -b + 5.0f * c + 2.0f * d;
    const float q2 = 2.0f * c + 5.0f * d - e;
    const float t0 = a - 2.0f * b + c, s0 = a - 4.0f * b + 3.0f * c;
    const float t1 = b - 2.0f * c + d, s1 = d - b;
    const float t2 = c - 2.0f * d + e, s2 = 3.0f * c - 4.0f * d + e;
    const float k13 = 13.0f / 12.0f;
    float d0 = k13 * t0 * t0 + 0.25f * s0 * s0 + eps;
    float d1 = k13 * t1 * t1 + 0.25f * s1 * s1 + eps;
    float d2 = k13 * t2 * t2 + 0.25f * s2 * s2 + eps;
    const float a0 = 0.1f * fast_rcp(d0 * d0);
    const float a1 = 0.6f * fast_rcp(d1 * d1);
    const float a2 = 0.3f * fast_rcp(d2 * d2);
    return (a0 * q0 + a1 * q1 + a2 * q2) * fast_rcp(6.0f * (a0 + a1 + a2));
}

template <typename T>
__device__ __forceinline__ T linup5(T a, T b, T c, T d, T e) {
    return (T(2) * a - T(13) * b + T(47) * c + T(27) * d - T(3) * e) * (T(1) / T(60));
}

template <int RECON, typename T>
__device__ __forceinline__ T recon5(T a, T b, T c, T d, T e, T eps) {
    if constexpr (RECON == 1)
        return linup5<T>(a, b, c, d, e);
    else
        return weno5(a, b, c, d, e, eps);
}

// ---------------------------------------------------------------------------
// the face flux
// ---------------------------------------------------------------------------

template <int DIM, int RECON, int Y, typename T>
__device__ __forceinline__ void face_flux(const Stencil<DIM>& st, const SchemeK& sk,
                                          double (&Fo)[DIM + 2]) {
    constexpr int NV = DIM + 2;
    constexpr int E = NV - 1;
    const double gam = sk.gamma, gm1 = sk.gamma - 1.0;

    // (1) face reference state with the metric-order interpolation
    double w[8];
    const double Vf = face_interp<Y>(st.V);
    double sf[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
#pragma unroll
        for (int r = 0; r < 8; ++r) w[r] = st.s[r][c];
        sf[c] = face_interp<Y>(w);
    }
    double Qs[NV], us[DIM], ps = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) Qs[v] = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) us[c] = 0.0;
    if (sk.reform) {
        const double iVf = 1.0 / Vf;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
#pragma unroll
            for (int r = 0; r < 8; ++r) w[r] = st.q[r][v] * st.V[r];
            Qs[v] = face_interp<Y>(w) * iVf;
        }
        const double irs = 1.0 / Qs[0];
        double m2 = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            us[c] = Qs[1 + c] * irs;
            m2 += Qs[1 + c] * us[c];
        }
        ps = gm1 * (Qs[E] - 0.5 * m2);
    }
    // (2) reference face flux F(Q*) . s_f
    double Fts[NV];
    {
        double U = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) U += us[c] * sf[c];
        Fts[0] = Qs[0] * U;
#pragma unroll
        for (int c = 0; c < DIM; ++c) Fts[1 + c] = Qs[1 + c] * U + ps * sf[c];
        Fts[E] = (Qs[E] + ps) * U;
    }

    // unit normal and eigenvalue scale sigma = |s_f| / (1/J)_f
    double s2 = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) s2 += sf[c] * sf[c];
    const double snorm = sqrt(s2);
    const double isn = 1.0 / snorm;
    T n[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) n[c] = T(sf[c] * isn);
    const T sigma = T(snorm / Vf);

    // (3) reference-subtracted values at m = i-2..i+3 (slots 1..6), plus the
    // node velocities/sound speeds for the LF speeds and the Roe states
    T dQ[6][NV], dF[6][NV];
    T mxm = T(0), mx0 = T(0), mxp = T(0);
    double rhoL = 0, rhoR = 0, uL[DIM], uR[DIM], HL = 0, HR = 0;
#pragma unroll
    for (int r = 1; r <= 6; ++r) {
        const double rho = st.q[r][0];
        const double ir = 1.0 / rho;
        double u[DIM], m2 = 0.0, U = 0.0, Us = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            u[c] = st.q[r][1 + c] * ir;
            m2 += st.q[r][1 + c] * u[c];
            U += u[c] * st.s[r][c];
            Us += us[c] * st.s[r][c];
        }
        const double p = gm1 * (st.q[r][E] - 0.5 * m2);
        const double dp = p - ps;
        dF[r - 1][0] = T(rho * U - Qs[0] * Us);
#pragma unroll
        for (int c = 0; c < DIM; ++c)
            dF[r - 1][1 + c] = T(st.q[r][1 + c] * U - Qs[1 + c] * Us + dp * st.s[r][c]);
        dF[r - 1][E] = T((st.q[r][E] + p) * U - (Qs[E] + ps) * Us);
#pragma unroll
        for (int v = 0; v < NV; ++v) dQ[r - 1][v] = T((st.q[r][v] - Qs[v]) * st.V[r]);
        // LF speeds
        T un = T(0);
#pragma unroll
        for (int c = 0; c < DIM; ++c) un += n[c] * T(u[c]);
        const T cs = vsqrt<T>(T(gam * p * ir));
        mxm = fmax(mxm, fabs(un - cs));
        mx0 = fmax(mx0, fabs(un));
        mxp = fmax(mxp, fabs(un + cs));
        if (r == 3) {
            rhoL = rho;
            HL = (st.q[r][E] + p) * ir;
#pragma unroll
            for (int c = 0; c < DIM; ++c) uL[c] = u[c];
        }
        if (r == 4) {
            rhoR = rho;
            HR = (st.q[r][E] + p) * ir;
#pragma unroll
            for (int c = 0; c < DIM; ++c) uR[c] = u[c];
        }
    }
    const T lam0 = sigma * mxm, lamm = sigma * mx0, lamL = sigma * mxp;

    // (4) Roe average and characteristic basis
    const T wL = vsqrt<T>(T(rhoL)), wR = vsqrt<T>(T(rhoR));
    const T iw = rcp<T>(wL + wR);
    T uh[DIM];
    T q2 = T(0), un = T(0);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        uh[c] = (wL * T(uL[c]) + wR * T(uR[c])) * iw;
        q2 += uh[c] * uh[c];
        un += uh[c] * n[c];
    }
    const T Hh = (wL * T(HL) + wR * T(HR)) * iw;
    const T c2 = T(gm1) * (Hh - T(0.5) * q2);
    const T ch = vsqrt<T>(c2);
    const T ic = rcp<T>(ch);
    const T b2 = T(gm1) * rcp<T>(c2);
    const T hq2 = T(0.5) * q2;

    // tangent basis of the shear fields
    T t1[DIM], t2[3];
    if constexpr (DIM == 2) {
        t1[0] = -n[1];
        t1[1] = n[0];
    } else {
        // a = argmin |n_k|, components within 1e-10 count as tied and the
        // lowest k wins; t1 = normalize(n x e_a)
        const T tie = T(1e-10);
        const T a0 = fabs(n[0]), a1 = fabs(n[1]), a2 = fabs(n[2]);
        int a = 0;
        T am = a0;
        if (a1 < am - tie) { a = 1; am = a1; }
        if (a2 < am - tie) { a = 2; }
        T x0, x1, x2;
        if (a == 0) { x0 = T(0); x1 = n[2]; x2 = -n[1]; }
        else if (a == 1) { x0 = -n[2]; x1 = T(0); x2 = n[0]; }
        else { x0 = n[1]; x1 = -n[0]; x2 = T(0); }
        const T ix = rcp<T>(vsqrt<T>(x0 * x0 + x1 * x1 + x2 * x2));
        t1[0] = x0 * ix;
        t1[1] = x1 * ix;
        t1[2] = x2 * ix;
        t2[0] = n[1] * t1[2] - n[2] * t1[1];
        t2[1] = n[2] * t1[0] - n[0] * t1[2];
        t2[2] = n[0] * t1[1] - n[1] * t1[0];
    }
    T ut1 = T(0), ut2 = T(0);
#pragma unroll
    for (int c = 0; c < DIM; ++c) ut1 += uh[c] * t1[c];
    if constexpr (DIM == 3) ut2 = uh[0] * t2[0] + uh[1] * t2[1] + uh[2] * t2[2];

    // (5)-(7): per characteristic field, project, split, reconstruct
    const T eps = T(sk.eps);
    T hs[NV];
    // acoustic and entropy fields share phi/psi: l_0 w = (phi - psi)/2,
    // l_1 w = w_0 - phi, l_E w = (phi + psi)/2 with
    // phi = b2 (|u|^2/2 w_0 - u.w_m + w_E), psi = (n.w_m - u_n w_0)/c
    T pF[6], sF[6], pQ[6], sQ[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        T uw = T(0), nw = T(0), uq = T(0), nq = T(0);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            uw += uh[c] * dF[r][1 + c];
            nw += n[c] * dF[r][1 + c];
            uq += uh[c] * dQ[r][1 + c];
            nq += n[c] * dQ[r][1 + c];
        }
        pF[r] = b2 * (hq2 * dF[r][0] - uw + dF[r][E]);
        sF[r] = (nw - un * dF[r][0]) * ic;
        pQ[r] = b2 * (hq2 * dQ[r][0] - uq + dQ[r][E]);
        sQ[r] = (nq - un * dQ[r][0]) * ic;
    }
    {
        // field 0 (u_n - c)
        T vp[6], vm[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            const T a = T(0.5) * (pF[r] - sF[r]);
            const T b = T(0.5) * (pQ[r] - sQ[r]);
            vp[r] = T(0.5) * (a + lam0 * b);
            vm[r] = T(0.5) * (a - lam0 * b);
        }
        hs[0] = recon5<RECON, T>(vp[0], vp[1], vp[2], vp[3], vp[4], eps) +
                recon5<RECON, T>(vm[5], vm[4], vm[3], vm[2], vm[1], eps);
    }
    {
        // field E (u_n + c)
        T vp[6], vm[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            const T a = T(0.5) * (pF[r] + sF[r]);
            const T b = T(0.5) * (pQ[r] + sQ[r]);
            vp[r] = T(0.5) * (a + lamL * b);
            vm[r] = T(0.5) * (a - lamL * b);
        }
        hs[E] = recon5<RECON, T>(vp[0], vp[1], vp[2], vp[3], vp[4], eps) +
                recon5<RECON, T>(vm[5], vm[4], vm[3], vm[2], vm[1], eps);
    }
    {
        // field 1 (entropy, u_n)
        T vp[6], vm[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            const T a = dF[r][0] - pF[r];
            const T b = dQ[r][0] - pQ[r];
            vp[r] = T(0.5) * (a + lamm * b);
            vm[r] = T(0.5) * (a - lamm * b);
        }
        hs[1] = recon5<RECON, T>(vp[0], vp[1], vp[2], vp[3], vp[4], eps) +
                recon5<RECON, T>(vm[5], vm[4], vm[3], vm[2], vm[1], eps);
    }
    {
        // shear field along t1: l = (-u.t1, t1, 0)
        T vp[6], vm[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            T a = -ut1 * dF[r][0], b = -ut1 * dQ[r][0];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                a += t1[c] * dF[r][1 + c];
                b += t1[c] * dQ[r][1 + c];
            }
            vp[r] = T(0.5) * (a + lamm * b);
            vm[r] = T(0.5) * (a - lamm * b);
        }
        hs[2] = recon5<RECON, T>(vp[0], vp[1], vp[2], vp[3], vp[4], eps) +
                recon5<RECON, T>(vm[5], vm[4], vm[3], vm[2], vm[1], eps);
    }
    if constexpr (DIM == 3) {
        T vp[6], vm[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            T a = -ut2 * dF[r][0], b = -ut2 * dQ[r][0];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                a += t2[c] * dF[r][1 + c];
                b += t2[c] * dQ[r][1 + c];
            }
            vp[r] = T(0.5) * (a + lamm * b);
            vm[r] = T(0.5) * (a - lamm * b);
        }
        hs[3] = recon5<RECON, T>(vp[0], vp[1], vp[2], vp[3], vp[4], eps) +
                recon5<RECON, T>(vm[5], vm[4], vm[3], vm[2], vm[1], eps);
    }

    // (8) back-projection R h and add-back of the reference flux
    const T h0 = hs[0], h1 = hs[1], hE = hs[E];
    const T hsum = h0 + h1 + hE, hdif = hE - h0;
    Fo[0] = Fts[0] + double(hsum);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        T m = uh[c] * hsum + ch * n[c] * hdif + t1[c] * hs[2];
        if constexpr (DIM == 3) m += t2[c] * hs[3];
        Fo[1 + c] = Fts[1 + c] + double(m);
    }
    {
        T en = Hh * (h0 + hE) + ch * un * hdif + hq2 * h1 + ut1 * hs[2];
        if constexpr (DIM == 3) en += ut2 * hs[3];
        Fo[E] = Fts[E] + double(en);
    }
}

}  // namespace fpk
