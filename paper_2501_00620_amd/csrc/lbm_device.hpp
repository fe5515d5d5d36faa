// lbm_device.hpp -- per-site arithmetic of the bump-function D3Q19 step on gfx950.
//
// Method: Afrasiabian & Denniston, "A Novel Velocity Discretization for Lattice Boltzmann
// Method: Application to Compressible Flow" (arXiv:2501.00620), Sec. II B-C and Appendix A.
// Lattice units dx = dt = c = 1; c_s^2 = 1/3; omega = 1/(tau + 1/2) (Eq. 55).
//
// The forms used here are algebraic rearrangements chosen for few VALU operations:
//  * feq (Appendix A) grouped per lattice direction class.  Rest:
//      rho/9 (3 - 2|u|^2 - 6(ux^2 uy^2 + ux^2 uz^2 + uy^2 uz^2));
//    face along axis a with sign s (o_a = |u|^2 - u_a^2):
//      rho/18 (1 + 3 s u_a + 2 u_a^2 - 2 o_a + 6 u_a^2 o_a);
//    edge in the (a,b) plane with q = s_a u_a + s_b u_b:
//      rho/36 (1 - u_a^2 - u_b^2 - 6 u_a^2 u_b^2 + 3 q (1 + q)).
//  * the forcing populations with the moments of Eqs. 58-61 in Hermite form,
//      Phi_i = w_i [3 e_i.F + 9/2 (e_i.S.e_i - tr S / 3)],
//    whose zeroth, first and second moments are 0, F and S on D3Q19.
//  * the isotropic derivative d_a phi = 3 sum_i w_i e_ia phi(x + e_i) applied to the sources
//    R = rho b and X_abg = rho u*_g b_ab as one sum over neighbours: with
//    v_i = sum_a e_ia R_a. (x + e_i),  F = -3 sum_i w_i v_i  and
//    S_bg = -3 sum_i w_i (v_ib u_g + v_ig u_b)(x + e_i).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 19;
constexpr int NB = 6;     // bbar components xx yy zz xy xz yz
constexpr int NSRC = 9;   // gradient sources per site: R (6) then u* (3)
constexpr int NFIELD = Q + NB;

// Velocity set and order of the paper (rows 2-4 of Table I).
constexpr int EX[Q] = {0, 1, 0, -1, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0};
constexpr int EY[Q] = {0, 0, 1, 0, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1};
constexpr int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
// Index of -e_i (half-way bounce-back).
constexpr int OPP[Q] = {0, 3, 4, 1, 2, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
// Weights w_i = feq_i(u = 0) / rho (Appendix A at rest): 1/3, 1/18 (faces), 1/36 (edges).
constexpr double WQ[Q] = {1.0 / 3, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                          1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                          1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// ------------------------------------------------------------------------------------------
// Storage codecs.  S = 0: double, 1: float, 2: fp16, 3: bf16.  What is stored is always the
// deviation of a field from its reference value (d_i or beta, see below); the 16-bit codes h
// hold deviation / scale[k] (k = field: 0..18 populations, 19..24 b), so the deviation decodes
// as scale[k] * h.  ref[k] is the reference value itself, added back only when the state is
// read out in absolute terms.
// ------------------------------------------------------------------------------------------
struct Codec {
    double ref[NFIELD];
    float scale[NFIELD];
    float inv[NFIELD];
};

template <int S> struct Storage;

template <> struct Storage<0> {
    using T = double;
    using C = double;
    static __device__ __forceinline__ C load(const T *p, size_t i, int, const Codec &) { return p[i]; }
    static __device__ __forceinline__ void store(T *p, size_t i, int, C v, const Codec &, unsigned &) { p[i] = v; }
};

template <> struct Storage<1> {
    using T = float;
    using C = float;
    static __device__ __forceinline__ C load(const T *p, size_t i, int, const Codec &) { return p[i]; }
    static __device__ __forceinline__ void store(T *p, size_t i, int, C v, const Codec &, unsigned &) { p[i] = v; }
};

__device__ __forceinline__ float half_bits_to_float(uint16_t b) {
    return (float)__builtin_bit_cast(_Float16, b);
}
// Overflow of a 16-bit code.  Conversion rounds to nearest even, so a finite value turns into
// +-inf exactly when its magnitude reaches the midpoint between the largest finite code and the
// next power of two: 65520 for fp16, (2 - 2^-8) 2^127 for bf16.  Such a value is stored as +-inf
// (nothing is clamped) and sets the range flag; a NaN is stored as NaN without the flag, since
// it comes only from a state that is already non-finite, which the health check counts.
constexpr float HALF_OVERFLOW = 65520.0f;
__device__ __forceinline__ float bf16_overflow() { return __uint_as_float(0x7f7f8000u); }

// float -> fp16 code, round to nearest even (hardware conversion).
__device__ __forceinline__ uint16_t float_to_half_bits(float h, unsigned &sat) {
    if (fabsf(h) >= HALF_OVERFLOW) sat = 1u;
    return __builtin_bit_cast(uint16_t, (_Float16)h);
}
__device__ __forceinline__ float bf16_bits_to_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
// float -> bf16 code, round to nearest even on the dropped 16 bits; NaN stays NaN.
__device__ __forceinline__ uint16_t float_to_bf16_bits(float h, unsigned &sat) {
    uint32_t u = __float_as_uint(h);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)0x7fc0u;
    if (fabsf(h) >= bf16_overflow()) sat = 1u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <> struct Storage<2> {
    using T = uint16_t;
    using C = float;
    static __device__ __forceinline__ C load(const T *p, size_t i, int k, const Codec &c) {
        return c.scale[k] * half_bits_to_float(p[i]);
    }
    static __device__ __forceinline__ void store(T *p, size_t i, int k, C v, const Codec &c, unsigned &sat) {
        p[i] = float_to_half_bits(v * c.inv[k], sat);
    }
};

template <> struct Storage<3> {
    using T = uint16_t;
    using C = float;
    static __device__ __forceinline__ C load(const T *p, size_t i, int k, const Codec &c) {
        return c.scale[k] * bf16_bits_to_float(p[i]);
    }
    static __device__ __forceinline__ void store(T *p, size_t i, int k, C v, const Codec &c, unsigned &sat) {
        p[i] = float_to_bf16_bits(v * c.inv[k], sat);
    }
};

// ------------------------------------------------------------------------------------------
// Per-site arithmetic (compute type C) in deviation variables.
//
// Every precision stores and computes deviations from the rest equilibrium at the reference
// state (rho_ref, T_ref):  d_i = fbar_i - w_i rho_ref  and  beta = bbar - b_ref with
// b_ref = (T_ref - 1/3) I  (beq at rest, Appendix A).  The macroscopic quantities then come
// without cancellation:
//    rho - rho_ref = sum d_i,   j = sum d_i e_i   (sum w_i e_i = 0),
//    P := tr Pi - rho = sum d_i (|e_i|^2 - 1) = sum_edges d_i - d_0   (sum w_i |e_i|^2 = 1),
//    theta := T - T_ref = (P + rho tr beta - rho |u|^2) / (3 rho)    (energy-conserving T),
//    beq - b_ref = theta I + u u / 3,
//    feq_i - w_i rho_ref = w_i (rho - rho_ref) + rho (feq_i(1, u) - w_i).
// The isotropic derivative of rho*b is taken of R' = rho b - rho_ref b_ref (a constant
// removed, same gradient); the second-moment source rho u b = u (R' + rho_ref b_ref) keeps it.
// ------------------------------------------------------------------------------------------
template <typename C> struct StepConst {
    C omega;      // 1/(tau + 1/2)
    C half_omega; // omega/2: b = bbar - (omega/2)(bbar - beq) (Eqs. 62-65)
    C fcoef;      // 1 - omega/2 = tau/(tau + 1/2), the forcing weight of Eq. 55
    C rho_ref;    // reference density of the deviation variables
    C theta_ref;  // T_ref - 1/3, the diagonal of b_ref
    C K;          // rho_ref * theta_ref
    C om1;        // 1 - omega
    C ghost;      // 1 - omega_g / omega: the non-hydrodynamic moments' own rate (0: single rate)
    C au[3];      // uniform body-force acceleration (when force_u)
    int force_u;  // 1: a uniform body force acts (no acceleration field)
    C uwb[3];     // velocity of the wall below plane 0 (walls; tangential)
    C uwt[3];     // velocity of the wall above plane nz - 1
    int iso;      // prescribed temperature (theta per site or constant)
};

// feq_i - w_i rho_ref (Appendix A, grouped form; see the header comment).
template <typename C>
__device__ __forceinline__ void equilibrium_dev(C drho, C rho, C ux, C uy, C uz, C f[Q]) {
    const C x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
    const C r9 = rho * C(1.0 / 9.0), r18 = rho * C(1.0 / 18.0), r36 = rho * C(1.0 / 36.0);
    const C d3 = drho * C(1.0 / 3.0), d18 = drho * C(1.0 / 18.0), d36 = drho * C(1.0 / 36.0);
    f[0] = d3 - r9 * (C(2) * (x2 + y2 + z2) + C(6) * (x2 * y2 + x2 * z2 + y2 * z2));
    const C ox = y2 + z2, oy = x2 + z2, oz = x2 + y2;
    const C ax = d18 + r18 * (C(2) * (x2 - ox) + C(6) * x2 * ox);
    const C ay = d18 + r18 * (C(2) * (y2 - oy) + C(6) * y2 * oy);
    const C az = d18 + r18 * (C(2) * (z2 - oz) + C(6) * z2 * oz);
    const C tx = r18 * C(3) * ux, ty = r18 * C(3) * uy, tz = r18 * C(3) * uz;
    f[1] = ax + tx;
    f[3] = ax - tx;
    f[2] = ay + ty;
    f[4] = ay - ty;
    f[5] = az + tz;
    f[6] = az - tz;
    const C bxy = d36 - r36 * (oz + C(6) * x2 * y2);
    const C bxz = d36 - r36 * (oy + C(6) * x2 * z2);
    const C byz = d36 - r36 * (ox + C(6) * y2 * z2);
    const C r12 = rho * C(1.0 / 12.0);  // 3 rho / 36
    C q;
    q = ux + uy;  f[7] = bxy + r12 * q * (C(1) + q);
    q = -q;       f[10] = bxy + r12 * q * (C(1) + q);
    q = ux - uy;  f[8] = bxy + r12 * q * (C(1) + q);
    q = -q;       f[9] = bxy + r12 * q * (C(1) + q);
    q = ux + uz;  f[11] = bxz + r12 * q * (C(1) + q);
    q = -q;       f[14] = bxz + r12 * q * (C(1) + q);
    q = ux - uz;  f[12] = bxz + r12 * q * (C(1) + q);
    q = -q;       f[13] = bxz + r12 * q * (C(1) + q);
    q = uy + uz;  f[15] = byz + r12 * q * (C(1) + q);
    q = -q;       f[18] = byz + r12 * q * (C(1) + q);
    q = uy - uz;  f[16] = byz + r12 * q * (C(1) + q);
    q = -q;       f[17] = byz + r12 * q * (C(1) + q);
}

// beq - b_ref = theta I + u u / 3 (Appendix A / Eq. 36 with P = rho T I).
template <typename C>
__device__ __forceinline__ void variance_eq_dev(C ux, C uy, C uz, C theta, C b[NB]) {
    const C third = C(1.0 / 3.0);
    b[0] = fma(ux * ux, third, theta);
    b[1] = fma(uy * uy, third, theta);
    b[2] = fma(uz * uz, third, theta);
    b[3] = ux * uy * third;
    b[4] = ux * uz * third;
    b[5] = uy * uz * third;
}

// 1/x.  Single precision: the hardware reciprocal (about 1 ulp, and not unbiased) refined by one
// Newton-Raphson step r' = r + r (1 - x r), which leaves an error of about half an ulp; double:
// correctly rounded division.
template <typename C> __device__ __forceinline__ C recip(C x) { return C(1) / x; }
template <> __device__ __forceinline__ float recip<float>(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Moments of the deviation populations.
template <typename C> struct PopMoments {
    C drho, rho, jx, jy, jz, P;
};
template <typename C>
__device__ __forceinline__ PopMoments<C> pop_moments(const C d[Q], C rho_ref) {
    PopMoments<C> m;
    const C faces = ((d[1] + d[3]) + (d[2] + d[4])) + (d[5] + d[6]);
    const C edges = (((d[7] + d[8]) + (d[9] + d[10])) + ((d[11] + d[12]) + (d[13] + d[14]))) +
                    ((d[15] + d[16]) + (d[17] + d[18]));
    m.drho = (d[0] + faces) + edges;
    m.rho = rho_ref + m.drho;
    m.P = edges - d[0];
    m.jx = ((d[1] - d[3]) + (d[7] + d[8]) - (d[9] + d[10])) + ((d[11] + d[12]) - (d[13] + d[14]));
    m.jy = ((d[2] - d[4]) + (d[7] - d[8]) + (d[9] - d[10])) + ((d[15] + d[16]) - (d[17] + d[18]));
    m.jz = ((d[5] - d[6]) + (d[11] - d[12]) + (d[13] - d[14])) + ((d[15] - d[16]) + (d[17] - d[18]));
    return m;
}

// Step 1: predictor velocity and temperature, and the gradient sources R' and u*.
// b = bbar - (omega/2)(bbar - beq(u*, T*)) is the physical variance of Eqs. 62-65 with the
// uncorrected velocity inside beq, as the paper allows after Eq. 68.
template <typename C>
__device__ __forceinline__ void predictor_sources(const PopMoments<C> &m, const C beta[NB], C theta_iso,
                                                  const StepConst<C> &k, C src[NSRC]) {
    const C inv = recip(m.rho);
    const C ux = m.jx * inv, uy = m.jy * inv, uz = m.jz * inv;
    const C u2 = ux * ux + uy * uy + uz * uz;
    const C trb = beta[0] + beta[1] + beta[2];
    const C theta = k.iso ? theta_iso : (m.P + m.rho * (trb - u2)) * inv * C(1.0 / 3.0);
    C beq[NB];
    variance_eq_dev(ux, uy, uz, theta, beq);
    C bp[NB];
#pragma unroll
    for (int c = 0; c < NB; c++) bp[c] = beta[c] - k.half_omega * (beta[c] - beq[c]);
    const C dK = m.drho * k.theta_ref;  // (rho - rho_ref) theta_ref on the diagonal
#pragma unroll
    for (int c = 0; c < 3; c++) src[c] = fma(m.rho, bp[c], dK);
#pragma unroll
    for (int c = 3; c < NB; c++) src[c] = m.rho * bp[c];
    src[6] = ux;
    src[7] = uy;
    src[8] = uz;
}

// Accumulates the isotropic-gradient forcing moments over the 18 neighbours.
template <typename C> struct GradAcc {
    C fF[3], fS[6];  // face sums (weight 1/18)
    C eF[3], eS[6];  // edge sums (weight 1/36)
};

// The diagonal S sums collect v_b u_b once; grad_finish doubles them.  HASK: T_ref != 1/3, so
// the second-moment source carries the constant rho_ref b_ref = K I as well.
template <typename C, int I, bool HASK = true>
__device__ __forceinline__ void grad_add(GradAcc<C> &g, const C s[NSRC], C K) {
    // v = sum_a e_ia R'_a.   R' rows: x = (xx, xy, xz), y = (xy, yy, yz), z = (xz, yz, zz);
    // the second-moment source uses the full R = R' + K I, i.e. v + K e_i.
    constexpr int ex = EX[I], ey = EY[I], ez = EZ[I];
    const C vx = C(ex) * s[0] + C(ey) * s[3] + C(ez) * s[4];
    const C vy = C(ex) * s[3] + C(ey) * s[1] + C(ez) * s[5];
    const C vz = C(ex) * s[4] + C(ey) * s[5] + C(ez) * s[2];
    C wx = vx, wy = vy, wz = vz;
    if constexpr (HASK) {
        wx = vx + C(ex) * K;
        wy = vy + C(ey) * K;
        wz = vz + C(ez) * K;
    }
    const C ux = s[6], uy = s[7], uz = s[8];
    constexpr bool face = (ex * ex + ey * ey + ez * ez) == 1;
    C *F = face ? g.fF : g.eF;
    C *S = face ? g.fS : g.eS;
    F[0] += vx;
    F[1] += vy;
    F[2] += vz;
    S[0] = fma(wx, ux, S[0]);
    S[1] = fma(wy, uy, S[1]);
    S[2] = fma(wz, uz, S[2]);
    S[3] = fma(wx, uy, fma(wy, ux, S[3]));
    S[4] = fma(wx, uz, fma(wz, ux, S[4]));
    S[5] = fma(wy, uz, fma(wz, uy, S[5]));
}

// The same term for a neighbour one plane beyond a wall, from the three planes of its column
// inside the wall, s0 (the wall-adjacent plane), s1, s2: the variance pressure R is mirrored
// (R(s0)), the products R u* are extrapolated to second order, 3 X(s0) - 3 X(s1) + X(s2).
template <typename C, int I, bool HASK = true>
__device__ __forceinline__ void grad_add_wall(GradAcc<C> &g, const C s0[NSRC], const C s1[NSRC], const C s2[NSRC],
                                              C K) {
    constexpr int ex = EX[I], ey = EY[I], ez = EZ[I];
    constexpr bool face = (ex * ex + ey * ey + ez * ez) == 1;
    C *F = face ? g.fF : g.eF;
    C *S = face ? g.fS : g.eS;
    F[0] += C(ex) * s0[0] + C(ey) * s0[3] + C(ez) * s0[4];
    F[1] += C(ex) * s0[3] + C(ey) * s0[1] + C(ez) * s0[5];
    F[2] += C(ex) * s0[4] + C(ey) * s0[5] + C(ez) * s0[2];
    auto add = [&](const C *s, C c) {
        C wx = C(ex) * s[0] + C(ey) * s[3] + C(ez) * s[4];
        C wy = C(ex) * s[3] + C(ey) * s[1] + C(ez) * s[5];
        C wz = C(ex) * s[4] + C(ey) * s[5] + C(ez) * s[2];
        if constexpr (HASK) {
            wx += C(ex) * K;
            wy += C(ey) * K;
            wz += C(ez) * K;
        }
        wx *= c;
        wy *= c;
        wz *= c;
        const C ux = s[6], uy = s[7], uz = s[8];
        S[0] = fma(wx, ux, S[0]);
        S[1] = fma(wy, uy, S[1]);
        S[2] = fma(wz, uz, S[2]);
        S[3] = fma(wx, uy, fma(wy, ux, S[3]));
        S[4] = fma(wx, uz, fma(wz, ux, S[4]));
        S[5] = fma(wy, uz, fma(wz, uy, S[5]));
    };
    add(s0, C(3));
    add(s1, C(-3));
    add(s2, C(1));
}

template <typename C>
__device__ __forceinline__ void grad_init(GradAcc<C> &g) {
#pragma unroll
    for (int c = 0; c < 3; c++) g.fF[c] = g.eF[c] = C(0);
#pragma unroll
    for (int c = 0; c < 6; c++) g.fS[c] = g.eS[c] = C(0);
}

// F = -3 (face/18 + edge/36) = -(face/6 + edge/12), likewise S (diagonal sums doubled).
template <typename C>
__device__ __forceinline__ void grad_finish(const GradAcc<C> &g, C F[3], C S[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) F[c] = -(g.fF[c] * C(1.0 / 6.0) + g.eF[c] * C(1.0 / 12.0));
#pragma unroll
    for (int c = 0; c < 3; c++) S[c] = -(g.fS[c] * C(1.0 / 3.0) + g.eS[c] * C(1.0 / 6.0));
#pragma unroll
    for (int c = 3; c < 6; c++) S[c] = -(g.fS[c] * C(1.0 / 6.0) + g.eS[c] * C(1.0 / 12.0));
}

// The same forcing moments on a lattice of one z plane, from the in-plane faces (directions 1-4,
// in the face sums) and in-plane edges (7-10, in the edge sums) alone: each face offset also
// stands for the two z edges reading the same site (weight 1/18 + 2/36 = 1/9), whose z parts
// cancel, and the +-z faces at the site itself cancel.  F = -3 (face/9 + edge/36), S likewise
// with the diagonal sums doubled.
template <typename C>
__device__ __forceinline__ void grad_finish_thin(const GradAcc<C> &g, C F[3], C S[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) F[c] = -(g.fF[c] * C(1.0 / 3.0) + g.eF[c] * C(1.0 / 12.0));
#pragma unroll
    for (int c = 0; c < 3; c++) S[c] = -(g.fS[c] * C(2.0 / 3.0) + g.eS[c] * C(1.0 / 6.0));
#pragma unroll
    for (int c = 3; c < 6; c++) S[c] = -(g.fS[c] * C(1.0 / 3.0) + g.eS[c] * C(1.0 / 12.0));
}

// The body-force acceleration at site s: the field (3 planes of n values) if there is one, else
// the uniform vector of the step constants.
template <typename C>
__device__ __forceinline__ void site_accel(const StepConst<C> &k, const C *accel, size_t n, size_t s, C a[3]) {
    if (accel) {
        a[0] = accel[s];
        a[1] = accel[n + s];
        a[2] = accel[2 * n + s];
    } else {
        a[0] = k.au[0];
        a[1] = k.au[1];
        a[2] = k.au[2];
    }
}

// A body-force acceleration a in the forcing moments, in the manner of a Guo forcing:
// F += rho a and S += rho (u a + a u), u the corrected velocity of Eq. 57 (which, formed from the
// new F by collide, carries half of rho a).
template <typename C>
__device__ __forceinline__ void add_body_force(const PopMoments<C> &m, const C a[3], C F[3], C S[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) F[c] = fma(m.rho, a[c], F[c]);
    const C inv = recip(m.rho);
    const C ux = (m.jx + C(0.5) * F[0]) * inv;  // as collide forms it
    const C uy = (m.jy + C(0.5) * F[1]) * inv;
    const C uz = (m.jz + C(0.5) * F[2]) * inv;
    S[0] = fma(C(2) * m.rho, ux * a[0], S[0]);
    S[1] = fma(C(2) * m.rho, uy * a[1], S[1]);
    S[2] = fma(C(2) * m.rho, uz * a[2], S[2]);
    S[3] = fma(m.rho, fma(ux, a[1], uy * a[0]), S[3]);
    S[4] = fma(m.rho, fma(ux, a[2], uz * a[0]), S[4]);
    S[5] = fma(m.rho, fma(uy, a[2], uz * a[1]), S[5]);
}

// Steps 3-5: corrected moments, equilibria, forcing and the BGK update, in place on the
// deviations d and beta.  Returns the corrected u and theta = T - T_ref if asked.
//
// Each population is updated as d' = (1 - omega) d + c with c = omega (feq - w rho_ref) + g,
// g = (1 - omega/2) Phi.  Opposite velocities i, i' share the even part P and flip the sign of
// the odd part M of c:  c_i = P + M,  c_i' = P - M.  Per pair (axis a, or plane (a,b) with
// q = s_a u_a + s_b u_b):
//   faces:  P = omega [drho/18 + rho/18 (2 u_a^2 - 2 o_a + 6 u_a^2 o_a)] + (fcoef/4)(S_aa - trS/3)
//           M = omega rho u_a / 6 + (fcoef/6) F_a  = G_a / 6,  G = omega j + F
//   edges:  P = omega [drho/36 - rho/36 (u_a^2 + u_b^2 + 6 u_a^2 u_b^2) + rho q^2 / 12]
//               + (fcoef/8)(S_aa + S_bb - trS/3) + s_a s_b (fcoef/4) S_ab
//           M = omega rho q / 12 + (fcoef/12)(s_a F_a + s_b F_b)  = (s_a G_a + s_b G_b) / 12
//   rest:   c = omega [drho/3 - rho/9 (2|u|^2 + 6(ux^2 uy^2 + ux^2 uz^2 + uy^2 uz^2))] - fcoef trS/2
// (the grouped Appendix A equilibrium and the Hermite-form forcing written above).
template <typename C>
__device__ __forceinline__ void collide(C d[Q], C beta[NB], const PopMoments<C> &m, const C F[3],
                                        const C S[6], C theta_iso, const StepConst<C> &k, C *out_u = nullptr,
                                        C *out_theta = nullptr) {
    const C inv = recip(m.rho);
    const C ux = (m.jx + C(0.5) * F[0]) * inv;  // Eq. 57
    const C uy = (m.jy + C(0.5) * F[1]) * inv;
    const C uz = (m.jz + C(0.5) * F[2]) * inv;
    const C trS = S[0] + S[1] + S[2];
    const C x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
    C theta;
    if (k.iso) {
        theta = theta_iso;
    } else {
        const C trb = beta[0] + beta[1] + beta[2];
        theta = (m.P + C(0.5) * trS + m.rho * (trb - (x2 + y2 + z2))) * inv * C(1.0 / 3.0);
    }
    if (out_u) {
        out_u[0] = ux;
        out_u[1] = uy;
        out_u[2] = uz;
    }
    if (out_theta) *out_theta = theta;

    // beta <- beta + omega (beq - beta), beq - b_ref = theta I + u u / 3
    const C third = C(1.0 / 3.0);
    beta[0] = fma(k.omega, fma(x2, third, theta) - beta[0], beta[0]);
    beta[1] = fma(k.omega, fma(y2, third, theta) - beta[1], beta[1]);
    beta[2] = fma(k.omega, fma(z2, third, theta) - beta[2], beta[2]);
    beta[3] = fma(k.omega, ux * uy * third - beta[3], beta[3]);
    beta[4] = fma(k.omega, ux * uz * third - beta[4], beta[4]);
    beta[5] = fma(k.omega, uy * uz * third - beta[5], beta[5]);

    const C om = k.omega, om1 = k.om1, fc = k.fcoef;
    const C wr = om * m.rho, wd = om * m.drho;
    const C wr9 = wr * C(1.0 / 9.0), wr18 = wr * C(1.0 / 18.0), wr36 = wr * C(1.0 / 36.0);
    const C wr12 = wr * C(1.0 / 12.0);
    const C wd18 = wd * C(1.0 / 18.0), wd36 = wd * C(1.0 / 36.0);
    const C t3 = trS * third;
    const C fc4 = fc * C(0.25), fc8 = fc * C(0.125);
    // Odd parts.  The momentum the update hands out is G = omega rho u + (1 - omega/2) F
    // = omega j + F (Eq. 57 with u = (j + F/2)/rho), formed from j directly.  Each edge pair gets
    // H_a +- H_b with H = G/12, and each face pair the remainder G_a/2 - 4 H_a, so that the
    // population momenta sum to G up to the rounding of single operations.  (Splitting G as
    // G/6 per face and G/12 per edge with rounded constants would hand out (1 + 3e-8) G in
    // single precision, a bias that compounds over many steps.)
    const C Gx = fma(om, m.jx, F[0]), Gy = fma(om, m.jy, F[1]), Gz = fma(om, m.jz, F[2]);
    const C Hx = Gx * C(1.0 / 12.0), Hy = Gy * C(1.0 / 12.0), Hz = Gz * C(1.0 / 12.0);
    const C xy = x2 * y2, xz = x2 * z2, yz = y2 * z2;
    const C ox = y2 + z2, oy = x2 + z2, oz = x2 + y2;

    // rest
    d[0] = fma(om1, d[0], fma(wd, third, -wr9 * fma(C(2), x2 + ox, C(6) * (xy + xz + yz))) - fc * C(0.5) * trS);

    // faces: pairs (1,3) x, (2,4) y, (5,6) z
    auto face = [&](int ip, int im, C a2, C oa, C Ga, C Ha, C Saa) {
        const C P = fma(wr18, fma(C(2), a2 - oa, C(6) * a2 * oa), wd18) + fc4 * (Saa - t3);
        const C M = fma(C(-4), Ha, C(0.5) * Ga);
        d[ip] = fma(om1, d[ip], P + M);
        d[im] = fma(om1, d[im], P - M);
    };
    face(1, 3, x2, ox, Gx, Hx, S[0]);
    face(2, 4, y2, oy, Gy, Hy, S[1]);
    face(5, 6, z2, oz, Gz, Hz, S[2]);

    // edges: in the (a,b) plane, pairs (+a+b, -a-b) and (+a-b, -a+b)
    auto edges = [&](int ipp, int imm, int ipm, int imp, C a2b2, C a2b2x, C ua, C ub, C Ha, C Hb, C Saa, C Sbb,
                     C Sab) {
        const C base = fma(-wr36, fma(C(6), a2b2x, a2b2), wd36) + fc8 * (Saa + Sbb - t3);
        const C sab = fc4 * Sab;
        C q = ua + ub;
        C P = fma(wr12, q * q, base) + sab;
        C M = Ha + Hb;
        d[ipp] = fma(om1, d[ipp], P + M);
        d[imm] = fma(om1, d[imm], P - M);
        q = ua - ub;
        P = fma(wr12, q * q, base) - sab;
        M = Ha - Hb;
        d[ipm] = fma(om1, d[ipm], P + M);
        d[imp] = fma(om1, d[imp], P - M);
    };
    edges(7, 10, 8, 9, oz, xy, ux, uy, Hx, Hy, S[0], S[1], S[3]);
    edges(11, 14, 12, 13, oy, xz, ux, uz, Hx, Hz, S[0], S[2], S[4]);
    edges(15, 18, 16, 17, ox, yz, uy, uz, Hy, Hz, S[1], S[2], S[5]);
}

// Periodic neighbour offsets of a site: X/Y/Z[d+1] hold the x index, the row offset and the
// plane offset of coordinate (c + d) mod n for d = -1, 0, 1 (valid for any n >= 1).
struct Nbr {
    int X[3];
    int Y[3];
    int Z[3];
    __device__ __forceinline__ int at(int dx, int dy, int dz) const { return Z[dz + 1] + Y[dy + 1] + X[dx + 1]; }
};

__device__ __forceinline__ Nbr make_nbr(int x, int y, int z, int nx, int ny, int nz) {
    Nbr o;
    const int nxy = nx * ny;
    o.X[0] = x == 0 ? nx - 1 : x - 1;
    o.X[1] = x;
    o.X[2] = x == nx - 1 ? 0 : x + 1;
    o.Y[0] = (y == 0 ? ny - 1 : y - 1) * nx;
    o.Y[1] = y * nx;
    o.Y[2] = (y == ny - 1 ? 0 : y + 1) * nx;
    o.Z[0] = (z == 0 ? nz - 1 : z - 1) * nxy;
    o.Z[1] = z * nxy;
    o.Z[2] = (z == nz - 1 ? 0 : z + 1) * nxy;
    return o;
}

// compile-time loop helper
template <int I, int N> struct Unroll {
    template <typename Fn> static __device__ __forceinline__ void run(Fn &&fn) {
        fn(std::integral_constant<int, I>{});
        Unroll<I + 1, N>::run(fn);
    }
};
template <int N> struct Unroll<N, N> {
    template <typename Fn> static __device__ __forceinline__ void run(Fn &&) {}
};

// Rows 11-19 of Table I (Appendix B), the non-hydrodynamic moments, each scaled to integers
// (a row's scale cancels in ghost_relax).
constexpr int GHOST_ROWS[9][Q] = {
    {0, -2, 0, 2, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0},
    {0, 0, -2, 0, 2, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, -2, 2, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, -1, -1, 1, 1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1},
    {0, 1, 1, 1, 1, -2, -2, -2, -2, -2, -2, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0, 0, 0, -1, -1, -1, -1, 1, 1, 1, 1},
    {1, -2, -2, -2, -2, -2, -2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
};
constexpr double ghost_norm(int a) {  // sum_j w_j r_j^2 of ghost row a
    double s = 0.0;
    for (int j = 0; j < Q; j++) s += WQ[j] * GHOST_ROWS[a][j] * GHOST_ROWS[a][j];
    return s;
}

// The non-hydrodynamic moments of Table I (rows 11-19, integer-scaled as GHOST_ROWS) of d.
template <typename C> __device__ __forceinline__ void ghost_moments(const C d[Q], C m[9]) {
    Unroll<0, 9>::run([&](auto A) {
        C acc = C(0);
        Unroll<0, Q>::run([&](auto J) {
            constexpr int r = GHOST_ROWS[A][J];
            if constexpr (r != 0) acc = fma(C(r), d[J], acc);
        });
        m[A] = acc;
    });
}

// Relaxation of the non-hydrodynamic moments at their own rate omega_g (Table I rows 11-19),
// applied after the single-rate collision d0 -> d, given m0 = ghost_moments(d0).  In the Table I
// basis the rates are diagonal, Phi has no components on these rows, and rows 1-10 keep omega, so
// the update differs from the single-rate one by (omega - omega_g) m_a(d0 - deq) on each ghost
// row a, mapped back with the inverse of Table I (w_i r_i / sum_j w_j r_j^2).  The single-rate
// step gives m_a(d0 - deq) = m_a(d0 - d) / omega, so with cg = 1 - omega_g / omega
//   d_i += cg w_i r_i (m_a(d0) - m_a(d)) / sum_j w_j r_j^2.
// Carrying the 9 moments of d0 across the collision instead of its 19 populations keeps the
// fused sweep's register budget.
template <typename C>
__device__ __forceinline__ void ghost_relax(const C m0[9], C d[Q], C cg) {
    C m1[9];
    ghost_moments(d, m1);
    C add[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) add[i] = C(0);
    Unroll<0, 9>::run([&](auto A) {
        const C g = (m0[A] - m1[A]) * (cg * C(1.0 / ghost_norm(A)));
        Unroll<0, Q>::run([&](auto I) {
            constexpr int r = GHOST_ROWS[A][I];
            if constexpr (r != 0) add[I] = fma(C(WQ[I] * r), g, add[I]);
        });
    });
#pragma unroll
    for (int i = 0; i < Q; i++) d[i] += add[i];
}

// Standard lattice Boltzmann comparator (Sec. I, Eq. 4; lattice units, c_s^2 = 1/3): the
// second-order Hermite equilibrium at temperature T = 1/3 + th, in deviation form
//   feq_i - w_i rho_ref = w_i (rho - rho_ref)
//                         + rho w_i [3 e.u + 9/2 (e.u)^2 - 3/2 |u|^2 + 9/2 th (|e|^2 - 1)].
template <typename C>
__device__ __forceinline__ void equilibrium_std_dev(C drho, C rho, C ux, C uy, C uz, C th, C f[Q]) {
    const C u2 = ux * ux + uy * uy + uz * uz;
    const C a = fma(C(-1.5), u2, C(-4.5) * th);  // the |e|^2 = 0 part of the bracket
    Unroll<0, Q>::run([&](auto I) {
        constexpr int ex = EX[I], ey = EY[I], ez = EZ[I];
        constexpr int e2 = ex * ex + ey * ey + ez * ez;
        const C eu = C(ex) * ux + C(ey) * uy + C(ez) * uz;
        const C br = fma(eu, fma(C(4.5), eu, C(3)), fma(C(4.5 * e2), th, a));
        f[I] = C(WQ[I]) * fma(rho, br, drho);
    });
}

// Forcing populations from their moments F and S (Eqs. 58-61 with no ghost moments), in Hermite
// form: Phi_i = w_i [3 e_i.F + 9/2 (e_i e_i - I/3) : S].  S is ordered xx yy zz xy xz yz.
template <typename C>
__device__ __forceinline__ void forcing_pops(const C F[3], const C S[6], C phi[Q]) {
    const C t3 = (S[0] + S[1] + S[2]) * C(1.0 / 3.0);
    Unroll<0, Q>::run([&](auto I) {
        constexpr int ex = EX[I], ey = EY[I], ez = EZ[I];
        const C eF = C(ex) * F[0] + C(ey) * F[1] + C(ez) * F[2];
        const C eSe = C(ex * ex) * S[0] + C(ey * ey) * S[1] + C(ez * ez) * S[2] +
                      C(2 * ex * ey) * S[3] + C(2 * ex * ez) * S[4] + C(2 * ey * ez) * S[5];
        phi[I] = C(WQ[I]) * fma(C(3), eF, C(4.5) * (eSe - t3));
    });
}

}  // namespace lbm
