// Device-side physics of one element for the TLED + Pennes step, single
// precision, written in "small quantities" so that nothing is formed by
// subtracting nearly equal O(1) numbers:
//   - the displacement gradient H = F - I is kept, not F;
//   - the elastic part is H_e = F_e - I, Green strain E = (H_e + H_e^T + H_e^T H_e)/2;
//   - J - 1 = tr H + ((tr H)^2 - tr H^2)/2 + det H (exact expansion of det(I + H));
//   - J^(-2/3) - 1 = expm1(-2/3 log1p(J - 1));
//   - I - I1/3 C^-1 = 2 C^-1 dev E and I4bar - 1 = (J^-2/3 - 1) + 2 J^-2/3 a.E.a.
// Algebraically these are the textbook forms of the Table 5 model (Eq. 9)
// evaluated on the elastic deformation (Eq. 8) and pulled back (Eq. 10).
#pragma once

#include <hip/hip_runtime.h>

namespace tled {

// Kernel-side material constants (single precision, derived on the host).
struct KMat {
    float mu, kappa, eta;         // moduli at T0
    float alpha, alpha_m, alpha_n; // expansion coefficients (alpha_m: along the fibre m, alpha_n: along n)
    float k, k_m;                 // conductivities
    // Temperature laws are evaluated on the rise dT = T - T0 with the ramp start
    // as an offset from T0 formed in FP64 on the host (off = T0 - T_start): an
    // absolute temperature in FP32 is quantised to 3e-5 K near 310 K, which the
    // steep shrinkage ramp would turn into strain errors.
    float muT_off, muT_inv, muT_drop;
    float sh_off, sh_inv, sh_eps;
    float ck_off, ck_inv;         // c(T), k(T) ramp
    float c_lo, c_hi, kr_hi;      // c at lo/hi; k_hi / k
    float pc1[4], pc2[4];         // Prony: dt g/(dt + tau), tau/(dt + tau)
    float hgk;                    // hourglass: hg_coef (kappa + 4 mu / 3)
    int n_prony;
    int expan_mode, cond_mode, muT_on, shrink_on, ckT_on;
};

struct Sym3 {
    float xx, yy, zz, xy, yz, xz;
};

__device__ __forceinline__ float clamp01f(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }

// Hardware reciprocal (v_rcp_f32, within 1 ulp).  Every reciprocal here is of a
// quantity near 1 or of a well-scaled determinant, so the IEEE division
// sequence is not needed.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// (1 + x)^(-2/3) - 1.  Binomial series to x^5 for |x| < 0.02 (truncation below
// 3e-11, i.e. < 3e-9 relative), else expm1(-2/3 log1p(x)).
__device__ __forceinline__ float pow_m23_m1(float x) {
    if (fabsf(x) < 0.02f)
        return x * (-2.0f / 3.0f +
                    x * (5.0f / 9.0f + x * (-40.0f / 81.0f + x * (110.0f / 243.0f + x * (-308.0f / 729.0f)))));
    return expm1f(-(2.0f / 3.0f) * log1pf(x));
}

// Symmetric product (A B + (A B)^T)/2 of two symmetric matrices.
__device__ __forceinline__ Sym3 sym_prod(const Sym3 &A, const Sym3 &B) {
    float m00 = A.xx * B.xx + A.xy * B.xy + A.xz * B.xz;
    float m11 = A.xy * B.xy + A.yy * B.yy + A.yz * B.yz;
    float m22 = A.xz * B.xz + A.yz * B.yz + A.zz * B.zz;
    float m01 = A.xx * B.xy + A.xy * B.yy + A.xz * B.yz;
    float m10 = A.xy * B.xx + A.yy * B.xy + A.yz * B.xz;
    float m12 = A.xy * B.xz + A.yy * B.yz + A.yz * B.zz;
    float m21 = A.xz * B.xy + A.yz * B.yy + A.zz * B.yz;
    float m02 = A.xx * B.xz + A.xy * B.yz + A.xz * B.zz;
    float m20 = A.xz * B.xx + A.yz * B.xy + A.zz * B.xz;
    return Sym3{m00, m11, m22, 0.5f * (m01 + m10), 0.5f * (m12 + m21), 0.5f * (m02 + m20)};
}

// (J - 1) of I + A from the invariants of A, and det A.
__device__ __forceinline__ float det_m1(const float A[9]) {
    float i1 = A[0] + A[4] + A[8];
    float trA2 = A[0] * A[0] + A[4] * A[4] + A[8] * A[8] +
                 2.0f * (A[1] * A[3] + A[2] * A[6] + A[5] * A[7]);
    float i2 = 0.5f * (i1 * i1 - trA2);
    float i3 = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
               A[2] * (A[3] * A[7] - A[4] * A[6]);
    return i1 + i2 + i3;
}

// Adjugate of a symmetric matrix.
__device__ __forceinline__ Sym3 sym_adj(const Sym3 &C) {
    return Sym3{C.yy * C.zz - C.yz * C.yz, C.xx * C.zz - C.xz * C.xz, C.xx * C.yy - C.xy * C.xy,
                C.xz * C.yz - C.xy * C.zz, C.xy * C.xz - C.xx * C.yz, C.xy * C.yz - C.xz * C.yy};
}

// Result of the per-element physics: PV = V0 F S~ (first Piola times volume,
// row-major 3x3), qV = V0 K0 grad T (pulled-back heat flux times volume),
// psiV = V0 det(Fth) Psi (only when requested), Jmin = min(det F, J_el).
struct ElemOut {
    float PV[9];
    float qV[3];
    float psiV;
    float Jmin;
};

// Thermal stretch (Section 3.2): lambda - 1 = alpha dT for the expansion
// coefficient of one axis, times the optional shrinkage factor.
__device__ __forceinline__ float stretch_m1(const KMat &m, float alpha, float dTe) {
    float a = alpha * dTe;
    if (m.shrink_on) {
        const float s1 = m.sh_eps * clamp01f((dTe + m.sh_off) * m.sh_inv);
        a = a + s1 + s1 * a;
    }
    return a;
}

// Octahedral decoding of a unit vector stored as two floats.
__device__ __forceinline__ void oct_decode(float x, float y, float a[3]) {
    float z = 1.0f - fabsf(x) - fabsf(y);
    float t = fmaxf(-z, 0.0f);
    x += (x >= 0.0f) ? -t : t;
    y += (y >= 0.0f) ? -t : t;
    float r = rsqrtf(x * x + y * y + z * z);
    a[0] = x * r; a[1] = y * r; a[2] = z * r;
}

// He += beta (F v) (x) v for a unit axis v (F = I + H): one axis term of
// F F_th^-1 with F_th^-1 = I / lambda_i + sum_v beta_v v (x) v (Eq. 11).
__device__ __forceinline__ void add_axis_term(float He[9], const float H[9], const float v[3], float beta) {
    const float Fv[3] = {v[0] + H[0] * v[0] + H[1] * v[1] + H[2] * v[2],
                         v[1] + H[3] * v[0] + H[4] * v[1] + H[5] * v[2],
                         v[2] + H[6] * v[0] + H[7] * v[1] + H[8] * v[2]};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) He[3 * i + j] += beta * Fv[i] * v[j];
}

// Per-element physics.  H: displacement gradient (row-major), gT: reference
// temperature gradient, dTe: element temperature rise over T0, a: unit fibre,
// theta: Prony state (n_prony x 6, updated in place), aniso + 2 e: the
// element's two float4 of anisotropy data (second expansion axis in
// octahedral coordinates, conductivity tensor: (n.x, n.y, Dxx, Dyy),
// (Dzz, Dxy, Dyz, Dxz)), read only inside the orthotropic expansion and tensor
// conduction branches.  ANISO = false compiles those two modes out (the
// kernels for every other mode then keep the register budget of the
// isotropic and transversely isotropic code); ANISO = true handles every mode.
template <int NP, bool ANISO>
__device__ __forceinline__ void element_physics(const KMat &m, const float H[9], const float gT[3],
                                                float dTe, const float a[3], float V0, float *theta,
                                                bool want_psi, ElemOut &o, const float4 *__restrict__ aniso,
                                                int e) {
    // ---- thermal split, Eqs. 7-8, 11
    const float li1 = stretch_m1(m, m.alpha, dTe);
    const float li = 1.0f + li1, inv_li = rcp(li);
    float He[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) He[i] = H[i] * inv_li;
    He[0] -= li1 * inv_li;
    He[4] -= li1 * inv_li;
    He[8] -= li1 * inv_li;
    float beta = 0.0f, lm = 1.0f;
    if (!ANISO) {
        if (m.expan_mode == 1) {
            // F_e = F/li + beta (F a) (x) a, beta = 1/lm - 1/li = (li1 - lm1)/(li lm)
            const float lm1 = stretch_m1(m, m.alpha_m, dTe);
            lm = 1.0f + lm1;
            beta = (li1 - lm1) * inv_li * rcp(lm);
            add_axis_term(He, H, a, beta);
        }
    } else if (m.expan_mode != 0) {
        // F_e = F/li + b_m (F m) (x) m [+ b_n (F n) (x) n], b = 1/l - 1/li = (li1 - l1)/(li l)
        const float lm1 = stretch_m1(m, m.alpha_m, dTe);
        add_axis_term(He, H, a, (li1 - lm1) * inv_li * rcp(1.0f + lm1));
        if (m.expan_mode == 2) {
            float nv[3];
            const float4 q = aniso[2 * size_t(e)];
            oct_decode(q.x, q.y, nv);
            const float ln1 = stretch_m1(m, m.alpha_n, dTe);
            add_axis_term(He, H, nv, (li1 - ln1) * inv_li * rcp(1.0f + ln1));
        }
    }
    // ---- Green strain of the elastic part
    Sym3 E;
    E.xx = He[0] + 0.5f * (He[0] * He[0] + He[3] * He[3] + He[6] * He[6]);
    E.yy = He[4] + 0.5f * (He[1] * He[1] + He[4] * He[4] + He[7] * He[7]);
    E.zz = He[8] + 0.5f * (He[2] * He[2] + He[5] * He[5] + He[8] * He[8]);
    E.xy = 0.5f * (He[1] + He[3] + He[0] * He[1] + He[3] * He[4] + He[6] * He[7]);
    E.yz = 0.5f * (He[5] + He[7] + He[1] * He[2] + He[4] * He[5] + He[7] * He[8]);
    E.xz = 0.5f * (He[2] + He[6] + He[0] * He[2] + He[3] * He[5] + He[6] * He[8]);
    const float Jm1 = det_m1(He);
    const float J = 1.0f + Jm1;
    const float j23m1 = pow_m23_m1(Jm1);
    const float j23 = 1.0f + j23m1;
    // C = I + 2E, C^-1 = adj(C) / J^2
    Sym3 C{1.0f + 2.0f * E.xx, 1.0f + 2.0f * E.yy, 1.0f + 2.0f * E.zz, 2.0f * E.xy, 2.0f * E.yz, 2.0f * E.xz};
    Sym3 Ci = sym_adj(C);
    const float invJ2 = rcp(J * J);
    Ci.xx *= invJ2; Ci.yy *= invJ2; Ci.zz *= invJ2; Ci.xy *= invJ2; Ci.yz *= invJ2; Ci.xz *= invJ2;
    const float trE = E.xx + E.yy + E.zz;
    Sym3 dev{E.xx - trE * (1.0f / 3.0f), E.yy - trE * (1.0f / 3.0f), E.zz - trE * (1.0f / 3.0f), E.xy, E.yz, E.xz};
    Sym3 M = sym_prod(Ci, dev);  // C^-1 dev E  (= (I - I1/3 C^-1)/2)
    float scale = 1.0f;
    if (m.muT_on) scale = 1.0f - m.muT_drop * clamp01f((dTe + m.muT_off) * m.muT_inv);
    const float mu = m.mu * scale, eta = m.eta * scale;
    const float aEa = a[0] * (E.xx * a[0] + E.xy * a[1] + E.xz * a[2]) +
                      a[1] * (E.xy * a[0] + E.yy * a[1] + E.yz * a[2]) +
                      a[2] * (E.xz * a[0] + E.yz * a[1] + E.zz * a[2]);
    const float I4 = 1.0f + 2.0f * aEa;
    const float I4b1 = j23m1 + 2.0f * j23 * aEa;  // I4bar - 1
    const float ciso = 2.0f * mu * j23;
    const float cfib = 2.0f * eta * I4b1 * j23;
    const float cvol = m.kappa * J * Jm1;
    const float cfc = cvol - cfib * I4 * (1.0f / 3.0f);
    Sym3 S;  // S_i, Eq. 9
    S.xx = ciso * M.xx + cfib * a[0] * a[0] + cfc * Ci.xx;
    S.yy = ciso * M.yy + cfib * a[1] * a[1] + cfc * Ci.yy;
    S.zz = ciso * M.zz + cfib * a[2] * a[2] + cfc * Ci.zz;
    S.xy = ciso * M.xy + cfib * a[0] * a[1] + cfc * Ci.xy;
    S.yz = ciso * M.yz + cfib * a[1] * a[2] + cfc * Ci.yz;
    S.xz = ciso * M.xz + cfib * a[0] * a[2] + cfc * Ci.xz;
    // ---- pull-back, Eq. 10
    float detFth;
    if (m.expan_mode == 0) {
        detFth = li * li * li;
        S.xx *= li; S.yy *= li; S.zz *= li; S.xy *= li; S.yz *= li; S.xz *= li;
    } else if (!ANISO) {
        // det(Fth) Fth^-1 S Fth^-T, Fth^-1 = I/li + beta a(x)a
        detFth = li * li * lm;
        float Sa[3] = {S.xx * a[0] + S.xy * a[1] + S.xz * a[2], S.xy * a[0] + S.yy * a[1] + S.yz * a[2],
                       S.xz * a[0] + S.yz * a[1] + S.zz * a[2]};
        float aSa = a[0] * Sa[0] + a[1] * Sa[1] + a[2] * Sa[2];
        float c0 = detFth * inv_li * inv_li, c1 = detFth * beta * inv_li, c2 = detFth * beta * beta * aSa;
        S = Sym3{c0 * S.xx + c1 * 2.0f * a[0] * Sa[0] + c2 * a[0] * a[0],
                 c0 * S.yy + c1 * 2.0f * a[1] * Sa[1] + c2 * a[1] * a[1],
                 c0 * S.zz + c1 * 2.0f * a[2] * Sa[2] + c2 * a[2] * a[2],
                 c0 * S.xy + c1 * (a[0] * Sa[1] + Sa[0] * a[1]) + c2 * a[0] * a[1],
                 c0 * S.yz + c1 * (a[1] * Sa[2] + Sa[1] * a[2]) + c2 * a[1] * a[2],
                 c0 * S.xz + c1 * (a[0] * Sa[2] + Sa[0] * a[2]) + c2 * a[0] * a[2]};
    } else {
        // det(Fth) P S P with P = Fth^-1 = I/li + b_m m (x) m + b_n n (x) n (m = a; b_n = 0
        // in the transversely isotropic mode):
        //   P S P = S/li^2 + (1/li) sum_v b_v (v (S v)^T + (S v) v^T) + sum_{v,w} b_v b_w (v.S w) v (x) w
        const float lm1 = stretch_m1(m, m.alpha_m, dTe), lm = 1.0f + lm1;
        const float bm = (li1 - lm1) * inv_li * rcp(lm);
        float nv[3] = {0.0f, 0.0f, 0.0f}, bn = 0.0f, ln = li;
        if (m.expan_mode == 2) {
            const float4 q = aniso[2 * size_t(e)];
            oct_decode(q.x, q.y, nv);
            const float ln1 = stretch_m1(m, m.alpha_n, dTe);
            ln = 1.0f + ln1;
            bn = (li1 - ln1) * inv_li * rcp(ln);
        }
        detFth = li * lm * ln;
        const float Sa[3] = {S.xx * a[0] + S.xy * a[1] + S.xz * a[2], S.xy * a[0] + S.yy * a[1] + S.yz * a[2],
                             S.xz * a[0] + S.yz * a[1] + S.zz * a[2]};
        const float Sn[3] = {S.xx * nv[0] + S.xy * nv[1] + S.xz * nv[2], S.xy * nv[0] + S.yy * nv[1] + S.yz * nv[2],
                             S.xz * nv[0] + S.yz * nv[1] + S.zz * nv[2]};
        const float aSa = a[0] * Sa[0] + a[1] * Sa[1] + a[2] * Sa[2];
        const float nSn = nv[0] * Sn[0] + nv[1] * Sn[1] + nv[2] * Sn[2];
        const float aSn = a[0] * Sn[0] + a[1] * Sn[1] + a[2] * Sn[2];
        const float c0 = detFth * inv_li * inv_li, cm = detFth * bm * inv_li, cn = detFth * bn * inv_li;
        const float cmm = detFth * bm * bm * aSa, cnn = detFth * bn * bn * nSn, cmn = detFth * bm * bn * aSn;
#define TLED_PSP(i, j)                                                                                       \
    (cm * (a[i] * Sa[j] + Sa[i] * a[j]) + cn * (nv[i] * Sn[j] + Sn[i] * nv[j]) + cmm * a[i] * a[j] +            \
     cnn * nv[i] * nv[j] + cmn * (a[i] * nv[j] + nv[i] * a[j]))
        S = Sym3{c0 * S.xx + TLED_PSP(0, 0), c0 * S.yy + TLED_PSP(1, 1), c0 * S.zz + TLED_PSP(2, 2),
                 c0 * S.xy + TLED_PSP(0, 1), c0 * S.yz + TLED_PSP(1, 2), c0 * S.xz + TLED_PSP(0, 2)};
#undef TLED_PSP
    }
    if (want_psi) {
        float I1b3 = 3.0f * j23m1 + 2.0f * j23 * trE;  // I1bar - 3
        o.psiV = V0 * detFth * (0.5f * mu * I1b3 + 0.5f * eta * I4b1 * I4b1 + 0.5f * m.kappa * Jm1 * Jm1);
    }
    // ---- Prony relaxation on the total stress
    Sym3 St = S;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        float *t = theta + 6 * p;
        const float c1 = m.pc1[p], c2 = m.pc2[p];
        t[0] = c1 * S.xx + c2 * t[0];
        t[1] = c1 * S.yy + c2 * t[1];
        t[2] = c1 * S.zz + c2 * t[2];
        t[3] = c1 * S.xy + c2 * t[3];
        t[4] = c1 * S.yz + c2 * t[4];
        t[5] = c1 * S.xz + c2 * t[5];
        St.xx -= t[0]; St.yy -= t[1]; St.zz -= t[2]; St.xy -= t[3]; St.yz -= t[4]; St.xz -= t[5];
    }
    // ---- PV = V0 (I + H) S~
    const float Sm[9] = {St.xx, St.xy, St.xz, St.xy, St.yy, St.yz, St.xz, St.yz, St.zz};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            o.PV[3 * i + j] = V0 * (Sm[3 * i + j] + H[3 * i] * Sm[j] + H[3 * i + 1] * Sm[3 + j] +
                                    H[3 * i + 2] * Sm[6 + j]);
    // ---- conduction with the total F, Eq. 16: K0 = J F^-1 D F^-T
    const float Jt1 = det_m1(H);
    const float Jt = 1.0f + Jt1;
    float kscale = 1.0f;
    if (m.ckT_on) kscale = 1.0f + clamp01f((dTe + m.ck_off) * m.ck_inv) * (m.kr_hi - 1.0f);
    float K[6];
    if (m.cond_mode == 0) {
        // J k C^-1 = k adj(C) / J with C = I + H + H^T + H^T H
        Sym3 Ct{1.0f + 2.0f * H[0] + H[0] * H[0] + H[3] * H[3] + H[6] * H[6],
                1.0f + 2.0f * H[4] + H[1] * H[1] + H[4] * H[4] + H[7] * H[7],
                1.0f + 2.0f * H[8] + H[2] * H[2] + H[5] * H[5] + H[8] * H[8],
                H[1] + H[3] + H[0] * H[1] + H[3] * H[4] + H[6] * H[7],
                H[5] + H[7] + H[1] * H[2] + H[4] * H[5] + H[7] * H[8],
                H[2] + H[6] + H[0] * H[2] + H[3] * H[5] + H[6] * H[8]};
        Sym3 A = sym_adj(Ct);
        const float f = m.k * kscale * rcp(Jt);
        K[0] = f * A.xx; K[1] = f * A.yy; K[2] = f * A.zz; K[3] = f * A.xy; K[4] = f * A.yz; K[5] = f * A.xz;
    } else {
        // adj(F) D adj(F)^T / J
        const float F[9] = {1.0f + H[0], H[1], H[2], H[3], 1.0f + H[4], H[5], H[6], H[7], 1.0f + H[8]};
        float Ad[9] = {F[4] * F[8] - F[5] * F[7], F[2] * F[7] - F[1] * F[8], F[1] * F[5] - F[2] * F[4],
                       F[5] * F[6] - F[3] * F[8], F[0] * F[8] - F[2] * F[6], F[2] * F[3] - F[0] * F[5],
                       F[3] * F[7] - F[4] * F[6], F[1] * F[6] - F[0] * F[7], F[0] * F[4] - F[1] * F[3]};
        const float iJt = rcp(Jt);
        float r[3][3];
        if (!ANISO || m.cond_mode == 1) {
            // D = k I + (k_m - k) a a
            const float kk = m.k * kscale, km = m.k_m * kscale;
            float Aa[3] = {Ad[0] * a[0] + Ad[1] * a[1] + Ad[2] * a[2], Ad[3] * a[0] + Ad[4] * a[1] + Ad[5] * a[2],
                           Ad[6] * a[0] + Ad[7] * a[1] + Ad[8] * a[2]};
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    r[i][j] = (kk * (Ad[3 * i] * Ad[3 * j] + Ad[3 * i + 1] * Ad[3 * j + 1] +
                                     Ad[3 * i + 2] * Ad[3 * j + 2]) +
                               (km - kk) * Aa[i] * Aa[j]) * iJt;
        } else {
            // the element's tensor D (times k(T)/k)
            const float4 d0 = aniso[2 * size_t(e)], d1 = aniso[2 * size_t(e) + 1];
            const float Dm[9] = {d0.z, d1.y, d1.w, d1.y, d0.w, d1.z, d1.w, d1.z, d1.x};
            float AD[9];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    AD[3 * i + j] = Ad[3 * i] * Dm[j] + Ad[3 * i + 1] * Dm[3 + j] + Ad[3 * i + 2] * Dm[6 + j];
            const float f = kscale * iJt;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    r[i][j] = (AD[3 * i] * Ad[3 * j] + AD[3 * i + 1] * Ad[3 * j + 1] + AD[3 * i + 2] * Ad[3 * j + 2]) * f;
        }
        K[0] = r[0][0]; K[1] = r[1][1]; K[2] = r[2][2]; K[3] = r[0][1]; K[4] = r[1][2]; K[5] = r[0][2];
    }
    o.qV[0] = V0 * (K[0] * gT[0] + K[3] * gT[1] + K[5] * gT[2]);
    o.qV[1] = V0 * (K[3] * gT[0] + K[1] * gT[1] + K[4] * gT[2]);
    o.qV[2] = V0 * (K[5] * gT[0] + K[4] * gT[1] + K[2] * gT[2]);
    o.Jmin = fminf(J, Jt);
}

}  // namespace tled
