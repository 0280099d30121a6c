/*
 * tled_oracle.c -- plain, serial, double-precision CPU reference of the
 * coupled thermo-visco-hyperelastic total-Lagrangian explicit dynamics (TLED)
 * + explicit Pennes bioheat time step of Zhang, Lay, Roberts and Chauhan,
 * "Towards real-time finite-strain anisotropic thermo-visco-elastodynamic
 * analysis of soft tissues for thermal ablative therapy" (arXiv 2009.10400).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the oracle the GPU library is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no source, header, table or helper
 * with the GPU path and includes nothing from it.
 *
 * It is written for a reader holding the paper: every routine follows the
 * textbook form of the equation it cites (C = F^T F, I1 - 3 by subtraction,
 * inverses by adjugate, the position form of the central difference), in the
 * paper's order, with no blocking, fusion or reordering.  Serial loops with a
 * scatter-add assembly; nothing is tuned.
 *
 * Readings where the paper is silent or garbled (each also listed in the
 * design notes of the repository):
 *   - conduction enters the Pennes update with a minus sign (heat flows from
 *     hot to cold; the matrix of Eq. 15 is positive semi-definite), Eq. 12-14/20;
 *   - one integration point per element; the element temperature used for the
 *     thermal stretch and for temperature-dependent properties is the mean of
 *     the nodal temperatures;
 *   - lumped heat capacity, perfusion and source loads use reference volumes;
 *   - Prony terms act on the total pulled-back stress of Eq. 10, start from
 *     zero and are updated with the current stress before it is relaxed;
 *   - both fields advance from the state at step n (Jacobi coupling);
 *   - the H8 hourglass control is a Flanagan-Belytschko-type stiffness on
 *     total-Lagrangian hourglass vectors with coefficient
 *     hg_coef * (kappa + 4 mu / 3) * V0 * sum_a |dh_a/dX|^2 / 8;
 *   - critical time step min_e L_e / c_d with c_d = sqrt((kappa + 4mu/3 + 4eta)/rho),
 *     L_e = 3 V0 / A_max (T4) or V0 / A_max (H8);
 *   - T4 elements with negative volume are repaired by swapping their last two
 *     nodes; a degenerate element or an inverted H8 is an error;
 *   - the orthotropic expansion of Eq. 11 takes m = the fibre a0 and n = the
 *     per-element second axis made orthonormal to m; a per-element conductivity
 *     tensor is the D of Eq. 15 as given (not rotated with the tissue), scaled by
 *     k(T)/k when the conductivity is temperature-dependent.
 *
 * Parity unpinned: the hourglass coefficient and the critical-time-step
 * formula are readings, not the paper's numbers (the hourglass force is pinned
 * by its invariants, it vanishes on affine fields and conserves momentum, and by
 * its closed form on an undistorted cube).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Material record (the oracle's own definition).                         */
/* ---------------------------------------------------------------------- */
typedef struct {
    double rho;          /* reference mass density, kg/m^3                       */
    double mu;           /* shear modulus, Pa (Table 5 model)                   */
    double kappa;        /* bulk modulus, Pa                                    */
    double eta;          /* fibre (anisotropic) coefficient eta_a, Pa           */
    double alpha;        /* thermal expansion coefficient, 1/K (isotropic part) */
    double alpha_m;      /* expansion along the fibre m = a0 (expan_mode 1, 2), 1/K */
    double alpha_n;      /* expansion along the second axis n (expan_mode 2), 1/K */
    double T0;           /* stress-free reference temperature, K               */
    double k;            /* thermal conductivity, W/(m K)                      */
    double k_m;          /* conductivity along the fibre (cond_mode 1)          */
    double c;            /* specific heat capacity, J/(kg K)                   */
    double wbcb;         /* perfusion w_b c_b, W/(m^3 K)                       */
    double T_art;        /* arterial blood temperature, K                      */
    double Q_met;        /* metabolic heat generation, W/m^3                   */
    double g[4];         /* Prony relative moduli phi_i                         */
    double tau[4];       /* Prony relaxation times tau_i, s                     */
    double muT_lo, muT_hi, muT_drop;          /* mu(T), eta(T) linear drop    */
    double shrink_T, shrink_width, shrink_eps; /* shrinkage ramp              */
    double ckT_lo, ckT_hi, c_hi, k_hi;        /* c(T), k(T) linear laws       */
    double hg_coef;      /* hourglass coefficient (H8)                         */
    int32_t n_prony;     /* number of Prony terms, 0..4                        */
    int32_t expan_mode;  /* 0: F_th = lambda I; 1: transversely isotropic; 2: orthotropic (Eq. 11) */
    int32_t cond_mode;   /* 0: D = k I; 1: D = k I + (k_m - k) a0 (x) a0; 2: per-element tensor */
    int32_t muT_on;      /* 1: temperature-dependent mu and eta                  */
    int32_t shrink_on;   /* 1: shrinkage factor on the thermal stretch          */
    int32_t ckT_on;      /* 1: temperature-dependent c and k                    */
} orc_material;

typedef struct {
    int32_t npe;
    int64_t nn, ne;
    double *X;        /* nn x 3 reference coordinates                         */
    int32_t *conn;    /* ne x npe (orientation repaired)                      */
    double *a0;       /* ne x 3 unit fibre directions                         */
    double *n0;       /* ne x 3 second expansion axes (expan_mode 2), or NULL   */
    double *Dc;       /* ne x 6 conductivity tensors xx yy zz xy yz xz (cond_mode 2), or NULL */
    double *q;        /* ne regional source density, W/m^3                    */
    uint8_t *fix;     /* nn: bit0..2 fixed u_x,u_y,u_z ; bit3 fixed T          */
    double *Tfix;     /* nn prescribed temperatures (where bit3)              */
    double t_on, t_off, dt, gamma;
    orc_material m;
    /* precomputed */
    double *dhdx;     /* ne x npe x 3 spatial derivatives dh_a/dX             */
    double *V0;       /* ne element reference volumes                         */
    double *gam;      /* ne x 4 x 8 hourglass vectors (H8)                    */
    double *khg;      /* ne hourglass stiffness (H8)                          */
    double *Vl;       /* nn lumped reference volume                           */
    double *M;        /* nn lumped mass                                       */
    double *Kb;       /* nn lumped perfusion                                  */
    double *Qm;       /* nn lumped metabolic load                            */
    double *Qr;       /* nn lumped regional source load                       */
    double dt_cr;
    int64_t n_swapped;
} orc_sim;

enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_MESH = -2, ORC_E_OOM = -5 };

/* ---------------------------------------------------------------------- */
/* 3x3 helpers, row-major A[3*i+j].                                         */
/* ---------------------------------------------------------------------- */
static double det3(const double *A)
{
    return A[0] * (A[4] * A[8] - A[5] * A[7])
         - A[1] * (A[3] * A[8] - A[5] * A[6])
         + A[2] * (A[3] * A[7] - A[4] * A[6]);
}

static void inv3(const double *A, double *B)
{
    double d = det3(A);
    B[0] = (A[4] * A[8] - A[5] * A[7]) / d;
    B[1] = (A[2] * A[7] - A[1] * A[8]) / d;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / d;
    B[3] = (A[5] * A[6] - A[3] * A[8]) / d;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / d;
    B[5] = (A[2] * A[3] - A[0] * A[5]) / d;
    B[6] = (A[3] * A[7] - A[4] * A[6]) / d;
    B[7] = (A[1] * A[6] - A[0] * A[7]) / d;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / d;
}

static void mul3(const double *A, const double *B, double *C)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = s;
        }
}

static void transpose3(const double *A, double *B)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[3 * i + j] = A[3 * j + i];
}

static double clamp01(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

/* ---------------------------------------------------------------------- */
/* Material laws.                                                          */
/* ---------------------------------------------------------------------- */

/* Thermal stretch ratios, lambda ~= 1 + alpha (T - T0) (Section 3.2, after
 * Eq. 11), optionally times a reversible shrinkage factor: li across the axes,
 * lm along m (the fibre), ln along n. */
static void thermal_stretch(const orc_material *m, double Te, double *li, double *lm, double *ln)
{
    double dT = Te - m->T0;
    double a = 1.0 + m->alpha * dT;
    double b = (m->expan_mode == 1 || m->expan_mode == 2) ? 1.0 + m->alpha_m * dT : a;
    double c = (m->expan_mode == 2) ? 1.0 + m->alpha_n * dT : a;
    if (m->shrink_on) {
        double s = 1.0 + m->shrink_eps * clamp01((Te - m->shrink_T) / m->shrink_width);
        a *= s;
        b *= s;
        c *= s;
    }
    *li = a;
    *lm = b;
    *ln = c;
}

/* Unit axes of Eq. 11: m = a / |a|, and n made orthogonal to m and unit length
 * (Gram-Schmidt; the paper takes m and n orthonormal).  Returns 0 when n is
 * (numerically) parallel to m. */
static int expansion_axes(const double *a_in, const double *n_in, double *mv, double *nv)
{
    double an = sqrt(a_in[0] * a_in[0] + a_in[1] * a_in[1] + a_in[2] * a_in[2]);
    for (int i = 0; i < 3; ++i) mv[i] = a_in[i] / an;
    if (!n_in) { nv[0] = nv[1] = nv[2] = 0.0; return 1; }
    double nn0 = sqrt(n_in[0] * n_in[0] + n_in[1] * n_in[1] + n_in[2] * n_in[2]);
    double d = n_in[0] * mv[0] + n_in[1] * mv[1] + n_in[2] * mv[2];
    double w[3] = {n_in[0] - d * mv[0], n_in[1] - d * mv[1], n_in[2] - d * mv[2]};
    double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (!(wn > 1e-6 * nn0)) return 0;
    for (int i = 0; i < 3; ++i) nv[i] = w[i] / wn;
    return 1;
}

/* Scale of mu and eta at temperature T (temperature-dependent mechanics). */
static double mech_scale(const orc_material *m, double T)
{
    if (!m->muT_on) return 1.0;
    return 1.0 - m->muT_drop * clamp01((T - m->muT_lo) / (m->muT_hi - m->muT_lo));
}

/* Linear c(T) and k(T) between (ckT_lo: c, k) and (ckT_hi: c_hi, k_hi), clamped (Table 5). */
static double heat_capacity(const orc_material *m, double T)
{
    if (!m->ckT_on) return m->c;
    double w = clamp01((T - m->ckT_lo) / (m->ckT_hi - m->ckT_lo));
    return m->c + w * (m->c_hi - m->c);
}

static double conductivity_scale(const orc_material *m, double T)
{
    if (!m->ckT_on) return 1.0;
    double w = clamp01((T - m->ckT_lo) / (m->ckT_hi - m->ckT_lo));
    return (m->k + w * (m->k_hi - m->k)) / m->k;
}

/*
 * Total second Piola-Kirchhoff stress S0 (Eqs. 7-10) for the transversely
 * isotropic neo-Hookean model of Table 5,
 *   Psi = mu/2 (I1bar - 3) + eta/2 (I4bar - 1)^2 + kappa/2 (J - 1)^2,
 * evaluated on the elastic part Fe = F Fth^-1 (Eq. 8), S_i = 2 dPsi/dC_i
 * (Eq. 9), pulled back with det(Fth) Fth^-1 S_i Fth^-T (Eq. 10).
 * Fth = lambda_i I + (lambda_m - lambda_i) m (x) m + (lambda_n - lambda_i) n (x) n
 * (Eq. 11) with m the unit fibre a and n the second axis (n_in, made orthonormal
 * to m; may be NULL outside the orthotropic mode).  The transversely isotropic
 * form has lambda_n = lambda_i and the isotropic one lambda_m = lambda_n = lambda_i.
 * psi returns det(Fth) Psi, the strain energy per unit reference volume.
 * Returns J of the elastic part.
 */
double orc_stress(const orc_material *m, const double *F, const double *a_in, const double *n_in,
                  double Te, double *S0, double *psi)
{
    double a[3], nv[3];
    expansion_axes(a_in, m->expan_mode == 2 ? n_in : NULL, a, nv);
    double A0[9], N0[9], I3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            A0[3 * i + j] = a[i] * a[j];
            N0[3 * i + j] = nv[i] * nv[j];
        }

    double li, lm, ln;
    thermal_stretch(m, Te, &li, &lm, &ln);
    double Fth[9], Fth_inv[9], Fth_invT[9];
    for (int i = 0; i < 9; ++i) Fth[i] = li * I3[i] + (lm - li) * A0[i] + (ln - li) * N0[i];
    inv3(Fth, Fth_inv);
    transpose3(Fth_inv, Fth_invT);
    double detFth = det3(Fth);

    double Fe[9], FeT[9], Ce[9], Ce_inv[9];
    mul3(F, Fth_inv, Fe);
    transpose3(Fe, FeT);
    mul3(FeT, Fe, Ce);
    double J = det3(Fe);
    double I1 = Ce[0] + Ce[4] + Ce[8];
    double I4 = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) I4 += a[i] * Ce[3 * i + j] * a[j];
    inv3(Ce, Ce_inv);

    double s = mech_scale(m, Te);
    double mu = m->mu * s, eta = m->eta * s, kappa = m->kappa;
    double J23 = pow(J, -2.0 / 3.0);
    double I1bar = J23 * I1, I4bar = J23 * I4;

    double Si[9];
    for (int i = 0; i < 9; ++i) {
        Si[i] = mu * J23 * (I3[i] - I1 / 3.0 * Ce_inv[i])
              + 2.0 * eta * (I4bar - 1.0) * J23 * (A0[i] - I4 / 3.0 * Ce_inv[i])
              + kappa * J * (J - 1.0) * Ce_inv[i];
    }
    double T1[9], T2[9];
    mul3(Fth_inv, Si, T1);
    mul3(T1, Fth_invT, T2);
    for (int i = 0; i < 9; ++i) S0[i] = detFth * T2[i];
    if (psi)
        *psi = detFth * (0.5 * mu * (I1bar - 3.0) + 0.5 * eta * (I4bar - 1.0) * (I4bar - 1.0)
                         + 0.5 * kappa * (J - 1.0) * (J - 1.0));
    return J;
}

/* ---------------------------------------------------------------------- */
/* Element geometry (the precomputed total-Lagrangian quantities).          */
/* ---------------------------------------------------------------------- */

/* H8 local node signs (xi, eta, zeta), node order (---),(+--),(++-),(-+-),
 * (--+),(+-+),(+++),(-++). */
static const double H8_XI[8]   = {-1, 1, 1, -1, -1, 1, 1, -1};
static const double H8_ETA[8]  = {-1, -1, 1, 1, -1, -1, 1, 1};
static const double H8_ZETA[8] = {-1, -1, -1, -1, 1, 1, 1, 1};

/* T4: D = [X2-X1 | X3-X1 | X4-X1], V0 = det D / 6, dh_{k+1}/dX = row k of D^-1,
 * dh_1/dX = -(sum of the others).  Returns det D. */
static double t4_geometry(const double *Xe, double *dhdx, double *V0)
{
    double D[9], Dinv[9];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) D[3 * i + k] = Xe[3 * (k + 1) + i] - Xe[i];
    double d = det3(D);
    if (d == 0.0) return d;
    inv3(D, Dinv);
    for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) {
            dhdx[3 * (k + 1) + j] = Dinv[3 * k + j];
            s += Dinv[3 * k + j];
        }
        dhdx[j] = -s;
    }
    *V0 = d / 6.0;
    return d;
}

/* H8 with one integration point at the centre: dh_a/dxi = (xi_a, eta_a, zeta_a)/8,
 * J0 = sum_a X_a (x) dh_a/dxi, dh_a/dX = J0^-T dh_a/dxi, V0 = 8 det J0 (Eqs. 18, 25).
 * Also the hourglass vectors gamma_alpha = h_alpha - (dh/dX)(X^T h_alpha).  Returns det J0. */
static double h8_geometry(const double *Xe, double *dhdx, double *V0, double *gam)
{
    double J0[9] = {0}, J0inv[9];
    double dNdxi[8][3];
    for (int a = 0; a < 8; ++a) {
        dNdxi[a][0] = H8_XI[a] / 8.0;
        dNdxi[a][1] = H8_ETA[a] / 8.0;
        dNdxi[a][2] = H8_ZETA[a] / 8.0;
    }
    for (int a = 0; a < 8; ++a)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) J0[3 * i + j] += Xe[3 * a + i] * dNdxi[a][j];
    double d = det3(J0);
    if (!(d > 0.0)) return d;
    inv3(J0, J0inv);
    for (int a = 0; a < 8; ++a)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += dNdxi[a][k] * J0inv[3 * k + j];
            dhdx[3 * a + j] = s;
        }
    *V0 = 8.0 * d;
    if (gam) {
        double h[4][8];
        for (int a = 0; a < 8; ++a) {
            h[0][a] = H8_ETA[a] * H8_ZETA[a];
            h[1][a] = H8_ZETA[a] * H8_XI[a];
            h[2][a] = H8_XI[a] * H8_ETA[a];
            h[3][a] = H8_XI[a] * H8_ETA[a] * H8_ZETA[a];
        }
        for (int al = 0; al < 4; ++al) {
            double c[3] = {0, 0, 0};
            for (int b = 0; b < 8; ++b)
                for (int i = 0; i < 3; ++i) c[i] += Xe[3 * b + i] * h[al][b];
            for (int a = 0; a < 8; ++a) {
                double s = 0.0;
                for (int i = 0; i < 3; ++i) s += dhdx[3 * a + i] * c[i];
                gam[8 * al + a] = h[al][a] - s;
            }
        }
    }
    return d;
}

static double tri_area(const double *p, const double *q, const double *r)
{
    double u[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
    double v[3] = {r[0] - p[0], r[1] - p[1], r[2] - p[2]};
    double w[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
    return 0.5 * sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
}

static double quad_area(const double *p0, const double *p1, const double *p2, const double *p3)
{
    double d1[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
    double d2[3] = {p3[0] - p1[0], p3[1] - p1[1], p3[2] - p1[2]};
    double w[3] = {d1[1] * d2[2] - d1[2] * d2[1], d1[2] * d2[0] - d1[0] * d2[2], d1[0] * d2[1] - d1[1] * d2[0]};
    return 0.5 * sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
}

/* Characteristic length for the critical time step. */
static double element_length(int npe, const double *Xe, double V0)
{
    double amax = 0.0, A;
    if (npe == 4) {
        static const int f[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
        for (int i = 0; i < 4; ++i) {
            A = tri_area(Xe + 3 * f[i][0], Xe + 3 * f[i][1], Xe + 3 * f[i][2]);
            if (A > amax) amax = A;
        }
        return 3.0 * V0 / amax;
    }
    static const int f[6][4] = {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 3, 7, 4},
                                {1, 2, 6, 5}, {0, 1, 5, 4}, {3, 2, 6, 7}};
    for (int i = 0; i < 6; ++i) {
        A = quad_area(Xe + 3 * f[i][0], Xe + 3 * f[i][1], Xe + 3 * f[i][2], Xe + 3 * f[i][3]);
        if (A > amax) amax = A;
    }
    return V0 / amax;
}

/* ---------------------------------------------------------------------- */
/* One element: nodal forces (Eqs. 24-28) and conduction loads (Eq. 16).  */
/* ---------------------------------------------------------------------- */
typedef struct {
    double psi;    /* strain energy of the element (J), incl. hourglass      */
    double J;      /* det F                                                 */
} elem_info;

static void element_compute(const orc_material *m, int npe, const double *dhdx, double V0,
                            const double *gam, double khg,
                            const double *ue, const double *Te_nodes, const double *a,
                            const double *nax, const double *Dc,
                            double *theta, double dt, double *f, double *h, elem_info *info)
{
    /* Eq. 17: F = u_e^T (L h) + I, i.e. F_ij = delta_ij + sum_a u_a,i dh_a/dX_j */
    double F[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (int ai = 0; ai < npe; ++ai)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) F[3 * i + j] += ue[3 * ai + i] * dhdx[3 * ai + j];

    double Te = 0.0;
    for (int ai = 0; ai < npe; ++ai) Te += Te_nodes[ai];
    Te /= (double)npe;

    double S0[9], psi;
    orc_stress(m, F, a, nax, Te, S0, &psi);

    /* Prony recursion on the total stress (after Eq. 27):
     * theta_i <- dt phi_i/(dt + tau_i) S + tau_i/(dt + tau_i) theta_i ; S~ = S - sum theta_i */
    double St[9];
    for (int i = 0; i < 9; ++i) St[i] = S0[i];
    static const int sym[9] = {0, 3, 5, 3, 1, 4, 5, 4, 2}; /* (xx yy zz xy yz xz) */
    for (int p = 0; p < m->n_prony; ++p) {
        double c1 = dt * m->g[p] / (dt + m->tau[p]);
        double c2 = m->tau[p] / (dt + m->tau[p]);
        double *th = theta + 6 * p;
        double Sv[6] = {S0[0], S0[4], S0[8], S0[1], S0[5], S0[2]};
        for (int c = 0; c < 6; ++c) th[c] = c1 * Sv[c] + c2 * th[c];
        for (int i = 0; i < 9; ++i) St[i] -= th[sym[i]];
    }

    /* Eq. 28 with one point: f_a = V0 F S~ dh_a/dX */
    double P[9];
    mul3(F, St, P);
    for (int ai = 0; ai < npe; ++ai)
        for (int i = 0; i < 3; ++i) {
            double s = 0.0;
            for (int j = 0; j < 3; ++j) s += P[3 * i + j] * dhdx[3 * ai + j];
            f[3 * ai + i] = V0 * s;
        }

    double e_hg = 0.0;
    if (npe == 8 && gam) {
        /* hourglass: f_a += khg sum_alpha gamma_alpha,a (gamma_alpha . u) */
        for (int al = 0; al < 4; ++al) {
            double q[3] = {0, 0, 0};
            for (int b = 0; b < 8; ++b)
                for (int i = 0; i < 3; ++i) q[i] += gam[8 * al + b] * ue[3 * b + i];
            for (int ai = 0; ai < 8; ++ai)
                for (int i = 0; i < 3; ++i) f[3 * ai + i] += khg * gam[8 * al + ai] * q[i];
            e_hg += 0.5 * khg * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        }
    }

    /* Eq. 16 (Eqs. 18-19 with one point):
     * K_e = V0 det(F) (L h F^-1) D (L h F^-1)^T, f_ther = K_e T_e, with D the
     * element conductivity tensor of Eq. 15 (times k(T)/k when temperature-dependent) */
    double Finv[9];
    inv3(F, Finv);
    double J = det3(F);
    double kT = m->k * conductivity_scale(m, Te);
    double kmT = m->k_m * conductivity_scale(m, Te);
    double an = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    double D[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            D[3 * i + j] = (i == j) ? kT : 0.0;
            if (m->cond_mode == 1) D[3 * i + j] += (kmT - kT) * (a[i] / an) * (a[j] / an);
        }
    if (m->cond_mode == 2) {
        static const int comp[9] = {0, 3, 5, 3, 1, 4, 5, 4, 2}; /* (xx yy zz xy yz xz) */
        double ks = conductivity_scale(m, Te);
        for (int i = 0; i < 9; ++i) D[i] = ks * Dc[comp[i]];
    }
    double BF[8][3];
    for (int ai = 0; ai < npe; ++ai)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += dhdx[3 * ai + k] * Finv[3 * k + j];
            BF[ai][j] = s;
        }
    for (int ai = 0; ai < npe; ++ai) {
        double s = 0.0;
        for (int b = 0; b < npe; ++b) {
            double kab = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) kab += BF[ai][i] * D[3 * i + j] * BF[b][j];
            s += V0 * J * kab * Te_nodes[b];
        }
        h[ai] = s;
    }

    if (info) {
        info->psi = V0 * psi + e_hg;
        info->J = J;
    }
}

/* Element-level entry for the closed-form and finite-difference tests.
 * Xe npe x 3, ue npe x 3, Te npe, theta n_prony x 6 (in/out), outputs f npe x 3, h npe.
 * Returns 0, or ORC_E_MESH for a degenerate element. */
int orc_element(const orc_material *m, int32_t npe, const double *Xe, const double *ue,
                const double *Te, const double *a0, const double *n0, const double *Dc,
                double *theta, double dt, double *f, double *h, double *energy)
{
    if (m->expan_mode == 2) {
        double mv[3], nv[3];
        if (!n0 || !expansion_axes(a0, n0, mv, nv)) return ORC_E_ARG;
    }
    if (m->cond_mode == 2 && !Dc) return ORC_E_ARG;
    double dhdx[24], V0 = 0.0, gam[32];
    double d;
    if (npe == 4) d = t4_geometry(Xe, dhdx, &V0);
    else if (npe == 8) d = h8_geometry(Xe, dhdx, &V0, gam);
    else return ORC_E_ARG;
    if (!(d > 0.0)) return ORC_E_MESH;
    double khg = 0.0;
    if (npe == 8) {
        double s = 0.0;
        for (int i = 0; i < 24; ++i) s += dhdx[i] * dhdx[i];
        khg = m->hg_coef * (m->kappa + 4.0 * m->mu / 3.0) * V0 * s / 8.0;
    }
    double th0[24] = {0};
    elem_info info;
    element_compute(m, npe, dhdx, V0, npe == 8 ? gam : NULL, khg, ue, Te, a0, n0, Dc,
                    theta ? theta : th0, dt, f, h, &info);
    if (energy) *energy = info.psi;
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Problem set-up: copies inputs, precomputes geometry and lumped matrices. */
/* ---------------------------------------------------------------------- */
void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->X); free(s->conn); free(s->a0); free(s->n0); free(s->Dc); free(s->q); free(s->fix); free(s->Tfix);
    free(s->dhdx); free(s->V0); free(s->gam); free(s->khg);
    free(s->Vl); free(s->M); free(s->Kb); free(s->Qm); free(s->Qr);
    free(s);
}

int orc_create(orc_sim **out, int32_t npe, int64_t nn, const double *X, int64_t ne,
               const int32_t *conn, const double *a0, const double *n0, const double *Dc,
               const double *q, const uint8_t *fix,
               const double *Tfix, const orc_material *m, double t_on, double t_off,
               double dt, double gamma)
{
    *out = NULL;
    if ((npe != 4 && npe != 8) || nn <= 0 || ne <= 0 || !X || !conn || !m) return ORC_E_ARG;
    if (m->n_prony < 0 || m->n_prony > 4) return ORC_E_ARG;
    if ((m->expan_mode == 2 && !n0) || (m->cond_mode == 2 && !Dc)) return ORC_E_ARG;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    if (!s) return ORC_E_OOM;
    s->npe = npe; s->nn = nn; s->ne = ne; s->m = *m;
    s->t_on = t_on; s->t_off = t_off; s->dt = dt; s->gamma = gamma;
    s->X = malloc(sizeof(double) * 3 * nn);
    s->conn = malloc(sizeof(int32_t) * npe * ne);
    s->a0 = malloc(sizeof(double) * 3 * ne);
    s->q = calloc(ne, sizeof(double));
    s->fix = calloc(nn, 1);
    s->Tfix = calloc(nn, sizeof(double));
    s->dhdx = malloc(sizeof(double) * 3 * npe * ne);
    s->V0 = malloc(sizeof(double) * ne);
    s->gam = (npe == 8) ? malloc(sizeof(double) * 32 * ne) : NULL;
    s->khg = calloc(ne, sizeof(double));
    s->Vl = calloc(nn, sizeof(double));
    s->M = calloc(nn, sizeof(double));
    s->Kb = calloc(nn, sizeof(double));
    s->Qm = calloc(nn, sizeof(double));
    s->Qr = calloc(nn, sizeof(double));
    if (!s->X || !s->conn || !s->a0 || !s->q || !s->fix || !s->Tfix || !s->dhdx || !s->V0 ||
        (npe == 8 && !s->gam) || !s->khg || !s->Vl || !s->M || !s->Kb || !s->Qm || !s->Qr) {
        orc_destroy(s);
        return ORC_E_OOM;
    }
    memcpy(s->X, X, sizeof(double) * 3 * nn);
    memcpy(s->conn, conn, sizeof(int32_t) * npe * ne);
    for (int64_t e = 0; e < ne; ++e) {
        if (a0) { s->a0[3 * e] = a0[3 * e]; s->a0[3 * e + 1] = a0[3 * e + 1]; s->a0[3 * e + 2] = a0[3 * e + 2]; }
        else { s->a0[3 * e] = 1.0; s->a0[3 * e + 1] = 0.0; s->a0[3 * e + 2] = 0.0; }
    }
    if (m->expan_mode == 2) {
        s->n0 = malloc(sizeof(double) * 3 * ne);
        if (!s->n0) { orc_destroy(s); return ORC_E_OOM; }
        memcpy(s->n0, n0, sizeof(double) * 3 * ne);
        for (int64_t e = 0; e < ne; ++e) {
            double mv[3], nv[3];
            if (!expansion_axes(s->a0 + 3 * e, s->n0 + 3 * e, mv, nv)) { orc_destroy(s); return ORC_E_ARG; }
        }
    }
    if (m->cond_mode == 2) {
        s->Dc = malloc(sizeof(double) * 6 * ne);
        if (!s->Dc) { orc_destroy(s); return ORC_E_OOM; }
        memcpy(s->Dc, Dc, sizeof(double) * 6 * ne);
    }
    if (q) memcpy(s->q, q, sizeof(double) * ne);
    if (fix) memcpy(s->fix, fix, nn);
    if (Tfix) memcpy(s->Tfix, Tfix, sizeof(double) * nn);

    double cd = sqrt((m->kappa + 4.0 * m->mu / 3.0 + 4.0 * m->eta) / m->rho);
    s->dt_cr = INFINITY;
    for (int64_t e = 0; e < ne; ++e) {
        int32_t *c = s->conn + (int64_t)npe * e;
        double Xe[24];
        for (int a = 0; a < npe; ++a) {
            if (c[a] < 0 || c[a] >= nn) { orc_destroy(s); return ORC_E_MESH; }
            for (int i = 0; i < 3; ++i) Xe[3 * a + i] = s->X[3 * (int64_t)c[a] + i];
        }
        double *dh = s->dhdx + (int64_t)3 * npe * e;
        double d;
        if (npe == 4) {
            d = t4_geometry(Xe, dh, &s->V0[e]);
            if (d < 0.0) {            /* repair orientation: swap the last two nodes */
                int32_t t = c[2]; c[2] = c[3]; c[3] = t;
                for (int i = 0; i < 3; ++i) { double x = Xe[6 + i]; Xe[6 + i] = Xe[9 + i]; Xe[9 + i] = x; }
                d = t4_geometry(Xe, dh, &s->V0[e]);
                s->n_swapped++;
            }
            if (!(d > 0.0)) { orc_destroy(s); return ORC_E_MESH; }
        } else {
            d = h8_geometry(Xe, dh, &s->V0[e], s->gam + 32 * e);
            if (!(d > 0.0)) { orc_destroy(s); return ORC_E_MESH; }
            double ss = 0.0;
            for (int i = 0; i < 24; ++i) ss += dh[i] * dh[i];
            s->khg[e] = m->hg_coef * (m->kappa + 4.0 * m->mu / 3.0) * s->V0[e] * ss / 8.0;
        }
        double L = element_length(npe, Xe, s->V0[e]);
        double dte = L / cd;
        if (dte < s->dt_cr) s->dt_cr = dte;
        /* lumping with reference volumes */
        for (int a = 0; a < npe; ++a) {
            s->Vl[c[a]] += s->V0[e] / npe;
            s->Qr[c[a]] += s->q[e] * s->V0[e] / npe;
        }
    }
    for (int64_t a = 0; a < nn; ++a) {
        s->M[a] = m->rho * s->Vl[a];
        s->Kb[a] = m->wbcb * s->Vl[a];
        s->Qm[a] = m->Q_met * s->Vl[a];
    }
    *out = s;
    return ORC_OK;
}

double orc_critical_dt(const orc_sim *s) { return s->dt_cr; }
int64_t orc_n_swapped(const orc_sim *s) { return s->n_swapped; }

void orc_lumped(const orc_sim *s, double *Vl, double *M, double *Kb, double *Qm, double *Qr)
{
    for (int64_t a = 0; a < s->nn; ++a) {
        if (Vl) Vl[a] = s->Vl[a];
        if (M) M[a] = s->M[a];
        if (Kb) Kb[a] = s->Kb[a];
        if (Qm) Qm[a] = s->Qm[a];
        if (Qr) Qr[a] = s->Qr[a];
    }
}

void orc_geometry(const orc_sim *s, int32_t *conn, double *dhdx, double *V0)
{
    if (conn) memcpy(conn, s->conn, sizeof(int32_t) * s->npe * s->ne);
    if (dhdx) memcpy(dhdx, s->dhdx, sizeof(double) * 3 * s->npe * s->ne);
    if (V0) memcpy(V0, s->V0, sizeof(double) * s->ne);
}

/* Element loop of one step: internal forces Fint (nn x 3), conduction loads Hc (nn),
 * updated Prony state; returns strain energy and min det F through the pointers. */
static void element_loop(const orc_sim *s, const double *u, const double *T, double *theta,
                         double *Fint, double *Hc, double *energy, double *minJ)
{
    int npe = s->npe;
    memset(Fint, 0, sizeof(double) * 3 * s->nn);
    memset(Hc, 0, sizeof(double) * s->nn);
    double E = 0.0, Jmin = INFINITY;
    for (int64_t e = 0; e < s->ne; ++e) {
        const int32_t *c = s->conn + (int64_t)npe * e;
        double ue[24], Te[8], f[24], h[8];
        for (int a = 0; a < npe; ++a) {
            for (int i = 0; i < 3; ++i) ue[3 * a + i] = u[3 * (int64_t)c[a] + i];
            Te[a] = T[c[a]];
        }
        elem_info info;
        element_compute(&s->m, npe, s->dhdx + (int64_t)3 * npe * e, s->V0[e],
                        npe == 8 ? s->gam + 32 * e : NULL, s->khg[e], ue, Te, s->a0 + 3 * e,
                        s->n0 ? s->n0 + 3 * e : NULL, s->Dc ? s->Dc + 6 * e : NULL,
                        theta + (int64_t)6 * s->m.n_prony * e, s->dt, f, h, &info);
        for (int a = 0; a < npe; ++a) {
            for (int i = 0; i < 3; ++i) Fint[3 * (int64_t)c[a] + i] += f[3 * a + i];
            Hc[c[a]] += h[a];
        }
        E += info.psi;
        if (info.J < Jmin) Jmin = info.J;
    }
    *energy = E;
    *minJ = Jmin;
}

/* Conduction loads K(u) T for a given state (no Prony update), for the patch tests. */
int orc_loads(const orc_sim *s, const double *u, const double *T, double *Fint, double *Hc)
{
    int64_t nth = (int64_t)6 * s->m.n_prony * s->ne;
    double *theta = calloc(nth > 0 ? nth : 1, sizeof(double));
    if (!theta) return ORC_E_OOM;
    double E, Jm;
    element_loop(s, u, T, theta, Fint, Hc, &E, &Jm);
    free(theta);
    return ORC_OK;
}

/*
 * Advance nsteps from step index step0.  State in/out:
 *   u, u_prev  nn x 3  displacement at steps n and n-1
 *   T          nn      absolute temperature, K
 *   theta      ne x n_prony x 6 Prony state (xx yy zz xy yz xz)
 * monitors (nsteps x 6, may be NULL) receives per step n:
 *   [0] strain energy of u^n (incl. hourglass), [1] 1/2 sum M |v^{n+1/2}|^2,
 *   [2] 1/2 sum M v^{n-1/2}.v^{n+1/2}, [3] max T^{n+1}, [4] sum rho c Vl T^{n+1},
 *   [5] min det F at step n.
 * Explicit Pennes update: Eq. 20 with the conduction sign of the reading above.
 * Displacement update: the central difference of Eq. 27 with R = 0, D = gamma M.
 */
int orc_run(const orc_sim *s, int64_t nsteps, int64_t step0, double *u, double *u_prev,
            double *T, double *theta, double *monitors)
{
    int64_t nn = s->nn;
    double *Fint = malloc(sizeof(double) * 3 * nn);
    double *Hc = malloc(sizeof(double) * nn);
    double *un = malloc(sizeof(double) * 3 * nn);
    double *Tn = malloc(sizeof(double) * nn);
    if (!Fint || !Hc || !un || !Tn) { free(Fint); free(Hc); free(un); free(Tn); return ORC_E_OOM; }
    const double dt = s->dt, g = s->gamma;
    for (int64_t it = 0; it < nsteps; ++it) {
        int64_t n = step0 + it;
        double t = (double)n * dt;
        double src = (t >= s->t_on && t < s->t_off) ? 1.0 : 0.0;
        double E, Jmin;
        element_loop(s, u, T, theta, Fint, Hc, &E, &Jmin);
        double ke_half = 0.0, ke_cross = 0.0, Tmax = -INFINITY, heat = 0.0;
        for (int64_t a = 0; a < nn; ++a) {
            /* Eq. 20 */
            double Ca = s->m.rho * heat_capacity(&s->m, T[a]) * s->Vl[a];
            double Tnew = T[a] + dt / Ca * (-Hc[a] - s->Kb[a] * (T[a] - s->m.T_art) + s->Qm[a] + src * s->Qr[a]);
            if (s->fix[a] & 8) Tnew = s->Tfix[a];
            Tn[a] = Tnew;
            /* Eq. 27 */
            double M = s->M[a];
            double den = g * M / (2.0 * dt) + M / (dt * dt);
            for (int i = 0; i < 3; ++i) {
                int64_t k = 3 * a + i;
                double unew = (-Fint[k] + 2.0 * M / (dt * dt) * u[k]
                               + (g * M / (2.0 * dt) - M / (dt * dt)) * u_prev[k]) / den;
                if (s->fix[a] & (1 << i)) unew = 0.0;
                un[k] = unew;
                double vp = (unew - u[k]) / dt, vm = (u[k] - u_prev[k]) / dt;
                ke_half += 0.5 * M * vp * vp;
                ke_cross += 0.5 * M * vm * vp;
            }
            if (Tnew > Tmax) Tmax = Tnew;
            heat += s->m.rho * heat_capacity(&s->m, Tnew) * s->Vl[a] * Tnew;
        }
        memcpy(u_prev, u, sizeof(double) * 3 * nn);
        memcpy(u, un, sizeof(double) * 3 * nn);
        memcpy(T, Tn, sizeof(double) * nn);
        if (monitors) {
            double *mo = monitors + 6 * it;
            mo[0] = E; mo[1] = ke_half; mo[2] = ke_cross; mo[3] = Tmax; mo[4] = heat; mo[5] = Jmin;
        }
    }
    free(Fint); free(Hc); free(un); free(Tn);
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Thermal dose.  Section 7 names thermal-damage models as the clinical    */
/* measures of an ablation besides an isotherm; their published             */
/* definitions, one time step's contribution at the temperature the step   */
/* ends at (a rectangle rule in time):                                     */
/*   CEM43 (Sapareto and Dewey), cumulative equivalent minutes at 43 C:    */
/*     (dt / 60) R^(43 - T_C), R = 0.5 for T_C >= 43 C, 0.25 below;         */
/*   Arrhenius damage integral (Henriques and Moritz):                     */
/*     dt A exp(-Ea / (R_gas T)), T in kelvin, R_gas = 8.314462618 J/(mol K); */
/*     nothing is added when A <= 0.                                       */
/* ---------------------------------------------------------------------- */
void orc_thermal_dose(int64_t nn, const double *T, double dt, double A, double Ea, double *cem43, double *omega)
{
    const double R_gas = 8.314462618;
    for (int64_t a = 0; a < nn; ++a) {
        double Tc = T[a] - 273.15;
        double R = Tc >= 43.0 ? 0.5 : 0.25;
        cem43[a] += dt / 60.0 * pow(R, 43.0 - Tc);
        if (A > 0.0) omega[a] += dt * A * exp(-Ea / (R_gas * T[a]));
    }
}
