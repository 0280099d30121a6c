// HIP kernels of one coupled TLED + Pennes time step for CDNA4 (gfx950).
//
// Two variants share the element physics of device_math.h:
//   two-pass: element kernel (one thread per element) writes its npe nodal
//     (force, heat) contributions; node kernel (one thread per node) sums its
//     incident contributions in a fixed order and advances the node;
//   fused patch: one workgroup per patch of contiguous elements stages the
//     patch nodes in LDS, computes the elements, assembles and advances the
//     patch-interior nodes in LDS, and writes partial sums for the nodes it
//     shares with other patches; a shared-node kernel finishes those.
// No atomics in the assembly; every sum has a fixed order, so a run is
// bitwise reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_math.h"
#include "kernels.h"

#include <hip/hip_ext.h>

// Launch with optional timing: with a start/stop event pair the events are taken
// by the dispatch itself (hipExtLaunchKernelGGL), so no extra packets sit
// between kernels and the elapsed time is the kernel's own duration.
#define TLED_LAUNCH(ev, kern, grid, block, lds, stream, ...)                                              \
    do {                                                                                                  \
        if (ev) hipExtLaunchKernelGGL(kern, grid, block, lds, stream, (ev)->start, (ev)->stop, 0, __VA_ARGS__); \
        else hipLaunchKernelGGL(kern, grid, block, lds, stream, __VA_ARGS__);                             \
    } while (0)


namespace tled {

// Workgroups are dispatched round-robin over the XCDs; map them so that
// consecutive logical blocks (neighbouring elements in the locality order)
// run on the same XCD and share its L2.
__device__ __forceinline__ int xcd_block(int b, int G) {
    const int q = G / kNumXcd, r = G % kNumXcd;
    const int x = b % kNumXcd, i = b / kNumXcd;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__device__ __forceinline__ bool finite4(float4 v) {
    return isfinite(v.x) && isfinite(v.y) && isfinite(v.z) && isfinite(v.w);
}

// Block-wide sum of a double, then one partial per block (fixed order).
template <int BS>
__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < BS / 64; ++i) s += sh[i];
    __syncthreads();
    return s;
}

template <int BS>
__device__ __forceinline__ float block_max(float v, float *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    float s = -INFINITY;
    if (threadIdx.x == 0)
        for (int i = 0; i < BS / 64; ++i) s = fmaxf(s, sh[i]);
    __syncthreads();
    return s;
}

__device__ __forceinline__ void raise_flags(unsigned *status, bool nonfinite, bool inverted) {
    // one atomic per wavefront, only when something went wrong
    unsigned f = (nonfinite ? TLED_FLAG_NONFINITE : 0u) | (inverted ? TLED_FLAG_INVERTED : 0u);
    unsigned long long any = __ballot(f != 0u);
    if (any) {
        unsigned fw = f;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) fw |= __shfl_xor(fw, o);
        if ((threadIdx.x & 63) == 0) atomicOr(status, fw);
    }
}

// ---------------------------------------------------------------- element math

struct ElemResultT4 {
    float4 o[4];
    float psiV;
    bool nonfinite, inverted;
};

// T4 geometry: rows b_k = dh_{k}/dX of local nodes 1..3 (node 0 is minus their sum), V0, fibre.
struct GeoT4 {
    float b[3][3];
    float V0;
    float a[3];
};

// From the precomputed planes g0,g1,g2 = (b1, b2, b3, V0, fibre in octahedral coordinates).
__device__ __forceinline__ GeoT4 t4_geo_planes(float4 g0, float4 g1, float4 g2) {
    GeoT4 g;
    g.b[0][0] = g0.x; g.b[0][1] = g0.y; g.b[0][2] = g0.z;
    g.b[1][0] = g0.w; g.b[1][1] = g1.x; g.b[1][2] = g1.y;
    g.b[2][0] = g1.z; g.b[2][1] = g1.w; g.b[2][2] = g2.x;
    g.V0 = g2.y;
    oct_decode(g2.z, g2.w, g.a);
    return g;
}

// From reference coordinates (relative to the patch centroid): with edge columns
// e_k = X_k - X_0, D^-1 has rows (e2 x e3, e3 x e1, e1 x e2) / det D and V0 = det D / 6.
__device__ __forceinline__ GeoT4 t4_geo_coords(const float4 x[4], float2 fib) {
    GeoT4 g;
    const float e[3][3] = {{x[1].x - x[0].x, x[1].y - x[0].y, x[1].z - x[0].z},
                           {x[2].x - x[0].x, x[2].y - x[0].y, x[2].z - x[0].z},
                           {x[3].x - x[0].x, x[3].y - x[0].y, x[3].z - x[0].z}};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float *p = e[(k + 1) % 3], *q = e[(k + 2) % 3];
        g.b[k][0] = p[1] * q[2] - p[2] * q[1];
        g.b[k][1] = p[2] * q[0] - p[0] * q[2];
        g.b[k][2] = p[0] * q[1] - p[1] * q[0];
    }
    const float det = e[0][0] * g.b[0][0] + e[0][1] * g.b[0][1] + e[0][2] * g.b[0][2];
    const float inv = rcp(det);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        g.b[k][0] *= inv; g.b[k][1] *= inv; g.b[k][2] *= inv;
    }
    g.V0 = det * (1.0f / 6.0f);
    oct_decode(fib.x, fib.y, g.a);
    return g;
}

// T4 element: node data u4 = (ux, uy, uz, dT).
template <int NP, bool MON, bool ANISO>
__device__ __forceinline__ void t4_compute(const KMat &m, const float4 u[4], const GeoT4 &g, float *th,
                                           ElemResultT4 &r, const float4 *__restrict__ aniso, int e) {
    float d[3][4];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        d[k][0] = u[k + 1].x - u[0].x;
        d[k][1] = u[k + 1].y - u[0].y;
        d[k][2] = u[k + 1].z - u[0].z;
        d[k][3] = u[k + 1].w - u[0].w;
    }
    float H[9], gT[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            H[3 * i + j] = d[0][i] * g.b[0][j] + d[1][i] * g.b[1][j] + d[2][i] * g.b[2][j];
#pragma unroll
    for (int j = 0; j < 3; ++j) gT[j] = d[0][3] * g.b[0][j] + d[1][3] * g.b[1][j] + d[2][3] * g.b[2][j];
    const float dTe = 0.25f * (u[0].w + u[1].w + u[2].w + u[3].w);
    ElemOut eo;
    element_physics<NP, ANISO>(m, H, gT, dTe, g.a, g.V0, th, MON, eo, aniso, e);
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float *b = g.b[k];
        float4 f;
        f.x = eo.PV[0] * b[0] + eo.PV[1] * b[1] + eo.PV[2] * b[2];
        f.y = eo.PV[3] * b[0] + eo.PV[4] * b[1] + eo.PV[5] * b[2];
        f.z = eo.PV[6] * b[0] + eo.PV[7] * b[1] + eo.PV[8] * b[2];
        f.w = eo.qV[0] * b[0] + eo.qV[1] * b[1] + eo.qV[2] * b[2];
        r.o[k + 1] = f;
        s.x += f.x; s.y += f.y; s.z += f.z; s.w += f.w;
    }
    r.o[0] = make_float4(-s.x, -s.y, -s.z, -s.w);
    r.psiV = MON ? eo.psiV : 0.0f;
    r.inverted = !(eo.Jmin > 0.0f);
    r.nonfinite = !(finite4(r.o[0]) && finite4(r.o[1]) && finite4(r.o[2]) && finite4(r.o[3]));
}

// H8 local nodes carry the natural-coordinate signs (xi, eta, zeta) = (---), (+--),
// (++-), (-+-), (--+), (+-+), (+++), (-++); the hourglass base vectors are eta zeta,
// zeta xi, xi eta, xi eta zeta.

struct ElemResultH8 {
    float4 o[8];
    float psiV;
    bool nonfinite, inverted;
};

// H8 geometry: G = J0^-T (dh_a/dX = G s_a / 8), V0, fibre, c_alpha = X^T h_alpha, k_hg.
struct GeoH8 {
    float G[9];
    float V0;
    float a[3];
    float c[12];
    float khg;
};

__device__ __forceinline__ GeoH8 h8_geo_planes(float4 g0, float4 g1, float4 g2, float4 h0, float4 h1, float4 h2,
                                               float khg) {
    GeoH8 g;
    g.G[0] = g0.x; g.G[1] = g0.y; g.G[2] = g0.z; g.G[3] = g0.w; g.G[4] = g1.x;
    g.G[5] = g1.y; g.G[6] = g1.z; g.G[7] = g1.w; g.G[8] = g2.x;
    g.V0 = g2.y;
    oct_decode(g2.z, g2.w, g.a);
    const float c[12] = {h0.x, h0.y, h0.z, h0.w, h1.x, h1.y, h1.z, h1.w, h2.x, h2.y, h2.z, h2.w};
#pragma unroll
    for (int i = 0; i < 12; ++i) g.c[i] = c[i];
    g.khg = khg;
    return g;
}

// Walsh-Hadamard butterflies over the eight nodes of an H8, taken in the binary
// order of their natural-coordinate signs (bit 0: xi > 0, bit 1: eta > 0,
// bit 2: zeta > 0; node n sits at position kH8Bin[n], and the map is its own
// inverse).  The sign functions of the element are the products
// prod_{d in m} s_d over subsets m of the three directions: m = 1, 2, 4 are
// xi, eta, zeta (the one-point gradient), m = 6, 5, 3, 7 the hourglass modes
// eta zeta, zeta xi, xi eta, xi eta zeta, m = 0 the constant.  wht8 turns
// nodal values v into all eight sums sum_b f_m(b) v_b (24 additions instead of
// 56 for the seven sums formed one by one); iwht8 turns coefficients of the
// eight functions into nodal values.
__device__ constexpr int kH8Bin[8] = {0, 1, 3, 2, 4, 5, 7, 6};

__device__ __forceinline__ void wht8(float v[8]) {
#pragma unroll
    for (int h = 1; h < 8; h <<= 1)
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (!(i & h)) {
                const float a = v[i], b = v[i + h];
                v[i] = b + a;
                v[i + h] = b - a;
            }
}

__device__ __forceinline__ void iwht8(float v[8]) {
#pragma unroll
    for (int h = 1; h < 8; h <<= 1)
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (!(i & h)) {
                const float a = v[i], b = v[i + h];
                v[i] = a - b;
                v[i + h] = a + b;
            }
}

// From reference coordinates: J0 = sum_a X_a (x) s_a / 8, G = J0^-T, V0 = 8 det J0,
// c_alpha = sum_a h_alpha,a X_a, k_hg = hg (kappa + 4 mu / 3) V0 tr(G^T G) / 64
// (sum_a |G s_a / 8|^2 = tr(G^T G) / 8 since sum_a s_a s_a^T = 8 I).  The sums are
// the sign-function sums of each coordinate (wht8); they do not see a common
// translation of the nodes.
__device__ __forceinline__ GeoH8 h8_geo_coords(const float4 x[8], float2 fib, float hgk) {
    GeoH8 g;
    float J[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        float v[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const float4 xb = x[kH8Bin[b]];
            v[b] = i == 0 ? xb.x : (i == 1 ? xb.y : xb.z);
        }
        wht8(v);
        J[3 * i] = 0.125f * v[1];
        J[3 * i + 1] = 0.125f * v[2];
        J[3 * i + 2] = 0.125f * v[4];
        g.c[i] = v[6];          // eta zeta
        g.c[3 + i] = v[5];      // zeta xi
        g.c[6 + i] = v[3];      // xi eta
        g.c[9 + i] = v[7];      // xi eta zeta
    }
    // G = J0^-T = cof(J0) / det J0
    const float cof[9] = {J[4] * J[8] - J[5] * J[7], J[5] * J[6] - J[3] * J[8], J[3] * J[7] - J[4] * J[6],
                          J[2] * J[7] - J[1] * J[8], J[0] * J[8] - J[2] * J[6], J[1] * J[6] - J[0] * J[7],
                          J[1] * J[5] - J[2] * J[4], J[2] * J[3] - J[0] * J[5], J[0] * J[4] - J[1] * J[3]};
    const float det = J[0] * cof[0] + J[1] * cof[1] + J[2] * cof[2];
    const float inv = rcp(det);
    float tr = 0.f;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        g.G[i] = cof[i] * inv;
        tr += g.G[i] * g.G[i];
    }
    g.V0 = 8.0f * det;
    g.khg = hgk * g.V0 * tr * (1.0f / 64.0f);
    oct_decode(fib.x, fib.y, g.a);
    return g;
}

template <int NP, bool MON, bool ANISO>
__device__ __forceinline__ void h8_compute(const KMat &m, const float4 u[8], const GeoH8 &g, float *th,
                                           ElemResultH8 &r, const float4 *__restrict__ aniso, int e) {
    const float *G = g.G;
    const float *c = g.c;
    const float V0 = g.V0, khg = g.khg;
    const float *a = g.a;
    // sign-function sums of every nodal component (wht8): U_ik = sum_a u_a,i s_a,k,
    // t_k = sum_a dT_a s_a,k, hourglass sums hu_alpha,i = sum_a h_alpha,a u_a,i
    float U[3][3], t[3], hu[4][3], dsum;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float v[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const float4 ub = u[kH8Bin[b]];
            v[b] = i == 0 ? ub.x : (i == 1 ? ub.y : (i == 2 ? ub.z : ub.w));
        }
        wht8(v);
        if (i < 3) {
            U[i][0] = v[1]; U[i][1] = v[2]; U[i][2] = v[4];
            hu[0][i] = v[6]; hu[1][i] = v[5]; hu[2][i] = v[3]; hu[3][i] = v[7];
        } else {
            t[0] = v[1]; t[1] = v[2]; t[2] = v[4];
            dsum = v[0];
        }
    }
    float H[9], gT[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            H[3 * i + j] = 0.125f * (U[i][0] * G[3 * j] + U[i][1] * G[3 * j + 1] + U[i][2] * G[3 * j + 2]);
#pragma unroll
    for (int j = 0; j < 3; ++j) gT[j] = 0.125f * (G[3 * j] * t[0] + G[3 * j + 1] * t[1] + G[3 * j + 2] * t[2]);
    const float dTe = 0.125f * dsum;
    ElemOut eo;
    element_physics<NP, ANISO>(m, H, gT, dTe, a, V0, th, MON, eo, aniso, e);
    // hourglass: q_alpha = sum_a h_alpha,a u_a - H c_alpha ; W = sum_alpha q_alpha c_alpha^T
    float q[4][3], W[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    float ehg = 0.f;
#pragma unroll
    for (int al = 0; al < 4; ++al) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
            q[al][i] = hu[al][i] - (H[3 * i] * c[3 * al] + H[3 * i + 1] * c[3 * al + 1] + H[3 * i + 2] * c[3 * al + 2]);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) W[3 * i + j] += q[al][i] * c[3 * al + j];
        ehg += q[al][0] * q[al][0] + q[al][1] * q[al][1] + q[al][2] * q[al][2];
    }
    // f_a = Q s_a + khg sum_alpha h_alpha,a q_alpha with Q = (PV - khg W) G / 8 ; h_a = s_a . (G^T qV / 8)
    float Q[9], rq[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float acc = 0.f;
#pragma unroll
            for (int j = 0; j < 3; ++j) acc += (eo.PV[3 * i + j] - khg * W[3 * i + j]) * G[3 * j + k];
            Q[3 * i + k] = 0.125f * acc;
        }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        rq[k] = 0.125f * (G[k] * eo.qV[0] + G[3 + k] * eo.qV[1] + G[6 + k] * eo.qV[2]);
    // nodal values from the coefficients of the sign functions (iwht8):
    // f_a = Q s_a + khg sum_alpha h_alpha,a q_alpha, heat s_a . rq
    float fv[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float* v = fv[i];
        if (i < 3) {
            v[0] = 0.f;
            v[1] = Q[3 * i]; v[2] = Q[3 * i + 1]; v[4] = Q[3 * i + 2];
            v[6] = khg * q[0][i]; v[5] = khg * q[1][i]; v[3] = khg * q[2][i]; v[7] = khg * q[3][i];
        } else {
            v[0] = 0.f; v[3] = 0.f; v[5] = 0.f; v[6] = 0.f; v[7] = 0.f;
            v[1] = rq[0]; v[2] = rq[1]; v[4] = rq[2];
        }
        iwht8(v);
    }
    bool nf = false;
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        const int b = kH8Bin[n];
        const float4 f = make_float4(fv[0][b], fv[1][b], fv[2][b], fv[3][b]);
        r.o[n] = f;
        nf |= !finite4(f);
    }
    r.psiV = MON ? eo.psiV + 0.5f * khg * ehg : 0.0f;
    r.inverted = !(eo.Jmin > 0.0f);
    r.nonfinite = nf;
}

// Prony state of element e: the 6 np components in float4 planes (components
// 4k..4k+3 of all elements, element-major), then one float2 plane when 6 np is
// not a multiple of 4 (same layout as theta_index on the host).
__device__ __forceinline__ void load_theta(const float *__restrict__ theta, size_t ne, size_t e, int np, float *th) {
    const int n4 = 6 * np / 4;
    for (int k = 0; k < n4; ++k) {
        const float4 v = reinterpret_cast<const float4 *>(theta)[size_t(k) * ne + e];
        th[4 * k] = v.x; th[4 * k + 1] = v.y; th[4 * k + 2] = v.z; th[4 * k + 3] = v.w;
    }
    if (6 * np % 4) {
        const float2 v = reinterpret_cast<const float2 *>(theta + 4 * size_t(n4) * ne)[e];
        th[4 * n4] = v.x; th[4 * n4 + 1] = v.y;
    }
}
__device__ __forceinline__ void store_theta(float *__restrict__ theta, size_t ne, size_t e, int np, const float *th) {
    const int n4 = 6 * np / 4;
    for (int k = 0; k < n4; ++k)
        reinterpret_cast<float4 *>(theta)[size_t(k) * ne + e] =
            make_float4(th[4 * k], th[4 * k + 1], th[4 * k + 2], th[4 * k + 3]);
    if (6 * np % 4)
        reinterpret_cast<float2 *>(theta + 4 * size_t(n4) * ne)[e] = make_float2(th[4 * n4], th[4 * n4 + 1]);
}

// ---------------------------------------------------------------- node update

struct NodeNew {
    float4 u, v;
    bool nonfinite;
};

// Eq. 20 (temperature, forward Euler; conduction with a minus sign) and the
// velocity form of the central difference of Eq. 27 (R = 0, D = gamma M):
//   v+ = A v- - B f,  A = (1 - gamma dt/2)/(1 + gamma dt/2),  B = dt / (M (1 + gamma dt/2)),
//   u+ = u + dt v+.
__device__ __forceinline__ NodeNew node_advance(const NodeParams &p, float4 u, float4 v, float4 th, unsigned mk,
                                                float4 acc, float src) {
    NodeNew r;
    float dT = u.w;
    if (!(mk & 8u)) {
        float dtC = th.x;
        if (p.ckT_on) {
            float w = clamp01f((dT + p.ck_off) * p.ck_inv);
            dtC = dtC / (p.c_lo + w * (p.c_hi - p.c_lo));
        }
        dT = dT + dtC * (-acc.w - th.y * dT + th.z + src * th.w);
    }
    const float B = v.w;
    float vx = (mk & 1u) ? 0.f : p.A * v.x - B * acc.x;
    float vy = (mk & 2u) ? 0.f : p.A * v.y - B * acc.y;
    float vz = (mk & 4u) ? 0.f : p.A * v.z - B * acc.z;
    r.v = make_float4(vx, vy, vz, B);
    r.u = make_float4((mk & 1u) ? 0.f : u.x + p.dt * vx, (mk & 2u) ? 0.f : u.y + p.dt * vy,
                      (mk & 4u) ? 0.f : u.z + p.dt * vz, dT);
    r.nonfinite = !(finite4(r.u) && isfinite(vx) && isfinite(vy) && isfinite(vz));
    return r;
}

struct NodeMon {
    double ke;
    float tmax, tmin;
    double abl;
};

__device__ __forceinline__ void node_monitor(const NodeParams &p, const NodeNew &r, float Vl, NodeMon &mo) {
    mo.ke += 0.5 * double(p.rho) * double(Vl) * double(r.v.x * r.v.x + r.v.y * r.v.y + r.v.z * r.v.z);
    float T = p.T0 + r.u.w;
    mo.tmax = fmaxf(mo.tmax, T);
    mo.tmin = fminf(mo.tmin, T);
    if (T >= p.abl_T) mo.abl += double(Vl);
}

template <int BS>
__device__ __forceinline__ void write_node_partials(NodeMon mo, double *part, int idx, double *shd, float *shf) {
    double ke = block_sum<BS>(mo.ke, shd);
    double abl = block_sum<BS>(mo.abl, shd);
    float tmax = block_max<BS>(mo.tmax, shf);
    float tmin = -block_max<BS>(-mo.tmin, shf);
    if (threadIdx.x == 0) {
        double *pp = part + 4 * size_t(idx);
        pp[0] = ke; pp[1] = tmax; pp[2] = tmin; pp[3] = abl;
    }
}

__device__ __forceinline__ float source_switch(const NodeParams &p, const long long *step_base, int j) {
    const long long n = *step_base + j;
    return (n >= p.n_on && n < p.n_off) ? 1.0f : 0.0f;
}

// Sum of a shared node's partials [k0, k1) in their stored order (groups of four
// independent loads).  The shared-node kernels and the fused patch kernel both
// use it, so a shared node's update has the same bits wherever it is computed.
__device__ __forceinline__ float4 sum_node_partials(const float4 *partial, int k0, int k1) {
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int k = k0; k < k1; k += 4) {
        float4 o[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) o[q] = (k + q < k1) ? partial[k + q] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc.x += o[q].x; acc.y += o[q].y; acc.z += o[q].z; acc.w += o[q].w;
        }
    }
    return acc;
}

// One step's thermal dose of node a at its end-of-step temperature rise dT,
// in FP64 (CEM43 rates reach 2^(T - 43 C) per minute, far beyond FP32 at
// ablation temperatures, and the sums run over 10^5 steps):
//   CEM43 (Sapareto and Dewey): (dt / 60) R^(43 - T_C), R = 0.5 at T_C >= 43
//   and 0.25 below, i.e. 2^x resp. 2^(2x) with x = T - 316.15 K;
//   Arrhenius (Henriques and Moritz): dt A exp(-Ea / (R_gas T)).
__device__ __forceinline__ void add_thermal_dose(double2 *dose, const DoseParams &q, size_t a, float dT) {
    const double x = double(dT) - q.cem_off;
    double2 d = dose[a];
    d.x += q.dt_min * exp2(x >= 0.0 ? x : 2.0 * x);
    if (q.arrhenius) d.y += q.dt * exp(q.lnA - q.EaR / (q.T0 + double(dT)));
    dose[a] = d;
}

// Runs after a step's node updates (only when the dose is enabled, so the
// solver kernels carry no trace of it).
__global__ __launch_bounds__(kBlock) void dose_kernel(const float4 *__restrict__ nu4, int nn,
                                                      double2 *__restrict__ dose, DoseParams q) {
    const int a = int(blockIdx.x) * kBlock + int(threadIdx.x);
    if (a < nn) add_thermal_dose(dose, q, size_t(a), nu4[a].w);
}

// ---------------------------------------------------------------- two-pass kernels

template <int NP, bool MON, bool ANISO>
__global__ __launch_bounds__(kBlock) void t4_element_kernel(
    const int4 *__restrict__ conn, const float4 *__restrict__ g0, const float4 *__restrict__ g1,
    const float4 *__restrict__ g2, const float4 *__restrict__ nu4, float *__restrict__ theta,
    float4 *__restrict__ out, int ne, KMat m, unsigned *__restrict__ status, double *__restrict__ part,
    const float4 *__restrict__ aniso) {
    __shared__ double shd[kBlock / 64];
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int e = blk * kBlock + threadIdx.x;
    float psi = 0.f;
    bool nf = false, inv = false;
    if (e < ne) {
        const int4 c = conn[e];
        float4 u[4] = {nu4[c.x], nu4[c.y], nu4[c.z], nu4[c.w]};
        float th[6 * NP + 1];
        load_theta(theta, ne, e, NP, th);
        ElemResultT4 r;
        t4_compute<NP, MON, ANISO>(m, u, t4_geo_planes(g0[e], g1[e], g2[e]), th, r, aniso, e);
        store_theta(theta, ne, e, NP, th);
#pragma unroll
        for (int k = 0; k < 4; ++k) out[4 * size_t(e) + k] = r.o[k];
        psi = r.psiV;
        nf = r.nonfinite;
        inv = r.inverted;
    }
    raise_flags(status, nf, inv);
    if (MON) {
        double s = block_sum<kBlock>(double(psi), shd);
        if (threadIdx.x == 0) part[blk] = s;
    }
}

template <int NP, bool MON, bool ANISO>
__global__ __launch_bounds__(kBlock) void h8_element_kernel(
    const int4 *__restrict__ conn0, const int4 *__restrict__ conn1, const float4 *__restrict__ g0,
    const float4 *__restrict__ g1, const float4 *__restrict__ g2, const float4 *__restrict__ hg0,
    const float4 *__restrict__ hg1, const float4 *__restrict__ hg2, const float *__restrict__ khg,
    const float4 *__restrict__ nu4, float *__restrict__ theta, float4 *__restrict__ out, int ne, KMat m,
    unsigned *__restrict__ status, double *__restrict__ part, const float4 *__restrict__ aniso) {
    __shared__ double shd[kBlock / 64];
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int e = blk * kBlock + threadIdx.x;
    float psi = 0.f;
    bool nf = false, inv = false;
    if (e < ne) {
        const int4 ca = conn0[e], cb = conn1[e];
        float4 u[8] = {nu4[ca.x], nu4[ca.y], nu4[ca.z], nu4[ca.w], nu4[cb.x], nu4[cb.y], nu4[cb.z], nu4[cb.w]};
        float th[6 * NP + 1];
        load_theta(theta, ne, e, NP, th);
        ElemResultH8 r;
        h8_compute<NP, MON, ANISO>(m, u, h8_geo_planes(g0[e], g1[e], g2[e], hg0[e], hg1[e], hg2[e], khg[e]), th, r,
                            aniso, e);
        store_theta(theta, ne, e, NP, th);
#pragma unroll
        for (int k = 0; k < 8; ++k) out[8 * size_t(e) + k] = r.o[k];
        psi = r.psiV;
        nf = r.nonfinite;
        inv = r.inverted;
    }
    raise_flags(status, nf, inv);
    if (MON) {
        double s = block_sum<kBlock>(double(psi), shd);
        if (threadIdx.x == 0) part[blk] = s;
    }
}

template <bool MON>
__global__ __launch_bounds__(kBlock) void node_kernel(
    const int *__restrict__ rowptr, const int *__restrict__ inc, const float4 *__restrict__ out,
    float4 *__restrict__ nu4, float4 *__restrict__ nv4, const float4 *__restrict__ nth,
    const uint8_t *__restrict__ mask, const float *__restrict__ Vl, int nn, NodeParams p,
    const long long *__restrict__ step_base, int j, unsigned *__restrict__ status, double *__restrict__ part) {
    __shared__ double shd[kBlock / 64];
    __shared__ float shf[kBlock / 64];
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int a = blk * kBlock + threadIdx.x;
    const float src = source_switch(p, step_base, j);
    NodeMon mo{0.0, -INFINITY, INFINITY, 0.0};
    bool nf = false;
    if (a < nn) {
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        const int k1 = rowptr[a + 1];
        for (int k = rowptr[a]; k < k1; ++k) {
            const float4 o = out[inc[k]];
            acc.x += o.x; acc.y += o.y; acc.z += o.z; acc.w += o.w;
        }
        NodeNew r = node_advance(p, nu4[a], nv4[a], nth[a], mask[a], acc, src);
        nu4[a] = r.u;
        nv4[a] = r.v;
        nf = r.nonfinite;
        if (MON) node_monitor(p, r, Vl[a], mo);
    }
    raise_flags(status, nf, false);
    if (MON) write_node_partials<kBlock>(mo, part, blk, shd, shf);
}

// ---------------------------------------------------------------- fused patch kernels

// One workgroup of BS threads per patch.  LDS: local node state and reference
// coordinates (float4 each per local node) and the element-slot outputs
// (float4 per element slot, grouped by local node: each element writes its
// slots at their precomputed positions, and each node sums its contiguous run).  GEOX: element geometry rebuilt from the staged
// coordinates (else read from the precomputed planes).  ANISO: the orthotropic
// expansion and tensor conduction modes are compiled in.
// A value the whole wavefront shares, read from memory that the kernel also
// writes elsewhere: the compiler cannot prove it unchanged since the kernel
// started, so it would keep it in vector registers (and branch on it per lane);
// readfirstlane puts every word in a scalar register.
template <typename T>
__device__ __forceinline__ T uniform_load(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "word-sized fields");
    int w[sizeof(T) / 4];
    __builtin_memcpy(w, p, sizeof(T));      // the words of the value (memcpy: no type punning)
#pragma unroll
    for (int i = 0; i < int(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    T v;
    __builtin_memcpy(&v, w, sizeof(T));
    return v;
}
__device__ __forceinline__ int uniform_int(const int *p) { return __builtin_amdgcn_readfirstlane(*p); }

// UNI: several patches per workgroup (loads after earlier stores in the same
// kernel), so the per-patch values are read with uniform_load.
// FUSED (single problems): the shared nodes have not yet been advanced by the
// previous step.  Every patch holding one sums its partials of that step and
// advances it while staging (the shared-node kernel's arithmetic, so the same
// bits); the patch that wrote the node's first partial stores the update, into
// the other buffer of the pair the step reads its shared state from.
template <int NPE, int NP, bool MON, int BS, bool GEOX, bool BATCH, bool ANISO, bool UNI = false, bool FUSED = false>
__device__ __forceinline__ void patch_work(const PatchArgs &A, const int pid, const int j, float4 *lds, double *shd,
                                           float *shf) {
    // BATCH: per-scenario constants and end steps; else the single problem's
    // constants at index 0 (no scenario lookups, fewer scalar registers live)
    int sc = 0;
    if (BATCH) {
        sc = UNI ? uniform_int(A.patch_scen + pid) : A.patch_scen[pid];
        const long long end = UNI ? uniform_load(A.scen_end + sc) : A.scen_end[sc];
        if (*A.step_base + j >= end) {   // this scenario has finished: hold it
            if (MON && threadIdx.x == 0) {
                A.part_elem[pid] = 0.0;
                double *pp = A.part_node + 4 * size_t(pid);
                pp[0] = 0.0; pp[1] = -INFINITY; pp[2] = INFINITY; pp[3] = 0.0;
            }
            return;
        }
    }
    const KMat m = UNI ? uniform_load(A.km + sc) : A.km[sc];
    const NodeParams p = UNI ? uniform_load(A.np + sc) : A.np[sc];
    const int e0 = UNI ? uniform_int(A.elem_begin + pid) : A.elem_begin[pid];
    const int e1 = UNI ? uniform_int(A.elem_begin + pid + 1) : A.elem_begin[pid + 1];
    const int ib = UNI ? uniform_int(A.int_begin + pid) : A.int_begin[pid];
    const int ie = UNI ? uniform_int(A.int_begin + pid + 1) : A.int_begin[pid + 1];
    const int sb = UNI ? uniform_int(A.shared_begin + pid) : A.shared_begin[pid];
    const int se = UNI ? uniform_int(A.shared_begin + pid + 1) : A.shared_begin[pid + 1];
    const int nint = ie - ib, nloc = nint + (se - sb);
    float4 *lnode = lds;                                   // nloc: (u, dT)
    float4 *lxyz = lds + A.max_nodes;                      // nloc: reference coordinates (GEOX)
    float4 *lout = lds + (GEOX ? 2 : 1) * A.max_nodes;     // (e1 - e0) * NPE
    const float *gx = GEOX ? A.lX + 3 * size_t(UNI ? uniform_int(A.lx_begin + pid) : A.lx_begin[pid]) : nullptr;
    // Stage the local nodes.  The node ids of a thread's first two local nodes
    // are requested before their data, so the id -> data chain is paid once.
    // GEOX: the fourth float of a shared node's staged coordinate carries the
    // position of its partial (read in the node phase without a global load).
    bool nf_stage = false;
    if (FUSED) {
        const float src_prev = source_switch(p, A.step_base, j - 1);
        for (int l = threadIdx.x; l < nloc; l += BS) {
            if (l < nint) {
                lnode[l] = A.nu4[ib + l];
                if (GEOX) lxyz[l] = make_float4(gx[3 * l], gx[3 * l + 1], gx[3 * l + 2], 0.f);
            } else {
                const int q = sb + l - nint;
                const int id = A.shared_ids[q], pp = A.ppos[q];
                const int2 kr = A.srange[q];                       // independent of the id
                const int sn = id - A.n_interior;
                const float4 u0 = A.su_in[sn], v0 = A.sv_in[sn], th = A.nth[id];
                const unsigned mk = A.mask[id];
                const float4 acc = sum_node_partials(A.partial_prev, kr.x, kr.y);
                const NodeNew r = node_advance(p, u0, v0, th, mk, acc, src_prev);
                lnode[l] = r.u;
                if (GEOX) lxyz[l] = make_float4(gx[3 * l], gx[3 * l + 1], gx[3 * l + 2], __int_as_float(pp));
                if (pp == kr.x) {
                    A.su_out[sn] = r.u;
                    A.sv_out[sn] = r.v;
                    nf_stage |= r.nonfinite;
                }
            }
        }
    } else {
        int nid[2];
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int l = threadIdx.x + it * BS;
            nid[it] = l < nint ? ib + l : (l < nloc ? A.shared_ids[sb + l - nint] : -1);
        }
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int l = threadIdx.x + it * BS;
            if (l < nloc) {
                lnode[l] = A.nu4[nid[it]];
                if (GEOX)
                    lxyz[l] = make_float4(gx[3 * l], gx[3 * l + 1], gx[3 * l + 2],
                                          __int_as_float(l < nint ? 0 : A.ppos[sb + l - nint]));
            }
        }
        for (int l = threadIdx.x + 2 * BS; l < nloc; l += BS) {
            lnode[l] = (l < nint) ? A.nu4[ib + l] : A.nu4[A.shared_ids[sb + l - nint]];
            if (GEOX)
                lxyz[l] = make_float4(gx[3 * l], gx[3 * l + 1], gx[3 * l + 2],
                                      __int_as_float(l < nint ? 0 : A.ppos[sb + l - nint]));
        }
    }
    __syncthreads();
    float psi = 0.f;
    bool nf = nf_stage, inv = false;
    for (int e = e0 + threadIdx.x; e < e1; e += BS) {
        float th[6 * NP + 1];
        load_theta(A.theta, A.ne, e, NP, th);
        if (NPE == 4) {
            const ushort4 c = reinterpret_cast<const ushort4 *>(A.lconn)[e];
            const ushort4 ps = reinterpret_cast<const ushort4 *>(A.lpos)[e];   // independent of c
            float4 u[4] = {lnode[c.x], lnode[c.y], lnode[c.z], lnode[c.w]};
            GeoT4 g;
            if (GEOX) {
                const float4 x[4] = {lxyz[c.x], lxyz[c.y], lxyz[c.z], lxyz[c.w]};
                g = t4_geo_coords(x, A.fib[e]);
            } else {
                g = t4_geo_planes(A.g0[e], A.g1[e], A.g2[e]);
            }
            ElemResultT4 r;
            t4_compute<NP, MON, ANISO>(m, u, g, th, r, A.aniso, e);
            lout[ps.x] = r.o[0];
            lout[ps.y] = r.o[1];
            lout[ps.z] = r.o[2];
            lout[ps.w] = r.o[3];
            psi += r.psiV;
            nf |= r.nonfinite;
            inv |= r.inverted;
        } else {
            const ushort4 ca = reinterpret_cast<const ushort4 *>(A.lconn)[2 * e];
            const ushort4 cb = reinterpret_cast<const ushort4 *>(A.lconn)[2 * e + 1];
            const ushort4 pa = reinterpret_cast<const ushort4 *>(A.lpos)[2 * e];
            const ushort4 pb = reinterpret_cast<const ushort4 *>(A.lpos)[2 * e + 1];
            float4 u[8] = {lnode[ca.x], lnode[ca.y], lnode[ca.z], lnode[ca.w],
                           lnode[cb.x], lnode[cb.y], lnode[cb.z], lnode[cb.w]};
            GeoH8 g;
            if (GEOX) {
                const float4 x[8] = {lxyz[ca.x], lxyz[ca.y], lxyz[ca.z], lxyz[ca.w],
                                     lxyz[cb.x], lxyz[cb.y], lxyz[cb.z], lxyz[cb.w]};
                g = h8_geo_coords(x, A.fib[e], m.hgk);
            } else {
                g = h8_geo_planes(A.g0[e], A.g1[e], A.g2[e], A.hg0[e], A.hg1[e], A.hg2[e], A.khg[e]);
            }
            ElemResultH8 r;
            h8_compute<NP, MON, ANISO>(m, u, g, th, r, A.aniso, e);
            lout[pa.x] = r.o[0];
            lout[pa.y] = r.o[1];
            lout[pa.z] = r.o[2];
            lout[pa.w] = r.o[3];
            lout[pb.x] = r.o[4];
            lout[pb.y] = r.o[5];
            lout[pb.z] = r.o[6];
            lout[pb.w] = r.o[7];
            psi += r.psiV;
            nf |= r.nonfinite;
            inv |= r.inverted;
        }
        store_theta(A.theta, A.ne, e, NP, th);
    }
    __syncthreads();
    // assemble local nodes in a fixed order
    const float src = source_switch(p, A.step_base, j);
    const uint16_t *lrow = A.lrow + (UNI ? uniform_int(A.lrow_begin + pid) : A.lrow_begin[pid]);
    NodeMon mo{0.0, -INFINITY, INFINITY, 0.0};
    for (int l = threadIdx.x; l < nloc; l += BS) {
        const bool interior = l < nint;
        const int a = ib + (interior ? l : 0);
        float4 v0 = make_float4(0.f, 0.f, 0.f, 0.f), th = v0;
        unsigned mk = 0;
        if (interior) {   // node constants first: their latency overlaps the LDS gather
            v0 = A.nv4[a];
            th = A.nth[a];
            mk = A.mask[a];
        }
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        // the node's slots are the contiguous LDS positions k0 .. k1 (element
        // order): summed in that order, with no global index loads
        const int k0 = lrow[l], k1 = lrow[l + 1];
        for (int k = k0; k < k1; ++k) {
            const float4 o = lout[k];
            acc.x += o.x; acc.y += o.y; acc.z += o.z; acc.w += o.w;
        }
        if (interior) {
            NodeNew r = node_advance(p, lnode[l], v0, th, mk, acc, src);
            A.nu4[a] = r.u;
            A.nv4[a] = r.v;
            nf |= r.nonfinite;
            if (MON) node_monitor(p, r, A.Vl[a], mo);
        } else {
            A.partial[GEOX ? __float_as_int(lxyz[l].w) : A.ppos[sb + l - nint]] = acc;
        }
    }
    raise_flags(A.status, nf, inv);
    if (MON) {
        double s = block_sum<BS>(double(psi), shd);
        if (threadIdx.x == 0) A.part_elem[pid] = s;
        write_node_partials<BS>(mo, A.part_node, pid, shd, shf);
    }
}

// One workgroup per patch (a launch covers the first gridDim.x patches).
// H8 with precomputed geometry: compiled for four waves per SIMD (at most 128
// VGPRs, a few values spilled), which its LDS footprint allows; 3 waves per SIMD
// at 144 VGPRs otherwise.  Rebuilding the geometry needs the staged coordinates
// in LDS, which leave room for three workgroups per CU only.
template <int NPE, int NP, bool MON, int BS, bool GEOX, bool BATCH, bool ANISO, bool FUSED = false>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(NPE == 8 && !GEOX ? 4 : 1)))
void patch_kernel(PatchArgs A, int j) {
    extern __shared__ float4 lds[];
    __shared__ double shd[BS / 64];
    __shared__ float shf[BS / 64];
    patch_work<NPE, NP, MON, BS, GEOX, BATCH, ANISO, false, FUSED>(A, xcd_block(blockIdx.x, gridDim.x), j, lds, shd,
                                                                  shf);
}

// Batch scenarios still running at `step`: the union positions run in order of
// descending end step, so they are the first m positions with pos_end > step.
__device__ __forceinline__ int running_positions(const PatchArgs &A, long long step) {
    int lo = 0, hi = A.n_pos;   // first position whose end step is <= step
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (A.pos_end[mid] > step) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Persistent form of the batch patch kernel: launched with the workgroups that
// are resident at once, which walk the step's patches (all patches at a monitor
// step, where finished ones write neutral monitor partials; else only those of
// the scenarios still running: their count for the step was left by the
// previous step's shared-node kernel in the slot of the step's parity, so one
// captured graph serves every step).  The workgroups of XCD x (dispatch is
// round-robin over the XCDs) take the x-th eighth of the patches in a strided
// walk, so that neighbouring patches, which share nodes, stay in one L2.  The
// assignment is static: pulling patches one by one from device-wide counters
// measured 3.8 times slower (every pull is an atomic on one of a few
// addresses, served in order at the coherence point of the XCDs).  No
// workgroup waits for another.
template <int NPE, int NP, bool MON, bool GEOX>
__global__ __launch_bounds__(kBlock) void patch_queue_kernel(PatchArgs A, int j) {
    extern __shared__ float4 lds[];
    __shared__ double shd[kBlock / 64];
    __shared__ float shf[kBlock / 64];
    const long long step = *A.step_base + j;
    const int n = MON ? A.n_patches : int(A.qcount[2 * (step & 1)]);
    const int G = int(gridDim.x), x = int(blockIdx.x) % kNumXcd, i = int(blockIdx.x) / kNumXcd;
    const int gx = G / kNumXcd + (x < G % kNumXcd ? 1 : 0);          // workgroups on XCD x
    const int lo = int((long long)n * x / kNumXcd), hi = int((long long)n * (x + 1) / kNumXcd);
    for (int pid = lo + i; pid < hi; pid += gx)
        patch_work<NPE, NP, MON, kBlock, GEOX, true, false, true>(A, pid, j, lds, shd, shf);
}

template <bool MON, bool BATCH>
__global__ __launch_bounds__(kBlock) void shared_node_kernel(PatchArgs A, int j) {
    __shared__ double shd[kBlock / 64];
    __shared__ float shf[kBlock / 64];
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int s = blk * kBlock + threadIdx.x;
    NodeMon mo{0.0, -INFINITY, INFINITY, 0.0};
    bool nf = false;
    const int sc = (BATCH && s < A.n_shared) ? A.shared_scen[s] : 0;
    const long long step = *A.step_base + j;
    if (s < A.n_shared && (!BATCH || step < A.scen_end[sc])) {
        const NodeParams p = A.np[sc];
        const float src = (step >= p.n_on && step < p.n_off) ? 1.0f : 0.0f;
        const int a = A.n_interior + s;
        const float4 u0 = A.su_in[s], v0 = A.sv_in[s], th = A.nth[a];   // independent of the partials
        const unsigned mk = A.mask[a];
        const float4 acc = sum_node_partials(A.partial, A.srow[s], A.srow[s + 1]);
        NodeNew r = node_advance(p, u0, v0, th, mk, acc, src);
        A.nu4[a] = r.u;
        A.nv4[a] = r.v;
        nf = r.nonfinite;
        if (MON) node_monitor(p, r, A.Vl[a], mo);
    }
    raise_flags(A.status, nf, false);
    if (MON) write_node_partials<kBlock>(mo, A.part_node + 4 * size_t(A.n_patches), blk, shd, shf);
}

// Shared-node kernel of the persistent schedule: a fixed grid strides over the
// shared nodes of the scenarios still running (all of them at a monitor step),
// counted on the device; block 0 also counts the next step's running patches
// and shared nodes.
template <bool MON>
__global__ __launch_bounds__(kBlock) void shared_node_queue_kernel(PatchArgs A, int j) {
    __shared__ double shd[kBlock / 64];
    __shared__ float shf[kBlock / 64];
    const long long step = *A.step_base + j;
    const int64_t n = MON ? int64_t(A.n_shared) : int64_t(A.qcount[2 * (step & 1) + 1]);
    // the running scenarios' patch and shared-node counts of the next step, into
    // the other parity's slots (read by the next step's kernels only)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int m = running_positions(A, step + 1);
        long long *nx = A.qcount + 2 * ((step + 1) & 1);
        nx[0] = m ? A.pos_patch_hi[m - 1] : 0;
        nx[1] = m ? A.pos_shared_hi[m - 1] : 0;
    }
    NodeMon mo{0.0, -INFINITY, INFINITY, 0.0};
    bool nf = false;
    for (int64_t s = int64_t(blockIdx.x) * kBlock + threadIdx.x; s < n; s += int64_t(gridDim.x) * kBlock) {
        const int sc = A.shared_scen[s];
        if (step >= A.scen_end[sc]) continue;
        const NodeParams p = A.np[sc];
        const float src = (step >= p.n_on && step < p.n_off) ? 1.0f : 0.0f;
        const int64_t a = A.n_interior + s;
        const float4 u0 = A.nu4[a], v0 = A.nv4[a], th = A.nth[a];
        const unsigned mk = A.mask[a];
        const float4 acc = sum_node_partials(A.partial, A.srow[s], A.srow[s + 1]);
        NodeNew r = node_advance(p, u0, v0, th, mk, acc, src);
        A.nu4[a] = r.u;
        A.nv4[a] = r.v;
        nf |= r.nonfinite;
        if (MON) node_monitor(p, r, A.Vl[a], mo);
    }
    raise_flags(A.status, nf, false);
    if (MON) write_node_partials<kBlock>(mo, A.part_node + 4 * size_t(A.n_patches), int(blockIdx.x), shd, shf);
}

// ---------------------------------------------------------------- monitors

// One block: sums the per-block partials in a fixed order, writes the monitor
// record and advances the device step counter by the chunk length.
__global__ __launch_bounds__(kBlock) void finish_kernel(const double *__restrict__ part_elem, int n_elem_parts,
                                                        const double *__restrict__ part_node, int n_node_parts,
                                                        long long *step_base, int k, const unsigned *status,
                                                        DevMonitors *mon) {
    __shared__ double shd[kBlock / 64];
    __shared__ float shf[kBlock / 64];
    double se = 0.0, ke = 0.0, abl = 0.0;
    float tmax = -INFINITY, tmin = INFINITY;
    // unrolled so that several loads are in flight; the additions keep their order
#pragma unroll 4
    for (int i = threadIdx.x; i < n_elem_parts; i += kBlock) se += part_elem[i];
#pragma unroll 4
    for (int i = threadIdx.x; i < n_node_parts; i += kBlock) {
        ke += part_node[4 * i];
        tmax = fmaxf(tmax, float(part_node[4 * i + 1]));
        tmin = fminf(tmin, float(part_node[4 * i + 2]));
        abl += part_node[4 * i + 3];
    }
    se = block_sum<kBlock>(se, shd);
    ke = block_sum<kBlock>(ke, shd);
    abl = block_sum<kBlock>(abl, shd);
    tmax = block_max<kBlock>(tmax, shf);
    tmin = -block_max<kBlock>(-tmin, shf);
    if (threadIdx.x == 0) {
        const long long n = *step_base + k;
        *step_base = n;
        mon->step = n;
        mon->strain = se;
        mon->kinetic = ke;
        mon->T_max = tmax;
        mon->T_min = tmin;
        mon->ablated = abl;
        mon->flags = *status;
    }
}

// ---------------------------------------------------------------- launchers

namespace {
template <int NP, bool ANISO>
void launch_t4_element_a(bool mon, const TwoPassArgs &a, const KMat &m, hipStream_t s, const LaunchTiming *ev) {
    dim3 grid((a.ne + kBlock - 1) / kBlock);
    if (mon)
        TLED_LAUNCH(ev, (t4_element_kernel<NP, true, ANISO>), grid, dim3(kBlock), 0, s, a.conn4, a.g0, a.g1, a.g2,
                    a.nu4, a.theta, a.out, a.ne, m, a.status, a.part_elem, a.aniso);
    else
        TLED_LAUNCH(ev, (t4_element_kernel<NP, false, ANISO>), grid, dim3(kBlock), 0, s, a.conn4, a.g0, a.g1, a.g2,
                    a.nu4, a.theta, a.out, a.ne, m, a.status, a.part_elem, a.aniso);
}
template <int NP, bool ANISO>
void launch_h8_element_a(bool mon, const TwoPassArgs &a, const KMat &m, hipStream_t s, const LaunchTiming *ev) {
    dim3 grid((a.ne + kBlock - 1) / kBlock);
    if (mon)
        TLED_LAUNCH(ev, (h8_element_kernel<NP, true, ANISO>), grid, dim3(kBlock), 0, s, a.conn4, a.conn4b, a.g0, a.g1,
                    a.g2, a.hg0, a.hg1, a.hg2, a.khg, a.nu4, a.theta, a.out, a.ne, m, a.status, a.part_elem, a.aniso);
    else
        TLED_LAUNCH(ev, (h8_element_kernel<NP, false, ANISO>), grid, dim3(kBlock), 0, s, a.conn4, a.conn4b, a.g0,
                    a.g1, a.g2, a.hg0, a.hg1, a.hg2, a.khg, a.nu4, a.theta, a.out, a.ne, m, a.status, a.part_elem,
                    a.aniso);
}
// The anisotropy plane is present exactly when the orthotropic expansion or the tensor conduction is on.
template <int NP>
void launch_t4_element(bool mon, const TwoPassArgs &a, const KMat &m, hipStream_t s, const LaunchTiming *ev) {
    if (a.aniso) launch_t4_element_a<NP, true>(mon, a, m, s, ev);
    else launch_t4_element_a<NP, false>(mon, a, m, s, ev);
}
template <int NP>
void launch_h8_element(bool mon, const TwoPassArgs &a, const KMat &m, hipStream_t s, const LaunchTiming *ev) {
    if (a.aniso) launch_h8_element_a<NP, true>(mon, a, m, s, ev);
    else launch_h8_element_a<NP, false>(mon, a, m, s, ev);
}

// occ != nullptr: report the resident workgroups per CU of the instantiation
// instead of launching it.
template <int NPE, int NP, int BS, bool GEOX, bool BATCH, bool ANISO = false, bool FUSED = false>
void launch_patch_g(bool mon, const PatchArgs &a, int j, size_t lds, hipStream_t s, int *occ,
                    const LaunchTiming *ev) {
    if (occ) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                occ, reinterpret_cast<const void *>(&patch_kernel<NPE, NP, false, BS, GEOX, BATCH, ANISO, FUSED>),
                BS, lds) != hipSuccess)
            *occ = -1;
        return;
    }
    dim3 grid(a.n_patches);
    if (mon)
        TLED_LAUNCH(ev, (patch_kernel<NPE, NP, true, BS, GEOX, BATCH, ANISO, FUSED>), grid, dim3(BS), lds, s, a, j);
    else
        TLED_LAUNCH(ev, (patch_kernel<NPE, NP, false, BS, GEOX, BATCH, ANISO, FUSED>), grid, dim3(BS), lds, s, a, j);
}

// Batches run with 256-thread workgroups only; so do single problems with the
// orthotropic expansion or the tensor conduction (the anisotropy plane is
// present exactly then).  The fused form exists for single problems with the
// geometry rebuilt from coordinates, 256 threads and no anisotropy plane (the
// library enables it only then).
template <int NPE, int NP>
void launch_patch_np(bool mon, bool geox, int bs, bool batch, const PatchArgs &a, int j, size_t lds,
                     hipStream_t s, int *occ, const LaunchTiming *ev, bool fused) {
    if (fused) {
        launch_patch_g<NPE, NP, 256, true, false, false, true>(mon, a, j, lds, s, occ, ev);
    } else if (a.aniso && !batch) {
        if (geox) launch_patch_g<NPE, NP, 256, true, false, true>(mon, a, j, lds, s, occ, ev);
        else launch_patch_g<NPE, NP, 256, false, false, true>(mon, a, j, lds, s, occ, ev);
    } else if (batch) {
        if (geox) launch_patch_g<NPE, NP, 256, true, true>(mon, a, j, lds, s, occ, ev);
        else launch_patch_g<NPE, NP, 256, false, true>(mon, a, j, lds, s, occ, ev);
    } else if (NPE == 4 && bs == 512) {
        if constexpr (NPE == 4) {   // 512-thread workgroups exist for T4 only
            if (geox) launch_patch_g<NPE, NP, 512, true, false>(mon, a, j, lds, s, occ, ev);
            else launch_patch_g<NPE, NP, 512, false, false>(mon, a, j, lds, s, occ, ev);
        }
    } else {
        if (geox) launch_patch_g<NPE, NP, 256, true, false>(mon, a, j, lds, s, occ, ev);
        else launch_patch_g<NPE, NP, 256, false, false>(mon, a, j, lds, s, occ, ev);
    }
}
}  // namespace

void launch_element(int npe, int np, bool mon, const TwoPassArgs &a, const KMat &m, hipStream_t s,
                    const LaunchTiming *ev) {
    if (a.ne == 0) return;
    if (npe == 4) {
        switch (np) {
            case 0: launch_t4_element<0>(mon, a, m, s, ev); break;
            case 1: launch_t4_element<1>(mon, a, m, s, ev); break;
            case 2: launch_t4_element<2>(mon, a, m, s, ev); break;
            case 3: launch_t4_element<3>(mon, a, m, s, ev); break;
            default: launch_t4_element<4>(mon, a, m, s, ev); break;
        }
    } else {
        switch (np) {
            case 0: launch_h8_element<0>(mon, a, m, s, ev); break;
            case 1: launch_h8_element<1>(mon, a, m, s, ev); break;
            case 2: launch_h8_element<2>(mon, a, m, s, ev); break;
            case 3: launch_h8_element<3>(mon, a, m, s, ev); break;
            default: launch_h8_element<4>(mon, a, m, s, ev); break;
        }
    }
}

void launch_dose(const float4 *nu4, int nn, double2 *dose, const DoseParams &q, hipStream_t s) {
    if (nn > 0) hipLaunchKernelGGL(dose_kernel, dim3((nn + kBlock - 1) / kBlock), dim3(kBlock), 0, s, nu4, nn, dose, q);
}

void launch_node(bool mon, const TwoPassArgs &a, const NodeParams &p, int j, hipStream_t s, const LaunchTiming *ev) {
    dim3 grid((a.nn + kBlock - 1) / kBlock);
    if (mon)
        TLED_LAUNCH(ev, (node_kernel<true>), grid, dim3(kBlock), 0, s, a.rowptr, a.inc, a.out, a.nu4, a.nv4, a.nth,
                    a.mask, a.Vl, a.nn, p, a.step_base, j, a.status, a.part_node);
    else
        TLED_LAUNCH(ev, (node_kernel<false>), grid, dim3(kBlock), 0, s, a.rowptr, a.inc, a.out, a.nu4, a.nv4, a.nth,
                    a.mask, a.Vl, a.nn, p, a.step_base, j, a.status, a.part_node);
}

namespace {
void patch_dispatch(int npe, int np, bool mon, bool geox, int bs, bool batch, const PatchArgs &a, int j,
                    hipStream_t s, int *occ, const LaunchTiming *ev, bool fused) {
    const size_t lds = patch_lds_bytes(npe, geox, a);
    if (npe == 4) {
        switch (np) {
            case 0: launch_patch_np<4, 0>(mon, geox, bs, batch, a, j, lds, s, occ, ev, fused); break;
            case 1: launch_patch_np<4, 1>(mon, geox, bs, batch, a, j, lds, s, occ, ev, fused); break;
            case 2: launch_patch_np<4, 2>(mon, geox, bs, batch, a, j, lds, s, occ, ev, fused); break;
            case 3: launch_patch_np<4, 3>(mon, geox, bs, batch, a, j, lds, s, occ, ev, fused); break;
            default: launch_patch_np<4, 4>(mon, geox, bs, batch, a, j, lds, s, occ, ev, fused); break;
        }
    } else {
        switch (np) {
            case 0: launch_patch_np<8, 0>(mon, geox, bs, batch, a, j, lds, s, occ, ev, fused); break;
            case 1: launch_patch_np<8, 1>(mon, geox, bs, batch, a, j, lds, s, occ, ev, fused); break;
            case 2: launch_patch_np<8, 2>(mon, geox, bs, batch, a, j, lds, s, occ, ev, fused); break;
            case 3: launch_patch_np<8, 3>(mon, geox, bs, batch, a, j, lds, s, occ, ev, fused); break;
            default: launch_patch_np<8, 4>(mon, geox, bs, batch, a, j, lds, s, occ, ev, fused); break;
        }
    }
}
}  // namespace

void launch_patch(int npe, int np, bool mon, bool geox, int bs, bool batch, const PatchArgs &a, int j,
                  hipStream_t s, const LaunchTiming *ev, bool fused) {
    patch_dispatch(npe, np, mon, geox, bs, batch, a, j, s, nullptr, ev, fused);
}

namespace {
// occ != nullptr: report resident workgroups per CU instead of launching.
template <int NPE, int NP, bool GEOX>
void launch_queue_g(bool mon, const PatchArgs &a, int j, int grid, size_t lds, hipStream_t s, int *occ,
                    const LaunchTiming *ev) {
    if (occ) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                occ, reinterpret_cast<const void *>(&patch_queue_kernel<NPE, NP, false, GEOX>), kBlock, lds) !=
            hipSuccess)
            *occ = -1;
        return;
    }
    if (mon) TLED_LAUNCH(ev, (patch_queue_kernel<NPE, NP, true, GEOX>), dim3(grid), dim3(kBlock), lds, s, a, j);
    else TLED_LAUNCH(ev, (patch_queue_kernel<NPE, NP, false, GEOX>), dim3(grid), dim3(kBlock), lds, s, a, j);
}
template <int NPE>
void queue_np(int np, bool mon, bool geox, const PatchArgs &a, int j, int grid, size_t lds, hipStream_t s, int *occ,
              const LaunchTiming *ev) {
#define TLED_QNP(NPV)                                                            \
    if (geox) launch_queue_g<NPE, NPV, true>(mon, a, j, grid, lds, s, occ, ev);  \
    else launch_queue_g<NPE, NPV, false>(mon, a, j, grid, lds, s, occ, ev);
    switch (np) {
        case 0: TLED_QNP(0) break;
        case 1: TLED_QNP(1) break;
        case 2: TLED_QNP(2) break;
        case 3: TLED_QNP(3) break;
        default: TLED_QNP(4) break;
    }
#undef TLED_QNP
}
}  // namespace

void launch_patch_queue(int npe, int np, bool mon, bool geox, const PatchArgs &a, int j, int grid, hipStream_t s,
                        const LaunchTiming *ev) {
    const size_t lds = patch_lds_bytes(npe, geox, a);
    if (npe == 4) queue_np<4>(np, mon, geox, a, j, grid, lds, s, nullptr, ev);
    else queue_np<8>(np, mon, geox, a, j, grid, lds, s, nullptr, ev);
}

int patch_queue_occupancy(int npe, int np, bool geox, const PatchArgs &a) {
    int occ = 0;
    const size_t lds = patch_lds_bytes(npe, geox, a);
    if (npe == 4) queue_np<4>(np, false, geox, a, 0, 1, lds, nullptr, &occ, nullptr);
    else queue_np<8>(np, false, geox, a, 0, 1, lds, nullptr, &occ, nullptr);
    return occ;
}

void launch_shared_nodes_queue(bool mon, const PatchArgs &a, int j, int grid, hipStream_t s, const LaunchTiming *ev) {
    if (mon) TLED_LAUNCH(ev, (shared_node_queue_kernel<true>), dim3(grid), dim3(kBlock), 0, s, a, j);
    else TLED_LAUNCH(ev, (shared_node_queue_kernel<false>), dim3(grid), dim3(kBlock), 0, s, a, j);
}

int patch_occupancy(int npe, int np, bool geox, int bs, bool batch, const PatchArgs &a, bool fused) {
    int occ = 0;
    patch_dispatch(npe, np, false, geox, bs, batch, a, 0, nullptr, &occ, nullptr, fused);
    return occ;
}

void launch_shared_nodes(bool mon, bool batch, const PatchArgs &a, int j, hipStream_t s, const LaunchTiming *ev) {
    const int nb = int((a.n_shared + kBlock - 1) / kBlock);
    if (nb == 0) return;
    dim3 grid(nb);
    if (batch) {
        if (mon) TLED_LAUNCH(ev, (shared_node_kernel<true, true>), grid, dim3(kBlock), 0, s, a, j);
        else TLED_LAUNCH(ev, (shared_node_kernel<false, true>), grid, dim3(kBlock), 0, s, a, j);
    } else {
        if (mon) TLED_LAUNCH(ev, (shared_node_kernel<true, false>), grid, dim3(kBlock), 0, s, a, j);
        else TLED_LAUNCH(ev, (shared_node_kernel<false, false>), grid, dim3(kBlock), 0, s, a, j);
    }
}

// One block per scenario: max T and the lumped volume at or above T_abl (fixed-order reduction).
__global__ __launch_bounds__(kBlock) void scenario_monitor_kernel(const float4 *__restrict__ nu4,
                                                                  const float *__restrict__ Vl,
                                                                  const long long *__restrict__ ranges,
                                                                  const NodeParams *__restrict__ np, float T_abl,
                                                                  double *__restrict__ out) {
    __shared__ double shd[kBlock / 64];
    __shared__ float shf[kBlock / 64];
    const int sc = blockIdx.x;
    const float T0 = np[sc].T0;
    float tmax = -INFINITY;
    double vol = 0.0;
    for (int r = 0; r < 2; ++r) {
        const long long lo = ranges[4 * sc + 2 * r], hi = ranges[4 * sc + 2 * r + 1];
        for (long long a = lo + threadIdx.x; a < hi; a += kBlock) {
            const float T = T0 + nu4[a].w;
            tmax = fmaxf(tmax, T);
            if (T >= T_abl) vol += double(Vl[a]);
        }
    }
    vol = block_sum<kBlock>(vol, shd);
    tmax = block_max<kBlock>(tmax, shf);
    if (threadIdx.x == 0) {
        out[2 * sc] = tmax;
        out[2 * sc + 1] = vol;
    }
}

void launch_scenario_monitors(const float4 *nu4, const float *Vl, const long long *ranges, const NodeParams *np,
                              int n_scen, float T_abl, double *out, hipStream_t s) {
    if (n_scen <= 0) return;
    hipLaunchKernelGGL(scenario_monitor_kernel, dim3(n_scen), dim3(kBlock), 0, s, nu4, Vl, ranges, np, T_abl, out);
}

void launch_finish(const double *part_elem, int n_elem_parts, const double *part_node, int n_node_parts,
                   long long *step_base, int k, const unsigned *status, DevMonitors *mon, hipStream_t s) {
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(kBlock), 0, s, part_elem, n_elem_parts, part_node, n_node_parts,
                       step_base, k, status, mon);
}

size_t patch_lds_bytes(int npe, bool geox, const PatchArgs &a) {
    return sizeof(float4) * ((geox ? 2 : 1) * size_t(a.max_nodes) + size_t(a.max_elems) * npe);
}

}  // namespace tled

// ---------------------------------------------------------------- field export

namespace tled {

__global__ __launch_bounds__(kBlock) void export_fields_kernel(const float4 *__restrict__ nu4,
                                                               const int *__restrict__ new2old, int nn, float T0,
                                                               float *__restrict__ u_dst, float *__restrict__ T_dst) {
    const int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= nn) return;
    const float4 u = nu4[a];
    const int o = new2old[a];
    if (u_dst) {
        u_dst[3 * size_t(o)] = u.x;
        u_dst[3 * size_t(o) + 1] = u.y;
        u_dst[3 * size_t(o) + 2] = u.z;
    }
    if (T_dst) T_dst[o] = T0 + u.w;
}

void launch_export_fields(const float4 *nu4, const int *new2old, int nn, float T0, float *u_dst, float *T_dst,
                          hipStream_t s) {
    if (nn == 0) return;
    hipLaunchKernelGGL(export_fields_kernel, dim3((nn + kBlock - 1) / kBlock), dim3(kBlock), 0, s, nu4, new2old, nn,
                       T0, u_dst, T_dst);
}

}  // namespace tled
