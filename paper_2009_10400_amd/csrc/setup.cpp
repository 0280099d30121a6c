// Host-side set-up of the TLED solver, in double precision: validation,
// orientation repair, element geometry, lumped matrices, critical time step,
// locality reordering and the assembly lists of both kernel variants.
//
// The geometry is the total-Lagrangian precompute of Section 5 (spatial
// derivatives, initial volumes, initial Jacobian, mass): it is done once,
// here, and rounded to single precision once when uploaded.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <numeric>
#include <system_error>
#include <thread>

#include "tled_internal.h"

namespace tled {
namespace {

// H8 natural-coordinate signs of the local nodes (---),(+--),(++-),(-+-),(--+),(+-+),(+++),(-++).
const int kHexSign[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                            {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

// Hourglass base vectors eta*zeta, zeta*xi, xi*eta, xi*eta*zeta at the nodes.
inline int hourglass_base(int alpha, int a) {
    const int *s = kHexSign[a];
    switch (alpha) {
        case 0: return s[1] * s[2];
        case 1: return s[2] * s[0];
        case 2: return s[0] * s[1];
        default: return s[0] * s[1] * s[2];
    }
}

inline double det3(const double m[9]) {
    return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
           m[2] * (m[3] * m[7] - m[4] * m[6]);
}

// Inverse through the cofactor matrix; returns the determinant.
inline double invert3(const double m[9], double r[9]) {
    double c[9] = {m[4] * m[8] - m[5] * m[7], m[5] * m[6] - m[3] * m[8], m[3] * m[7] - m[4] * m[6],
                   m[2] * m[7] - m[1] * m[8], m[0] * m[8] - m[2] * m[6], m[1] * m[6] - m[0] * m[7],
                   m[1] * m[5] - m[2] * m[4], m[2] * m[3] - m[0] * m[5], m[0] * m[4] - m[1] * m[3]};
    double d = m[0] * c[0] + m[1] * c[1] + m[2] * c[2];
    // r = adj(m) / d, adj = cofactor^T
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r[3 * i + j] = c[3 * j + i] / d;
    return d;
}

inline double norm_cross(const double *u, const double *v) {
    double w0 = u[1] * v[2] - u[2] * v[1], w1 = u[2] * v[0] - u[0] * v[2], w2 = u[0] * v[1] - u[1] * v[0];
    return std::sqrt(w0 * w0 + w1 * w1 + w2 * w2);
}

struct ElemGeo {
    double geo[9];   // T4: rows dh/dX of local nodes 1..3 ; H8: G = J0^-T
    double V0;
    double hgc[12];  // H8 only
    double sum_dh2;  // sum_a |dh_a/dX|^2
    double L;        // characteristic length
};

// T4 geometry from the edge matrix D (columns X_k - X_0, k = 1..3):
// dh_k/dX = row k-1 of D^-1, V0 = det D / 6.
double tet_geometry(const double *Xe, ElemGeo *g) {
    double D[9];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) D[3 * i + k] = Xe[3 * (k + 1) + i] - Xe[i];
    double d = det3(D);
    if (!(d > 0.0)) return d;
    double Di[9];
    invert3(D, Di);
    std::memcpy(g->geo, Di, sizeof(Di));
    g->V0 = d / 6.0;
    double s = 0.0, r0[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j) {
            s += Di[3 * k + j] * Di[3 * k + j];
            r0[j] -= Di[3 * k + j];
        }
    g->sum_dh2 = s + r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2];
    // length = 3 V0 / largest face area
    static const int face[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    double amax = 0.0;
    for (auto &f : face) {
        const double *p = Xe + 3 * f[0], *q = Xe + 3 * f[1], *r = Xe + 3 * f[2];
        double u[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
        double v[3] = {r[0] - p[0], r[1] - p[1], r[2] - p[2]};
        amax = std::max(amax, 0.5 * norm_cross(u, v));
    }
    g->L = 3.0 * g->V0 / amax;
    return d;
}

// H8 one-point geometry: J0 = sum_a X_a (x) s_a / 8 (derivatives of the
// trilinear shape functions at the centre), G = J0^-T so dh_a/dX = G s_a / 8,
// V0 = 8 det J0; hourglass c_alpha = sum_a X_a h_alpha,a.
double hex_geometry(const double *Xe, ElemGeo *g) {
    double J0[9] = {0};
    double Xr[24];
    for (int a = 0; a < 8; ++a)
        for (int i = 0; i < 3; ++i) Xr[3 * a + i] = Xe[3 * a + i] - Xe[i];  // translation-free
    for (int a = 0; a < 8; ++a)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) J0[3 * i + j] += Xr[3 * a + i] * kHexSign[a][j] / 8.0;
    double d = det3(J0);
    if (!(d > 0.0)) return d;
    double Ji[9];
    invert3(J0, Ji);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) g->geo[3 * i + j] = Ji[3 * j + i];  // G = J0^-T
    g->V0 = 8.0 * d;
    double s = 0.0;
    for (int a = 0; a < 8; ++a)
        for (int j = 0; j < 3; ++j) {
            double dh = (g->geo[3 * j] * kHexSign[a][0] + g->geo[3 * j + 1] * kHexSign[a][1] +
                         g->geo[3 * j + 2] * kHexSign[a][2]) / 8.0;
            s += dh * dh;
        }
    g->sum_dh2 = s;
    for (int al = 0; al < 4; ++al)
        for (int i = 0; i < 3; ++i) {
            double c = 0.0;
            for (int a = 0; a < 8; ++a) c += Xr[3 * a + i] * hourglass_base(al, a);
            g->hgc[3 * al + i] = c;
        }
    static const int face[6][4] = {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 3, 7, 4},
                                   {1, 2, 6, 5}, {0, 1, 5, 4}, {3, 2, 6, 7}};
    double amax = 0.0;
    for (auto &f : face) {
        const double *p0 = Xe + 3 * f[0], *p1 = Xe + 3 * f[1], *p2 = Xe + 3 * f[2], *p3 = Xe + 3 * f[3];
        double d1[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
        double d2[3] = {p3[0] - p1[0], p3[1] - p1[1], p3[2] - p1[2]};
        amax = std::max(amax, 0.5 * norm_cross(d1, d2));
    }
    g->L = g->V0 / amax;
    return d;
}

double wave_speed(const tled_material &m) {
    return std::sqrt((m.kappa + 4.0 * m.mu / 3.0 + 4.0 * m.eta) / m.rho);
}

tled_status check_inputs(const HostProblem &p, std::string *err) {
    if (!p.have_mesh) { *err = "mesh not set"; return TLED_E_STATE; }
    if (!p.have_mat) { *err = "material not set"; return TLED_E_STATE; }
    const tled_material &m = p.mat;
    if (!(m.rho > 0) || !(m.mu > 0) || !(m.kappa > 0) || m.eta < 0 || !(m.c > 0) || m.k < 0 ||
        m.wbcb < 0 || m.n_prony < 0 || m.n_prony > 4) {
        *err = "material out of range (rho, mu, kappa, c > 0; eta, k, wbcb >= 0; 0 <= n_prony <= 4)";
        return TLED_E_ARG;
    }
    double gs = 0.0;
    for (int i = 0; i < m.n_prony; ++i) {
        if (!(m.tau[i] > 0) || m.g[i] < 0) { *err = "Prony terms need tau > 0, g >= 0"; return TLED_E_ARG; }
        gs += m.g[i];
    }
    if (gs >= 1.0) { *err = "Prony moduli must sum below 1"; return TLED_E_ARG; }
    if (m.muT_on && !(m.muT_hi > m.muT_lo)) { *err = "muT_hi must exceed muT_lo"; return TLED_E_ARG; }
    if (m.shrink_on && !(m.shrink_width > 0)) { *err = "shrink_width must be > 0"; return TLED_E_ARG; }
    if (m.ckT_on && !(m.ckT_hi > m.ckT_lo)) { *err = "ckT_hi must exceed ckT_lo"; return TLED_E_ARG; }
    if (m.ckT_on && (!(m.c_hi > 0) || m.k_hi < 0)) { *err = "c_hi > 0 and k_hi >= 0 required"; return TLED_E_ARG; }
    if (m.expan_mode < 0 || m.expan_mode > 2 || m.cond_mode < 0 || m.cond_mode > 2) {
        *err = "expan_mode and cond_mode must be 0, 1 or 2"; return TLED_E_ARG;
    }
    if (m.expan_mode == 2 && int64_t(p.n0.size()) != 3 * p.ne) {
        *err = "expan_mode 2 needs the second expansion axes (tled_set_expansion_axes)"; return TLED_E_ARG;
    }
    if (m.cond_mode == 2 && int64_t(p.Dc.size()) != 6 * p.ne) {
        *err = "cond_mode 2 needs the element conductivity tensors (tled_set_conductivity)"; return TLED_E_ARG;
    }
    if (m.cond_mode == 2) {
        // each tensor symmetric positive semi-definite: all principal minors >= 0 (to rounding)
        for (int64_t e = 0; e < p.ne; ++e) {
            const double *d = &p.Dc[6 * e];
            const double xx = d[0], yy = d[1], zz = d[2], xy = d[3], yz = d[4], xz = d[5];
            bool finite = true;
            for (int i = 0; i < 6; ++i) finite = finite && std::isfinite(d[i]);
            const double sc = std::max({std::fabs(xx), std::fabs(yy), std::fabs(zz), std::fabs(xy), std::fabs(yz),
                                        std::fabs(xz)});
            const double tol = 1e-12 * sc * sc, tol3 = 1e-12 * sc * sc * sc;
            const double det3 = xx * (yy * zz - yz * yz) - xy * (xy * zz - yz * xz) + xz * (xy * yz - yy * xz);
            if (!finite || xx < 0 || yy < 0 || zz < 0 || xx * yy - xy * xy < -tol || yy * zz - yz * yz < -tol ||
                xx * zz - xz * xz < -tol || det3 < -tol3) {
                *err = "conductivity tensor of element " + std::to_string(e) + " is not symmetric positive semi-definite";
                return TLED_E_ARG;
            }
        }
    }
    return TLED_OK;
}

// Elements in caller order with repaired orientation; geometry per element.
// f(lo, hi) over [0, n) cut into `threads` contiguous ranges, one host thread
// each (the calling thread takes the first, and any range whose thread could
// not be started).  Callers only write disjoint ranges, so the result does not
// depend on the thread count.
template <class F>
void parallel_ranges(int64_t n, int threads, F f) {
    const int t = int(std::max<int64_t>(1, std::min<int64_t>(threads, n / 4096)));
    if (t <= 1) { f(int64_t(0), n); return; }
    std::vector<std::thread> pool;
    int started = 1;
    for (; started < t; ++started) {
        try {
            const int i = started;
            pool.emplace_back([&, i] { f(n * i / t, n * (i + 1) / t); });
        } catch (const std::system_error &) {
            break;
        }
    }
    for (int i = started; i < t; ++i) f(n * i / t, n * (i + 1) / t);
    f(int64_t(0), n / t);
    for (auto &th : pool) th.join();
}

// Starts up to `extra` host threads running `work` (which takes its items from
// a shared counter, so the calling thread finishes whatever they do not);
// stops at the first thread that cannot be started.
template <class F>
std::vector<std::thread> start_workers(int extra, F &work) {
    std::vector<std::thread> pool;
    for (int t = 0; t < extra; ++t) {
        try {
            pool.emplace_back(work);
        } catch (const std::system_error &) {
            break;
        }
    }
    return pool;
}

tled_status element_pass(const HostProblem &p, std::vector<int32_t> *conn, std::vector<ElemGeo> *geo,
                         int64_t *n_swapped, std::string *err, int threads = 1) {
    const int npe = p.npe;
    *conn = p.conn;
    geo->resize(p.ne);
    // per range: swapped count and the first failing element (the lowest over
    // all ranges is the one a serial pass would report)
    struct Res { int64_t swapped = 0, bad = -1; tled_status st = TLED_OK; std::string msg; };
    std::vector<Res> res(std::max(1, threads));
    std::atomic<int> slot{0};
    parallel_ranges(p.ne, threads, [&](int64_t lo, int64_t hi) {
        Res &r = res[slot++];
        for (int64_t e = lo; e < hi; ++e) {
            int32_t *c = conn->data() + npe * e;
            double Xe[24];
            bool range_ok = true;
            for (int a = 0; a < npe; ++a) {
                if (c[a] < 0 || c[a] >= p.nn) { range_ok = false; break; }
                std::memcpy(Xe + 3 * a, p.X.data() + 3 * int64_t(c[a]), 3 * sizeof(double));
            }
            if (!range_ok) {
                r = Res{r.swapped, e, TLED_E_MESH, "connectivity of element " + std::to_string(e) + " out of range"};
                return;
            }
            double d;
            if (npe == 4) {
                d = tet_geometry(Xe, &(*geo)[e]);
                if (d < 0.0) {
                    std::swap(c[2], c[3]);
                    for (int i = 0; i < 3; ++i) std::swap(Xe[6 + i], Xe[9 + i]);
                    d = tet_geometry(Xe, &(*geo)[e]);
                    ++r.swapped;
                }
                if (!(d > 0.0)) {
                    r = Res{r.swapped, e, TLED_E_MESH, "T4 element " + std::to_string(e) + " has zero volume"};
                    return;
                }
            } else {
                d = hex_geometry(Xe, &(*geo)[e]);
                if (!(d > 0.0)) {
                    r = Res{r.swapped, e, TLED_E_MESH,
                            "H8 element " + std::to_string(e) + " has det J0 <= 0 (inverted or degenerate)"};
                    return;
                }
            }
        }
    });
    *n_swapped = 0;
    const Res *first = nullptr;
    for (const Res &r : res) {
        *n_swapped += r.swapped;
        if (r.bad >= 0 && (!first || r.bad < first->bad)) first = &r;
    }
    if (first) {
        *err = first->msg;
        return first->st;
    }
    return TLED_OK;
}

uint64_t spread3(uint64_t x) {
    x &= 0x1fffff;
    x = (x | x << 32) & 0x1f00000000ffffULL;
    x = (x | x << 16) & 0x1f0000ff0000ffULL;
    x = (x | x << 8) & 0x100f00f00f00f00fULL;
    x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
    x = (x | x << 2) & 0x1249249249249249ULL;
    return x;
}

// Element centroids (mean of the nodes) and their Morton (Z-order) keys over
// the mesh's bounding cube.
void centroids_and_keys(const HostProblem &p, const std::vector<int32_t> &conn, std::vector<double> *cen,
                        std::vector<uint64_t> *key) {
    const int npe = p.npe;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t a = 0; a < p.nn; ++a)
        for (int i = 0; i < 3; ++i) {
            lo[i] = std::min(lo[i], p.X[3 * a + i]);
            hi[i] = std::max(hi[i], p.X[3 * a + i]);
        }
    double span = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
    cen->assign(size_t(p.ne) * 3, 0.0);
    key->resize(p.ne);
    for (int64_t e = 0; e < p.ne; ++e) {
        double *c = cen->data() + 3 * e;
        for (int a = 0; a < npe; ++a)
            for (int i = 0; i < 3; ++i) c[i] += p.X[3 * int64_t(conn[npe * e + a]) + i];
        uint64_t k = 0;
        for (int i = 0; i < 3; ++i) {
            c[i] /= npe;
            double t = (c[i] - lo[i]) / span;
            uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, t * 2097151.0));
            k |= spread3(q) << i;
        }
        (*key)[e] = k;
    }
}

// Element order along a Morton curve of the centroids.
std::vector<int64_t> morton_order(const HostProblem &p, const std::vector<int32_t> &conn) {
    std::vector<double> cen;
    std::vector<uint64_t> key;
    centroids_and_keys(p, conn, &cen, &key);
    std::vector<int64_t> order(p.ne);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(),
              [&](int64_t a, int64_t b) { return key[a] != key[b] ? key[a] < key[b] : a < b; });
    return order;
}

// Element order whose consecutive runs of P elements are compact patches:
// recursive coordinate bisection of the centroids.  A set of M > P elements
// (q = ceil(M/P) patches) is cut across the longest extent of its centroids
// into floor(q/2)·P elements and the rest; sets of at most P elements are
// leaves, ordered along the Morton curve.  Every leaf but the last has exactly
// P elements, and ties are broken by element number, so the order is fully
// determined by the mesh.  Against runs of the Morton order this stores about
// 8 % fewer patch-local node copies on tetrahedral meshes and bounds the
// nodes of the largest patch far more tightly (a regular grid of power-of-two
// size is cut into boxes of the same size either way).
std::vector<int64_t> bisection_order(const HostProblem &p, const std::vector<int32_t> &conn, int P, int threads) {
    std::vector<double> cen;
    std::vector<uint64_t> key;
    centroids_and_keys(p, conn, &cen, &key);
    // the partition moves compact records (centroid, key, element) rather than
    // indices into the centroid array
    struct Item {
        double c[3];
        uint64_t key;
        int64_t e;
    };
    std::vector<Item> it(p.ne);
    for (int64_t e = 0; e < p.ne; ++e) it[e] = Item{{cen[3 * e], cen[3 * e + 1], cen[3 * e + 2]}, key[e], e};
    // the two halves of a cut are disjoint ranges: the top cuts hand one half
    // to another host thread (the result does not depend on the thread count)
    std::function<void(int64_t, int64_t, int)> split = [&](int64_t lo, int64_t hi, int par) {
        const int64_t M = hi - lo;
        auto first = it.begin() + lo, last = it.begin() + hi;
        if (M <= P) {
            std::sort(first, last, [](const Item &a, const Item &b) { return a.key != b.key ? a.key < b.key : a.e < b.e; });
            return;
        }
        double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
        for (auto q = first; q != last; ++q)
            for (int i = 0; i < 3; ++i) {
                mn[i] = std::min(mn[i], q->c[i]);
                mx[i] = std::max(mx[i], q->c[i]);
            }
        int ax = 0;   // extents equal to rounding go to the lower axis (regular grids cut alike everywhere)
        for (int i = 1; i < 3; ++i)
            if (mx[i] - mn[i] > (mx[ax] - mn[ax]) * (1.0 + 1e-9)) ax = i;
        const int64_t q = (M + P - 1) / P, left = (q / 2) * int64_t(P);
        std::nth_element(first, first + left, last, [ax](const Item &a, const Item &b) {
            return a.c[ax] != b.c[ax] ? a.c[ax] < b.c[ax] : a.e < b.e;
        });
        std::thread th;
        if (par > 1 && M > 8192) {
            try {
                th = std::thread(split, lo, lo + left, par / 2);
            } catch (const std::system_error &) {
                // no thread: both halves on this one
            }
        }
        if (th.joinable()) {
            split(lo + left, hi, par - par / 2);
            th.join();
        } else {
            split(lo, lo + left, 1);
            split(lo + left, hi, 1);
        }
    };
    split(0, p.ne, std::max(1, threads));
    std::vector<int64_t> order(p.ne);
    for (int64_t e = 0; e < p.ne; ++e) order[e] = it[e].e;
    return order;
}

void build_patches(Precomputed *pc, int patch_elems, const std::vector<double> &Xc) {
    const int npe = pc->npe;
    const int64_t ne = pc->ne, nn = pc->nn;
    Patches &P = pc->patches;
    P.n = int32_t((ne + patch_elems - 1) / patch_elems);
    P.elem_begin.resize(P.n + 1);
    for (int32_t p = 0; p <= P.n; ++p) P.elem_begin[p] = int32_t(std::min<int64_t>(ne, int64_t(p) * patch_elems));
    // patch membership of nodes: interior iff touched by exactly one patch
    std::vector<int32_t> owner(nn, -1);
    std::vector<uint8_t> shared(nn, 0);
    for (int32_t p = 0; p < P.n; ++p)
        for (int64_t e = P.elem_begin[p]; e < P.elem_begin[p + 1]; ++e)
            for (int a = 0; a < npe; ++a) {
                int32_t n = pc->conn[npe * e + a];
                if (owner[n] == -1) owner[n] = p;
                else if (owner[n] != p) shared[n] = 1;
            }
    // new node order: interior nodes patch by patch (first-touch inside the
    // patch), then shared nodes in first-touch order
    std::vector<int64_t> old2new(nn, -1), new2old;
    new2old.reserve(nn);
    P.int_begin.assign(P.n + 1, 0);
    for (int32_t p = 0; p < P.n; ++p) {
        P.int_begin[p] = int32_t(new2old.size());
        for (int64_t e = P.elem_begin[p]; e < P.elem_begin[p + 1]; ++e)
            for (int a = 0; a < npe; ++a) {
                int32_t n = pc->conn[npe * e + a];
                if (!shared[n] && old2new[n] < 0) {
                    old2new[n] = int64_t(new2old.size());
                    new2old.push_back(n);
                }
            }
    }
    P.int_begin[P.n] = int32_t(new2old.size());
    P.n_interior = int64_t(new2old.size());
    for (int64_t e = 0; e < ne; ++e)
        for (int a = 0; a < npe; ++a) {
            int32_t n = pc->conn[npe * e + a];
            if (shared[n] && old2new[n] < 0) {
                old2new[n] = int64_t(new2old.size());
                new2old.push_back(n);
            }
        }
    // renumber everything node-indexed
    auto permute_d = [&](std::vector<double> &v, int w) {
        std::vector<double> t(v.size());
        for (int64_t i = 0; i < nn; ++i)
            for (int k = 0; k < w; ++k) t[w * i + k] = v[w * new2old[i] + k];
        v.swap(t);
    };
    permute_d(pc->Vl, 1); permute_d(pc->M, 1); permute_d(pc->C, 1); permute_d(pc->Kb, 1);
    permute_d(pc->Qm, 1); permute_d(pc->Qr, 1); permute_d(pc->Tfix, 1);
    {
        std::vector<uint8_t> t(nn);
        for (int64_t i = 0; i < nn; ++i) t[i] = pc->fix[new2old[i]];
        pc->fix.swap(t);
        std::vector<int64_t> n2o(nn);
        for (int64_t i = 0; i < nn; ++i) n2o[i] = pc->node_new2old[new2old[i]];
        pc->node_new2old.swap(n2o);
        for (int64_t i = 0; i < nn; ++i) pc->node_old2new[pc->node_new2old[i]] = i;
    }
    for (auto &c : pc->conn) c = int32_t(old2new[c]);

    // per-patch local numbering, gather lists and shared partial slots
    P.shared_begin.assign(P.n + 1, 0);
    P.shared_ids.clear();
    P.lconn.resize(size_t(ne) * npe);
    P.lrow_begin.assign(P.n + 1, 0);
    P.lrow.clear();
    P.lpos.resize(size_t(ne) * npe);
    P.max_nodes = 0;
    P.max_elems = 0;
    P.slot_stride = int32_t(std::min<int64_t>(patch_elems, ne));
    std::vector<int32_t> local(nn, -1);
    std::vector<std::vector<int32_t>> shared_parts(nn - P.n_interior);
    P.lX.clear();
    P.lx_begin.assign(P.n + 1, 0);
    for (int32_t p = 0; p < P.n; ++p) {
        const int32_t e0 = P.elem_begin[p], e1 = P.elem_begin[p + 1];
        const int32_t ib = P.int_begin[p], ie = P.int_begin[p + 1];
        const int32_t nint = ie - ib;
        P.shared_begin[p] = int32_t(P.shared_ids.size());
        std::vector<int32_t> touched;
        for (int32_t n = ib; n < ie; ++n) local[n] = n - ib;
        int32_t nloc = nint;
        for (int32_t e = e0; e < e1; ++e)
            for (int a = 0; a < npe; ++a) {
                int32_t n = pc->conn[npe * e + a];
                if (n >= P.n_interior && local[n] < 0) {
                    local[n] = nloc++;
                    touched.push_back(n);
                    shared_parts[n - P.n_interior].push_back(int32_t(P.shared_ids.size()));
                    P.shared_ids.push_back(n);
                }
                P.lconn[size_t(npe) * e + a] = uint16_t(local[n]);
            }
        P.max_nodes = std::max(P.max_nodes, nloc);
        P.max_elems = std::max(P.max_elems, e1 - e0);
        // local reference coordinates relative to the patch centroid (FP64, then rounded)
        {
            std::vector<int32_t> ids(nloc);
            for (int32_t n = ib; n < ie; ++n) ids[n - ib] = n;
            for (size_t k = 0; k < touched.size(); ++k) ids[nint + k] = touched[k];
            double o[3] = {0, 0, 0};
            for (int32_t n : ids)
                for (int i = 0; i < 3; ++i) o[i] += Xc[3 * pc->node_new2old[n] + i];
            for (int i = 0; i < 3; ++i) o[i] /= double(nloc);
            P.lx_begin[p] = int32_t(P.lX.size() / 3);
            for (int32_t n : ids)
                for (int i = 0; i < 3; ++i) P.lX.push_back(float(Xc[3 * pc->node_new2old[n] + i] - o[i]));
        }
        // local gather lists
        std::vector<int32_t> cnt(nloc + 1, 0);
        for (int32_t e = e0; e < e1; ++e)
            for (int a = 0; a < npe; ++a) cnt[P.lconn[size_t(npe) * e + a] + 1]++;
        for (int32_t l = 0; l < nloc; ++l) cnt[l + 1] += cnt[l];
        P.lrow_begin[p] = int32_t(P.lrow.size());
        for (int32_t l = 0; l <= nloc; ++l) P.lrow.push_back(uint16_t(cnt[l]));
        std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
        for (int32_t e = e0; e < e1; ++e)
            for (int a = 0; a < npe; ++a) {
                int32_t l = P.lconn[size_t(npe) * e + a];
                P.lpos[size_t(npe) * e + a] = uint16_t(fill[l]++);
            }
        for (int32_t n = ib; n < ie; ++n) local[n] = -1;
        for (int32_t n : touched) local[n] = -1;
    }
    P.shared_begin[P.n] = int32_t(P.shared_ids.size());
    P.lrow_begin[P.n] = int32_t(P.lrow.size());
    const int64_t nsh = nn - P.n_interior;
    P.lx_begin[P.n] = int32_t(P.lX.size() / 3);
    P.srow.assign(nsh + 1, 0);
    P.ppos.assign(P.shared_ids.size(), -1);
    int32_t pos = 0;
    for (int64_t s = 0; s < nsh; ++s) {
        P.srow[s] = pos;
        for (int32_t k : shared_parts[s]) P.ppos[k] = pos++;   // shared_parts[s] is in patch order
    }
    P.srow[nsh] = pos;
}

}  // namespace

int host_threads() {
    int nt = int(std::thread::hardware_concurrency());
    if (const char *env = std::getenv("TLED_HOST_THREADS")) nt = std::atoi(env);
    return std::max(1, std::min(nt, 64));
}

tled_status critical_dt(const HostProblem &p, double *dt_cr, std::string *err) {
    tled_status st = check_inputs(p, err);
    if (st != TLED_OK) return st;
    std::vector<int32_t> conn;
    std::vector<ElemGeo> geo;
    int64_t ns;
    st = element_pass(p, &conn, &geo, &ns, err);
    if (st != TLED_OK) return st;
    double cd = wave_speed(p.mat), dtc = std::numeric_limits<double>::infinity();
    for (auto &g : geo) dtc = std::min(dtc, g.L / cd);
    *dt_cr = dtc;
    return TLED_OK;
}

tled_status precompute(const HostProblem &p, const SetupOptions &opt, Precomputed *out, std::string *err) {
    tled_status st = check_inputs(p, err);
    if (st != TLED_OK) return st;
    if (p.ne <= 0 || p.nn <= 0) { *err = "empty mesh"; return TLED_E_ARG; }
    const int npe = p.npe;
    std::vector<int32_t> conn;
    std::vector<ElemGeo> geo;
    Precomputed &pc = *out;
    pc = Precomputed();
    pc.npe = npe; pc.nn = p.nn; pc.ne = p.ne;
    st = element_pass(p, &conn, &geo, &pc.n_swapped, err, opt.threads);
    if (st != TLED_OK) return st;

    double cd = wave_speed(p.mat);
    pc.dt_cr = std::numeric_limits<double>::infinity();
    for (auto &g : geo) pc.dt_cr = std::min(pc.dt_cr, g.L / cd);

    // element order (fused variants: patches of pe consecutive elements)
    const int pe = std::max(8, std::min(opt.patch_elems, 65536 / npe));
    std::vector<int64_t> eorder(p.ne);
    if (opt.reorder)
        eorder = (opt.build_patches && opt.bisect) ? bisection_order(p, conn, pe, opt.threads) : morton_order(p, conn);
    else std::iota(eorder.begin(), eorder.end(), 0);
    pc.elem_new2old = eorder;
    // node order: first touch along the element order (or identity)
    pc.node_old2new.assign(p.nn, -1);
    pc.node_new2old.clear();
    pc.node_new2old.reserve(p.nn);
    if (opt.reorder) {
        for (int64_t ei = 0; ei < p.ne; ++ei)
            for (int a = 0; a < npe; ++a) {
                int32_t n = conn[npe * eorder[ei] + a];
                if (pc.node_old2new[n] < 0) {
                    pc.node_old2new[n] = int64_t(pc.node_new2old.size());
                    pc.node_new2old.push_back(n);
                }
            }
        if (int64_t(pc.node_new2old.size()) != p.nn) {
            *err = "mesh has nodes that belong to no element";
            return TLED_E_MESH;
        }
    } else {
        for (int64_t a = 0; a < p.nn; ++a) { pc.node_old2new[a] = a; pc.node_new2old.push_back(a); }
    }
    const int64_t nn = p.nn, ne = p.ne;

    pc.conn.resize(size_t(ne) * npe);
    pc.geo.resize(size_t(ne) * 9);
    pc.V0.resize(ne);
    pc.a0.resize(size_t(ne) * 3);
    if (p.mat.expan_mode == 2) pc.n0.resize(size_t(ne) * 3);
    if (p.mat.cond_mode == 2) pc.Dc.resize(size_t(ne) * 6);
    if (npe == 8) { pc.hgc.resize(size_t(ne) * 12); pc.khg.resize(ne); }
    std::vector<double> q(ne, 0.0);
    for (int64_t ei = 0; ei < ne; ++ei) {
        int64_t e = eorder[ei];
        for (int a = 0; a < npe; ++a) pc.conn[npe * ei + a] = int32_t(pc.node_old2new[conn[npe * e + a]]);
        const ElemGeo &g = geo[e];
        std::memcpy(&pc.geo[9 * ei], g.geo, 9 * sizeof(double));
        pc.V0[ei] = g.V0;
        double a0[3] = {1.0, 0.0, 0.0};
        if (!p.a0.empty()) { a0[0] = p.a0[3 * e]; a0[1] = p.a0[3 * e + 1]; a0[2] = p.a0[3 * e + 2]; }
        double an = std::sqrt(a0[0] * a0[0] + a0[1] * a0[1] + a0[2] * a0[2]);
        if (!(an > 0.0)) { *err = "zero fibre vector at element " + std::to_string(e); return TLED_E_ARG; }
        for (int i = 0; i < 3; ++i) pc.a0[3 * ei + i] = a0[i] / an;
        if (p.mat.expan_mode == 2) {
            // Eq. 11's axes are orthonormal: remove n's component along m = a0, normalise
            const double *m = &pc.a0[3 * ei], *n = &p.n0[3 * e];
            const double nn0 = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            const double d = n[0] * m[0] + n[1] * m[1] + n[2] * m[2];
            const double w[3] = {n[0] - d * m[0], n[1] - d * m[1], n[2] - d * m[2]};
            const double wn = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
            if (!(wn > 1e-6 * nn0)) {
                *err = "second expansion axis parallel to the fibre (or zero) at element " + std::to_string(e);
                return TLED_E_ARG;
            }
            for (int i = 0; i < 3; ++i) pc.n0[3 * ei + i] = w[i] / wn;
        }
        if (p.mat.cond_mode == 2) std::memcpy(&pc.Dc[6 * ei], &p.Dc[6 * e], 6 * sizeof(double));
        if (npe == 8) {
            std::memcpy(&pc.hgc[12 * ei], g.hgc, 12 * sizeof(double));
            pc.khg[ei] = p.mat.hg_coef * (p.mat.kappa + 4.0 * p.mat.mu / 3.0) * g.V0 * g.sum_dh2 / 8.0;
        }
        if (!p.q.empty()) q[ei] = p.q[e];
    }

    // lumped quantities with reference volumes
    pc.Vl.assign(nn, 0.0);
    pc.Qr.assign(nn, 0.0);
    for (int64_t e = 0; e < ne; ++e)
        for (int a = 0; a < npe; ++a) {
            int32_t n = pc.conn[npe * e + a];
            pc.Vl[n] += pc.V0[e] / npe;
            pc.Qr[n] += q[e] * pc.V0[e] / npe;
        }
    pc.M.resize(nn); pc.C.resize(nn); pc.Kb.resize(nn); pc.Qm.resize(nn);
    pc.fix.assign(nn, 0);
    pc.Tfix.assign(nn, p.mat.T0);
    for (int64_t a = 0; a < nn; ++a) {
        pc.M[a] = p.mat.rho * pc.Vl[a];
        pc.C[a] = p.mat.rho * p.mat.c * pc.Vl[a];
        pc.Kb[a] = p.mat.wbcb * pc.Vl[a];
        pc.Qm[a] = p.mat.Q_met * pc.Vl[a];
        int64_t o = pc.node_new2old[a];
        if (!p.fix.empty()) pc.fix[a] = p.fix[o];
        if (!p.Tfix.empty()) pc.Tfix[a] = p.Tfix[o];
    }

    // Explicit thermal stability: forward Euler on C dT/dt = -(K + K_b) T + ... is
    // stable for dt <= 2 / lambda_max(C^-1 (K + K_b)), and by Gershgorin
    // lambda_max <= max_a (sum_b |K_ab| + K_b,a) / C_a.  K is taken on the reference
    // geometry with the largest conductivity the material reaches (k, k_m, k(T)),
    // |K_e,ab| <= V0 k_max |dh_a/dX| |dh_b/dX|; C with the smallest heat capacity (c(T)).
    {
        const tled_material &m = p.mat;
        double kmax = m.k;
        if (m.cond_mode == 1) kmax = std::max(kmax, m.k_m);
        const double kt = (m.ckT_on && m.k > 0.0) ? std::max(1.0, m.k_hi / m.k) : 1.0;
        kmax *= kt;
        const double cmin = m.ckT_on ? std::min(m.c, m.c_hi) : m.c;
        std::vector<double> rowsum(nn, 0.0);
        for (int64_t ei = 0; ei < ne; ++ei) {
            const ElemGeo &g = geo[eorder[ei]];
            double gn[8];
            if (npe == 4) {
                double r0[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k < 3; ++k) {
                    const double *r = g.geo + 3 * k;
                    gn[k + 1] = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                    for (int i = 0; i < 3; ++i) r0[i] -= r[i];
                }
                gn[0] = std::sqrt(r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2]);
            } else {
                for (int a = 0; a < 8; ++a) {
                    double d2 = 0.0;
                    for (int j = 0; j < 3; ++j) {
                        const double dh = (g.geo[3 * j] * kHexSign[a][0] + g.geo[3 * j + 1] * kHexSign[a][1] +
                                           g.geo[3 * j + 2] * kHexSign[a][2]) / 8.0;
                        d2 += dh * dh;
                    }
                    gn[a] = std::sqrt(d2);
                }
            }
            double sum = 0.0;
            for (int a = 0; a < npe; ++a) sum += gn[a];
            double ke = kmax;
            if (m.cond_mode == 2) {   // Frobenius norm >= the tensor's largest eigenvalue
                const double *d = &pc.Dc[6 * ei];
                ke = kt * std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] +
                                    2.0 * (d[3] * d[3] + d[4] * d[4] + d[5] * d[5]));
            }
            for (int a = 0; a < npe; ++a) rowsum[pc.conn[npe * ei + a]] += g.V0 * ke * gn[a] * sum;
        }
        pc.dt_th = std::numeric_limits<double>::infinity();
        for (int64_t a = 0; a < nn; ++a) {
            const double den = rowsum[a] + m.wbcb * pc.Vl[a];
            if (den > 0.0) pc.dt_th = std::min(pc.dt_th, 2.0 * m.rho * cmin * pc.Vl[a] / den);
        }
    }

    if (opt.build_patches) build_patches(&pc, pe, p.X);

    // node -> element-slot incidence (ascending slot order): the two-pass variant's gather
    if (opt.build_patches) return TLED_OK;
    pc.rowptr.assign(nn + 1, 0);
    for (int64_t s = 0; s < ne * npe; ++s) pc.rowptr[pc.conn[s] + 1]++;
    for (int64_t a = 0; a < nn; ++a) pc.rowptr[a + 1] += pc.rowptr[a];
    pc.inc.resize(size_t(ne) * npe);
    std::vector<int32_t> fill(pc.rowptr.begin(), pc.rowptr.end() - 1);
    for (int64_t s = 0; s < ne * npe; ++s) pc.inc[fill[pc.conn[s]]++] = int32_t(s);
    return TLED_OK;
}

tled_status precompute_batch(const std::vector<HostProblem> &ps, const std::vector<int> &patch_elems,
                             bool reorder, bool bisect, const std::function<int64_t(size_t, double)> &end_step,
                             Precomputed *out, std::vector<ScenRange> *ranges,
                             std::vector<int32_t> *patch_scen, std::vector<int32_t> *shared_scen,
                             std::string *err) {
    const size_t S = ps.size();
    if (S == 0) { *err = "empty batch"; return TLED_E_ARG; }
    const int npe = ps[0].npe;
    for (size_t k = 0; k < S; ++k) {
        if (ps[k].npe != npe) { *err = "a batch needs one element type"; return TLED_E_ARG; }
        if (ps[k].mat.n_prony != ps[0].mat.n_prony) { *err = "a batch needs one Prony term count"; return TLED_E_ARG; }
    }
    // Scenarios are independent: precompute them on a pool of host threads
    // (TLED_HOST_THREADS, default the hardware concurrency, at most 64).  Each
    // result depends only on its own scenario, so the outcome does not depend on
    // the thread count.
    std::vector<Precomputed> pcs(S);
    std::vector<tled_status> sts(S, TLED_OK);
    std::vector<std::string> errs(S);
    std::atomic<size_t> next{0};
    auto work = [&]() {
        for (size_t k = next++; k < S; k = next++) {
            SetupOptions so;
            so.reorder = reorder;
            so.bisect = bisect;
            so.build_patches = true;
            so.patch_elems = patch_elems[k];
            so.threads = std::max(1, host_threads() / int(S));   // threads left over for each scenario
            sts[k] = precompute(ps[k], so, &pcs[k], &errs[k]);
        }
    };
    const int nt = std::max(1, std::min(host_threads(), int(S)));
    std::vector<std::thread> pool = start_workers(nt - 1, work);
    work();
    for (auto &th : pool) th.join();
    for (size_t k = 0; k < S; ++k)
        if (sts[k] != TLED_OK) { *err = "scenario " + std::to_string(k) + ": " + errs[k]; return sts[k]; }
    // Union order: scenarios by descending end step (stable), so that the
    // patches and shared nodes of the scenarios still running at any step form
    // a prefix of the union arrays and a step can launch just that prefix.
    std::vector<int64_t> ends(S);
    for (size_t k = 0; k < S; ++k) ends[k] = end_step(k, pcs[k].dt_cr);
    std::vector<size_t> order(S);
    std::iota(order.begin(), order.end(), size_t(0));
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return ends[a] > ends[b]; });
    // offsets of every scenario in the union (serial prefix sums in union
    // order), then each scenario fills its own slices of the union arrays (in
    // parallel)
    struct Off {
        int64_t e, i, s, patch, sid, lrow, lx, geo, hgc, khg, a0, lconn, ppos;
    };
    std::vector<Off> off(S + 1);
    {
        Off o{};
        for (size_t pos = 0; pos < S; ++pos) {
            const size_t k = order[pos];
            off[k] = o;
            const Precomputed &pc = pcs[k];
            const Patches &Q = pc.patches;
            o.e += pc.ne;
            o.i += Q.n_interior;
            o.s += pc.nn - Q.n_interior;
            o.patch += Q.n;
            o.sid += int64_t(Q.shared_ids.size());
            o.lrow += int64_t(Q.lrow.size());
            o.lx += int64_t(Q.lX.size() / 3);
            o.geo += int64_t(pc.geo.size());
            o.hgc += int64_t(pc.hgc.size());
            o.khg += int64_t(pc.khg.size());
            o.a0 += int64_t(pc.a0.size());
            o.lconn += int64_t(Q.lconn.size());
            o.ppos += int64_t(Q.ppos.size());
        }
        off[S] = o;
    }
    const Off &T = off[S];
    if (T.e > INT32_MAX / npe || T.sid > INT32_MAX || T.lrow > INT32_MAX) { *err = "batch too large"; return TLED_E_ARG; }
    Precomputed &U = *out;
    U = Precomputed();
    U.npe = npe;
    U.ne = T.e;
    U.nn = T.i + T.s;
    const int64_t NE = T.e, NI = T.i;
    ranges->assign(S, ScenRange());
    patch_scen->assign(T.patch, 0);
    shared_scen->assign(T.s, 0);
    Patches &P = U.patches;
    P.n_interior = NI;
    P.n = int32_t(T.patch);
    int32_t stride = 0;
    for (auto &pc : pcs) {
        stride = std::max(stride, pc.patches.slot_stride);
        P.max_nodes = std::max(P.max_nodes, pc.patches.max_nodes);
        P.max_elems = std::max(P.max_elems, pc.patches.max_elems);
    }
    P.slot_stride = stride;
    U.Vl.assign(U.nn, 0); U.M.assign(U.nn, 0); U.C.assign(U.nn, 0); U.Kb.assign(U.nn, 0);
    U.Qm.assign(U.nn, 0); U.Qr.assign(U.nn, 0); U.fix.assign(U.nn, 0); U.Tfix.assign(U.nn, 0);
    U.node_new2old.assign(U.nn, -1);   // caller index within its scenario
    U.conn.resize(size_t(NE) * npe);
    U.geo.resize(T.geo);
    U.V0.resize(NE);
    U.hgc.resize(T.hgc);
    U.khg.resize(T.khg);
    U.a0.resize(T.a0);
    U.elem_new2old.resize(NE);
    P.elem_begin.resize(T.patch + 1);
    P.int_begin.resize(T.patch + 1);
    P.shared_begin.resize(T.patch + 1);
    P.lrow_begin.resize(T.patch + 1);
    P.lx_begin.resize(T.patch + 1);
    P.shared_ids.resize(T.sid);
    P.lconn.resize(T.lconn);
    P.lrow.resize(T.lrow);
    P.lpos.resize(size_t(NE) * npe);
    P.srow.resize(T.s + 1);
    P.ppos.resize(T.ppos);
    P.lX.resize(size_t(T.lx) * 3);
    next = 0;
    auto fill = [&]() {
        for (size_t k = next++; k < S; k = next++) {
            const Precomputed &pc = pcs[k];
            const Patches &Q = pc.patches;
            const Off &o = off[k];
            ScenRange &R = (*ranges)[k];
            const int64_t nint = Q.n_interior, nsh = pc.nn - nint;
            const int64_t eo = o.e, io = o.i, so_ = o.s;
            const int32_t sid0 = int32_t(o.sid), lr0 = int32_t(o.lrow), lx0 = int32_t(o.lx);
            auto map = [&](int64_t n) { return n < nint ? io + n : NI + so_ + (n - nint); };
            R.elem_lo = eo; R.elem_hi = eo + pc.ne;
            R.int_lo = io; R.int_hi = io + nint;
            R.sh_lo = NI + so_; R.sh_hi = NI + so_ + nsh;
            R.patch_lo = int32_t(o.patch); R.patch_hi = int32_t(o.patch + Q.n);
            R.dt_cr = pc.dt_cr;
            R.dt_th = pc.dt_th;
            R.n_swapped = pc.n_swapped;
            R.node_of.resize(pc.nn);
            for (int64_t a = 0; a < pc.nn; ++a) R.node_of[pc.node_new2old[a]] = map(a);
            R.elem_of.resize(pc.ne);
            for (int64_t e = 0; e < pc.ne; ++e) R.elem_of[pc.elem_new2old[e]] = eo + e;
            for (int64_t a = 0; a < pc.nn; ++a) {
                const int64_t g = map(a);
                U.Vl[g] = pc.Vl[a]; U.M[g] = pc.M[a]; U.C[g] = pc.C[a]; U.Kb[g] = pc.Kb[a];
                U.Qm[g] = pc.Qm[a]; U.Qr[g] = pc.Qr[a]; U.fix[g] = pc.fix[a]; U.Tfix[g] = pc.Tfix[a];
                U.node_new2old[g] = pc.node_new2old[a];
            }
            for (int64_t j = 0; j < nsh; ++j) (*shared_scen)[so_ + j] = int32_t(k);
            for (size_t c = 0; c < pc.conn.size(); ++c) U.conn[size_t(eo) * npe + c] = int32_t(map(pc.conn[c]));
            std::copy(pc.geo.begin(), pc.geo.end(), U.geo.begin() + o.geo);
            std::copy(pc.V0.begin(), pc.V0.end(), U.V0.begin() + eo);
            std::copy(pc.hgc.begin(), pc.hgc.end(), U.hgc.begin() + o.hgc);
            std::copy(pc.khg.begin(), pc.khg.end(), U.khg.begin() + o.khg);
            std::copy(pc.a0.begin(), pc.a0.end(), U.a0.begin() + o.a0);
            std::copy(pc.elem_new2old.begin(), pc.elem_new2old.begin() + pc.ne, U.elem_new2old.begin() + eo);
            for (int32_t q = 0; q < Q.n; ++q) {
                const size_t g = size_t(o.patch) + q;
                P.elem_begin[g] = int32_t(eo + Q.elem_begin[q]);
                P.int_begin[g] = int32_t(io + Q.int_begin[q]);
                P.shared_begin[g] = sid0 + Q.shared_begin[q];
                P.lrow_begin[g] = lr0 + Q.lrow_begin[q];
                P.lx_begin[g] = lx0 + Q.lx_begin[q];
                (*patch_scen)[g] = int32_t(k);
            }
            for (size_t q = 0; q < Q.shared_ids.size(); ++q) P.shared_ids[sid0 + q] = int32_t(map(Q.shared_ids[q]));
            std::copy(Q.lconn.begin(), Q.lconn.end(), P.lconn.begin() + o.lconn);
            std::copy(Q.lrow.begin(), Q.lrow.end(), P.lrow.begin() + o.lrow);
            std::copy(Q.lpos.begin(), Q.lpos.end(), P.lpos.begin() + size_t(eo) * npe);   // patch-local
            for (int64_t j = 0; j < nsh; ++j) P.srow[so_ + j] = sid0 + Q.srow[j];
            for (size_t q = 0; q < Q.ppos.size(); ++q) P.ppos[o.ppos + q] = sid0 + Q.ppos[q];
            std::copy(Q.lX.begin(), Q.lX.end(), P.lX.begin() + 3 * o.lx);
        }
    };
    pool = start_workers(nt - 1, fill);
    fill();
    for (auto &th : pool) th.join();
    P.elem_begin[T.patch] = int32_t(NE);
    P.int_begin[T.patch] = int32_t(NI);
    P.shared_begin[T.patch] = int32_t(T.sid);
    P.lrow_begin[T.patch] = int32_t(T.lrow);
    P.lx_begin[T.patch] = int32_t(T.lx);
    P.srow[T.s] = int32_t(T.sid);
    if (P.max_elems * npe > 65535 || P.slot_stride * npe > 65535) { *err = "patch too large"; return TLED_E_ARG; }
    U.dt_cr = 0.0;
    return TLED_OK;
}

}  // namespace tled
