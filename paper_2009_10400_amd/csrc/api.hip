// C-ABI of the TLED + Pennes solver (declared in include/tled.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <numeric>
#include <climits>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "../../include/tled.h"
#include "kernels.h"
#include "tled_internal.h"

using namespace tled;

namespace {

constexpr uint64_t kStateMagic = 0x31534544454c5454ULL;  // "TTLEDES1"

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct tled_sim {
    int device = -1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *(*alloc)(size_t, void *) = nullptr;
    void (*release)(void *, void *) = nullptr;
    void *actx = nullptr;
    tled_options opt{};
    HostProblem prob;
    Precomputed pc;
    bool finalized = false;
    std::string err;
    std::vector<DevBuf> bufs;
    int64_t device_bytes = 0;
    int variant = 1;
    int np = 0;
    KMat km{};
    NodeParams nparams{};
    TwoPassArgs tp{};
    PatchArgs pa{};
    long long *d_step = nullptr;
    unsigned *d_status = nullptr;
    DevMonitors *d_mon = nullptr;
    double *d_part_elem = nullptr, *d_part_node = nullptr;
    int n_elem_parts = 0, n_node_parts = 0;
    int *d_new2old = nullptr;
    // instantiated hipGraphs of step chunks, keyed by chunk length and (batch)
    // the launched patch and shared-node counts baked into them; least
    // recently used first out
    struct GraphEntry {
        hipGraphExec_t exec;
        int k, np;
        int64_t ns;
        uint64_t used;
    };
    std::vector<GraphEntry> graphs;
    uint64_t graph_clock = 0;
    int64_t step = 0;
    std::vector<float> B;   // per-node velocity coefficient (kept for state writes)
    size_t theta_floats = 0;
    // scenarios: a single problem is a batch of one
    bool is_batch = false;
    std::vector<HostProblem> scen;
    std::vector<int64_t> scen_steps;
    std::vector<int32_t> scen_pe;
    std::vector<double> scen_cfl, scen_tend;   // > 0: dt and steps chosen at finalize
    std::vector<ScenRange> ranges;
    std::vector<int32_t> patch_scen, shared_scen;
    std::vector<KMat> scen_km;
    std::vector<NodeParams> scen_np;
    KMat *d_km = nullptr;
    NodeParams *d_np = nullptr;
    long long *d_ranges = nullptr;
    double *d_scen_mon = nullptr;
    // batch: union positions (scenarios by descending end step): end step, and
    // the patch and shared-node counts of the prefix ending at the position
    std::vector<int64_t> pos_end, pos_shared_hi;
    std::vector<int32_t> pos_patch_hi;
    // persistent schedule of a batch: grids of the patch and shared-node kernels
    bool queue = false;
    int q_grid = 0, q_sgrid = 0;
    // shared nodes advanced inside the next step's patch kernel: the second
    // partial buffer and the second shared-node state buffer (the first ones
    // are pa.partial and the shared tail of nu4, nv4)
    bool fuse = false;
    float4 *d_part2 = nullptr, *d_sux = nullptr, *d_svx = nullptr;
    // thermal dose (tled_set_thermal_dose): per node (CEM43 minutes, Arrhenius integral)
    bool dose_on = false;
    double dose_A = 0.0, dose_Ea = 0.0;
    double2 *d_dose = nullptr;
    DoseParams dq{};
};

namespace {

// Default elements per patch of a single problem.  H8: 256 (on a regular grid,
// 8x8x4-cell boxes).  T4: the patch kernel is fastest with patches as large as
// the LDS of four resident 256-thread workgroups per CU allows (about 500
// elements with bisection patches), but only 256 CUs x 4 = 1024 patches run at
// once, and a patch count just above a multiple of 1024 leaves a last round
// that keeps few CUs busy (measured on the 1M-tet ellipsoid: 2087 patches of
// 480 elements 31.9 us, 2019 patches of 496 elements 29.4 us).  So the count
// of rounds is the smallest one whose patches fit, and the patches are the
// smallest (a multiple of 8) that fill those rounds.  512-thread workgroups:
// two per CU, patches up to 704 elements (the 64 KB LDS of one workgroup).
int default_patch_elems(int npe, int64_t ne, int block_size) {
    if (npe != 4) return 256;
    const int64_t slots = 256 * (block_size == 512 ? 2 : 4), pe_max = block_size == 512 ? 704 : 504;
    for (int64_t k = 1;; ++k) {
        const int64_t pe = ((ne + k * slots - 1) / (k * slots) + 7) / 8 * 8;
        if (pe <= pe_max) return int(std::max<int64_t>(pe, 128));
    }
}

// Default kernel variant: fused patches for both element types; T4 rebuilds the
// geometry from the staged coordinates (variant 2), H8 reads the precomputed
// geometry planes (variant 3), whose smaller LDS footprint (no staged
// coordinates: 39.2 KB for 256-element patches, against 45.7 KB) lets four
// workgroups share a CU, and whose kernel is compiled for four waves per SIMD
// (64³ cube: 20.1 us per step against 23.0 us for variant 2).
int default_variant(int npe) { return npe == 8 ? 3 : 2; }

// Whether the shared nodes of a finalized handle are advanced inside the next
// step's patch kernel: asked for (shared_update = 1), single problems with kernel
// variant 2, 256-thread workgroups, no anisotropy plane, no thermal dose (its
// kernel reads every node's temperature after each step) and some shared node.
// Not the default: on the 1M-tet ellipsoid it saved under 1 % of a step in long
// runs and measured slower in runs of 20 steps.
bool fused_shared_nodes(const tled_sim *s) {
    const tled_material &m = s->prob.mat;
    return !s->is_batch && s->variant == 2 && (s->opt.block_size == 0 || s->opt.block_size == kBlock) &&
           m.expan_mode != 2 && m.cond_mode != 2 && s->opt.shared_update == 1 && !s->dose_on &&
           s->pc.nn > s->pc.patches.n_interior;
}

tled_status fail(tled_sim *s, tled_status st, const std::string &msg) {
    if (s) s->err = msg;
    return st;
}

#define HIPCHK(sim, expr)                                                                         \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(sim, TLED_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

void *dev_alloc(tled_sim *s, size_t bytes) {
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~size_t(255);
    void *p = nullptr;
    if (s->alloc) {
        p = s->alloc(bytes, s->actx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) {
        s->bufs.push_back({p, bytes});
        s->device_bytes += int64_t(bytes);
    }
    return p;
}

void drop_graphs(tled_sim *s) {
    for (auto &g : s->graphs) (void)hipGraphExecDestroy(g.exec);
    s->graphs.clear();
}

void free_device(tled_sim *s) {
    drop_graphs(s);
    for (auto &b : s->bufs) {
        if (s->release) s->release(b.p, s->actx);
        else (void)hipFree(b.p);
    }
    s->bufs.clear();
    s->device_bytes = 0;
}

template <typename T>
tled_status upload(tled_sim *s, T **dst, const std::vector<T> &src) {
    *dst = static_cast<T *>(dev_alloc(s, sizeof(T) * src.size()));
    if (!*dst) return fail(s, TLED_E_OOM, "device allocation failed");
    if (!src.empty()) HIPCHK(s, hipMemcpyAsync(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s->stream));
    return TLED_OK;
}

template <typename T>
tled_status zeros(tled_sim *s, T **dst, size_t n) {
    *dst = static_cast<T *>(dev_alloc(s, sizeof(T) * n));
    if (!*dst) return fail(s, TLED_E_OOM, "device allocation failed");
    HIPCHK(s, hipMemsetAsync(*dst, 0, sizeof(T) * std::max<size_t>(n, 1), s->stream));
    return TLED_OK;
}

#define TRY(expr)                                \
    do {                                         \
        tled_status st_ = (expr);                \
        if (st_ != TLED_OK) return st_;          \
    } while (0)

void oct_encode(const double a[3], float *x, float *y) {
    double s = std::fabs(a[0]) + std::fabs(a[1]) + std::fabs(a[2]);
    double px = a[0] / s, py = a[1] / s;
    if (a[2] < 0.0) {
        double qx = (1.0 - std::fabs(py)) * (px >= 0.0 ? 1.0 : -1.0);
        double qy = (1.0 - std::fabs(px)) * (py >= 0.0 ? 1.0 : -1.0);
        px = qx;
        py = qy;
    }
    *x = float(px);
    *y = float(py);
}

// First step index n >= 0 with n * dt >= t (the same double comparison as the method's clock).
long long first_step_at(double t, double dt) {
    if (!(t > 0.0)) return 0;
    if (std::isinf(t)) return LLONG_MAX;
    double g = std::ceil(t / dt);
    if (g > 9.0e18) return LLONG_MAX;
    long long n = (long long)g;
    while (n > 0 && double(n - 1) * dt >= t) --n;
    while (double(n) * dt < t) ++n;
    return n;
}

KMat make_kmat(const tled_material &m, double dt) {
    KMat k{};
    k.mu = float(m.mu); k.kappa = float(m.kappa); k.eta = float(m.eta);
    k.alpha = float(m.alpha); k.alpha_m = float(m.alpha_m); k.alpha_n = float(m.alpha_n);
    k.k = float(m.k); k.k_m = float(m.k_m);
    // ramp starts as offsets from T0, formed in FP64 (the kernels work on dT = T - T0)
    k.muT_off = float(m.T0 - m.muT_lo); k.muT_inv = m.muT_on ? float(1.0 / (m.muT_hi - m.muT_lo)) : 0.f;
    k.muT_drop = float(m.muT_drop);
    k.sh_off = float(m.T0 - m.shrink_T); k.sh_inv = m.shrink_on ? float(1.0 / m.shrink_width) : 0.f;
    k.sh_eps = float(m.shrink_eps);
    k.ck_off = float(m.T0 - m.ckT_lo); k.ck_inv = m.ckT_on ? float(1.0 / (m.ckT_hi - m.ckT_lo)) : 0.f;
    k.c_lo = float(m.c); k.c_hi = float(m.c_hi); k.kr_hi = m.k > 0 ? float(m.k_hi / m.k) : 1.f;
    for (int i = 0; i < 4; ++i) {
        if (i < m.n_prony) {
            k.pc1[i] = float(dt * m.g[i] / (dt + m.tau[i]));
            k.pc2[i] = float(m.tau[i] / (dt + m.tau[i]));
        }
    }
    k.hgk = float(m.hg_coef * (m.kappa + 4.0 * m.mu / 3.0));
    k.n_prony = m.n_prony;
    k.expan_mode = m.expan_mode; k.cond_mode = m.cond_mode; k.muT_on = m.muT_on;
    k.shrink_on = m.shrink_on; k.ckT_on = m.ckT_on;
    return k;
}

NodeParams make_nparams(const HostProblem &pr, const KMat &k, double abl_T) {
    const tled_material &m = pr.mat;
    const double dt = pr.dt, g = pr.gamma;
    NodeParams p{};
    p.A = float((1.0 - 0.5 * g * dt) / (1.0 + 0.5 * g * dt));
    p.dt = float(dt);
    p.T0 = float(m.T0);
    p.rho = float(m.rho);
    p.abl_T = float(abl_T);
    p.ck_off = k.ck_off; p.ck_inv = k.ck_inv; p.c_lo = k.c_lo; p.c_hi = k.c_hi;
    p.ckT_on = m.ckT_on;
    p.n_on = first_step_at(pr.t_on, dt);
    p.n_off = first_step_at(pr.t_off, dt);
    return p;
}

void build_kernel_constants(tled_sim *s) {
    const double abl = s->opt.ablation_T > 0 ? s->opt.ablation_T : 333.15;
    s->scen_km.clear();
    s->scen_np.clear();
    for (const HostProblem &pr : s->scen) {
        s->scen_km.push_back(make_kmat(pr.mat, pr.dt));
        s->scen_np.push_back(make_nparams(pr, s->scen_km.back(), abl));
    }
    s->km = s->scen_km[0];
    s->nparams = s->scen_np[0];
}

// Single-precision device layout of the precomputed data, then upload.
tled_status upload_all(tled_sim *s) {
    const Precomputed &pc = s->pc;
    const int npe = pc.npe;
    const int64_t ne = pc.ne, nn = pc.nn;
    if (nn > INT_MAX / 2 || ne * npe > INT_MAX) return fail(s, TLED_E_ARG, "mesh too large for 32-bit indices");
    s->np = s->scen[0].mat.n_prony;

    // element planes
    std::vector<float4> g0(ne), g1(ne), g2(ne), h0, h1, h2;
    std::vector<float2> fib(ne);
    std::vector<float> khg;
    std::vector<int4> c0(ne), c1;
    if (npe == 8) { h0.resize(ne); h1.resize(ne); h2.resize(ne); khg.resize(ne); c1.resize(ne); }
    for (int64_t e = 0; e < ne; ++e) {
        const double *G = &pc.geo[9 * e];
        float ox, oy;
        oct_encode(&pc.a0[3 * e], &ox, &oy);
        fib[e] = make_float2(ox, oy);
        g0[e] = make_float4(float(G[0]), float(G[1]), float(G[2]), float(G[3]));
        g1[e] = make_float4(float(G[4]), float(G[5]), float(G[6]), float(G[7]));
        g2[e] = make_float4(float(G[8]), float(pc.V0[e]), ox, oy);
        const int32_t *c = &pc.conn[size_t(npe) * e];
        c0[e] = make_int4(c[0], c[1], c[2], c[3]);
        if (npe == 8) {
            c1[e] = make_int4(c[4], c[5], c[6], c[7]);
            const double *h = &pc.hgc[12 * e];
            h0[e] = make_float4(float(h[0]), float(h[1]), float(h[2]), float(h[3]));
            h1[e] = make_float4(float(h[4]), float(h[5]), float(h[6]), float(h[7]));
            h2[e] = make_float4(float(h[8]), float(h[9]), float(h[10]), float(h[11]));
            khg[e] = float(pc.khg[e]);
        }
    }
    // anisotropy plane (orthotropic expansion axis, conductivity tensor): two
    // float4 per element, only when a mode reads it
    std::vector<float4> aniso;
    const tled_material &m0 = s->scen[0].mat;
    if (m0.expan_mode == 2 || m0.cond_mode == 2) {
        aniso.assign(2 * size_t(ne), make_float4(0.f, 0.f, 0.f, 0.f));
        for (int64_t e = 0; e < ne; ++e) {
            float nx = 0.f, ny = 0.f;
            if (m0.expan_mode == 2) oct_encode(&pc.n0[3 * e], &nx, &ny);
            float d[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (m0.cond_mode == 2)
                for (int i = 0; i < 6; ++i) d[i] = float(pc.Dc[6 * e + i]);
            aniso[2 * e] = make_float4(nx, ny, d[0], d[1]);
            aniso[2 * e + 1] = make_float4(d[2], d[3], d[4], d[5]);
        }
    }
    // node arrays (each node with the constants of its scenario)
    std::vector<int32_t> node_scen(nn, 0);
    for (size_t k = 0; k < s->ranges.size(); ++k) {
        for (int64_t a = s->ranges[k].int_lo; a < s->ranges[k].int_hi; ++a) node_scen[a] = int32_t(k);
        for (int64_t a = s->ranges[k].sh_lo; a < s->ranges[k].sh_hi; ++a) node_scen[a] = int32_t(k);
    }
    std::vector<float4> nu4(nn), nv4(nn), nth(nn);
    std::vector<float> Vl(nn);
    std::vector<uint8_t> mask(nn);
    s->B.assign(nn, 0.f);
    for (int64_t a = 0; a < nn; ++a) {
        const HostProblem &pr = s->scen[node_scen[a]];
        const tled_material &m = pr.mat;
        const double dt = pr.dt, half = 1.0 + 0.5 * pr.gamma * pr.dt;
        const uint8_t mk = pc.fix[a];
        mask[a] = mk;
        Vl[a] = float(pc.Vl[a]);
        s->B[a] = float(dt / (pc.M[a] * half));
        nv4[a] = make_float4(0.f, 0.f, 0.f, s->B[a]);
        double dT0 = (mk & 8) ? pc.Tfix[a] - m.T0 : 0.0;
        nu4[a] = make_float4(0.f, 0.f, 0.f, float(dT0));
        if (mk & 8) {
            nth[a] = make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
            double x = m.ckT_on ? dt / (m.rho * pc.Vl[a]) : dt / pc.C[a];
            nth[a] = make_float4(float(x), float(pc.Kb[a]), float(pc.Qm[a] + pc.Kb[a] * (m.T_art - m.T0)),
                                 float(pc.Qr[a]));
        }
    }
    std::vector<int> new2old(nn);
    for (int64_t a = 0; a < nn; ++a) new2old[a] = int(pc.node_new2old[a]);

    TwoPassArgs &t = s->tp;
    t = TwoPassArgs{};
    t.ne = int(ne);
    t.nn = int(nn);
    const float4 *cg0, *cg1, *cg2, *chg0 = nullptr, *chg1 = nullptr, *chg2 = nullptr;
    const float *ckhg = nullptr;
    float4 *dg0 = nullptr, *dg1 = nullptr, *dg2 = nullptr, *dh0 = nullptr, *dh1 = nullptr, *dh2 = nullptr;
    float *dkhg = nullptr;
    if (s->variant != 2) {   // variant 2 rebuilds the geometry from patch-local coordinates
        TRY(upload(s, &dg0, g0)); TRY(upload(s, &dg1, g1)); TRY(upload(s, &dg2, g2));
        if (npe == 8) {
            TRY(upload(s, &dh0, h0)); TRY(upload(s, &dh1, h1)); TRY(upload(s, &dh2, h2)); TRY(upload(s, &dkhg, khg));
        }
    }
    cg0 = dg0; cg1 = dg1; cg2 = dg2; chg0 = dh0; chg1 = dh1; chg2 = dh2; ckhg = dkhg;
    float4 *dnu4, *dnv4, *dnth;
    float *dVl;
    uint8_t *dmask;
    TRY(upload(s, &dnu4, nu4)); TRY(upload(s, &dnv4, nv4)); TRY(upload(s, &dnth, nth));
    TRY(upload(s, &dVl, Vl)); TRY(upload(s, &dmask, mask));
    TRY(upload(s, &s->d_new2old, new2old));
    float *dtheta;
    s->theta_floats = size_t(6) * s->np * ne;
    TRY(zeros(s, &dtheta, std::max<size_t>(s->theta_floats, 1)));
    TRY(zeros(s, &s->d_step, 1));
    TRY(zeros(s, &s->d_status, 1));
    TRY(zeros(s, &s->d_mon, 1));

    t.g0 = cg0; t.g1 = cg1; t.g2 = cg2; t.hg0 = chg0; t.hg1 = chg1; t.hg2 = chg2; t.khg = ckhg;
    if (!aniso.empty()) {
        float4 *dan;
        TRY(upload(s, &dan, aniso));
        t.aniso = dan;
    }
    t.nu4 = dnu4; t.nv4 = dnv4; t.nth = dnth; t.mask = dmask; t.Vl = dVl; t.theta = dtheta;
    t.step_base = s->d_step;
    t.status = s->d_status;
    if (s->dose_on) {
        TRY(zeros(s, &s->d_dose, size_t(nn)));
        DoseParams &q = s->dq;
        q.T0 = s->prob.mat.T0;
        q.cem_off = 316.15 - s->prob.mat.T0;
        q.dt = s->prob.dt;
        q.dt_min = s->prob.dt / 60.0;
        q.arrhenius = s->dose_A > 0.0 ? 1 : 0;
        q.lnA = s->dose_A > 0.0 ? std::log(s->dose_A) : 0.0;
        q.EaR = s->dose_Ea / 8.314462618;
    }

    if (s->variant == 1) {
        int4 *dc0, *dc1 = nullptr;
        TRY(upload(s, &dc0, c0));
        if (npe == 8) TRY(upload(s, &dc1, c1));
        t.conn4 = dc0; t.conn4b = dc1;
        float4 *dout;
        TRY(zeros(s, &dout, size_t(ne) * npe));
        t.out = dout;
        int *drow, *dinc;
        TRY(upload(s, &drow, pc.rowptr));
        TRY(upload(s, &dinc, pc.inc));
        t.rowptr = drow; t.inc = dinc;
        s->n_elem_parts = int((ne + kBlock - 1) / kBlock);
        s->n_node_parts = int((nn + kBlock - 1) / kBlock);
        TRY(zeros(s, &s->d_part_elem, s->n_elem_parts));
        TRY(zeros(s, &s->d_part_node, size_t(4) * s->n_node_parts));
        t.part_elem = s->d_part_elem;
        t.part_node = s->d_part_node;
    } else {
        const Patches &P = pc.patches;
        PatchArgs &a = s->pa;
        a = PatchArgs{};
        a.ne = int(ne); a.n_patches = P.n; a.max_nodes = P.max_nodes; a.max_elems = P.max_elems;
        a.n_interior = int(P.n_interior); a.n_shared = int(nn - P.n_interior);
        int *d;
        TRY(upload(s, &d, P.elem_begin)); a.elem_begin = d;
        TRY(upload(s, &d, P.int_begin)); a.int_begin = d;
        TRY(upload(s, &d, P.shared_begin)); a.shared_begin = d;
        TRY(upload(s, &d, P.shared_ids)); a.shared_ids = d;
        TRY(upload(s, &d, P.lrow_begin)); a.lrow_begin = d;
        TRY(upload(s, &d, P.srow)); a.srow = d;
        TRY(upload(s, &d, P.ppos)); a.ppos = d;
        a.slot_stride = P.slot_stride;
        TRY(upload(s, &d, P.lx_begin)); a.lx_begin = d;
        float *dlx;
        TRY(upload(s, &dlx, P.lX)); a.lX = dlx;
        float2 *dfib;
        TRY(upload(s, &dfib, fib)); a.fib = dfib;
        uint16_t *u16;
        TRY(upload(s, &u16, P.lconn)); a.lconn = u16;
        TRY(upload(s, &u16, P.lrow)); a.lrow = u16;
        TRY(upload(s, &u16, P.lpos)); a.lpos = u16;
        a.nu4 = dnu4; a.nv4 = dnv4; a.nth = dnth; a.mask = dmask; a.Vl = dVl; a.theta = dtheta;
        a.g0 = cg0; a.g1 = cg1; a.g2 = cg2; a.hg0 = chg0; a.hg1 = chg1; a.hg2 = chg2; a.khg = ckhg;
        a.aniso = t.aniso;
        float4 *dpart;
        TRY(zeros(s, &dpart, std::max<size_t>(P.shared_ids.size(), 1)));
        a.partial = dpart;
        a.su_in = dnu4 + a.n_interior;
        a.sv_in = dnv4 + a.n_interior;
        s->fuse = fused_shared_nodes(s);
        if (s->fuse) {
            // per shared entry, its node's range of partials
            std::vector<int32_t> sr(2 * P.shared_ids.size());
            for (size_t q = 0; q < P.shared_ids.size(); ++q) {
                const int64_t sn = P.shared_ids[q] - P.n_interior;
                sr[2 * q] = P.srow[sn];
                sr[2 * q + 1] = P.srow[sn + 1];
            }
            int *dsr;
            TRY(upload(s, &dsr, sr));
            a.srange = reinterpret_cast<const int2 *>(dsr);
            TRY(zeros(s, &s->d_part2, P.shared_ids.size()));
            TRY(zeros(s, &s->d_sux, size_t(a.n_shared)));
            TRY(zeros(s, &s->d_svx, size_t(a.n_shared)));
        }
        a.step_base = s->d_step;
        a.status = s->d_status;
        s->n_elem_parts = P.n;
        s->n_node_parts = P.n + int((a.n_shared + kBlock - 1) / kBlock);
        if (s->queue) {
            // as many patch workgroups as are resident at once (never more than the patches);
            // the shared-node kernel's fixed grid strides over the nodes
            int cus = 0;
            HIPCHK(s, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device));
            const int occ = patch_queue_occupancy(npe, s->np, s->variant == 2, a);
            if (occ <= 0) return fail(s, TLED_E_HIP, "persistent patch kernel does not fit on a CU");
            s->q_grid = std::max(1, std::min(a.n_patches, occ * cus));
            s->q_sgrid = int(std::max<int64_t>(1, std::min<int64_t>((a.n_shared + kBlock - 1) / kBlock, 8 * cus)));
            s->n_node_parts = P.n + s->q_sgrid;
        }
        TRY(zeros(s, &s->d_part_elem, s->n_elem_parts));
        TRY(zeros(s, &s->d_part_node, size_t(4) * s->n_node_parts));
        a.part_elem = s->d_part_elem;
        a.part_node = s->d_part_node;
        // scenario tables
        const size_t S = s->scen.size();
        std::vector<long long> end(S), rng(4 * S);
        for (size_t k = 0; k < S; ++k) {
            end[k] = s->scen_steps[k];
            rng[4 * k] = s->ranges[k].int_lo; rng[4 * k + 1] = s->ranges[k].int_hi;
            rng[4 * k + 2] = s->ranges[k].sh_lo; rng[4 * k + 3] = s->ranges[k].sh_hi;
        }
        TRY(upload(s, &s->d_km, s->scen_km)); a.km = s->d_km;
        TRY(upload(s, &s->d_np, s->scen_np)); a.np = s->d_np;
        TRY(upload(s, &d, s->patch_scen)); a.patch_scen = d;
        std::vector<int32_t> shs = s->shared_scen;
        if (shs.empty()) shs.push_back(0);
        TRY(upload(s, &d, shs)); a.shared_scen = d;
        long long *dl;
        TRY(upload(s, &dl, end)); a.scen_end = dl;
        TRY(upload(s, &s->d_ranges, rng));
        TRY(zeros(s, &s->d_scen_mon, 2 * S));
        if (s->queue) {
            std::vector<long long> pe(s->pos_end.begin(), s->pos_end.end()), ps(s->pos_shared_hi.begin(),
                                                                                s->pos_shared_hi.end());
            long long *dpe, *dps;
            TRY(upload(s, &dpe, pe));
            TRY(upload(s, &dps, ps));
            TRY(upload(s, &d, s->pos_patch_hi));
            a.pos_end = dpe; a.pos_shared_hi = dps; a.pos_patch_hi = d;
            a.n_pos = int(pe.size());
            long long *dqc;
            TRY(zeros(s, &dqc, 4));
            a.qcount = dqc;
        }
    }
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return TLED_OK;
}

// Scenario tables for a single problem: one scenario covering everything, never ending.
void single_scenario(tled_sim *s) {
    s->scen.assign(1, s->prob);
    s->scen_steps.assign(1, LLONG_MAX);
    ScenRange r;
    r.elem_lo = 0; r.elem_hi = s->pc.ne;
    const int64_t nint = s->variant >= 2 ? s->pc.patches.n_interior : s->pc.nn;
    r.int_lo = 0; r.int_hi = nint; r.sh_lo = nint; r.sh_hi = s->pc.nn;
    r.patch_lo = 0; r.patch_hi = s->pc.patches.n;
    s->ranges.assign(1, r);
    s->patch_scen.assign(std::max(s->pc.patches.n, 1), 0);
    s->shared_scen.assign(std::max<int64_t>(s->pc.nn - nint, 1), 0);
}

// Patches and shared nodes to launch at step `step`.  In a batch, the scenarios
// still running form a prefix of the union (descending end steps), so a step
// launches that prefix only (at least one workgroup each, so that every launch
// exists); a single problem launches everything.
void active_counts(const tled_sim *s, int64_t step, int *n_patches, int64_t *n_shared) {
    *n_patches = s->pa.n_patches;
    *n_shared = s->pa.n_shared;
    if (!s->is_batch || s->queue || s->pos_end.empty()) return;   // the persistent kernels count on the device
    const auto it = std::partition_point(s->pos_end.begin(), s->pos_end.end(), [&](int64_t e) { return e > step; });
    const size_t m = size_t(it - s->pos_end.begin());
    // never more than the union holds (a batch may have no shared node at all)
    *n_patches = std::min(s->pa.n_patches, std::max(1, m ? s->pos_patch_hi[m - 1] : 0));
    *n_shared = std::min<int64_t>(s->pa.n_shared, std::max<int64_t>(1, m ? s->pos_shared_hi[m - 1] : 0));
}

// Persistent schedule: the running scenarios' patch and shared-node counts of
// step `step`, written into that step's parity slot (the kernels keep the slots
// current from then on).  Asynchronous on the library's stream; `h` must stay
// alive until the stream has passed the copy.
tled_status set_queue_counts(tled_sim *s, int64_t step, long long h[2]) {
    if (!s->queue) return TLED_OK;
    const auto it = std::partition_point(s->pos_end.begin(), s->pos_end.end(), [&](int64_t e) { return e > step; });
    const size_t m = size_t(it - s->pos_end.begin());
    h[0] = m ? s->pos_patch_hi[m - 1] : 0;
    h[1] = m ? s->pos_shared_hi[m - 1] : 0;
    HIPCHK(s, hipMemcpyAsync(s->pa.qcount + 2 * (step & 1), h, 2 * sizeof(long long), hipMemcpyHostToDevice,
                             s->stream));
    return TLED_OK;
}

// Enqueue a chunk of k steps (eager, or under stream capture) starting at step
// step0.  Batch: a step that reduces no monitors launches the prefix of
// scenarios still running at that step (eager) or at step0 (under capture: the
// prefix at the chunk's first step, which covers every later step of the
// chunk; scenarios ending inside the chunk exit in the kernels); the last step
// launches everything, so that every monitor partial is rewritten.
// With ev (4 events per step + 2): the element/patch and node/shared-node
// launches of step j carry the pairs (4j, 4j+1) and (4j+2, 4j+3), taken by the
// dispatches themselves; the finish kernel is bracketed by the last two.
tled_status enqueue_chunk(tled_sim *s, int k, int64_t step0, bool captured,
                          std::vector<hipEvent_t> *ev = nullptr) {
    const int npe = s->pc.npe;
    const int bs = s->opt.block_size > 0 ? s->opt.block_size : kBlock;
    for (int j = 0; j < k; ++j) {
        const bool mon = (j == k - 1);
        PatchArgs pa = s->pa;
        if (s->is_batch && !mon) {
            int np;
            int64_t ns;
            active_counts(s, captured ? step0 : step0 + j, &np, &ns);
            pa.n_patches = np;
            pa.n_shared = int(ns);
        }
        LaunchTiming t0{}, t1{};
        if (ev) {
            t0 = LaunchTiming{(*ev)[4 * j], (*ev)[4 * j + 1]};
            t1 = LaunchTiming{(*ev)[4 * j + 2], (*ev)[4 * j + 3]};
        }
        if (s->queue) {
            launch_patch_queue(npe, s->np, mon, s->variant == 2, s->pa, j, s->q_grid, s->stream, ev ? &t0 : nullptr);
            launch_shared_nodes_queue(mon, s->pa, j, s->q_sgrid, s->stream, ev ? &t1 : nullptr);
            continue;
        }
        // Fused shared nodes (chunks of two or more steps): step j > 0's patch
        // kernel first advances the shared nodes by step j - 1 from that step's
        // partials; partials and shared state alternate between two buffers
        // (state buffer 0 is the shared tail of nu4, nv4); one shared-node
        // kernel after the chunk's last step writes the shared state to nu4, nv4.
        const bool fuse = s->fuse && k >= 2;
        bool shared_launch = s->variant != 1 && pa.n_shared > 0;
        if (fuse) {
            float4 *const part[2] = {s->pa.partial, s->d_part2};
            float4 *const su[2] = {s->pa.nu4 + pa.n_interior, s->d_sux};
            float4 *const sv[2] = {s->pa.nv4 + pa.n_interior, s->d_svx};
            pa.partial = part[j & 1];
            pa.partial_prev = part[(j + 1) & 1];
            pa.su_in = su[(j + 1) & 1];
            pa.sv_in = sv[(j + 1) & 1];
            pa.su_out = su[j & 1];
            pa.sv_out = sv[j & 1];
            launch_patch(npe, s->np, mon, true, bs, false, pa, j, s->stream, ev ? &t0 : nullptr, j > 0);
            shared_launch = (j == k - 1);
            if (shared_launch) {   // reads the state this step's patch kernel stored
                pa.su_in = su[j & 1];
                pa.sv_in = sv[j & 1];
            }
        } else if (s->variant == 1) {
            launch_element(npe, s->np, mon, s->tp, s->km, s->stream, ev ? &t0 : nullptr);
        } else {
            launch_patch(npe, s->np, mon, s->variant == 2, bs, s->is_batch, pa, j, s->stream, ev ? &t0 : nullptr);
        }
        if (s->variant == 1) launch_node(mon, s->tp, s->nparams, j, s->stream, ev ? &t1 : nullptr);
        else if (shared_launch) launch_shared_nodes(mon, s->is_batch, pa, j, s->stream, ev ? &t1 : nullptr);
        else if (ev) {   // no shared-node launch at this step: the timed launch takes zero time
            HIPCHK(s, hipEventRecord(t1.start, s->stream));
            HIPCHK(s, hipEventRecord(t1.stop, s->stream));
        }
        if (s->d_dose) launch_dose(s->tp.nu4, int(s->pc.nn), s->d_dose, s->dq, s->stream);
    }
    if (ev) HIPCHK(s, hipEventRecord((*ev)[4 * size_t(k)], s->stream));
    launch_finish(s->d_part_elem, s->n_elem_parts, s->d_part_node, s->n_node_parts, s->d_step, k, s->d_status,
                  s->d_mon, s->stream);
    if (ev) HIPCHK(s, hipEventRecord((*ev)[4 * size_t(k) + 1], s->stream));
    HIPCHK(s, hipGetLastError());
    return TLED_OK;
}

constexpr size_t kMaxGraphs = 8;

// The cached graph of a k-step chunk starting at step0, or null.
hipGraphExec_t find_graph(tled_sim *s, int k, int64_t step0) {
    int np;
    int64_t ns;
    active_counts(s, step0, &np, &ns);
    for (auto &g : s->graphs)
        if (g.k == k && g.np == np && g.ns == ns) {
            g.used = ++s->graph_clock;
            return g.exec;
        }
    return nullptr;
}

tled_status build_graph(tled_sim *s, int k, int64_t step0, hipGraphExec_t *out) {
    hipGraph_t g = nullptr;
    HIPCHK(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    tled_status st = enqueue_chunk(s, k, step0, true);
    hipError_t e = hipStreamEndCapture(s->stream, &g);
    if (st != TLED_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(s, TLED_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(s, TLED_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    // move the graph's launch data to the device now, not at its first launch
    e = hipGraphUpload(exec, s->stream);
    if (e != hipSuccess) {
        (void)hipGraphExecDestroy(exec);
        return fail(s, TLED_E_HIP, std::string("hipGraphUpload: ") + hipGetErrorString(e));
    }
    if (s->graphs.size() >= kMaxGraphs) {
        auto lru = std::min_element(s->graphs.begin(), s->graphs.end(),
                                    [](const tled_sim::GraphEntry &a, const tled_sim::GraphEntry &b) {
                                        return a.used < b.used;
                                    });
        (void)hipGraphExecDestroy(lru->exec);
        s->graphs.erase(lru);
    }
    tled_sim::GraphEntry ge{exec, k, 0, 0, ++s->graph_clock};
    active_counts(s, step0, &ge.np, &ge.ns);
    s->graphs.push_back(ge);
    *out = exec;
    return TLED_OK;
}

tled_status get_graph(tled_sim *s, int k, int64_t step0, hipGraphExec_t *out) {
    *out = find_graph(s, k, step0);
    return *out ? TLED_OK : build_graph(s, k, step0, out);
}

tled_status check_status(tled_sim *s) {
    unsigned flags = 0;
    HIPCHK(s, hipMemcpyAsync(&flags, s->d_status, sizeof(unsigned), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    if (flags) {
        std::string m = "device raised";
        if (flags & TLED_FLAG_NONFINITE) m += " non-finite values";
        if (flags & TLED_FLAG_INVERTED) m += " inverted elements (det F <= 0)";
        return fail(s, TLED_E_UNSTABLE, m);
    }
    return TLED_OK;
}

// LDS a patch workgroup may take: the device's per-workgroup limit less 1 KiB
// for the kernels' static reduction arrays (host-only handles assume 64 KiB).
tled_status patch_lds_limit(tled_sim *s, size_t *lim) {
    int v = 65536;
    if (s->device >= 0) HIPCHK(s, hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, s->device));
    *lim = size_t(v) - 1024;
    return TLED_OK;
}

tled_status need_device(tled_sim *s) {
    if (!s) return TLED_E_ARG;
    if (!s->finalized) return fail(s, TLED_E_STATE, "call tled_finalize first");
    if (s->device < 0) return fail(s, TLED_E_STATE, "host-only handle has no device state");
    HIPCHK(s, hipSetDevice(s->device));
    return TLED_OK;
}

tled_status need_single(tled_sim *s) {
    TRY(need_device(s));
    if (s->is_batch) return fail(s, TLED_E_STATE, "batch handle: use the tled_batch_* reads");
    return TLED_OK;
}

tled_status need_setup(tled_sim *s) {
    if (!s) return TLED_E_ARG;
    if (s->finalized) return fail(s, TLED_E_STATE, "problem already finalized");
    return TLED_OK;
}

tled_status need_single_setup(tled_sim *s) {
    TRY(need_setup(s));
    if (s->is_batch) return fail(s, TLED_E_STATE, "batch handle: use tled_batch_add");
    return TLED_OK;
}

}  // namespace

extern "C" {

const char *tled_status_string(tled_status s) {
    switch (s) {
        case TLED_OK: return "ok";
        case TLED_E_ARG: return "invalid argument";
        case TLED_E_MESH: return "invalid mesh";
        case TLED_E_STATE: return "call out of order";
        case TLED_E_HIP: return "HIP runtime error";
        case TLED_E_OOM: return "out of memory";
        case TLED_E_UNSTABLE: return "unstable (non-finite values or inverted elements)";
        case TLED_E_UNSUPPORTED: return "unsupported option";
    }
    return "unknown status";
}

const char *tled_last_error(const tled_sim *sim) { return sim ? sim->err.c_str() : "null handle"; }

tled_status tled_create(tled_sim **out, int device) {
    if (!out) return TLED_E_ARG;
    *out = nullptr;
    tled_sim *s = new (std::nothrow) tled_sim();
    if (!s) return TLED_E_OOM;
    s->opt.graph_steps = 50;
    s->device = device;
    if (device >= 0) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess || device >= n) {
            delete s;
            return e != hipSuccess ? TLED_E_HIP : TLED_E_ARG;
        }
        if (hipSetDevice(device) != hipSuccess) {
            delete s;
            return TLED_E_HIP;
        }
    } else if (device != -1) {
        delete s;
        return TLED_E_ARG;
    }
    *out = s;
    return TLED_OK;
}

void tled_destroy(tled_sim *sim) {
    if (!sim) return;
    if (sim->device >= 0) {
        (void)hipSetDevice(sim->device);
        if (sim->stream) (void)hipStreamSynchronize(sim->stream);
        free_device(sim);
        if (sim->own_stream && sim->stream) (void)hipStreamDestroy(sim->stream);
    }
    delete sim;
}

tled_status tled_set_allocator(tled_sim *sim, void *(*alloc)(size_t, void *), void (*release)(void *, void *),
                               void *ctx) {
    TRY(need_setup(sim));
    if ((alloc == nullptr) != (release == nullptr)) return fail(sim, TLED_E_ARG, "allocator needs both functions");
    sim->alloc = alloc;
    sim->release = release;
    sim->actx = ctx;
    return TLED_OK;
}

tled_status tled_set_stream(tled_sim *sim, void *hip_stream) {
    TRY(need_setup(sim));
    sim->stream = static_cast<hipStream_t>(hip_stream);
    sim->own_stream = false;
    return TLED_OK;
}

tled_status tled_set_options(tled_sim *sim, const tled_options *opt) {
    if (!sim || !opt) return TLED_E_ARG;
    if (opt->kernel_variant < 0 || opt->kernel_variant > 3) return fail(sim, TLED_E_ARG, "kernel_variant must be 0..3");
    if (opt->patch_elems < 0 || opt->patch_elems > 4096) return fail(sim, TLED_E_ARG, "patch_elems out of range");
    if (opt->reorder < -1 || opt->reorder > 2) return fail(sim, TLED_E_ARG, "reorder must be -1..2");
    if (opt->block_size != 0 && opt->block_size != 256 && opt->block_size != 512)
        return fail(sim, TLED_E_UNSUPPORTED, "block_size must be 256 or 512");
    if (opt->batch_schedule < 0 || opt->batch_schedule > 1) return fail(sim, TLED_E_ARG, "batch_schedule must be 0 or 1");
    if (opt->batch_schedule == 1 && !sim->is_batch)
        return fail(sim, TLED_E_ARG, "batch_schedule 1 (persistent) is for batch handles");
    if (opt->shared_update < 0 || opt->shared_update > 2) return fail(sim, TLED_E_ARG, "shared_update must be 0..2");
    if (sim->finalized && (opt->kernel_variant != sim->opt.kernel_variant || opt->reorder != sim->opt.reorder ||
                           opt->patch_elems != sim->opt.patch_elems || opt->batch_schedule != sim->opt.batch_schedule ||
                           opt->block_size != sim->opt.block_size || opt->shared_update != sim->opt.shared_update))
        return fail(sim, TLED_E_STATE, "layout options must be set before tled_finalize");
    sim->opt = *opt;
    if (sim->opt.graph_steps == 0) sim->opt.graph_steps = !sim->is_batch ? 50 : (sim->opt.batch_schedule == 1 ? 100 : -1);
    // captured graphs hold the kernel constants by value: capture again
    if (sim->finalized) drop_graphs(sim);
    if (sim->finalized) {
        build_kernel_constants(sim);
        if (sim->device >= 0 && sim->d_km) {
            HIPCHK(sim, hipMemcpyAsync(sim->d_km, sim->scen_km.data(), sizeof(KMat) * sim->scen_km.size(),
                                       hipMemcpyHostToDevice, sim->stream));
            HIPCHK(sim, hipMemcpyAsync(sim->d_np, sim->scen_np.data(), sizeof(NodeParams) * sim->scen_np.size(),
                                       hipMemcpyHostToDevice, sim->stream));
            HIPCHK(sim, hipStreamSynchronize(sim->stream));
        }
    }
    return TLED_OK;
}

tled_status tled_set_mesh(tled_sim *sim, int elem_type, int64_t n_nodes, const double *X, int64_t n_elems,
                          const int32_t *conn) {
    TRY(need_single_setup(sim));
    if (elem_type != TLED_T4 && elem_type != TLED_H8) return fail(sim, TLED_E_ARG, "elem_type must be 4 or 8");
    if (n_nodes <= 0 || n_elems <= 0 || !X || !conn) return fail(sim, TLED_E_ARG, "empty mesh or null array");
    if (n_nodes > (int64_t(1) << 30) || n_elems * elem_type > INT_MAX)
        return fail(sim, TLED_E_ARG, "mesh exceeds 32-bit index range");
    HostProblem &p = sim->prob;
    p.npe = elem_type;
    p.nn = n_nodes;
    p.ne = n_elems;
    p.X.assign(X, X + 3 * n_nodes);
    for (int64_t i = 0; i < 3 * n_nodes; ++i)
        if (!std::isfinite(p.X[i])) return fail(sim, TLED_E_ARG, "non-finite coordinate");
    p.conn.assign(conn, conn + elem_type * n_elems);
    p.a0.clear();
    p.n0.clear();
    p.Dc.clear();
    p.q.clear();
    p.fix.assign(n_nodes, 0);
    p.Tfix.assign(n_nodes, 0.0);
    p.have_mesh = true;
    return TLED_OK;
}

tled_status tled_set_material(tled_sim *sim, const tled_material *m) {
    TRY(need_single_setup(sim));
    if (!m) return fail(sim, TLED_E_ARG, "null material");
    sim->prob.mat = *m;
    sim->prob.have_mat = true;
    return TLED_OK;
}

tled_status tled_set_fibres(tled_sim *sim, const double *a0) {
    TRY(need_single_setup(sim));
    if (!sim->prob.have_mesh) return fail(sim, TLED_E_STATE, "set the mesh first");
    if (!a0) { sim->prob.a0.clear(); return TLED_OK; }
    sim->prob.a0.assign(a0, a0 + 3 * sim->prob.ne);
    return TLED_OK;
}

tled_status tled_set_expansion_axes(tled_sim *sim, const double *n0) {
    TRY(need_single_setup(sim));
    if (!sim->prob.have_mesh) return fail(sim, TLED_E_STATE, "set the mesh first");
    if (!n0) { sim->prob.n0.clear(); return TLED_OK; }
    sim->prob.n0.assign(n0, n0 + 3 * sim->prob.ne);
    for (double v : sim->prob.n0)
        if (!std::isfinite(v)) { sim->prob.n0.clear(); return fail(sim, TLED_E_ARG, "non-finite expansion axis"); }
    return TLED_OK;
}

tled_status tled_set_conductivity(tled_sim *sim, const double *D) {
    TRY(need_single_setup(sim));
    if (!sim->prob.have_mesh) return fail(sim, TLED_E_STATE, "set the mesh first");
    if (!D) { sim->prob.Dc.clear(); return TLED_OK; }
    sim->prob.Dc.assign(D, D + 6 * sim->prob.ne);
    return TLED_OK;
}

tled_status tled_set_fixed_dofs(tled_sim *sim, int64_t n, const int32_t *node, const uint8_t *mask) {
    TRY(need_single_setup(sim));
    if (!sim->prob.have_mesh) return fail(sim, TLED_E_STATE, "set the mesh first");
    if (n < 0 || (n > 0 && (!node || !mask))) return fail(sim, TLED_E_ARG, "bad fixed-dof arrays");
    for (int64_t i = 0; i < n; ++i) {
        if (node[i] < 0 || node[i] >= sim->prob.nn) return fail(sim, TLED_E_ARG, "fixed node out of range");
        sim->prob.fix[node[i]] |= uint8_t(mask[i] & 7);
    }
    return TLED_OK;
}

tled_status tled_set_fixed_temperature(tled_sim *sim, int64_t n, const int32_t *node, const double *T) {
    TRY(need_single_setup(sim));
    if (!sim->prob.have_mesh) return fail(sim, TLED_E_STATE, "set the mesh first");
    if (n < 0 || (n > 0 && (!node || !T))) return fail(sim, TLED_E_ARG, "bad fixed-temperature arrays");
    for (int64_t i = 0; i < n; ++i) {
        if (node[i] < 0 || node[i] >= sim->prob.nn) return fail(sim, TLED_E_ARG, "fixed node out of range");
        if (!std::isfinite(T[i])) return fail(sim, TLED_E_ARG, "non-finite fixed temperature");
        sim->prob.fix[node[i]] |= 8;
        sim->prob.Tfix[node[i]] = T[i];
    }
    return TLED_OK;
}

tled_status tled_set_heat_source(tled_sim *sim, const double *q_elem, double t_on, double t_off) {
    TRY(need_single_setup(sim));
    if (!sim->prob.have_mesh) return fail(sim, TLED_E_STATE, "set the mesh first");
    if (std::isnan(t_on) || std::isnan(t_off)) return fail(sim, TLED_E_ARG, "NaN source window");
    if (q_elem) {
        sim->prob.q.assign(q_elem, q_elem + sim->prob.ne);
        for (double v : sim->prob.q)
            if (!std::isfinite(v)) return fail(sim, TLED_E_ARG, "non-finite source");
    } else {
        sim->prob.q.clear();
    }
    sim->prob.t_on = t_on;
    sim->prob.t_off = t_off;
    return TLED_OK;
}

tled_status tled_set_time(tled_sim *sim, double dt, double damping_gamma) {
    TRY(need_single_setup(sim));
    if (!(dt > 0.0) || !std::isfinite(dt) || !(damping_gamma >= 0.0) || !std::isfinite(damping_gamma))
        return fail(sim, TLED_E_ARG, "dt must be > 0 and gamma >= 0");
    if (0.5 * damping_gamma * dt >= 1.0) return fail(sim, TLED_E_ARG, "gamma * dt / 2 must stay below 1");
    sim->prob.dt = dt;
    sim->prob.gamma = damping_gamma;
    sim->prob.have_time = true;
    return TLED_OK;
}

tled_status tled_set_thermal_dose(tled_sim *sim, double arrhenius_A, double arrhenius_Ea) {
    if (!sim) return TLED_E_ARG;
    if (sim->is_batch) return fail(sim, TLED_E_UNSUPPORTED, "the thermal dose is for single problems");
    TRY(need_single_setup(sim));
    if (!(arrhenius_A >= 0.0) || !std::isfinite(arrhenius_A) || !(arrhenius_Ea >= 0.0) || !std::isfinite(arrhenius_Ea))
        return fail(sim, TLED_E_ARG, "Arrhenius A and Ea must be finite and >= 0");
    sim->dose_on = true;
    sim->dose_A = arrhenius_A;
    sim->dose_Ea = arrhenius_Ea;
    return TLED_OK;
}

tled_status tled_critical_dt(tled_sim *sim, double *dt_cr) {
    if (!sim || !dt_cr) return TLED_E_ARG;
    if (sim->finalized) {
        *dt_cr = sim->pc.dt_cr;
        return TLED_OK;
    }
    return critical_dt(sim->prob, dt_cr, &sim->err);
}

tled_status tled_finalize(tled_sim *sim) {
    TRY(need_single_setup(sim));
    if (!sim->prob.have_time) return fail(sim, TLED_E_STATE, "call tled_set_time first");
    int v = sim->opt.kernel_variant == 0 ? default_variant(sim->prob.npe) : sim->opt.kernel_variant;
    SetupOptions so;
    so.reorder = sim->opt.reorder >= 0;
    so.bisect = sim->opt.reorder != 2;
    so.build_patches = (v >= 2);
    so.threads = host_threads();
    so.patch_elems = sim->opt.patch_elems > 0
                         ? sim->opt.patch_elems
                         : default_patch_elems(sim->prob.npe, sim->prob.ne, sim->opt.block_size);
    if (sim->opt.block_size == 512 && sim->prob.npe == 8)
        return fail(sim, TLED_E_UNSUPPORTED, "block_size 512 is for T4 meshes only");
    if (sim->opt.block_size == 512 && (sim->prob.mat.expan_mode == 2 || sim->prob.mat.cond_mode == 2))
        return fail(sim, TLED_E_UNSUPPORTED,
                    "block_size 512 is not available with orthotropic expansion or tensor conduction");
    tled_status st = precompute(sim->prob, so, &sim->pc, &sim->err);
    if (st != TLED_OK) return st;
    if (sim->prob.dt > sim->pc.dt_cr)
        return fail(sim, TLED_E_ARG, "dt exceeds the critical time step " + std::to_string(sim->pc.dt_cr));
    if (sim->prob.dt > sim->pc.dt_th)
        return fail(sim, TLED_E_ARG, "dt exceeds the explicit thermal stability limit " +
                                         std::to_string(sim->pc.dt_th));
    sim->variant = v;
    if (v >= 2) {
        PatchArgs probe{};
        probe.max_nodes = sim->pc.patches.max_nodes;
        probe.max_elems = sim->pc.patches.max_elems;
        size_t lim = 0;
        TRY(patch_lds_limit(sim, &lim));
        if (patch_lds_bytes(sim->prob.npe, v == 2, probe) > lim)
            return fail(sim, TLED_E_ARG, "patch too large for LDS; lower patch_elems");
    }
    single_scenario(sim);
    build_kernel_constants(sim);
    if (sim->device >= 0) {
        HIPCHK(sim, hipSetDevice(sim->device));
        if (!sim->stream) {
            HIPCHK(sim, hipStreamCreateWithFlags(&sim->stream, hipStreamNonBlocking));
            sim->own_stream = true;
        }
        st = upload_all(sim);
        if (st != TLED_OK) {
            free_device(sim);
            return st;
        }
    }
    sim->step = 0;
    sim->finalized = true;
    return TLED_OK;
}

tled_status tled_step(tled_sim *sim, int64_t n_steps) {
    TRY(need_device(sim));
    if (n_steps < 0) return fail(sim, TLED_E_ARG, "negative step count");
    const int k = sim->opt.graph_steps;
    int64_t left = n_steps, cur = sim->step;
    if (k > 0) {
        while (left >= k) {
            // a batch's graph launches the prefix of scenarios running at its
            // first step: captured again when that prefix has changed
            hipGraphExec_t g;
            TRY(get_graph(sim, k, cur, &g));
            HIPCHK(sim, hipGraphLaunch(g, sim->stream));
            left -= k;
            cur += k;
        }
        // a shorter last chunk replays a graph of its length when one is cached
        // (tled_prepare_steps captures it), else it is enqueued eagerly
        if (left > 0) {
            if (hipGraphExec_t g = find_graph(sim, int(left), cur)) {
                HIPCHK(sim, hipGraphLaunch(g, sim->stream));
                cur += left;
                left = 0;
            }
        }
    }
    const int chunk = k > 0 ? k : 100;
    while (left > 0) {
        int c = int(std::min<int64_t>(left, chunk));
        TRY(enqueue_chunk(sim, c, cur, false));
        left -= c;
        cur += c;
    }
    sim->step += n_steps;
    return TLED_OK;
}

tled_status tled_prepare_steps(tled_sim *sim, int64_t n_steps) {
    TRY(need_device(sim));
    if (n_steps < 0) return fail(sim, TLED_E_ARG, "negative step count");
    const int k = sim->opt.graph_steps;
    if (k <= 0 || n_steps == 0) return TLED_OK;
    hipGraphExec_t g;
    const int64_t full = n_steps / k, rest = n_steps % k;
    int64_t cur = sim->step;
    if (full > 0) TRY(get_graph(sim, k, cur, &g));
    if (rest > 0) {
        // a batch's prefix may differ at the last chunk: capture at the step it starts
        TRY(get_graph(sim, int(rest), cur + full * k, &g));
    }
    return TLED_OK;
}

tled_status tled_sync(tled_sim *sim) {
    TRY(need_device(sim));
    HIPCHK(sim, hipStreamSynchronize(sim->stream));
    return check_status(sim);
}

tled_status tled_read_u(tled_sim *sim, double *u) {
    TRY(need_single(sim));
    if (!u) return fail(sim, TLED_E_ARG, "null output");
    const int64_t nn = sim->pc.nn;
    std::vector<float4> h(nn);
    HIPCHK(sim, hipMemcpyAsync(h.data(), sim->tp.nu4, sizeof(float4) * nn, hipMemcpyDeviceToHost, sim->stream));
    HIPCHK(sim, hipStreamSynchronize(sim->stream));
    for (int64_t a = 0; a < nn; ++a) {
        int64_t o = sim->pc.node_new2old[a];
        u[3 * o] = h[a].x; u[3 * o + 1] = h[a].y; u[3 * o + 2] = h[a].z;
    }
    return check_status(sim);
}

tled_status tled_read_T(tled_sim *sim, double *T) {
    TRY(need_single(sim));
    if (!T) return fail(sim, TLED_E_ARG, "null output");
    const int64_t nn = sim->pc.nn;
    std::vector<float4> h(nn);
    HIPCHK(sim, hipMemcpyAsync(h.data(), sim->tp.nu4, sizeof(float4) * nn, hipMemcpyDeviceToHost, sim->stream));
    HIPCHK(sim, hipStreamSynchronize(sim->stream));
    const double T0 = sim->prob.mat.T0;
    for (int64_t a = 0; a < nn; ++a) T[sim->pc.node_new2old[a]] = T0 + double(h[a].w);
    return check_status(sim);
}

tled_status tled_read_thermal_dose(tled_sim *sim, double *cem43, double *omega) {
    TRY(need_single(sim));
    if (!sim->dose_on) return fail(sim, TLED_E_STATE, "the thermal dose was not enabled before finalize");
    const int64_t nn = sim->pc.nn;
    std::vector<double2> h(nn);
    HIPCHK(sim, hipMemcpyAsync(h.data(), sim->d_dose, sizeof(double2) * nn, hipMemcpyDeviceToHost, sim->stream));
    HIPCHK(sim, hipStreamSynchronize(sim->stream));
    for (int64_t a = 0; a < nn; ++a) {
        const int64_t o = sim->pc.node_new2old[a];
        if (cem43) cem43[o] = h[a].x;
        if (omega) omega[o] = h[a].y;
    }
    return check_status(sim);
}

tled_status tled_copy_fields_device(tled_sim *sim, float *u_dst, float *T_dst) {
    TRY(need_single(sim));
    launch_export_fields(sim->tp.nu4, sim->d_new2old, int(sim->pc.nn), float(sim->prob.mat.T0), u_dst, T_dst,
                         sim->stream);
    HIPCHK(sim, hipGetLastError());
    return TLED_OK;
}

tled_status tled_get_monitors(tled_sim *sim, tled_monitors *out) {
    TRY(need_device(sim));
    if (!out) return fail(sim, TLED_E_ARG, "null output");
    DevMonitors m{};
    HIPCHK(sim, hipMemcpyAsync(&m, sim->d_mon, sizeof(m), hipMemcpyDeviceToHost, sim->stream));
    HIPCHK(sim, hipStreamSynchronize(sim->stream));
    std::memset(out, 0, sizeof(*out));
    out->step = m.step;
    out->t = double(m.step) * sim->prob.dt;
    out->kinetic = m.kinetic;
    out->strain = m.strain;
    out->T_max = m.T_max;
    out->T_min = m.T_min;
    out->ablated_volume = m.ablated;
    out->flags = m.flags;
    return check_status(sim);
}

tled_status tled_get_info(tled_sim *sim, tled_info *out) {
    if (!sim || !out) return TLED_E_ARG;
    std::memset(out, 0, sizeof(*out));
    out->n_nodes = sim->prob.nn;
    out->n_elems = sim->prob.ne;
    out->elem_type = sim->prob.npe;
    out->n_prony = sim->prob.mat.n_prony;
    out->dt = sim->prob.dt;
    if (sim->finalized) {
        out->n_swapped = sim->pc.n_swapped;
        out->kernel_variant = sim->variant;
        const bool fused = sim->variant >= 2;
        out->n_patches = fused ? sim->pc.patches.n : 0;
        out->n_shared_nodes = fused ? sim->pc.nn - sim->pc.patches.n_interior : 0;
        out->patch_max_nodes = fused ? sim->pc.patches.max_nodes : 0;
        if (fused) {
            PatchArgs probe{};
            probe.max_nodes = sim->pc.patches.max_nodes;
            probe.max_elems = sim->pc.patches.max_elems;
            out->patch_lds_bytes = int32_t(patch_lds_bytes(sim->prob.npe, sim->variant == 2, probe));
            const bool fs = fused_shared_nodes(sim);
            if (sim->device >= 0) {
                const int bs = sim->opt.block_size > 0 ? sim->opt.block_size : kBlock;
                out->patch_wgs_per_cu =
                    patch_occupancy(sim->prob.npe, sim->np, sim->variant == 2, bs, sim->is_batch, probe, fs);
            }
            if (out->n_shared_nodes > 0) out->shared_update = fs ? 1 : 2;
        }
        out->device_bytes = sim->device_bytes;
        out->dt_critical = sim->pc.dt_cr;
        out->dt_thermal = sim->pc.dt_th;
    }
    return TLED_OK;
}

tled_status tled_get_lumped(tled_sim *sim, double *Vl, double *M, double *C, double *Kb, double *Qm, double *Qr) {
    if (!sim) return TLED_E_ARG;
    if (sim->is_batch) return fail(sim, TLED_E_STATE, "not available on a batch handle");
    if (!sim->finalized) return fail(sim, TLED_E_STATE, "call tled_finalize first");
    const Precomputed &pc = sim->pc;
    for (int64_t a = 0; a < pc.nn; ++a) {
        int64_t o = pc.node_new2old[a];
        if (Vl) Vl[o] = pc.Vl[a];
        if (M) M[o] = pc.M[a];
        if (C) C[o] = pc.C[a];
        if (Kb) Kb[o] = pc.Kb[a];
        if (Qm) Qm[o] = pc.Qm[a];
        if (Qr) Qr[o] = pc.Qr[a];
    }
    return TLED_OK;
}

// Position of Prony component c (0 .. 6 np - 1) of internal element e in the
// device array: float4 planes of components 4k..4k+3, then a float2 plane.
static size_t theta_index(int c, int64_t e, int64_t ne, int np) {
    const int n4 = 6 * np / 4;
    if (c < 4 * n4) return size_t(c / 4) * 4 * size_t(ne) + 4 * size_t(e) + size_t(c % 4);
    return 4 * size_t(n4) * size_t(ne) + 2 * size_t(e) + size_t(c - 4 * n4);
}

tled_status tled_read_state(tled_sim *sim, double *u, double *v, double *T, double *theta, int64_t *step) {
    TRY(need_single(sim));
    const int64_t nn = sim->pc.nn, ne = sim->pc.ne;
    std::vector<float4> hu(nn), hv(nn);
    std::vector<float> ht(sim->theta_floats);
    HIPCHK(sim, hipMemcpyAsync(hu.data(), sim->tp.nu4, sizeof(float4) * nn, hipMemcpyDeviceToHost, sim->stream));
    HIPCHK(sim, hipMemcpyAsync(hv.data(), sim->tp.nv4, sizeof(float4) * nn, hipMemcpyDeviceToHost, sim->stream));
    if (!ht.empty())
        HIPCHK(sim, hipMemcpyAsync(ht.data(), sim->tp.theta, sizeof(float) * ht.size(), hipMemcpyDeviceToHost,
                                   sim->stream));
    long long st = 0;
    HIPCHK(sim, hipMemcpyAsync(&st, sim->d_step, sizeof(st), hipMemcpyDeviceToHost, sim->stream));
    HIPCHK(sim, hipStreamSynchronize(sim->stream));
    const double T0 = sim->prob.mat.T0;
    for (int64_t a = 0; a < nn; ++a) {
        int64_t o = sim->pc.node_new2old[a];
        if (u) { u[3 * o] = hu[a].x; u[3 * o + 1] = hu[a].y; u[3 * o + 2] = hu[a].z; }
        if (v) { v[3 * o] = hv[a].x; v[3 * o + 1] = hv[a].y; v[3 * o + 2] = hv[a].z; }
        if (T) T[o] = T0 + double(hu[a].w);
    }
    const int np = sim->np;
    if (theta)
        for (int64_t e = 0; e < ne; ++e) {
            int64_t o = sim->pc.elem_new2old[e];
            for (int k = 0; k < 6 * np; ++k) theta[6 * np * o + k] = ht[theta_index(k, e, ne, np)];
        }
    if (step) *step = st;
    return TLED_OK;
}

tled_status tled_write_state(tled_sim *sim, const double *u, const double *v, const double *T, const double *theta,
                             int64_t step) {
    TRY(need_single(sim));
    if (step < 0) return fail(sim, TLED_E_ARG, "negative step");
    const int64_t nn = sim->pc.nn, ne = sim->pc.ne;
    std::vector<float4> hu(nn), hv(nn);
    std::vector<float> ht(sim->theta_floats);
    HIPCHK(sim, hipMemcpyAsync(hu.data(), sim->tp.nu4, sizeof(float4) * nn, hipMemcpyDeviceToHost, sim->stream));
    HIPCHK(sim, hipMemcpyAsync(hv.data(), sim->tp.nv4, sizeof(float4) * nn, hipMemcpyDeviceToHost, sim->stream));
    if (!ht.empty())
        HIPCHK(sim, hipMemcpyAsync(ht.data(), sim->tp.theta, sizeof(float) * ht.size(), hipMemcpyDeviceToHost,
                                   sim->stream));
    HIPCHK(sim, hipStreamSynchronize(sim->stream));
    const double T0 = sim->prob.mat.T0;
    for (int64_t a = 0; a < nn; ++a) {
        int64_t o = sim->pc.node_new2old[a];
        const uint8_t mk = sim->pc.fix[a];
        if (u) hu[a] = make_float4(float(u[3 * o]), float(u[3 * o + 1]), float(u[3 * o + 2]), hu[a].w);
        if (v) hv[a] = make_float4(float(v[3 * o]), float(v[3 * o + 1]), float(v[3 * o + 2]), sim->B[a]);
        if (T) hu[a].w = float(T[o] - T0);
        if (mk & 1) { hu[a].x = 0.f; hv[a].x = 0.f; }
        if (mk & 2) { hu[a].y = 0.f; hv[a].y = 0.f; }
        if (mk & 4) { hu[a].z = 0.f; hv[a].z = 0.f; }
        if (mk & 8) hu[a].w = float(sim->pc.Tfix[a] - T0);
    }
    const int np = sim->np;
    if (theta)
        for (int64_t e = 0; e < ne; ++e) {
            int64_t o = sim->pc.elem_new2old[e];
            for (int k = 0; k < 6 * np; ++k) ht[theta_index(k, e, ne, np)] = float(theta[6 * np * o + k]);
        }
    long long st = step;
    HIPCHK(sim, hipMemcpyAsync(sim->tp.nu4, hu.data(), sizeof(float4) * nn, hipMemcpyHostToDevice, sim->stream));
    HIPCHK(sim, hipMemcpyAsync(sim->tp.nv4, hv.data(), sizeof(float4) * nn, hipMemcpyHostToDevice, sim->stream));
    if (!ht.empty())
        HIPCHK(sim, hipMemcpyAsync(sim->tp.theta, ht.data(), sizeof(float) * ht.size(), hipMemcpyHostToDevice,
                                   sim->stream));
    HIPCHK(sim, hipMemcpyAsync(sim->d_step, &st, sizeof(st), hipMemcpyHostToDevice, sim->stream));
    HIPCHK(sim, hipStreamSynchronize(sim->stream));
    sim->step = step;
    return TLED_OK;
}

tled_status tled_state_size(tled_sim *sim, size_t *bytes) {
    TRY(need_device(sim));
    if (!bytes) return fail(sim, TLED_E_ARG, "null output");
    *bytes = 64 + sizeof(float4) * 2 * size_t(sim->pc.nn) + sizeof(float) * sim->theta_floats +
             (sim->dose_on ? sizeof(double2) * size_t(sim->pc.nn) : 0);
    return TLED_OK;
}

tled_status tled_get_state(tled_sim *sim, void *buf) {
    TRY(need_device(sim));
    if (!buf) return fail(sim, TLED_E_ARG, "null buffer");
    char *b = static_cast<char *>(buf);
    const size_t nn = sim->pc.nn;
    uint64_t hdr[8] = {kStateMagic, uint64_t(sim->pc.nn), uint64_t(sim->pc.ne), uint64_t(sim->np),
                       uint64_t(sim->variant), 0, 0, uint64_t(sim->dose_on ? 1 : 0)};
    long long st = 0;
    HIPCHK(sim, hipMemcpyAsync(&st, sim->d_step, sizeof(st), hipMemcpyDeviceToHost, sim->stream));
    unsigned status = 0;
    HIPCHK(sim, hipMemcpyAsync(&status, sim->d_status, sizeof(status), hipMemcpyDeviceToHost, sim->stream));
    HIPCHK(sim, hipMemcpyAsync(b + 64, sim->tp.nu4, sizeof(float4) * nn, hipMemcpyDeviceToHost, sim->stream));
    HIPCHK(sim, hipMemcpyAsync(b + 64 + sizeof(float4) * nn, sim->tp.nv4, sizeof(float4) * nn, hipMemcpyDeviceToHost,
                               sim->stream));
    if (sim->theta_floats)
        HIPCHK(sim, hipMemcpyAsync(b + 64 + 2 * sizeof(float4) * nn, sim->tp.theta, sizeof(float) * sim->theta_floats,
                                   hipMemcpyDeviceToHost, sim->stream));
    if (sim->dose_on)
        HIPCHK(sim, hipMemcpyAsync(b + 64 + 2 * sizeof(float4) * nn + sizeof(float) * sim->theta_floats, sim->d_dose,
                                   sizeof(double2) * nn, hipMemcpyDeviceToHost, sim->stream));
    HIPCHK(sim, hipStreamSynchronize(sim->stream));
    hdr[5] = uint64_t(st);
    hdr[6] = status;
    std::memcpy(b, hdr, sizeof(hdr));
    return TLED_OK;
}

tled_status tled_set_state(tled_sim *sim, const void *buf) {
    TRY(need_device(sim));
    if (!buf) return fail(sim, TLED_E_ARG, "null buffer");
    const char *b = static_cast<const char *>(buf);
    uint64_t hdr[8];
    std::memcpy(hdr, b, sizeof(hdr));
    if (hdr[0] != kStateMagic || hdr[1] != uint64_t(sim->pc.nn) || hdr[2] != uint64_t(sim->pc.ne) ||
        hdr[3] != uint64_t(sim->np) || hdr[4] != uint64_t(sim->variant) || hdr[7] != uint64_t(sim->dose_on ? 1 : 0))
        return fail(sim, TLED_E_ARG, "state blob does not match this problem");
    const size_t nn = sim->pc.nn;
    long long st = (long long)hdr[5];
    unsigned status = unsigned(hdr[6]);
    HIPCHK(sim, hipMemcpyAsync(sim->tp.nu4, b + 64, sizeof(float4) * nn, hipMemcpyHostToDevice, sim->stream));
    HIPCHK(sim, hipMemcpyAsync(sim->tp.nv4, b + 64 + sizeof(float4) * nn, sizeof(float4) * nn, hipMemcpyHostToDevice,
                               sim->stream));
    if (sim->theta_floats)
        HIPCHK(sim, hipMemcpyAsync(sim->tp.theta, b + 64 + 2 * sizeof(float4) * nn, sizeof(float) * sim->theta_floats,
                                   hipMemcpyHostToDevice, sim->stream));
    if (sim->dose_on)
        HIPCHK(sim, hipMemcpyAsync(sim->d_dose, b + 64 + 2 * sizeof(float4) * nn + sizeof(float) * sim->theta_floats,
                                   sizeof(double2) * nn, hipMemcpyHostToDevice, sim->stream));
    HIPCHK(sim, hipMemcpyAsync(sim->d_step, &st, sizeof(st), hipMemcpyHostToDevice, sim->stream));
    HIPCHK(sim, hipMemcpyAsync(sim->d_status, &status, sizeof(status), hipMemcpyHostToDevice, sim->stream));
    long long qc[2];
    TRY(set_queue_counts(sim, st, qc));
    HIPCHK(sim, hipStreamSynchronize(sim->stream));
    sim->step = st;
    return TLED_OK;
}

// ------------------------------------------------------------------ batched scenarios

tled_status tled_batch_create(tled_batch **out, int device) {
    TRY(tled_create(out, device));
    (*out)->is_batch = true;
    (*out)->opt.graph_steps = -1;   // batches: eager steps, each launching exactly the running scenarios
    return TLED_OK;
}

void tled_batch_destroy(tled_batch *b) { tled_destroy(b); }

tled_status tled_batch_add(tled_batch *b, int elem_type, int64_t n_nodes, const double *X, int64_t n_elems,
                           const int32_t *conn, const tled_material *m, const double *a0, const double *q_elem,
                           double t_on, double t_off, int64_t n_fixed, const int32_t *fixed_nodes,
                           const uint8_t *fixed_mask, double dt, double damping_gamma, int64_t n_steps,
                           int32_t patch_elems, int32_t *index) {
    TRY(need_setup(b));
    if (!b->is_batch) return fail(b, TLED_E_STATE, "not a batch handle");
    if (elem_type != TLED_T4 && elem_type != TLED_H8) return fail(b, TLED_E_ARG, "elem_type must be 4 or 8");
    if (n_nodes <= 0 || n_elems <= 0 || !X || !conn || !m) return fail(b, TLED_E_ARG, "empty mesh or null array");
    if (n_nodes > (int64_t(1) << 30) || n_elems * elem_type > INT_MAX) return fail(b, TLED_E_ARG, "mesh too large");
    if (!(dt >= 0.0) || !std::isfinite(dt) || !(damping_gamma >= 0.0) || 0.5 * damping_gamma * dt >= 1.0)
        return fail(b, TLED_E_ARG, "dt must be >= 0, gamma >= 0, gamma dt / 2 < 1");
    if (n_steps < 0) return fail(b, TLED_E_ARG, "negative step count");
    if (patch_elems < 0 || patch_elems > 4096) return fail(b, TLED_E_ARG, "patch_elems out of range");
    if (std::isnan(t_on) || std::isnan(t_off)) return fail(b, TLED_E_ARG, "NaN source window");
    if (!b->scen.empty() && b->scen[0].npe != elem_type) return fail(b, TLED_E_ARG, "a batch needs one element type");
    if (!b->scen.empty() && b->scen[0].mat.n_prony != m->n_prony)
        return fail(b, TLED_E_ARG, "a batch needs one Prony term count");
    if (m->expan_mode == 2 || m->cond_mode == 2)
        return fail(b, TLED_E_UNSUPPORTED, "orthotropic expansion and tensor conduction are single-problem options");
    HostProblem p;
    p.npe = elem_type; p.nn = n_nodes; p.ne = n_elems;
    p.X.assign(X, X + 3 * n_nodes);
    for (double v : p.X)
        if (!std::isfinite(v)) return fail(b, TLED_E_ARG, "non-finite coordinate");
    p.conn.assign(conn, conn + elem_type * n_elems);
    if (a0) p.a0.assign(a0, a0 + 3 * n_elems);
    if (q_elem) p.q.assign(q_elem, q_elem + n_elems);
    for (double v : p.q)
        if (!std::isfinite(v)) return fail(b, TLED_E_ARG, "non-finite source");
    p.fix.assign(n_nodes, 0);
    p.Tfix.assign(n_nodes, 0.0);
    if (n_fixed < 0 || (n_fixed > 0 && (!fixed_nodes || !fixed_mask))) return fail(b, TLED_E_ARG, "bad fixed dofs");
    for (int64_t i = 0; i < n_fixed; ++i) {
        if (fixed_nodes[i] < 0 || fixed_nodes[i] >= n_nodes) return fail(b, TLED_E_ARG, "fixed node out of range");
        p.fix[fixed_nodes[i]] |= uint8_t(fixed_mask[i] & 7);
    }
    p.t_on = t_on; p.t_off = t_off; p.dt = dt; p.gamma = damping_gamma; p.mat = *m;
    p.have_mesh = p.have_mat = p.have_time = true;
    b->scen.push_back(std::move(p));
    b->scen_steps.push_back(n_steps);
    b->scen_pe.push_back(patch_elems);
    b->scen_cfl.push_back(0.0);
    b->scen_tend.push_back(0.0);
    if (index) *index = int32_t(b->scen.size() - 1);
    return TLED_OK;
}

tled_status tled_batch_set_duration(tled_batch *b, int32_t scenario, double cfl, double t_end) {
    TRY(need_setup(b));
    if (!b->is_batch) return fail(b, TLED_E_STATE, "not a batch handle");
    if (scenario < 0 || size_t(scenario) >= b->scen.size()) return fail(b, TLED_E_ARG, "scenario out of range");
    if (!(cfl > 0.0 && cfl <= 1.0) || !(t_end >= 0.0) || !std::isfinite(t_end))
        return fail(b, TLED_E_ARG, "need 0 < cfl <= 1 and a finite t_end >= 0");
    b->scen_cfl[scenario] = cfl;
    b->scen_tend[scenario] = t_end;
    return TLED_OK;
}

tled_status tled_batch_scenario_steps(tled_batch *b, int32_t scenario, double *dt, int64_t *n_steps) {
    if (!b || !b->is_batch) return b ? fail(b, TLED_E_STATE, "not a batch handle") : TLED_E_ARG;
    if (scenario < 0 || size_t(scenario) >= b->scen.size()) return fail(b, TLED_E_ARG, "scenario out of range");
    if (!b->finalized) return fail(b, TLED_E_STATE, "not finalized");
    if (dt) *dt = b->scen[scenario].dt;
    if (n_steps) *n_steps = b->scen_steps[scenario];
    return TLED_OK;
}

tled_status tled_batch_finalize(tled_batch *b) {
    TRY(need_setup(b));
    if (!b->is_batch) return fail(b, TLED_E_STATE, "not a batch handle");
    if (b->scen.empty()) return fail(b, TLED_E_STATE, "no scenario added");
    const int v = b->opt.kernel_variant == 0 ? default_variant(b->scen[0].npe) : b->opt.kernel_variant;
    if (v == 1) return fail(b, TLED_E_UNSUPPORTED, "batches run on the fused kernels (variant 2 or 3)");
    if (b->opt.block_size == 512)
        return fail(b, TLED_E_UNSUPPORTED, "batches run with 256-thread workgroups (block_size 0 or 256)");
    std::vector<int> pe(b->scen.size());
    for (size_t k = 0; k < pe.size(); ++k)
        pe[k] = b->scen_pe[k] > 0 ? b->scen_pe[k]
                                  : (b->opt.patch_elems > 0 ? b->opt.patch_elems : (b->scen[k].npe == 4 ? 448 : 256));
    // end steps as set below, for the union order (scenarios by descending end step)
    auto end_of = [b](size_t k, double dt_cr) -> int64_t {
        if (b->scen_cfl[k] > 0.0) {
            const double dt = b->scen_cfl[k] * dt_cr;
            return dt > 0.0 ? std::max<int64_t>(1, std::llround(b->scen_tend[k] / dt)) : 0;
        }
        return b->scen_steps[k];
    };
    tled_status st = precompute_batch(b->scen, pe, b->opt.reorder >= 0, b->opt.reorder != 2, end_of, &b->pc,
                                      &b->ranges, &b->patch_scen, &b->shared_scen, &b->err);
    if (st != TLED_OK) return st;
    for (size_t k = 0; k < b->scen.size(); ++k) {
        HostProblem &p = b->scen[k];
        if (b->scen_cfl[k] > 0.0) {
            p.dt = b->scen_cfl[k] * b->ranges[k].dt_cr;
            b->scen_steps[k] = std::max<int64_t>(1, std::llround(b->scen_tend[k] / p.dt));
        }
        if (!(p.dt > 0.0) || 0.5 * p.gamma * p.dt >= 1.0)
            return fail(b, TLED_E_ARG, "scenario " + std::to_string(k) + ": dt must be > 0 with gamma dt / 2 < 1");
    }
    for (size_t k = 0; k < b->scen.size(); ++k)
        if (b->scen[k].dt > b->ranges[k].dt_cr)
            return fail(b, TLED_E_ARG, "scenario " + std::to_string(k) + ": dt exceeds the critical step " +
                                           std::to_string(b->ranges[k].dt_cr));
        else if (b->scen[k].dt > b->ranges[k].dt_th)
            return fail(b, TLED_E_ARG, "scenario " + std::to_string(k) +
                                           ": dt exceeds the explicit thermal stability limit " +
                                           std::to_string(b->ranges[k].dt_th));
    PatchArgs probe{};
    probe.max_nodes = b->pc.patches.max_nodes;
    probe.max_elems = b->pc.patches.slot_stride;
    size_t lim = 0;
    TRY(patch_lds_limit(b, &lim));
    if (patch_lds_bytes(b->scen[0].npe, v == 2, probe) > lim)
        return fail(b, TLED_E_ARG, "patch too large for LDS; lower patch_elems");
    {
        const size_t S = b->scen.size();
        std::vector<size_t> pos(S);
        std::iota(pos.begin(), pos.end(), size_t(0));
        std::sort(pos.begin(), pos.end(), [&](size_t x, size_t y) { return b->ranges[x].patch_lo < b->ranges[y].patch_lo; });
        b->pos_end.resize(S);
        b->pos_patch_hi.resize(S);
        b->pos_shared_hi.resize(S);
        for (size_t m = 0; m < S; ++m) {
            const size_t k = pos[m];
            b->pos_end[m] = b->scen_steps[k];
            b->pos_patch_hi[m] = b->ranges[k].patch_hi;
            b->pos_shared_hi[m] = b->ranges[k].sh_hi - b->pc.patches.n_interior;
        }
        // not a prefix order (cannot happen: the union was ordered by these end steps): launch everything
        if (!std::is_sorted(b->pos_end.begin(), b->pos_end.end(), std::greater<int64_t>())) b->pos_end.clear();
    }
    b->queue = b->opt.batch_schedule == 1;
    if (b->queue && (b->pos_end.empty() || v != 2 && v != 3))
        return fail(b, TLED_E_STATE, "the persistent schedule needs the fused kernels and end-step ordered scenarios");
    b->variant = v;
    b->prob = b->scen[0];
    b->prob.nn = b->pc.nn;
    b->prob.ne = b->pc.ne;
    build_kernel_constants(b);
    if (b->device >= 0) {
        HIPCHK(b, hipSetDevice(b->device));
        if (!b->stream) {
            HIPCHK(b, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
            b->own_stream = true;
        }
        st = upload_all(b);
        if (st != TLED_OK) {
            free_device(b);
            return st;
        }
        long long qc[2];
        st = set_queue_counts(b, 0, qc);
        if (st == TLED_OK && hipStreamSynchronize(b->stream) != hipSuccess) st = fail(b, TLED_E_HIP, "stream sync");
        if (st != TLED_OK) {
            free_device(b);
            return st;
        }
    }
    b->step = 0;
    b->finalized = true;
    return TLED_OK;
}

tled_status tled_batch_run(tled_batch *b) {
    TRY(need_device(b));
    int64_t mx = 0;
    for (auto n : b->scen_steps) mx = std::max(mx, n);
    return mx > b->step ? tled_step(b, mx - b->step) : TLED_OK;
}

namespace {
// Copies the two node ranges of one scenario (patch-interior and shared) to the
// host and scatters them into caller numbering.
tled_status batch_read_one(tled_batch *b, int32_t scenario, double *u, double *T) {
    const ScenRange &R = b->ranges[scenario];
    const int64_t ni = R.int_hi - R.int_lo, ns = R.sh_hi - R.sh_lo;
    std::vector<float4> hi(size_t(std::max<int64_t>(ni, 0))), hs(size_t(std::max<int64_t>(ns, 0)));
    if (ni > 0)
        HIPCHK(b, hipMemcpyAsync(hi.data(), b->tp.nu4 + R.int_lo, sizeof(float4) * ni, hipMemcpyDeviceToHost,
                                 b->stream));
    if (ns > 0)
        HIPCHK(b, hipMemcpyAsync(hs.data(), b->tp.nu4 + R.sh_lo, sizeof(float4) * ns, hipMemcpyDeviceToHost,
                                 b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    const double T0 = b->scen[scenario].mat.T0;
    for (size_t i = 0; i < R.node_of.size(); ++i) {
        const int64_t g = R.node_of[i];
        const float4 v = (g >= R.int_lo && g < R.int_hi) ? hi[g - R.int_lo] : hs[g - R.sh_lo];
        if (u) { u[3 * i] = v.x; u[3 * i + 1] = v.y; u[3 * i + 2] = v.z; }
        if (T) T[i] = T0 + double(v.w);
    }
    return TLED_OK;
}
}  // namespace

tled_status tled_batch_read(tled_batch *b, int32_t scenario, double *u, double *T) {
    TRY(need_device(b));
    if (!b->is_batch) return fail(b, TLED_E_STATE, "not a batch handle");
    if (scenario < 0 || size_t(scenario) >= b->scen.size()) return fail(b, TLED_E_ARG, "scenario out of range");
    TRY(batch_read_one(b, scenario, u, T));
    return check_status(b);
}

tled_status tled_batch_read_all(tled_batch *b, double *u, double *T) {
    TRY(need_device(b));
    if (!b->is_batch) return fail(b, TLED_E_STATE, "not a batch handle");
    const int64_t nn = b->pc.nn;
    std::vector<float4> h(size_t(std::max<int64_t>(nn, 0)));
    HIPCHK(b, hipMemcpyAsync(h.data(), b->tp.nu4, sizeof(float4) * nn, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    int64_t off = 0;
    for (size_t k = 0; k < b->scen.size(); ++k) {
        const ScenRange &R = b->ranges[k];
        const double T0 = b->scen[k].mat.T0;
        for (size_t i = 0; i < R.node_of.size(); ++i) {
            const float4 v = h[R.node_of[i]];
            const int64_t o = off + int64_t(i);
            if (u) { u[3 * o] = v.x; u[3 * o + 1] = v.y; u[3 * o + 2] = v.z; }
            if (T) T[o] = T0 + double(v.w);
        }
        off += int64_t(R.node_of.size());
    }
    return check_status(b);
}

tled_status tled_batch_monitors(tled_batch *b, double ablation_T, double *T_max, double *ablated_volume) {
    TRY(need_device(b));
    if (!b->d_scen_mon) return fail(b, TLED_E_STATE, "scenario monitors need the fused kernels");
    const int S = int(b->scen.size());
    launch_scenario_monitors(b->tp.nu4, b->tp.Vl, b->d_ranges, b->d_np, S, float(ablation_T), b->d_scen_mon,
                             b->stream);
    HIPCHK(b, hipGetLastError());
    std::vector<double> h(2 * S);
    HIPCHK(b, hipMemcpyAsync(h.data(), b->d_scen_mon, sizeof(double) * 2 * S, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    for (int k = 0; k < S; ++k) {
        if (T_max) T_max[k] = h[2 * k];
        if (ablated_volume) ablated_volume[k] = h[2 * k + 1];
    }
    return check_status(b);
}

tled_status tled_batch_get_info(tled_batch *b, tled_batch_info *out) {
    if (!b || !out) return TLED_E_ARG;
    std::memset(out, 0, sizeof(*out));
    out->n_scenarios = int32_t(b->scen.size());
    for (auto n : b->scen_steps) out->max_steps = std::max<int64_t>(out->max_steps, n);
    for (auto &p : b->scen) out->n_elems += p.ne;
    for (auto &p : b->scen) out->n_nodes += p.nn;
    out->step = b->step;
    if (b->finalized) {
        out->n_patches = b->pc.patches.n;
        out->n_shared_nodes = b->pc.nn - b->pc.patches.n_interior;
        out->device_bytes = b->device_bytes;
        out->kernel_variant = b->variant;
    }
    return TLED_OK;
}

tled_status tled_kernel_times(tled_sim *sim, int64_t n_steps, double ms[3]) {
    TRY(need_device(sim));
    if (!ms || n_steps <= 0) return fail(sim, TLED_E_ARG, "need n_steps > 0 and an output array");
    ms[0] = ms[1] = ms[2] = 0.0;
    const int chunk = sim->opt.graph_steps > 0 ? sim->opt.graph_steps : 100;
    int64_t left = n_steps, chunks = 0, cur = sim->step;
    std::vector<hipEvent_t> ev(4 * size_t(chunk) + 2);
    for (auto &e : ev) HIPCHK(sim, hipEventCreate(&e));
    tled_status st = TLED_OK;
    while (left > 0 && st == TLED_OK) {
        int c = int(std::min<int64_t>(left, chunk));
        st = enqueue_chunk(sim, c, cur, false, &ev);
        if (st != TLED_OK) break;
        HIPCHK(sim, hipStreamSynchronize(sim->stream));
        for (int j = 0; j < c; ++j) {
            float a = 0.f, b = 0.f;
            HIPCHK(sim, hipEventElapsedTime(&a, ev[4 * j], ev[4 * j + 1]));
            HIPCHK(sim, hipEventElapsedTime(&b, ev[4 * j + 2], ev[4 * j + 3]));
            ms[0] += a;
            ms[1] += b;
        }
        float f = 0.f;
        HIPCHK(sim, hipEventElapsedTime(&f, ev[4 * size_t(c)], ev[4 * size_t(c) + 1]));
        ms[2] += f;
        ++chunks;
        left -= c;
        cur += c;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (st != TLED_OK) return st;
    sim->step += n_steps;
    ms[0] /= double(n_steps);
    ms[1] /= double(n_steps);
    ms[2] /= double(chunks);
    return check_status(sim);
}

}  // extern "C"
