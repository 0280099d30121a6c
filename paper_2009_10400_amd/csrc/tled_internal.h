// Internal host-side structures of the TLED library (no HIP types here, so
// the set-up code also builds with a plain C++ compiler).
#pragma once

#include <cstdint>
#include <limits>
#include <functional>
#include <string>
#include <vector>

#include "../../include/tled.h"

namespace tled {

// Problem as given by the caller (caller numbering, FP64).
struct HostProblem {
    int npe = 0;
    int64_t nn = 0, ne = 0;
    std::vector<double> X;          // nn * 3
    std::vector<int32_t> conn;      // ne * npe
    std::vector<double> a0;         // ne * 3, empty = (1,0,0)
    std::vector<double> n0;         // ne * 3 second expansion axes (expan_mode 2), else empty
    std::vector<double> Dc;         // ne * 6 conductivity tensors xx yy zz xy yz xz (cond_mode 2), else empty
    std::vector<double> q;          // ne, empty = 0
    std::vector<uint8_t> fix;       // nn, bit0..2 fixed u, bit3 fixed T
    std::vector<double> Tfix;       // nn
    double t_on = 0.0, t_off = std::numeric_limits<double>::infinity();
    double dt = 0.0, gamma = 0.0;
    tled_material mat{};
    bool have_mesh = false, have_mat = false, have_time = false;
};

// Patch partition of the fused variant.  Elements of patch p are the
// contiguous range [elem_begin[p], elem_begin[p+1]) of the internal element
// order; its nodes are the interior range [int_begin[p], int_begin[p+1]) of
// the internal node order (nodes touched by this patch only) followed by the
// shared nodes listed in shared_ids[shared_begin[p] .. shared_begin[p+1]).
struct Patches {
    int32_t n = 0;
    int32_t max_nodes = 0;                 // max local nodes over patches
    int32_t max_elems = 0;
    std::vector<int32_t> elem_begin;       // n + 1
    std::vector<int32_t> int_begin;        // n + 1 (interior node ranges)
    std::vector<int32_t> shared_begin;     // n + 1 (into shared_ids)
    std::vector<int32_t> shared_ids;       // internal node ids of shared nodes per patch
    std::vector<uint16_t> lconn;           // ne * npe local node indices
    // node-major element outputs: the patch's npe * n_elems element slots are
    // stored in LDS grouped by local node, local node l owning positions
    // lrow[off+l] .. lrow[off+l+1] (its slots in element order, then vertex
    // order); lpos[e * npe + a] is the position of element e's vertex a.
    std::vector<int32_t> lrow_begin;       // n + 1 offsets into lrow (each patch has nloc+1 entries)
    std::vector<uint16_t> lrow;            // row pointers, local to the patch
    std::vector<uint16_t> lpos;            // ne * npe positions, local to the patch
    int32_t slot_stride = 0;               // elements of the largest patch (sizes the LDS output array)
    // shared-node assembly: the partial of (patch p, local shared index j) is
    // written to partial slot ppos[shared_begin[p] + j]; slots are sorted by
    // node, then patch, so node n_interior + s sums the contiguous slots
    // srow[s] .. srow[s+1].
    int64_t n_interior = 0;                // nodes [0, n_interior) are interior
    std::vector<int32_t> srow;             // n_shared + 1
    std::vector<int32_t> ppos;             // shared_ids.size()
    // reference coordinates of every local node of every patch, relative to
    // the patch centroid (x, y, z per local node; patch p starts at lx_begin[p])
    std::vector<float> lX;
    std::vector<int32_t> lx_begin;         // n + 1
};

// Precomputed quantities in the internal (reordered) numbering, FP64.
struct Precomputed {
    int npe = 0;
    int64_t nn = 0, ne = 0;
    std::vector<int64_t> node_new2old, node_old2new, elem_new2old;
    std::vector<int32_t> conn;      // ne * npe internal node ids, orientation repaired
    std::vector<double> geo;        // ne * 9: T4 dh/dX rows of nodes 1..3; H8 G = J0^-T
    std::vector<double> V0;         // ne
    std::vector<double> hgc;        // ne * 12: H8 c_alpha = X^T h_alpha (alpha = 0..3)
    std::vector<double> khg;        // ne: H8 hourglass stiffness
    std::vector<double> a0;         // ne * 3 unit fibres
    std::vector<double> n0;         // ne * 3 unit second expansion axes, orthogonal to a0 (expan_mode 2)
    std::vector<double> Dc;         // ne * 6 conductivity tensors (cond_mode 2)
    std::vector<double> Vl, M, C, Kb, Qm, Qr;  // nn lumped quantities (C at T0)
    std::vector<uint8_t> fix;       // nn
    std::vector<double> Tfix;       // nn
    std::vector<int32_t> rowptr;    // nn + 1 node -> element-slot incidence (two-pass)
    std::vector<int32_t> inc;       // ne * npe values e * npe + s, ascending per node
    int64_t n_swapped = 0;
    double dt_cr = 0.0;
    double dt_th = 0.0;                      // explicit thermal stability bound (Gershgorin)
    Patches patches;
};

// Node and element ranges of one scenario of a batch in the union numbering.
struct ScenRange {
    int64_t elem_lo = 0, elem_hi = 0;     // elements
    int64_t int_lo = 0, int_hi = 0;       // patch-interior nodes
    int64_t sh_lo = 0, sh_hi = 0;         // shared nodes
    int32_t patch_lo = 0, patch_hi = 0;   // patches
    std::vector<int64_t> node_of;         // caller node index -> union internal index
    std::vector<int64_t> elem_of;         // caller element index -> union internal index
    double dt_cr = 0.0;
    double dt_th = 0.0;
    int64_t n_swapped = 0;
};

struct SetupOptions {
    bool reorder = true;
    bool build_patches = false;
    bool bisect = true;      // with reorder and build_patches: patches by coordinate bisection
    int patch_elems = 512;
    int threads = 1;         // host threads for the element pass and the bisection
};

// Host threads for set-up: the hardware concurrency, or TLED_HOST_THREADS, in 1..64.
int host_threads();

// Element geometry and critical step only (no reordering), for tled_critical_dt.
// Returns TLED_OK or TLED_E_MESH with a message.
tled_status critical_dt(const HostProblem &p, double *dt_cr, std::string *err);

// Full precompute.  Returns TLED_OK, TLED_E_MESH or TLED_E_ARG with a message.
tled_status precompute(const HostProblem &p, const SetupOptions &opt, Precomputed *out,
                       std::string *err);

// Batch of independent scenarios (same element type): each is precomputed with
// its own patch size, then all are concatenated into one union problem whose
// patch partition never mixes scenarios.  Scenarios enter the union in order
// of descending end_step(k, critical dt of k) (stable); node order of the
// union: all patch-interior nodes scenario by scenario, then all shared nodes
// scenario by scenario.  patch_scen / shared_scen give the scenario of each
// patch / shared node.
tled_status precompute_batch(const std::vector<HostProblem> &ps, const std::vector<int> &patch_elems,
                             bool reorder, bool bisect, const std::function<int64_t(size_t, double)> &end_step,
                             Precomputed *out, std::vector<ScenRange> *ranges,
                             std::vector<int32_t> *patch_scen, std::vector<int32_t> *shared_scen,
                             std::string *err);

}  // namespace tled
