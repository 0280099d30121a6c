// Launch interface of the TLED kernels (host side of kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tled.h"
#include "device_math.h"

namespace tled {

constexpr int kBlock = 256;   // threads per block (4 wavefronts of 64)
constexpr int kNumXcd = 8;    // accelerator complex dies of an MI355X

// Threads per workgroup of the fused patch kernel: 256 (4 wavefronts); T4 may
// also use 512.

// Node-update constants.
struct NodeParams {
    float A;          // (1 - gamma dt/2) / (1 + gamma dt/2)
    float dt;
    float T0;
    float rho;
    float abl_T;      // ablation threshold temperature, K
    float ck_off, ck_inv, c_lo, c_hi;  // c(T) law (when ckT_on) on dT: ramp start offset T0 - ckT_lo (FP64 -> FP32)
    int ckT_on;
    long long n_on, n_off;             // source active for n_on <= step < n_off
};

// Thermal dose accumulated per node when enabled (single problems): CEM43
// minutes and the Arrhenius damage integral, in FP64, from the node's
// end-of-step temperature rise dT, by a kernel of its own after each step.
struct DoseParams {
    double T0;        // reference temperature, K
    double cem_off;   // 316.15 K - T0 (43 C relative to T0)
    double dt_min;    // dt / 60
    double dt;        // s
    double lnA;       // ln of the Arrhenius frequency factor (1/s)
    double EaR;       // Ea / R_gas, K
    int arrhenius;    // 1: accumulate the Arrhenius integral
};

// Monitor record written by the finish kernel.
struct DevMonitors {
    long long step;
    double kinetic, strain, T_max, T_min, ablated;
    unsigned flags;
    unsigned pad;
};

struct TwoPassArgs {
    int ne, nn;
    const int4 *conn4, *conn4b;          // T4: conn4; H8: conn4 (nodes 0-3), conn4b (4-7)
    const float4 *g0, *g1, *g2;          // geometry planes
    const float4 *hg0, *hg1, *hg2;       // H8 hourglass c_alpha planes
    const float *khg;
    float4 *nu4, *nv4;                   // node state (u, dT), (v, B)
    const float4 *nth;                   // node thermal constants
    const uint8_t *mask;
    const float *Vl;
    float *theta;
    float4 *out;                         // ne * npe element-slot outputs
    const int *rowptr, *inc;
    const float4 *aniso;                 // 2 per element: (n_oct, Dxx, Dyy), (Dzz, Dxy, Dyz, Dxz), or null
    const long long *step_base;
    unsigned *status;
    double *part_elem, *part_node;
};

struct PatchArgs {
    int ne, n_patches, max_nodes, max_elems, slot_stride;
    int n_interior, n_shared;
    const int *elem_begin, *int_begin, *shared_begin, *shared_ids;
    const uint16_t *lconn, *lrow, *lpos;
    const int *lrow_begin;
    const int *srow, *ppos;
    const float *lX;            // per-patch local reference coordinates (x, y, z)
    const int *lx_begin;
    const float2 *fib;          // fibre, octahedral coordinates
    const float4 *aniso;        // 2 per element: (n_oct, Dxx, Dyy), (Dzz, Dxy, Dyz, Dxz), or null
    const float4 *g0, *g1, *g2, *hg0, *hg1, *hg2;   // precomputed geometry (plane variant)
    const float *khg;
    float4 *nu4, *nv4;
    const float4 *nth;
    const uint8_t *mask;
    const float *Vl;
    float *theta;
    float4 *partial;
    // Shared nodes updated inside the next step's patch kernel (single problems):
    // per shared entry (a patch's copy of a shared node) the range [x, y) of the
    // node's partials; the shared-node state the step starts from and the buffer
    // the first patch of each node writes the update to (n_shared each; the
    // shared-node kernel reads su_in, sv_in and writes nu4, nv4); the partials of
    // the previous step.
    const int2 *srange;
    const float4 *su_in, *sv_in;
    float4 *su_out, *sv_out;
    const float4 *partial_prev;
    const long long *step_base;
    unsigned *status;
    double *part_elem, *part_node;
    // scenario tables (a single problem is a batch of one scenario)
    const KMat *km;             // per scenario
    const NodeParams *np;       // per scenario
    const int *patch_scen;      // per patch
    const int *shared_scen;     // per shared node
    const long long *scen_end;  // per scenario: steps to run (the scenario holds afterwards)
    // persistent schedule of a batch: the union positions in order of
    // descending end step, with the patch and shared-node counts of the prefix
    // that ends at each position, and the running counts of the current and
    // next step
    long long *qcount;          // [parity of the step][patches, shared nodes] of the running scenarios
    const long long *pos_end;
    const int *pos_patch_hi;
    const long long *pos_shared_hi;
    int n_pos;
};

// Optional timing of one launch: both events are taken by the dispatch itself.
struct LaunchTiming {
    hipEvent_t start, stop;
};

void launch_element(int npe, int np, bool mon, const TwoPassArgs &a, const KMat &m, hipStream_t s,
                    const LaunchTiming *ev = nullptr);
// Thermal dose of every node at the temperature the step ended at (single problems).
void launch_dose(const float4 *nu4, int nn, double2 *dose, const DoseParams &q, hipStream_t s);
void launch_node(bool mon, const TwoPassArgs &a, const NodeParams &p, int j, hipStream_t s,
                 const LaunchTiming *ev = nullptr);
// batch: per-scenario constants and end steps (256-thread workgroups only).
// fused: the patch kernel first advances its shared nodes by the previous step
// (single problems, geometry rebuilt from coordinates, 256 threads, no
// anisotropy plane).
void launch_patch(int npe, int np, bool mon, bool geox, int bs, bool batch, const PatchArgs &a, int j,
                  hipStream_t s, const LaunchTiming *ev = nullptr, bool fused = false);
// Resident workgroups per CU of the patch kernel in this configuration (-1 on error).
int patch_occupancy(int npe, int np, bool geox, int bs, bool batch, const PatchArgs &a, bool fused = false);
void launch_shared_nodes(bool mon, bool batch, const PatchArgs &a, int j, hipStream_t s,
                         const LaunchTiming *ev = nullptr);
// Persistent schedule of a batch (256-thread workgroups): `grid` resident
// workgroups walk the step's patches, each XCD's workgroups an eighth of them;
// the shared-node kernel strides over the step's shared nodes with a fixed grid
// and counts the next step's running patches and shared nodes.
void launch_patch_queue(int npe, int np, bool mon, bool geox, const PatchArgs &a, int j, int grid, hipStream_t s,
                        const LaunchTiming *ev = nullptr);
int patch_queue_occupancy(int npe, int np, bool geox, const PatchArgs &a);
void launch_shared_nodes_queue(bool mon, const PatchArgs &a, int j, int grid, hipStream_t s,
                               const LaunchTiming *ev = nullptr);
// Per-scenario maximum temperature and lumped volume at or above T_abl, over the
// scenario's interior node range [int_lo, int_hi) and shared range [sh_lo, sh_hi).
void launch_scenario_monitors(const float4 *nu4, const float *Vl, const long long *ranges /* 4 per scenario */,
                              const NodeParams *np, int n_scen, float T_abl, double *out /* 2 per scenario */,
                              hipStream_t s);
void launch_finish(const double *part_elem, int n_elem_parts, const double *part_node, int n_node_parts,
                   long long *step_base, int k, const unsigned *status, DevMonitors *mon, hipStream_t s);
size_t patch_lds_bytes(int npe, bool geox, const PatchArgs &a);

}  // namespace tled

namespace tled {
void launch_export_fields(const float4 *nu4, const int *new2old, int nn, float T0, float *u_dst, float *T_dst,
                          hipStream_t s);
}  // namespace tled
