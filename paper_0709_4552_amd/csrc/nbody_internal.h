// Internal declarations shared by the translation units of libnbody.
// Not part of the public ABI (include/nbody.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nbody.h"

namespace nb {

constexpr int kWG = 256;          // threads per workgroup, every kernel
constexpr int kChunk = kWG;       // particles per scan chunk, one per thread (never crosses clusters)
constexpr int kLevels = 64;       // step levels tracked per cluster (level L: dt = 2^-L)
constexpr int kPlanThreads = 1024;

// Where the planner takes each cluster's block from.
constexpr int32_t kPlanFromLists = -1;   // n_act[c] particles at time t_next[c] (set by the host)
constexpr int32_t kPlanFromLevels = -2;  // next block of the block-step scheme, from the level counts

// bits of the device error word
enum : int32_t {
    kErrNonFinite = 1,
    kErrRange = 2,
    kErrNotDue = 4,
    kErrPlan = 8,
    kErrExtent = 16,
};

// Device-resident counters and scalars, one instance per context.
struct DevCtl {
    int32_t err;                   // error bits
    int32_t n_last;                // block size summed over clusters, last planned step
    int64_t total_items;           // force work items of the current plan
    int64_t part_used;             // partial-sum slots used by the current plan
    int64_t t_end_tick;            // clusters stop when their next time exceeds this
    unsigned long long clamps;     // steps clamped at the minimum
    unsigned long long steps;      // block steps with n > 0 (summed over clusters)
    unsigned long long updates;    // corrected particles
    double interactions;           // n*N summed
    int32_t any_active;            // at least one cluster active in the last plan
    int32_t cls;                   // shape class chosen by the last plan
    unsigned long long item_counter;  // work queue head of the force kernel
    int32_t s_max;                 // largest j-split of the current plan (0 = none)
    int32_t pad2;
};

// Host-visible copy of the fields the stepping loop polls (written by the last
// kernel of each captured batch of block steps into mapped pinned memory).
struct HostMirror {
    int32_t err;
    int32_t any_active;
};

constexpr int kMaxSlices = 1024;   // j-slices per cluster the planner may choose
// Workgroups of one launch do not run at equal speed, so when each takes a
// single long item the slowest sets the launch time.  The planner therefore
// sizes items against a virtual grid of 4x (2x) the resident one, so that the
// queue hands every workgroup several, once each workgroup has at least 16 (4)
// tile-units of work (i-blocks x j-tiles / grid); below that, slices of only a
// tile or two would cost more in per-item overhead than they save.
__host__ __device__ inline int64_t plan_grid(int64_t grid, int64_t nib, int64_t tiles) {
    const int64_t u = nib * tiles;
    return u >= 16 * grid ? 4 * grid : (u >= 4 * grid ? 2 * grid : grid);
}

// Launch-shape classes by block size: class k is used when the mean block
// size of the active clusters is >= min_n[k] (classes in decreasing order).
constexpr int kClasses = 5;
struct ClassTable {
    int32_t min_n[kClasses];
    int32_t ib[kClasses];     // i-particles per work item of the class's shape
    int32_t grid[kClasses];   // persistent workgroups of the class's launch
    int32_t jt[kClasses];     // j-slice granularity of the class's shape
};

// The plan of one evaluation of n of a single cluster's Nc particles: the
// shape class, the j-split S (slices of jl j-particles), and the work items
// and partial-sum slots that needs.  Candidate splits S = 1..kMaxSlices are
// ranked by plan_key (waves of items over the planning grid, then slice
// length, then S); the device planner ranks them across the lanes of a wave,
// the host (evaluations whose n it knows) in a loop: both take the same
// minimum, so both choose the same plan.
struct PlanChoice {
    int32_t cls, S, jl;
    int64_t items, parts;
};

__host__ __device__ inline int plan_class(const ClassTable &ct, int64_t n) {
    for (int k = 0; k < kClasses; k++)
        if (n >= ct.min_n[k])
            return k;
    return kClasses - 1;
}

// Rank of j-split S (INT64_MAX: not allowed).  Arithmetic in 32-bit integers
// (tiles < 2^23 for any cluster the ABI allows, S <= kMaxSlices) and
// waves = ceil(nib*Seff/grid) in FP64 (exact: the product is below 2^53, and a
// quotient that is not an integer lies at least 1/grid from one): software
// 64-bit divisions made the device loop the longest part of a small block
// step's first kernel.
__host__ __device__ inline int64_t plan_key(uint32_t S, uint32_t tiles32, double nibd,
                                            double inv_grid, int64_t grid, int64_t n,
                                            int64_t part_cap) {
    if (n <= 0 || (S > 1 && (int64_t)S * n > part_cap))
        return INT64_MAX;
    const uint32_t tps = (tiles32 + S - 1) / S;
    const uint32_t Seff = (tiles32 + tps - 1) / tps;
    const double q = nibd * (double)Seff;
    double wv = ceil(q * inv_grid);
    // the reciprocal product may round across an integer: step to the exact
    // ceiling
    if ((wv - 1.0) * (double)grid >= q)
        wv -= 1.0;
    else if (wv * (double)grid < q)
        wv += 1.0;
    const int64_t waves = (int64_t)wv;
    return ((waves * (int64_t)(tps + 1)) << 11) | (int64_t)(S - 1);
}

// The plan from the best key (INT64_MAX: S = 1).
__host__ __device__ inline PlanChoice plan_from_key(int64_t key, int cls, int64_t n, int64_t Nc,
                                                    int64_t tiles, int64_t j_tile, int64_t nib) {
    PlanChoice p{cls, 0, 0, 0, 0};
    const int64_t S = key == INT64_MAX ? 1 : (key & 2047) + 1;
    if (n > 0 && Nc > 0) {
        const int64_t tiles_per = (tiles + S - 1) / S;
        p.jl = (int32_t)(tiles_per * j_tile);
        p.S = (int32_t)((Nc + p.jl - 1) / p.jl);
        p.items = nib * p.S;
        p.parts = p.S > 1 ? (int64_t)p.S * n : 0;
    }
    return p;
}

// The same plan on the host: every candidate S in turn.
inline PlanChoice plan_on_host(const ClassTable &ct, int64_t n, int64_t Nc, int64_t part_cap) {
    const int cls = plan_class(ct, n);
    const int64_t j_tile = ct.jt[cls];
    const int64_t tiles = (Nc + j_tile - 1) / j_tile;
    const int64_t nib = (n + ct.ib[cls] - 1) / ct.ib[cls];
    const int64_t grid = plan_grid(ct.grid[cls], nib, tiles);
    const uint32_t tiles32 = (uint32_t)tiles;
    const double nibd = (double)nib, inv_grid = 1.0 / (double)grid;
    int64_t key = INT64_MAX;
    for (uint32_t S = 1; S <= (uint32_t)kMaxSlices && S <= tiles32; S++) {
        const int64_t k2 = plan_key(S, tiles32, nibd, inv_grid, grid, n, part_cap);
        key = k2 < key ? k2 : key;
    }
    return plan_from_key(key, cls, n, Nc, tiles, j_tile, nib);
}

// Predicted j-particle buffer.
//  mixed: P = (x_hi, y_hi, z_hi, m), Q = (x_lo, y_lo, z_lo, vx), R = (vy, vz)
//         with x_hi = q rint(x/q) on the fixed grid q (so x_hi_j - x_hi_i is
//         exact in FP32) and x_lo = fl32(x - x_hi); V = (vx_lo, vy_lo, vz_lo, 0)
//         with v_lo = fl32(v - fl32(v)), read only by the FP64 near field
//  fp64 : A = (x, y), B = (z, m), C = (vx, vy), D = vz
struct JBuf {
    float4 *P = nullptr;
    float4 *Q = nullptr;
    float2 *R = nullptr;
    float4 *V = nullptr;
    double2 *A = nullptr;
    double2 *B = nullptr;
    double2 *C = nullptr;
    double *D = nullptr;
};

// Caller state in device-pointer form (copied from nbody_state).
struct State {
    double *x, *y, *z, *vx, *vy, *vz, *ax, *ay, *az, *jx, *jy, *jz, *m;
    int64_t *tick;
    int8_t *lev;
};

// The particles of each cluster by block-step level, so that a block step
// finds its block without a scan (section 4.1, step 2: every particle on a
// level whose step divides the block time is due, and nothing else).  List
// (c, L) in buffer b holds cnt[b][c][L] particle indices of cluster c on
// level L, at idx + (b*nlev + L - lev_min)*n_total + off[c].  A block step
// gathers the lists of its due levels from buffer buf[c][L]; its force launch
// then switches each due level to the other buffer, emptied (nothing reads or
// writes the lists while it runs), and its corrector appends each corrected
// particle to the current list of its new level.
struct LevelLists {
    int32_t *idx;      // [2][nlev][n_total]
    int32_t *cnt;      // [2][C][kLevels]
    int32_t *buf;      // [C][kLevels] current buffer of each list
    int32_t nlev;      // lev_max - lev_min + 1
    int32_t lev_min;
    int32_t C;
    int64_t n_total;
};

// Work plan of one force evaluation, built on the device by k_plan.
struct PlanDev {
    int64_t *item_begin;   // [C+1] first work item of each cluster
    int32_t *S;            // [C] j-slices
    int32_t *jlen;         // [C] j-particles per slice (multiple of the tile)
    int64_t *part_begin;   // [C] first partial-sum slot of each cluster (S>1)
    int32_t *n_cur;        // [C] block size of the step being computed
    int64_t *t_cur;        // [C] time (ticks) of the step being computed
    int64_t *t_now;        // [C] time (ticks) of the cluster's last block step
    int32_t *lev_cnt;      // [C][kLevels] particles of the cluster on each step level
};

struct Params {
    int64_t n_total;
    int32_t C;
    double eps2;
    float eps2f;
    double eta, eta_init;
    int32_t dt_min_log2, dt_max_log2;
    int32_t lev_min, lev_max;       // -dt_max_log2, -dt_min_log2
    double tick;                    // 2^dt_min_log2
    int32_t precision;
    double grid_q;                  // mixed: quantum of the hi part of positions
    double grid_inv;                // 1 / grid_q
    const double4 *origin;          // mixed: [C] each cluster's origin (x, y, z, 0),
                                    // subtracted before the hi/lo split
};

// Mixed precision near field: a pair whose acceleration term may exceed
// kNearFrac*|a_i| (m_max/s > kNearFrac*|a_i|, with |a_i| the particle's last
// acceleration), or whose jerk term may exceed kNearFracJerk*|jerk_i|
// (m_max V_i s^{-3/2} > kNearFracJerk*|jerk_i|, with V_i = |v_i| + v_max the
// largest relative speed the cluster allows and |jerk_i| the particle's last
// jerk) is evaluated in FP64 instead of FP32.  The jerk sum cancels more than
// the acceleration sum: a pair term tens of times the total is common, and
// its FP32 rounding alone then costs ~1e-5 of the particle's jerk.
constexpr float kNearFrac = 0.1f;
constexpr float kNearFracJerk = 2.0f;
constexpr int kGridQLog2 = -16;  // hi parts on a 2^-16 grid: exact differences for |x| < 256
// Positions are split relative to their cluster's origin.  Within
// kMixedExtent of it every hi part is a float on the grid; a prediction
// beyond it raises kErrExtent.
constexpr double kMixedExtent = 256.0;
static_assert(kMixedExtent == (double)(1 << (24 + kGridQLog2)), "24-bit hi parts");

// Everything the force kernels need.
struct ForceArgs {
    JBuf jb;
    const int64_t *off;       // [C+1] cluster offsets (device)
    int32_t C;
    const int64_t *item_begin;
    const int32_t *S;
    const int32_t *jlen;
    const int64_t *part_begin;
    const int32_t *n_cur;
    const int64_t *total_items;   // &ctl->total_items
    const int32_t *i_list;        // slot-indexed active list
    int32_t slots_at_offsets;     // slot of (c,k) = off[c]+k if set, else k
    double *out_acc;              // [3][stride]
    double *out_jerk;             // [3][stride]
    double *out_pot;              // [stride] or null
    int64_t out_stride;
    double *part;                 // [7][part_cap]
    int64_t part_cap;
    int32_t *err;
    unsigned long long *item_counter;
    const int32_t *cls;           // class chosen by the plan
    int32_t cls_mask;             // this launch runs only if bit *cls is set
    int32_t fetch_lane;           // thread that pops the work queue (always 0); a
                                  // run-time value so the compiler cannot merge its
                                  // branch with other tid == 0 branches across the
                                  // barriers of the item loop
    int64_t n_total;
    double eps2;
    float eps2f;
    // mixed near field
    const double *hax, *hay, *haz;  // |a_i| hint: the particle's stored acceleration
    const double *hjx, *hjy, *hjz;  // |jerk_i| hint: the particle's stored jerk
    const double *m64;              // FP64 masses
    const float4 *nscale;           // [C] (largest mass, smallest mass, largest speed, 0)
    // block steps: the level lists whose due levels this launch switches to
    // fresh buffers (flip_lists = 0: explicit evaluations, no lists)
    LevelLists ll;
    int32_t flip_lists;
    int32_t lev_max;
    float near_frac;                // 0 disables the near field
    float near_frac_jerk;           // 0 disables its jerk criterion
    uint32_t cls_lj;                // lane-group launches: log2(j lanes) of class k
                                    // in bits 4k..4k+3
    // in-kernel prediction (lane-group launches, one cluster): classes in
    // fused_mask predict their j- and i-particles from the state to the
    // cluster's block time t_cur[0] instead of reading the j-buffer
    int32_t fused_mask;
    State st;
    const int64_t *t_cur;
    double tick, grid_q, grid_inv;
    const double4 *origin;          // the cluster's origin (in-kernel prediction)
    // a plan made on the host (one cluster, n known there): the force and
    // reduction kernels take it from here instead of the plan arrays
    int32_t host_plan;
    PlanChoice hp;
    int32_t hp_n;
};

// Third-order Taylor prediction of particle i to tick T (section 4.1, step
// 3), as the j-buffer record the force kernels read: mixed P = (x_hi, y_hi,
// z_hi, m), Q = (x_lo, y_lo, z_lo, vx), R = (vy, vz); FP64 A = (x, y),
// B = (z, m), C = (vx, vy), D = vz.  The prediction pass and the force
// kernels' in-kernel prediction both call these, so both give the same bits.
__device__ inline void predict_terms(const State &st, double tick, int64_t i, int64_t T,
                                     double &xp, double &yp, double &zp, double &vxp,
                                     double &vyp, double &vzp) {
    const double d = (double)(T - st.tick[i]) * tick;
    const double h = 0.5 * d, s6 = d * (1.0 / 6.0);
    const double ax = st.ax[i], ay = st.ay[i], az = st.az[i];
    const double jx = st.jx[i], jy = st.jy[i], jz = st.jz[i];
    const double vx = st.vx[i], vy = st.vy[i], vz = st.vz[i];
    // xp = x + d (v + d (a/2 + d j/6)),  vp = v + d (a + d j/2)
    xp = fma(d, fma(d, fma(s6, jx, 0.5 * ax), vx), st.x[i]);
    yp = fma(d, fma(d, fma(s6, jy, 0.5 * ay), vy), st.y[i]);
    zp = fma(d, fma(d, fma(s6, jz, 0.5 * az), vz), st.z[i]);
    vxp = fma(d, fma(h, jx, ax), vx);
    vyp = fma(d, fma(h, jy, ay), vy);
    vzp = fma(d, fma(h, jz, az), vz);
}

// The mixed j-record of a particle at (xp, vp) with mass m.
__device__ inline void split_mixed(double xp, double yp, double zp, double vxp, double vyp,
                                   double vzp, double m, double grid_q, double grid_inv,
                                   float4 &P, float4 &Q, float2 &R, float4 &V) {
    // hi on a fixed grid: differences of hi parts are exact, so the rounding
    // of x_j - x_i does not depend on i's low bits
    const float xh = (float)(rint(xp * grid_inv) * grid_q);
    const float yh = (float)(rint(yp * grid_inv) * grid_q);
    const float zh = (float)(rint(zp * grid_inv) * grid_q);
    P = make_float4(xh, yh, zh, (float)m);
    Q = make_float4((float)(xp - (double)xh), (float)(yp - (double)yh),
                    (float)(zp - (double)zh), (float)vxp);
    R = make_float2((float)vyp, (float)vzp);
    // what FP32 velocities drop: v = fl32(v) + v_lo to ~2^-48 |v|
    V = make_float4((float)(vxp - (double)Q.w), (float)(vyp - (double)R.x),
                    (float)(vzp - (double)R.y), 0.f);
}

// The mixed record of particle i predicted to tick T, its position taken
// relative to its cluster's origin o.  False when that relative position is
// kMixedExtent or more from o on some axis (NaN passes: the corrector flags it).
__device__ inline bool predict_mixed(const State &st, double tick, double grid_q, double grid_inv,
                                     const double4 &o, int64_t i, int64_t T, float4 &P, float4 &Q,
                                     float2 &R, float4 &V) {
    double xp, yp, zp, vxp, vyp, vzp;
    predict_terms(st, tick, i, T, xp, yp, zp, vxp, vyp, vzp);
    xp -= o.x;
    yp -= o.y;
    zp -= o.z;
    split_mixed(xp, yp, zp, vxp, vyp, vzp, st.m[i], grid_q, grid_inv, P, Q, R, V);
    return !(fabs(xp) >= kMixedExtent || fabs(yp) >= kMixedExtent || fabs(zp) >= kMixedExtent);
}

__device__ inline void predict_fp64(const State &st, double tick, int64_t i, int64_t T,
                                    double2 &A, double2 &B, double2 &C, double &D) {
    double xp, yp, zp, vxp, vyp, vzp;
    predict_terms(st, tick, i, T, xp, yp, zp, vxp, vyp, vzp);
    A = make_double2(xp, yp);
    B = make_double2(zp, st.m[i]);
    C = make_double2(vxp, vyp);
    D = vzp;
}

struct Shape {
    int i_per_lane;
    int j_lanes;
    int j_tile;
};

// A value every lane of the wave holds, made visibly uniform to the compiler.
// Loops and branches that contain barriers must depend only on such values:
// a barrier inside control flow the compiler treats as divergent (for example
// a loop whose exit reads LDS) is undefined and has deadlocked workgroups.
__device__ inline int64_t uniform_i64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline int32_t uniform_i32(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// One DPP lane move of a double (two 32-bit moves).  Rows that ROW_MASK leaves
// out receive 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ inline double dpp_move(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, CTRL, ROW_MASK, 0xF, false);
}

// Sum over each group of L consecutive lanes (L a power of two, <= 64) with
// DPP moves only, no LDS permutes: quad swaps (lane ^ 1, lane ^ 2), then the
// half-row and row mirrors (each pairs the two halves of an 8- and a 16-lane
// span), then the row broadcasts of lanes 15 and 31.  The last lane of each
// group (lane index L - 1 within it) ends with the group's sum; for L <= 16
// every lane of the group does.  The order of the additions is fixed.  Every
// lane of the wave must take part.
template <int L>
__device__ inline double group_sum(double v) {
    static_assert(L >= 1 && L <= 64 && (L & (L - 1)) == 0, "group of 1..64 lanes");
    if (L >= 2) v += dpp_move<0xB1>(v);        // quad_perm [1,0,3,2]
    if (L >= 4) v += dpp_move<0x4E>(v);        // quad_perm [2,3,0,1]
    if (L >= 8) v += dpp_move<0x141>(v);       // row_half_mirror
    if (L >= 16) v += dpp_move<0x140>(v);      // row_mirror
    if (L >= 32) v += dpp_move<0x142, 0xA>(v); // rows 1, 3 += lane 15 of rows 0, 2
    if (L >= 64) v += dpp_move<0x143, 0xC>(v); // rows 2, 3 += lane 31
    return v;
}

// The same with a group width known only at run time (uniform over the wave).
__device__ inline double group_sum_rt(double v, int L) {
    if (L >= 2) v += dpp_move<0xB1>(v);
    if (L >= 4) v += dpp_move<0x4E>(v);
    if (L >= 8) v += dpp_move<0x141>(v);
    if (L >= 16) v += dpp_move<0x140>(v);
    if (L >= 32) v += dpp_move<0x142, 0xA>(v);
    if (L >= 64) v += dpp_move<0x143, 0xC>(v);
    return v;
}

// ---- launchers (kernels_step.hip) -----------------------------------------
hipError_t launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);
hipError_t launch_iota_i32(int32_t *p, int64_t n, hipStream_t s);
hipError_t launch_set_i64(int64_t *p, int64_t v, hipStream_t s);
hipError_t launch_predict(const State &st, const Params &pr, const JBuf &jb, const int32_t *cid,
                          const int64_t *t_cur, const int32_t *n_cur, int64_t t_host,
                          int use_host_t, DevCtl *ctl, hipStream_t s);
hipError_t launch_prime(const State &st, const Params &pr, const int64_t *off,
                        const int32_t *chunk_c, const int64_t *chunk_b, int64_t n_chunks,
                        const PlanDev &pl, const LevelLists &ll, int64_t *t_min, int64_t *t_max,
                        DevCtl *ctl, hipStream_t s);
hipError_t launch_predict_gather(const State &st, const Params &pr, const JBuf &jb,
                                 const int64_t *off, const int32_t *chunk_c,
                                 const int64_t *chunk_b, int64_t n_chunks, const PlanDev &pl,
                                 const LevelLists &ll, int32_t *i_list, DevCtl *ctl, hipStream_t s);
hipError_t launch_plan(const Params &pr, const int64_t *off, const PlanDev &pl, int32_t *n_act,
                       int64_t *t_next, DevCtl *ctl, int64_t part_cap, const ClassTable &ct,
                       int32_t host_n, int64_t host_t, int32_t count_stats, hipStream_t s);
// fused_mask: classes whose force kernel predicts in the kernel; their blocks
// skip the prediction pass (compaction only)
hipError_t launch_plan_predict_gather(const State &st, const Params &pr, const JBuf &jb,
                                      const int64_t *off, const PlanDev &pl, const LevelLists &ll,
                                      int32_t *i_list, DevCtl *ctl, int64_t part_cap,
                                      const ClassTable &ct, int32_t fused_mask, hipStream_t s);
hipError_t launch_reduce(const ForceArgs &fa, const int32_t *cid, int64_t slot_space,
                         const int32_t *s_max, hipStream_t s);
hipError_t launch_reduce_correct(const ForceArgs &fa, const State &st, const Params &pr,
                                 const int32_t *cid, const PlanDev &pl, const LevelLists &ll,
                                 const int32_t *s_max, DevCtl *ctl, hipStream_t s);
hipError_t launch_correct(const State &st, const Params &pr, const int32_t *i_list,
                          int32_t slots_at_offsets, const int64_t *off, const int32_t *cid,
                          const int32_t *n_cur, const int64_t *t_cur, int64_t slot_space,
                          const double *acc_new, const double *jerk_new, int64_t in_stride,
                          DevCtl *ctl, hipStream_t s);
hipError_t launch_init_finish(const State &st, const Params &pr, const double *acc_new,
                              const double *jerk_new, int64_t stride, DevCtl *ctl,
                              hipStream_t s);
hipError_t launch_read_predicted(const Params &pr, const JBuf &jb, const int32_t *cid,
                                 double *pos, double *vel, hipStream_t s);
hipError_t launch_mirror(const DevCtl *ctl, HostMirror *mirror_dev, hipStream_t s);

// ---- force (kernels_force.hip) --------------------------------------------
bool force_shape_supported(const Shape &sh);
// Lane-group shapes (one i per lane group of 4-256 lanes) share one kernel;
// launch_force of such a shape needs fa.cls_lj filled for the classes in
// fa.cls_mask.
bool force_shape_grouped(const Shape &sh);
// pair_mass (mixed form only): near-field test per pair with m_j instead of
// the cluster's largest mass; for clusters whose masses are not all equal
int force_occupancy(const Shape &sh, int mixed, int want_pot, int exclude_self, int pair_mass);
int force_j_step(const Shape &sh);
hipError_t launch_force(const Shape &sh, int mixed, int want_pot, int exclude_self, int pair_mass,
                        const ForceArgs &fa, int grid, hipStream_t s);

}  // namespace nb
