// Host side of the C ABI declared in include/nbody.h: context, argument
// checks, launch sequencing, graph capture of the block step, autotuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "nbody.h"
#include "nbody_internal.h"

using namespace nb;

// Size classes whose block steps predict inside the force kernel by default:
// none.  Reading 14 state arrays per particle in the force kernel costs more
// latency than the streaming prediction pass saves (block steps to t = 1/8 at
// N = 196608 took 1.2% longer with classes 2-4 fused).
constexpr int32_t kDefaultFusedMask = 0;

struct nbody_ctx {
    Params pr{};
    double eps = 0.0;  // as given (pr holds eps^2)
    State st{};
    hipStream_t stream = nullptr;
    int device = 0;
    int n_cu = 256;

    std::vector<int64_t> off_h;
    int64_t max_cluster = 0;
    int64_t *off_d = nullptr;
    int32_t *cid_d = nullptr;
    int32_t *chunk_c_d = nullptr;
    int64_t *chunk_b_d = nullptr;
    int64_t n_chunks = 0;

    JBuf jb;
    int32_t *i_list_d = nullptr;
    int32_t *iota_d = nullptr;
    int32_t *n_act_d = nullptr;   // host-set block sizes (explicit and start-up evaluations)
    int64_t *t_next_d = nullptr;  // host-set block times; earliest next time when priming
    int64_t *t_max_d = nullptr;   // latest last time when priming
    PlanDev pl{};
    LevelLists ll{};  // particles by block-step level (the block of a step without a scan)
    double *acc_new = nullptr, *jerk_new = nullptr, *pot_new = nullptr;
    double *part = nullptr;
    int64_t part_cap = 0;
    DevCtl *ctl = nullptr;
    // [C] near-field scales of each cluster: largest mass, smallest mass,
    // largest speed (the mixed form's FP64 near-field test), from init / load
    float4 *nscale_d = nullptr;
    // [C] origin of each cluster's mixed records (x, y, z, 0), from init / load
    double4 *origin_d = nullptr;

    std::vector<void *> allocs;

    // host bookkeeping
    bool initialised = false;
    bool predicted = false;
    int64_t predicted_tick = -1;

    Shape cls_shape[kClasses];
    int cls_grid[kClasses];  // 0 = derive from occupancy
    int32_t cls_min_n[kClasses];
    int occ_cache[kClasses][2][2];  // occupancy per class, want_pot, exclude_self (0 = unknown)
    int pair_mass = 0;  // mixed form: some cluster's masses differ, near test per pair
    // block steps of one cluster: size classes whose lane-group force launch
    // predicts in the kernel (no prediction pass for their blocks)
    int32_t fused_mask = kDefaultFusedMask;

    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    // mapped pinned memory the last kernel of each captured batch writes, so
    // the stepping loop can poll it while the next batch is already queued
    HostMirror *mirror_h = nullptr;
    HostMirror *mirror_d = nullptr;
    hipEvent_t batch_ev[2] = {nullptr, nullptr};
};

namespace {

constexpr int kJTile = 256;
constexpr int kGraphBatch = 32;  // block steps per captured graph

int map_err(hipError_t e) {
    if (e == hipSuccess)
        return NBODY_OK;
    if (e == hipErrorOutOfMemory)
        return NBODY_ENOMEM;
    return NBODY_EDEVICE;
}

#define NB_TRY(expr)                       \
    do {                                   \
        hipError_t e__ = (expr);           \
        if (e__ != hipSuccess)             \
            return map_err(e__);           \
    } while (0)

template <typename T>
hipError_t dalloc(nbody_ctx *c, T **p, size_t count) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(1, count) * sizeof(T));
    if (e != hipSuccess)
        return e;
    c->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return hipSuccess;
}

int ib_of(const Shape &s) { return (kWG / s.j_lanes) * s.i_per_lane; }

bool is_multiple_tick(double t, int dt_min_log2, int64_t *tick) {
    if (!std::isfinite(t) || t < 0.0)
        return false;
    const double q = std::ldexp(t, -dt_min_log2);
    if (q > 9.0e18 || q != std::floor(q))
        return false;
    *tick = (int64_t)q;
    return true;
}

int grid_of(nbody_ctx *c, int cls, int want_pot, int excl) {
    if (c->cls_grid[cls] > 0)
        return c->cls_grid[cls];
    int &occ = c->occ_cache[cls][want_pot ? 1 : 0][excl ? 1 : 0];
    if (occ <= 0)
        occ = std::max(1, force_occupancy(c->cls_shape[cls], c->pr.precision == NBODY_PREC_MIXED,
                                          want_pot, excl, c->pair_mass));
    return occ * c->n_cu;
}

// class of a given mean block size (the same rule k_plan applies)
int class_of(const nbody_ctx *c, int64_t n_mean) {
    for (int k = 0; k < kClasses; k++)
        if (n_mean >= c->cls_min_n[k])
            return k;
    return kClasses - 1;
}

ClassTable class_table(nbody_ctx *c, int want_pot, int excl) {
    ClassTable ct{};
    for (int k = 0; k < kClasses; k++) {
        ct.min_n[k] = c->cls_min_n[k];
        ct.ib[k] = ib_of(c->cls_shape[k]);
        ct.grid[k] = grid_of(c, k, want_pot, excl);
        ct.jt[k] = force_j_step(c->cls_shape[k]);
    }
    return ct;
}

ForceArgs force_args(nbody_ctx *c, const int32_t *i_list, int slots_at_offsets, double *acc,
                     double *jerk, double *pot, int64_t stride) {
    ForceArgs fa{};
    fa.jb = c->jb;
    fa.off = c->off_d;
    fa.C = c->pr.C;
    fa.item_begin = c->pl.item_begin;
    fa.S = c->pl.S;
    fa.jlen = c->pl.jlen;
    fa.part_begin = c->pl.part_begin;
    fa.n_cur = c->pl.n_cur;
    fa.total_items = reinterpret_cast<const int64_t *>(&c->ctl->total_items);
    fa.i_list = i_list;
    fa.slots_at_offsets = slots_at_offsets;
    fa.out_acc = acc;
    fa.out_jerk = jerk;
    fa.out_pot = pot;
    fa.out_stride = stride;
    fa.part = c->part;
    fa.part_cap = c->part_cap;
    fa.err = &c->ctl->err;
    fa.item_counter = &c->ctl->item_counter;
    fa.cls = &c->ctl->cls;
    fa.fetch_lane = 0;
    fa.n_total = c->pr.n_total;
    fa.eps2 = c->pr.eps2;
    fa.eps2f = (float)c->pr.eps2;
    fa.hax = c->st.ax;
    fa.hay = c->st.ay;
    fa.haz = c->st.az;
    fa.hjx = c->st.jx;
    fa.hjy = c->st.jy;
    fa.hjz = c->st.jz;
    fa.m64 = c->st.m;
    fa.nscale = c->nscale_d;
    fa.near_frac = c->pr.precision == NBODY_PREC_MIXED ? kNearFrac : 0.f;
    fa.near_frac_jerk = c->pr.precision == NBODY_PREC_MIXED ? kNearFracJerk : 0.f;
    fa.fused_mask = 0;
    fa.st = c->st;
    fa.t_cur = c->pl.t_cur;
    fa.tick = c->pr.tick;
    fa.grid_q = c->pr.grid_q;
    fa.grid_inv = c->pr.grid_inv;
    fa.origin = c->origin_d;
    return fa;
}

// The force launches of a device-planned evaluation (or only class `only`):
// one per distinct launch among the classes, where classes share a launch if
// their shapes are equal, or both lane-group shapes (one kernel serves those),
// and their grids are equal; each launch runs only if the plan picked one of
// the classes it serves.
hipError_t launch_classes(nbody_ctx *c, ForceArgs fa, int mixed, int want_pot, int excl,
                          int only) {
    fa.cls_lj = 0;
    for (int k = 0; k < kClasses; k++) {
        int lg = 0;
        while ((1 << lg) < c->cls_shape[k].j_lanes)
            lg++;
        fa.cls_lj |= (uint32_t)lg << (4 * k);
    }
    int done = 0;
    for (int k = 0; k < kClasses; k++) {
        if ((only >= 0 && k != only) || (done >> k) & 1)
            continue;
        const Shape &sh = c->cls_shape[k];
        const bool grouped = force_shape_grouped(sh);
        const int grid = grid_of(c, k, want_pot, excl);
        int mask = 0;
        for (int q = k; q < kClasses; q++) {
            const Shape &o = c->cls_shape[q];
            const bool same = grouped ? force_shape_grouped(o)
                                      : (o.i_per_lane == sh.i_per_lane &&
                                         o.j_lanes == sh.j_lanes && o.j_tile == sh.j_tile);
            if ((only < 0 || q == only) && same && grid_of(c, q, want_pot, excl) == grid)
                mask |= 1 << q;
        }
        done |= mask;
        fa.cls_mask = mask;
        hipError_t e = launch_force(sh, mixed, want_pot, excl, c->pair_mass, fa, grid, c->stream);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// One force evaluation planned on the device.  host_n >= 0: the block size is
// known on the host (single cluster) and only that class's kernel is launched;
// otherwise every class kernel is launched and all but the planned one exit.
hipError_t enqueue_force(nbody_ctx *c, const int32_t *i_list, int slots_at_offsets,
                         int32_t host_n, int64_t host_t, int count_stats, double *acc,
                         double *jerk, double *pot, int64_t stride, int64_t slot_space) {
    const int excl = c->pr.eps2 == 0.0;
    const int want_pot = pot != nullptr;
    const int mixed = c->pr.precision == NBODY_PREC_MIXED;
    const ClassTable ct = class_table(c, want_pot, excl);
    int only = -1;
    ForceArgs fa = force_args(c, i_list, slots_at_offsets, acc, jerk, pot, stride);
    hipError_t e = hipSuccess;
    if (host_n >= 0 && c->pr.C == 1 && !count_stats) {
        // one cluster, n known here: plan on the host, launch only that
        // class's kernel, no plan kernel
        fa.host_plan = 1;
        fa.hp = plan_on_host(ct, host_n, c->pr.n_total, c->part_cap);
        fa.hp_n = host_n;
        only = fa.hp.cls;
    } else {
        if (host_n >= 0)
            only = class_of(c, host_n);
        e = launch_plan(c->pr, c->off_d, c->pl, c->n_act_d, c->t_next_d, c->ctl, c->part_cap,
                        ct, host_n, host_t, count_stats, c->stream);
        if (e != hipSuccess)
            return e;
    }
    e = launch_classes(c, fa, mixed, want_pot, excl, only);
    if (e != hipSuccess)
        return e;
    return launch_reduce(fa, c->cid_d, slot_space, &c->ctl->s_max, c->stream);
}

int read_ctl(nbody_ctx *c, DevCtl *out) {
    NB_TRY(hipStreamSynchronize(c->stream));
    NB_TRY(hipMemcpy(out, c->ctl, sizeof(DevCtl), hipMemcpyDeviceToHost));
    return NBODY_OK;
}

int consume_error(nbody_ctx *c, const DevCtl &h) {
    if (h.err == 0)
        return NBODY_OK;
    int32_t zero = 0;
    NB_TRY(hipMemcpy(&c->ctl->err, &zero, sizeof(zero), hipMemcpyHostToDevice));
    if (h.err & kErrRange)
        return NBODY_ERANGE;
    if (h.err & kErrNotDue)
        return NBODY_ESTATE;
    if (h.err & kErrExtent)  // its records are off the grid: what follows is not trusted
        return NBODY_EEXTENT;
    if (h.err & kErrNonFinite)
        return NBODY_ENONFINITE;
    return NBODY_EDEVICE;
}

// Level counts and times of the block-step scheme, rebuilt from the state
// (which the caller owns and the explicit entry points may have changed).
hipError_t enqueue_prime(nbody_ctx *c) {
    return launch_prime(c->st, c->pr, c->off_d, c->chunk_c_d, c->chunk_b_d, c->n_chunks, c->pl,
                        c->ll, c->t_next_d, c->t_max_d, c->ctl, c->stream);
}

// One block step of every active cluster (section 4.1): plan the next block
// from the level counts, predict and compact (one kernel for a single
// cluster, two for an ensemble), force, then reduce the j-split and correct in
// one pass.  Nothing here reads back to the host, so a batch of steps is
// captured into one graph.
hipError_t enqueue_block_step(nbody_ctx *c) {
    const int excl = c->pr.eps2 == 0.0;
    const int mixed = c->pr.precision == NBODY_PREC_MIXED;
    const ClassTable ct = class_table(c, 0, excl);
    // in-kernel prediction: one cluster, classes served by the lane-group launch
    int32_t fused = 0;
    if (c->pr.C == 1)
        for (int k = 0; k < kClasses; k++)
            if (((c->fused_mask >> k) & 1) && force_shape_grouped(c->cls_shape[k]))
                fused |= 1 << k;
    hipError_t e;
    if (c->pr.C == 1) {
        e = launch_plan_predict_gather(c->st, c->pr, c->jb, c->off_d, c->pl, c->ll, c->i_list_d,
                                       c->ctl, c->part_cap, ct, fused, c->stream);
    } else {
        e = launch_plan(c->pr, c->off_d, c->pl, c->n_act_d, c->t_next_d, c->ctl, c->part_cap, ct,
                        kPlanFromLevels, 0, 1, c->stream);
        if (e == hipSuccess)
            e = launch_predict_gather(c->st, c->pr, c->jb, c->off_d, c->chunk_c_d, c->chunk_b_d,
                                      c->n_chunks, c->pl, c->ll, c->i_list_d, c->ctl, c->stream);
    }
    if (e != hipSuccess)
        return e;
    ForceArgs fa = force_args(c, c->i_list_d, 1, c->acc_new, c->jerk_new, nullptr, c->pr.n_total);
    fa.fused_mask = fused;
    fa.ll = c->ll;
    fa.flip_lists = 1;
    fa.lev_max = c->pr.lev_max;
    e = launch_classes(c, fa, mixed, 0, excl, -1);
    if (e != hipSuccess)
        return e;
    return launch_reduce_correct(fa, c->st, c->pr, c->cid_d, c->pl, c->ll, &c->ctl->s_max,
                                 c->ctl, c->stream);
}

void drop_graph(nbody_ctx *c);

// Near-field scales of each cluster from host copies of the masses and the
// velocities (vel[q*N + i]): the largest and smallest |mass| and the largest
// speed, which bound a pair's acceleration and jerk terms in the mixed
// form's near-field test; and whether any cluster has unequal masses (then
// the mixed form tests every pair with its own m_j).
hipError_t upload_cluster_scales(nbody_ctx *c, const double *mh, const double *vh,
                                 const float4 *saved = nullptr) {
    const int64_t N = c->pr.n_total;
    std::vector<float4> sc(c->pr.C);
    bool unequal = false;
    for (int k = 0; k < c->pr.C; k++) {
        double mx = 0.0, mn = INFINITY, vmax = 0.0;
        const double m0 = mh[c->off_h[k]];
        for (int64_t i = c->off_h[k]; i < c->off_h[k + 1]; i++) {
            const double a = std::fabs(mh[i]);
            mx = std::max(mx, a);
            if (a > 0.0)  // the smallest mass that attracts
                mn = std::min(mn, a);
            unequal = unequal || mh[i] != m0;
            const double v2 = vh[i] * vh[i] + vh[N + i] * vh[N + i] + vh[2 * N + i] * vh[2 * N + i];
            vmax = std::max(vmax, std::sqrt(v2));
        }
        sc[k] = make_float4((float)mx, std::isfinite(mn) ? (float)mn : 0.f,
                            std::isfinite(vmax) ? (float)vmax : 0.f, 0.f);
    }
    // a resumed run keeps the scales its start-up set (the speeds at the
    // checkpoint differ), so it takes the same near-field decisions
    if (saved)
        for (int k = 0; k < c->pr.C; k++)
            sc[k] = saved[k];
    const int pm = (c->pr.precision == NBODY_PREC_MIXED && unequal) ? 1 : 0;
    if (pm != c->pair_mass) {
        c->pair_mass = pm;
        std::memset(c->occ_cache, 0, sizeof(c->occ_cache));
        drop_graph(c);
    }
    return hipMemcpy(c->nscale_d, sc.data(), sc.size() * sizeof(float4), hipMemcpyHostToDevice);
}

// Origins of the mixed records: the centre of each cluster's bounding box,
// rounded to a multiple of 64 so that a cluster around the coordinate origin
// keeps it (and its records their bits).  The FP64 form ignores them.
hipError_t upload_origins(nbody_ctx *c, const double *xh, const double4 *saved = nullptr) {
    const int64_t N = c->pr.n_total;
    std::vector<double4> o(c->pr.C, make_double4(0.0, 0.0, 0.0, 0.0));
    for (int k = 0; k < c->pr.C; k++) {
        double ctr[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < 3; q++) {
            double lo = INFINITY, hi = -INFINITY;
            for (int64_t i = c->off_h[k]; i < c->off_h[k + 1]; i++) {
                const double x = xh[q * N + i];
                if (std::isfinite(x)) {
                    lo = std::min(lo, x);
                    hi = std::max(hi, x);
                }
            }
            if (lo <= hi)
                ctr[q] = 64.0 * std::nearbyint((0.5 * lo + 0.5 * hi) * (1.0 / 64.0));
        }
        o[k] = make_double4(ctr[0], ctr[1], ctr[2], 0.0);
    }
    if (saved)
        for (int k = 0; k < c->pr.C; k++)
            o[k] = saved[k];
    return hipMemcpy(c->origin_d, o.data(), o.size() * sizeof(double4), hipMemcpyHostToDevice);
}

// ---- checkpoint file ----
// Little-endian binary: magic, version, the context's configuration (checked on
// load), statistics, tuning table, the near-field scales of each cluster (4
// floats), the origin of each cluster's mixed records (4 doubles; absent in
// version 2, whose runs used the coordinate origin), then the particle state
// as 13 FP64 arrays (x y z vx vy vz ax ay az jx jy jz m), int64 ticks and int8
// levels, and an FNV-1a 64-bit checksum of everything after the magic.
constexpr char kCkptMagic[8] = {'N', 'B', 'O', 'D', 'Y', 'C', 'K', 'P'};
constexpr uint32_t kCkptVersion = 3;

struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void add(const void *p, size_t n) {
        const unsigned char *b = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; i++) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    }
};

struct CkptWriter {
    FILE *f;
    Fnv sum;
    bool ok = true;
    void put(const void *p, size_t n) {
        if (ok && std::fwrite(p, 1, n, f) != n)
            ok = false;
        sum.add(p, n);
    }
};

struct CkptReader {
    FILE *f;
    Fnv sum;
    bool ok = true;
    void get(void *p, size_t n) {
        if (ok && std::fread(p, 1, n, f) != n)
            ok = false;
        if (ok)
            sum.add(p, n);
    }
};

// The configuration part of the header, in file order.
struct CkptConfig {
    int64_t n_total;
    int32_t n_clusters;
    int32_t precision;
    double eps, eta, eta_init;
    int32_t dt_min_log2, dt_max_log2;
};

CkptConfig ckpt_config(const nbody_ctx *c) {
    CkptConfig k{};
    k.n_total = c->pr.n_total;
    k.n_clusters = c->pr.C;
    k.precision = c->pr.precision;
    k.eps = c->eps;
    k.eta = c->pr.eta;
    k.eta_init = c->pr.eta_init;
    k.dt_min_log2 = c->pr.dt_min_log2;
    k.dt_max_log2 = c->pr.dt_max_log2;
    return k;
}

void drop_graph(nbody_ctx *c) {
    if (c->graph_exec)
        (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph)
        (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
}

// Capture kGraphBatch block steps on a private capture stream.
int build_graph(nbody_ctx *c) {
    drop_graph(c);
    (void)class_table(c, 0, c->pr.eps2 == 0.0);  // occupancy queries happen outside capture
    hipStream_t cap = nullptr;
    NB_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipStream_t user = c->stream;
    c->stream = cap;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int s = 0; s < kGraphBatch && e == hipSuccess; s++)
            e = enqueue_block_step(c);
        if (e == hipSuccess)
            e = launch_mirror(c->ctl, c->mirror_d, c->stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cap, &g);
        if (e == hipSuccess)
            e = e2;
        if (e == hipSuccess) {
            c->graph = g;
            e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    c->stream = user;
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        drop_graph(c);
        return map_err(e);
    }
    return NBODY_OK;
}

}  // namespace

extern "C" {

const char *nbody_strerror(int status) {
    switch (status) {
        case NBODY_OK: return "ok";
        case NBODY_EINVAL: return "invalid argument";
        case NBODY_ESTATE: return "call out of order or particle not due";
        case NBODY_ENOMEM: return "device out of memory";
        case NBODY_EDEVICE: return "HIP runtime error";
        case NBODY_ENONFINITE: return "non-finite value produced";
        case NBODY_EUNSUPPORTED: return "unsupported";
        case NBODY_ERANGE: return "particle index out of range";
        case NBODY_EIO: return "checkpoint file could not be written or read, or is damaged";
        case NBODY_ESCRATCH: return "more particles than the allocation-free evaluation holds";
        case NBODY_EEXTENT:
            return "mixed precision: a particle is 256 or more length units from its cluster's origin";
        default: return "unknown status";
    }
}

int nbody_create(const nbody_params *p, const nbody_state *s, void *stream, nbody_ctx **out) {
    if (!p || !s || !out)
        return NBODY_EINVAL;
    *out = nullptr;
    if (p->n_total < 1 || p->n_total > INT32_MAX || p->n_clusters < 1 ||
        p->n_clusters > p->n_total)
        return NBODY_EINVAL;
    if (!(p->eps >= 0.0) || !std::isfinite(p->eps) || !(p->eta > 0.0) || !std::isfinite(p->eta) ||
        !(p->eta_init > 0.0) || !std::isfinite(p->eta_init))
        return NBODY_EINVAL;
    if (p->dt_min_log2 < -40 || p->dt_max_log2 > 0 || p->dt_min_log2 > p->dt_max_log2)
        return NBODY_EINVAL;
    if (p->precision != NBODY_PREC_FP64 && p->precision != NBODY_PREC_MIXED)
        return NBODY_EINVAL;
    for (int c = 0; c < 3; c++)
        if (!s->pos[c] || !s->vel[c] || !s->acc[c] || !s->jerk[c])
            return NBODY_EINVAL;
    if (!s->mass || !s->t_tick || !s->level)
        return NBODY_EINVAL;
    std::vector<int64_t> off(p->n_clusters + 1);
    if (p->n_clusters == 1 && !p->cluster_offset) {
        off[0] = 0;
        off[1] = p->n_total;
    } else {
        if (!p->cluster_offset)
            return NBODY_EINVAL;
        for (int c = 0; c <= p->n_clusters; c++)
            off[c] = p->cluster_offset[c];
        if (off[0] != 0 || off[p->n_clusters] != p->n_total)
            return NBODY_EINVAL;
        for (int c = 0; c < p->n_clusters; c++)
            if (off[c + 1] <= off[c])
                return NBODY_EINVAL;
    }

    nbody_ctx *c = new (std::nothrow) nbody_ctx();
    if (!c)
        return NBODY_ENOMEM;
    c->stream = static_cast<hipStream_t>(stream);
    c->off_h = off;
    for (int k = 0; k < p->n_clusters; k++)
        c->max_cluster = std::max(c->max_cluster, off[k + 1] - off[k]);

    Params &pr = c->pr;
    pr.n_total = p->n_total;
    pr.C = p->n_clusters;
    c->eps = p->eps;
    pr.eps2 = p->eps * p->eps;
    pr.eps2f = (float)pr.eps2;
    pr.eta = p->eta;
    pr.eta_init = p->eta_init;
    pr.dt_min_log2 = p->dt_min_log2;
    pr.dt_max_log2 = p->dt_max_log2;
    pr.lev_min = -p->dt_max_log2;
    pr.lev_max = -p->dt_min_log2;
    pr.tick = std::ldexp(1.0, p->dt_min_log2);
    pr.precision = p->precision;
    pr.grid_q = std::ldexp(1.0, kGridQLog2);
    pr.grid_inv = std::ldexp(1.0, -kGridQLog2);

    State &st = c->st;
    st.x = s->pos[0]; st.y = s->pos[1]; st.z = s->pos[2];
    st.vx = s->vel[0]; st.vy = s->vel[1]; st.vz = s->vel[2];
    st.ax = s->acc[0]; st.ay = s->acc[1]; st.az = s->acc[2];
    st.jx = s->jerk[0]; st.jy = s->jerk[1]; st.jz = s->jerk[2];
    st.m = s->mass;
    st.tick = s->t_tick;
    st.lev = s->level;

    // default launch shapes by block size
    const Shape shapes[kClasses] = {{1, 1, kJTile}, {1, 4, kJTile}, {1, 16, kJTile},
                                    {1, 64, kJTile}, {1, 256, kJTile}};
    const int32_t min_n[kClasses] = {2048, 256, 32, 4, 0};
    for (int k = 0; k < kClasses; k++) {
        c->cls_shape[k] = shapes[k];
        c->cls_grid[k] = 0;
        c->cls_min_n[k] = min_n[k];
    }
    std::memset(c->occ_cache, 0, sizeof(c->occ_cache));

    int rc = NBODY_OK;
    auto fail = [&](hipError_t e) {
        rc = map_err(e);
        nbody_destroy(c);
        return rc;
    };
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess)
        return fail(e);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) ==
            hipSuccess &&
        cus > 0)
        c->n_cu = cus;

    const int64_t N = pr.n_total, C = pr.C;
    // chunk list for selection: chunks never cross clusters
    std::vector<int32_t> chunk_c;
    std::vector<int64_t> chunk_b;
    std::vector<int32_t> cid(N);
    for (int64_t k = 0; k < C; k++) {
        for (int64_t b = off[k]; b < off[k + 1]; b += kChunk) {
            chunk_c.push_back((int32_t)k);
            chunk_b.push_back(b);
        }
        for (int64_t i = off[k]; i < off[k + 1]; i++)
            cid[i] = (int32_t)k;
    }
    c->n_chunks = (int64_t)chunk_c.size();
    // partial sums: enough for any j-split the planner may choose
    c->part_cap = std::max<int64_t>(1 << 20, std::min<int64_t>(16 << 20, 8 * N));

    const bool mixed = pr.precision == NBODY_PREC_MIXED;
    if ((e = dalloc(c, &c->off_d, C + 1)) != hipSuccess || (e = dalloc(c, &c->cid_d, N)) != hipSuccess ||
        (e = dalloc(c, &c->chunk_c_d, c->n_chunks)) != hipSuccess ||
        (e = dalloc(c, &c->chunk_b_d, c->n_chunks)) != hipSuccess ||
        (e = dalloc(c, &c->i_list_d, N)) != hipSuccess || (e = dalloc(c, &c->iota_d, N)) != hipSuccess ||
        (e = dalloc(c, &c->n_act_d, C)) != hipSuccess || (e = dalloc(c, &c->t_next_d, C)) != hipSuccess ||
        (e = dalloc(c, &c->pl.item_begin, C + 1)) != hipSuccess ||
        (e = dalloc(c, &c->pl.S, C)) != hipSuccess || (e = dalloc(c, &c->pl.jlen, C)) != hipSuccess ||
        (e = dalloc(c, &c->pl.part_begin, C)) != hipSuccess ||
        (e = dalloc(c, &c->pl.n_cur, C)) != hipSuccess || (e = dalloc(c, &c->pl.t_cur, C)) != hipSuccess ||
        (e = dalloc(c, &c->pl.t_now, C)) != hipSuccess ||
        (e = dalloc(c, &c->pl.lev_cnt, C * kLevels)) != hipSuccess ||
        (e = dalloc(c, &c->t_max_d, C)) != hipSuccess ||
        (e = dalloc(c, &c->acc_new, 3 * N)) != hipSuccess ||
        (e = dalloc(c, &c->jerk_new, 3 * N)) != hipSuccess ||
        (e = dalloc(c, &c->pot_new, N)) != hipSuccess ||
        (e = dalloc(c, &c->part, 7 * c->part_cap)) != hipSuccess ||
        (e = dalloc(c, &c->ctl, 1)) != hipSuccess || (e = dalloc(c, &c->nscale_d, C)) != hipSuccess ||
        (e = dalloc(c, &c->origin_d, C)) != hipSuccess)
        return fail(e);
    c->pr.origin = c->origin_d;
    // level lists: two buffers of one list per level and cluster, each list
    // able to hold its whole cluster
    c->ll.nlev = pr.lev_max - pr.lev_min + 1;
    c->ll.lev_min = pr.lev_min;
    c->ll.C = (int32_t)C;
    c->ll.n_total = N;
    if ((e = dalloc(c, &c->ll.idx, 2 * (size_t)c->ll.nlev * N)) != hipSuccess ||
        (e = dalloc(c, &c->ll.cnt, 2 * C * kLevels)) != hipSuccess ||
        (e = dalloc(c, &c->ll.buf, C * kLevels)) != hipSuccess)
        return fail(e);
    if (mixed) {
        if ((e = dalloc(c, &c->jb.P, N)) != hipSuccess || (e = dalloc(c, &c->jb.Q, N)) != hipSuccess ||
            (e = dalloc(c, &c->jb.R, N)) != hipSuccess || (e = dalloc(c, &c->jb.V, N)) != hipSuccess)
            return fail(e);
    } else {
        if ((e = dalloc(c, &c->jb.A, N)) != hipSuccess || (e = dalloc(c, &c->jb.B, N)) != hipSuccess ||
            (e = dalloc(c, &c->jb.C, N)) != hipSuccess || (e = dalloc(c, &c->jb.D, N)) != hipSuccess)
            return fail(e);
    }
    if ((e = hipMemcpy(c->off_d, off.data(), (C + 1) * sizeof(int64_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->cid_d, cid.data(), N * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->chunk_c_d, chunk_c.data(), c->n_chunks * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->chunk_b_d, chunk_b.data(), c->n_chunks * sizeof(int64_t), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e);
    {
        void *hm = nullptr;
        if ((e = hipHostMalloc(&hm, sizeof(HostMirror), hipHostMallocMapped)) != hipSuccess)
            return fail(e);
        c->mirror_h = static_cast<HostMirror *>(hm);
        void *dm = nullptr;
        if ((e = hipHostGetDevicePointer(&dm, hm, 0)) != hipSuccess)
            return fail(e);
        c->mirror_d = static_cast<HostMirror *>(dm);
        for (int q = 0; q < 2; q++)
            if ((e = hipEventCreateWithFlags(&c->batch_ev[q], hipEventDisableTiming)) != hipSuccess)
                return fail(e);
    }
    DevCtl h{};
    h.t_end_tick = LLONG_MAX;
    if ((e = hipMemcpy(c->ctl, &h, sizeof(h), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e);
    {
        // no near-field scales until init / load (the mixed force refuses to
        // run before either)
        const std::vector<float4> zero(C, make_float4(0.f, 0.f, 0.f, 0.f));
        const std::vector<double4> zero_o(C, make_double4(0.0, 0.0, 0.0, 0.0));
        if ((e = hipMemcpy(c->nscale_d, zero.data(), C * sizeof(float4), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(c->origin_d, zero_o.data(), C * sizeof(double4), hipMemcpyHostToDevice)) != hipSuccess)
            return fail(e);
    }
    if ((e = launch_iota_i32(c->iota_d, N, c->stream)) != hipSuccess ||
        (e = launch_fill_i32(c->i_list_d, 0, N, c->stream)) != hipSuccess ||
        (e = launch_fill_i32(c->n_act_d, 0, C, c->stream)) != hipSuccess ||
        (e = launch_fill_i64(c->t_next_d, LLONG_MAX, C, c->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess)
        return fail(e);
    *out = c;
    return NBODY_OK;
}

int nbody_destroy(nbody_ctx *c) {
    if (!c)
        return NBODY_EINVAL;
    if (c->stream)
        (void)hipStreamSynchronize(c->stream);
    else
        (void)hipDeviceSynchronize();
    drop_graph(c);
    for (void *p : c->allocs)
        (void)hipFree(p);
    for (int q = 0; q < 2; q++)
        if (c->batch_ev[q])
            (void)hipEventDestroy(c->batch_ev[q]);
    if (c->mirror_h)
        (void)hipHostFree(c->mirror_h);
    delete c;
    return NBODY_OK;
}

int nbody_init(nbody_ctx *c) {
    if (!c)
        return NBODY_EINVAL;
    const int64_t N = c->pr.n_total;
    DevCtl h{};
    h.t_end_tick = LLONG_MAX;
    NB_TRY(hipStreamSynchronize(c->stream));
    NB_TRY(hipMemcpy(c->ctl, &h, sizeof(h), hipMemcpyHostToDevice));
    // zero a and jerk so the t = 0 prediction is exactly the positions
    for (int q = 0; q < 3; q++) {
        double *a[3] = {c->st.ax, c->st.ay, c->st.az};
        double *j[3] = {c->st.jx, c->st.jy, c->st.jz};
        NB_TRY(launch_fill_f64(a[q], 0.0, N, c->stream));
        NB_TRY(launch_fill_f64(j[q], 0.0, N, c->stream));
    }
    NB_TRY(launch_fill_i64(c->st.tick, 0, N, c->stream));
    NB_TRY(launch_fill_i32(c->n_act_d, 0, c->pr.C, c->stream));
    NB_TRY(launch_fill_i64(c->t_next_d, LLONG_MAX, c->pr.C, c->stream));
    {
        std::vector<double> mh(N), xh(3 * N), vh(3 * N);
        NB_TRY(hipStreamSynchronize(c->stream));
        NB_TRY(hipMemcpy(mh.data(), c->st.m, N * sizeof(double), hipMemcpyDeviceToHost));
        const double *xs[3] = {c->st.x, c->st.y, c->st.z};
        const double *vs[3] = {c->st.vx, c->st.vy, c->st.vz};
        for (int q = 0; q < 3; q++) {
            NB_TRY(hipMemcpy(xh.data() + q * N, xs[q], N * sizeof(double), hipMemcpyDeviceToHost));
            NB_TRY(hipMemcpy(vh.data() + q * N, vs[q], N * sizeof(double), hipMemcpyDeviceToHost));
        }
        NB_TRY(upload_cluster_scales(c, mh.data(), vh.data()));
        NB_TRY(upload_origins(c, xh.data()));
    }
    NB_TRY(launch_predict(c->st, c->pr, c->jb, c->cid_d, nullptr, nullptr, 0, 1, c->ctl, c->stream));
    // full sweep of every cluster: active list = identity, n_c = N_c, t = 0
    std::vector<int32_t> nc(c->pr.C);
    for (int k = 0; k < c->pr.C; k++)
        nc[k] = (int32_t)(c->off_h[k + 1] - c->off_h[k]);
    // mixed: a first sweep without near field gives |a| for the thresholds
    const int passes = c->pr.precision == NBODY_PREC_MIXED ? 2 : 1;
    for (int pass = 0; pass < passes; pass++) {
        // only the last pass's start-up steps count as clamped
        NB_TRY(launch_set_i64(reinterpret_cast<int64_t *>(&c->ctl->clamps), 0, c->stream));
        NB_TRY(hipMemcpyAsync(c->n_act_d, nc.data(), nc.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, c->stream));
        NB_TRY(launch_fill_i64(c->t_next_d, 0, c->pr.C, c->stream));
        NB_TRY(enqueue_force(c, c->iota_d, 1, kPlanFromLists, 0, 0, c->acc_new, c->jerk_new, nullptr, N, N));
        NB_TRY(launch_init_finish(c->st, c->pr, c->acc_new, c->jerk_new, N, c->ctl, c->stream));
        NB_TRY(hipStreamSynchronize(c->stream));  // nc must outlive the async copy
    }
    c->initialised = true;
    c->predicted = true;
    c->predicted_tick = 0;
    DevCtl hc;
    int rc = read_ctl(c, &hc);
    if (rc != NBODY_OK)
        return rc;
    return consume_error(c, hc);
}

int nbody_predict(nbody_ctx *c, double t) {
    if (!c)
        return NBODY_EINVAL;
    if (c->pr.C != 1)
        return NBODY_EUNSUPPORTED;
    int64_t tick;
    if (!is_multiple_tick(t, c->pr.dt_min_log2, &tick))
        return NBODY_EINVAL;
    NB_TRY(launch_predict(c->st, c->pr, c->jb, c->cid_d, nullptr, nullptr, tick, 1, c->ctl,
                          c->stream));
    c->predicted = true;
    c->predicted_tick = tick;
    return NBODY_OK;
}

int nbody_force_jerk(nbody_ctx *c, const int32_t *i_list, int64_t n, double t, double *acc,
                     double *jerk, double *pot) {
    if (!c || !i_list || !acc || !jerk)
        return NBODY_EINVAL;
    if (c->pr.C != 1)
        return NBODY_EUNSUPPORTED;
    if (n < 1 || n > c->pr.n_total)
        return NBODY_EINVAL;
    int64_t tick;
    if (!is_multiple_tick(t, c->pr.dt_min_log2, &tick))
        return NBODY_EINVAL;
    if (!c->predicted || c->predicted_tick != tick)
        return NBODY_ESTATE;
    // the mixed form's near-field test needs the scales and the stored
    // acceleration and jerk that nbody_init / nbody_load provide
    if (c->pr.precision == NBODY_PREC_MIXED && !c->initialised)
        return NBODY_ESTATE;
    NB_TRY(enqueue_force(c, i_list, 0, (int32_t)n, tick, 0, acc, jerk, pot, n, n));
    return NBODY_OK;
}

int nbody_correct(nbody_ctx *c, const int32_t *i_list, int64_t n, double t, const double *acc,
                  const double *jerk) {
    if (!c || !i_list || !acc || !jerk)
        return NBODY_EINVAL;
    if (c->pr.C != 1)
        return NBODY_EUNSUPPORTED;
    if (n < 1 || n > c->pr.n_total)
        return NBODY_EINVAL;
    int64_t tick;
    if (!is_multiple_tick(t, c->pr.dt_min_log2, &tick))
        return NBODY_EINVAL;
    if (!c->initialised)
        return NBODY_ESTATE;
    // the corrector reads n and t from the plan arrays; set them for this call
    const int32_t nn = (int32_t)n;
    NB_TRY(launch_fill_i32(c->pl.n_cur, nn, 1, c->stream));
    NB_TRY(launch_set_i64(c->pl.t_cur, tick, c->stream));
    NB_TRY(launch_correct(c->st, c->pr, i_list, 0, c->off_d, c->cid_d, c->pl.n_cur, c->pl.t_cur,
                          n, acc, jerk, n, c->ctl, c->stream));
    c->predicted = false;
    return NBODY_OK;
}

int nbody_step_block(nbody_ctx *c, double *t_out, int64_t *n_out) {
    if (!c)
        return NBODY_EINVAL;
    if (!c->initialised)
        return NBODY_ESTATE;
    NB_TRY(launch_set_i64(reinterpret_cast<int64_t *>(&c->ctl->t_end_tick), LLONG_MAX, c->stream));
    NB_TRY(enqueue_prime(c));
    DevCtl h;
    int rc = read_ctl(c, &h);
    if (rc != NBODY_OK)
        return rc;
    if (h.err)
        return consume_error(c, h);
    NB_TRY(enqueue_block_step(c));
    c->predicted = false;
    if (!t_out && !n_out)
        return NBODY_OK;
    rc = read_ctl(c, &h);
    if (rc != NBODY_OK)
        return rc;
    if (n_out)
        *n_out = h.n_last;
    if (t_out) {
        int64_t tk = 0;
        NB_TRY(hipMemcpy(&tk, c->pl.t_cur, sizeof(tk), hipMemcpyDeviceToHost));
        *t_out = std::ldexp((double)tk, c->pr.dt_min_log2);
    }
    return consume_error(c, h);
}

int nbody_run_until(nbody_ctx *c, double t_end, int64_t *n_steps_out) {
    if (!c)
        return NBODY_EINVAL;
    if (!c->initialised)
        return NBODY_ESTATE;
    int64_t tick;
    if (!is_multiple_tick(t_end, c->pr.dt_min_log2, &tick))
        return NBODY_EINVAL;
    NB_TRY(launch_set_i64(reinterpret_cast<int64_t *>(&c->ctl->t_end_tick), tick, c->stream));
    if (!c->graph_exec) {
        int rc = build_graph(c);
        if (rc != NBODY_OK)
            return rc;
    }
    NB_TRY(enqueue_prime(c));
    DevCtl h;
    int rc = read_ctl(c, &h);
    if (rc != NBODY_OK)
        return rc;
    if (h.err)
        return consume_error(c, h);
    const unsigned long long steps0 = h.steps;
    // Two batches in flight: while batch k runs, batch k+1 is already queued,
    // so the GPU does not wait for the host to look at batch k's outcome.
    // Batches after the last active step plan nothing and exit at once.
    c->mirror_h->err = 0;
    c->mirror_h->any_active = 1;
    int64_t launched = 0, waited = 0;
    for (;;) {
        while (launched - waited < 2) {
            NB_TRY(hipGraphLaunch(c->graph_exec, c->stream));
            NB_TRY(hipEventRecord(c->batch_ev[launched & 1], c->stream));
            launched++;
        }
        NB_TRY(hipEventSynchronize(c->batch_ev[waited & 1]));
        waited++;
        // the mirror holds the end of batch `waited` or of a later one
        const volatile HostMirror *m = c->mirror_h;
        if (m->err || !m->any_active)
            break;
    }
    rc = read_ctl(c, &h);  // waits for the batch still in flight
    if (rc != NBODY_OK)
        return rc;
    c->predicted = false;
    if (n_steps_out)
        *n_steps_out = (int64_t)(h.steps - steps0);
    return consume_error(c, h);
}

int nbody_sync(nbody_ctx *c) {
    if (!c)
        return NBODY_EINVAL;
    DevCtl h;
    int rc = read_ctl(c, &h);
    if (rc != NBODY_OK)
        return rc;
    return consume_error(c, h);
}

int nbody_get_stats(nbody_ctx *c, nbody_stats *out) {
    if (!c || !out)
        return NBODY_EINVAL;
    DevCtl h;
    int rc = read_ctl(c, &h);
    if (rc != NBODY_OK)
        return rc;
    out->block_steps = (int64_t)h.steps;
    out->updates = (int64_t)h.updates;
    out->interactions = h.interactions;
    out->dt_clamped = (int64_t)h.clamps;
    return consume_error(c, h);
}

int nbody_read_predicted(nbody_ctx *c, double *pos, double *vel) {
    if (!c || !pos || !vel)
        return NBODY_EINVAL;
    if (!c->predicted)
        return NBODY_ESTATE;
    NB_TRY(launch_read_predicted(c->pr, c->jb, c->cid_d, pos, vel, c->stream));
    return NBODY_OK;
}

int nbody_get_tuning(const nbody_ctx *c, nbody_tuning *out) {
    if (!c || !out || out->size_class < 0 || out->size_class >= kClasses)
        return NBODY_EINVAL;
    const int k = out->size_class;
    out->i_per_lane = c->cls_shape[k].i_per_lane;
    out->j_lanes = c->cls_shape[k].j_lanes;
    out->j_tile = c->cls_shape[k].j_tile;
    out->grid = c->cls_grid[k];
    return NBODY_OK;
}

int nbody_set_tuning(nbody_ctx *c, const nbody_tuning *t) {
    if (!c || !t || t->size_class < 0 || t->size_class >= kClasses)
        return NBODY_EINVAL;
    const Shape sh{t->i_per_lane, t->j_lanes, t->j_tile};
    if (!force_shape_supported(sh) || t->grid < 0)
        return NBODY_EINVAL;
    const int k = t->size_class;
    c->cls_shape[k] = sh;
    c->cls_grid[k] = t->grid;
    std::memset(c->occ_cache[k], 0, sizeof(c->occ_cache[k]));
    drop_graph(c);
    return NBODY_OK;
}

int nbody_set_fused_predict(nbody_ctx *c, int32_t class_mask) {
    if (!c || class_mask < 0 || class_mask >= (1 << kClasses))
        return NBODY_EINVAL;
    c->fused_mask = class_mask;
    drop_graph(c);
    return NBODY_OK;
}

int nbody_autotune(nbody_ctx *c, int64_t n_probe, nbody_tuning *best, double *best_ms) {
    if (!c || !best || n_probe < 1 || n_probe > c->max_cluster)
        return NBODY_EINVAL;
    if (!c->initialised)
        return NBODY_ESTATE;
    const int64_t N = c->pr.n_total;
    // per-cluster block sizes and their mean over clusters
    std::vector<int32_t> nc(c->pr.C);
    int64_t sum = 0;
    for (int k = 0; k < c->pr.C; k++) {
        nc[k] = (int32_t)std::min<int64_t>(n_probe, c->off_h[k + 1] - c->off_h[k]);
        sum += nc[k];
    }
    const int cls = class_of(c, sum / c->pr.C);
    // the time the j-particle buffer was predicted to, where known (the near
    // field's FP64 velocities are predicted to the evaluation time)
    const int64_t t_probe = c->predicted ? c->predicted_tick : 0;
    static const Shape cand[] = {{1, 1, 256}, {2, 1, 256}, {1, 4, 256}, {1, 16, 256},
                                 {1, 64, 256}, {1, 256, 256}};
    const Shape keep = c->cls_shape[cls];
    const int keep_grid = c->cls_grid[cls];
    hipEvent_t e0, e1;
    NB_TRY(hipEventCreate(&e0));
    NB_TRY(hipEventCreate(&e1));
    // every candidate's time; the pick is made below
    double cand_t[sizeof(cand) / sizeof(cand[0])];
    int rc = NBODY_OK;
    int ci = 0;
    for (const Shape &sh : cand) {
        c->cls_shape[cls] = sh;
        c->cls_grid[cls] = 0;
        std::memset(c->occ_cache[cls], 0, sizeof(c->occ_cache[cls]));
        float ms_min = 1e30f;
        for (int rep = 0; rep < 5 && rc == NBODY_OK; rep++) {
            hipError_t e = hipSuccess;
            if (c->pr.C == 1) {
                e = hipEventRecord(e0, c->stream);
                if (e == hipSuccess)
                    e = enqueue_force(c, c->iota_d, 0, nc[0], t_probe, 0, c->acc_new,
                                      c->jerk_new, nullptr, N, nc[0]);
            } else {
                e = hipMemcpyAsync(c->n_act_d, nc.data(), nc.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, c->stream);
                if (e == hipSuccess)
                    e = launch_fill_i64(c->t_next_d, t_probe, c->pr.C, c->stream);
                if (e == hipSuccess)
                    e = hipEventRecord(e0, c->stream);
                if (e == hipSuccess)
                    e = enqueue_force(c, c->iota_d, 1, kPlanFromLists, 0, 0, c->acc_new, c->jerk_new,
                                      nullptr, N, N);
            }
            if (e == hipSuccess)
                e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess)
                e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess)
                e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = map_err(e);
                break;
            }
            if (rep > 0)  // the first call warms caches and code
                ms_min = std::min(ms_min, ms);
        }
        if (rc != NBODY_OK)
            break;
        cand_t[ci++] = ms_min;
    }
    // The fastest shape; if that is a lane-group shape, the widest lane group
    // within 3% of it instead: the blocks a class meets in a run are spread
    // around the probe size, and uneven over the clusters of an ensemble, and
    // wider groups lose less on blocks smaller than the probe (all lane-group
    // shapes share one launch, so the choice adds no launch to a step).
    double best_t = 1e300;
    Shape best_s = keep;
    if (rc == NBODY_OK) {
        int fq = 0;
        for (int q = 1; q < ci; q++)
            if (cand_t[q] < cand_t[fq])
                fq = q;
        best_t = cand_t[fq];
        best_s = cand[fq];
        if (force_shape_grouped(best_s)) {
            const double lim = 1.03 * cand_t[fq];
            for (int q = 0; q < ci; q++)
                if (force_shape_grouped(cand[q]) && cand_t[q] <= lim &&
                    cand[q].j_lanes > best_s.j_lanes) {
                    best_t = cand_t[q];
                    best_s = cand[q];
                }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the device plan arrays were used as scratch; leave no pending block
    (void)launch_fill_i32(c->n_act_d, 0, c->pr.C, c->stream);
    (void)launch_fill_i64(c->t_next_d, LLONG_MAX, c->pr.C, c->stream);
    if (rc != NBODY_OK) {
        c->cls_shape[cls] = keep;
        c->cls_grid[cls] = keep_grid;
        std::memset(c->occ_cache[cls], 0, sizeof(c->occ_cache[cls]));
        return rc;
    }
    c->cls_shape[cls] = best_s;
    c->cls_grid[cls] = 0;
    std::memset(c->occ_cache[cls], 0, sizeof(c->occ_cache[cls]));
    drop_graph(c);
    best->size_class = cls;
    best->i_per_lane = best_s.i_per_lane;
    best->j_lanes = best_s.j_lanes;
    best->j_tile = best_s.j_tile;
    best->grid = 0;
    if (best_ms)
        *best_ms = best_t;
    DevCtl h;
    rc = read_ctl(c, &h);
    if (rc != NBODY_OK)
        return rc;
    return consume_error(c, h);
}

int nbody_save(nbody_ctx *c, const char *path) {
    if (!c || !path)
        return NBODY_EINVAL;
    if (!c->initialised)
        return NBODY_ESTATE;
    DevCtl h;
    int rc = read_ctl(c, &h);
    if (rc != NBODY_OK)
        return rc;
    if (h.err)
        return consume_error(c, h);
    const int64_t N = c->pr.n_total;
    const State &st = c->st;
    const double *src[13] = {st.x,  st.y,  st.z,  st.vx, st.vy, st.vz, st.ax,
                             st.ay, st.az, st.jx, st.jy, st.jz, st.m};
    std::vector<double> buf;
    std::vector<int64_t> tick;
    std::vector<int8_t> lev;
    try {
        buf.resize(13 * (size_t)N);
        tick.resize(N);
        lev.resize(N);
    } catch (const std::bad_alloc &) {
        return NBODY_ENOMEM;
    }
    for (int q = 0; q < 13; q++)
        NB_TRY(hipMemcpy(buf.data() + q * N, src[q], N * sizeof(double), hipMemcpyDeviceToHost));
    NB_TRY(hipMemcpy(tick.data(), st.tick, N * sizeof(int64_t), hipMemcpyDeviceToHost));
    NB_TRY(hipMemcpy(lev.data(), st.lev, N * sizeof(int8_t), hipMemcpyDeviceToHost));
    std::vector<float4> scales(c->pr.C);
    NB_TRY(hipMemcpy(scales.data(), c->nscale_d, scales.size() * sizeof(float4),
                     hipMemcpyDeviceToHost));
    std::vector<double4> origins(c->pr.C);
    NB_TRY(hipMemcpy(origins.data(), c->origin_d, origins.size() * sizeof(double4),
                     hipMemcpyDeviceToHost));

    // write beside the target, then rename: an existing checkpoint is replaced
    // only by a complete one
    const std::string tmp = std::string(path) + ".part";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f)
        return NBODY_EIO;
    CkptWriter w{f};
    if (std::fwrite(kCkptMagic, 1, sizeof(kCkptMagic), f) != sizeof(kCkptMagic))
        w.ok = false;
    const CkptConfig k = ckpt_config(c);
    w.put(&kCkptVersion, sizeof(kCkptVersion));
    w.put(&k.n_total, 8);
    w.put(&k.n_clusters, 4);
    w.put(&k.precision, 4);
    w.put(&k.eps, 8);
    w.put(&k.eta, 8);
    w.put(&k.eta_init, 8);
    w.put(&k.dt_min_log2, 4);
    w.put(&k.dt_max_log2, 4);
    w.put(c->off_h.data(), (c->off_h.size()) * sizeof(int64_t));
    const uint64_t stats[3] = {h.steps, h.updates, h.clamps};
    w.put(stats, sizeof(stats));
    w.put(&h.interactions, sizeof(double));
    for (int q = 0; q < kClasses; q++) {
        const int32_t t[4] = {c->cls_shape[q].i_per_lane, c->cls_shape[q].j_lanes,
                              c->cls_shape[q].j_tile, c->cls_grid[q]};
        w.put(t, sizeof(t));
    }
    w.put(scales.data(), scales.size() * sizeof(float4));
    w.put(origins.data(), origins.size() * sizeof(double4));
    w.put(buf.data(), buf.size() * sizeof(double));
    w.put(tick.data(), tick.size() * sizeof(int64_t));
    w.put(lev.data(), lev.size());
    const uint64_t sum = w.sum.h;
    if (w.ok && std::fwrite(&sum, 1, sizeof(sum), f) != sizeof(sum))
        w.ok = false;
    if (std::fclose(f) != 0)
        w.ok = false;
    if (w.ok && std::rename(tmp.c_str(), path) != 0)
        w.ok = false;
    if (!w.ok) {
        (void)std::remove(tmp.c_str());
        return NBODY_EIO;
    }
    return NBODY_OK;
}

int nbody_load(nbody_ctx *c, const char *path) {
    if (!c || !path)
        return NBODY_EINVAL;
    FILE *f = std::fopen(path, "rb");
    if (!f)
        return NBODY_EIO;
    auto done = [&](int rc) {
        std::fclose(f);
        return rc;
    };
    char magic[sizeof(kCkptMagic)];
    if (std::fread(magic, 1, sizeof(magic), f) != sizeof(magic) ||
        std::memcmp(magic, kCkptMagic, sizeof(magic)) != 0)
        return done(NBODY_EIO);
    CkptReader r{f};
    uint32_t ver = 0;
    r.get(&ver, sizeof(ver));
    if (!r.ok || (ver != kCkptVersion && ver != 2))
        return done(NBODY_EIO);
    CkptConfig k{};
    r.get(&k.n_total, 8);
    r.get(&k.n_clusters, 4);
    r.get(&k.precision, 4);
    r.get(&k.eps, 8);
    r.get(&k.eta, 8);
    r.get(&k.eta_init, 8);
    r.get(&k.dt_min_log2, 4);
    r.get(&k.dt_max_log2, 4);
    if (!r.ok)
        return done(NBODY_EIO);
    const CkptConfig mine = ckpt_config(c);
    // a checkpoint of another configuration: refuse before reading further
    if (k.n_total != mine.n_total || k.n_clusters != mine.n_clusters ||
        k.precision != mine.precision || k.eps != mine.eps || k.eta != mine.eta ||
        k.eta_init != mine.eta_init || k.dt_min_log2 != mine.dt_min_log2 ||
        k.dt_max_log2 != mine.dt_max_log2)
        return done(NBODY_EINVAL);
    std::vector<int64_t> off(c->off_h.size());
    r.get(off.data(), off.size() * sizeof(int64_t));
    if (!r.ok)
        return done(NBODY_EIO);
    if (off != c->off_h)
        return done(NBODY_EINVAL);
    uint64_t stats[3];
    double interactions = 0.0;
    r.get(stats, sizeof(stats));
    r.get(&interactions, sizeof(double));
    Shape shape[kClasses];
    int32_t grid[kClasses];
    for (int q = 0; q < kClasses; q++) {
        int32_t t[4] = {0, 0, 0, 0};
        r.get(t, sizeof(t));
        shape[q] = Shape{t[0], t[1], t[2]};
        grid[q] = t[3];
    }
    const int64_t N = c->pr.n_total;
    std::vector<double> buf;
    std::vector<int64_t> tick;
    std::vector<int8_t> lev;
    std::vector<float4> scales;
    std::vector<double4> origins;
    try {
        buf.resize(13 * (size_t)N);
        tick.resize(N);
        lev.resize(N);
        scales.resize(c->pr.C);
        origins.assign(c->pr.C, make_double4(0.0, 0.0, 0.0, 0.0));
    } catch (const std::bad_alloc &) {
        return done(NBODY_ENOMEM);
    }
    r.get(scales.data(), scales.size() * sizeof(float4));
    if (ver >= 3)
        r.get(origins.data(), origins.size() * sizeof(double4));
    r.get(buf.data(), buf.size() * sizeof(double));
    r.get(tick.data(), tick.size() * sizeof(int64_t));
    r.get(lev.data(), lev.size());
    uint64_t stored = 0;
    if (!r.ok || std::fread(&stored, 1, sizeof(stored), f) != sizeof(stored) ||
        stored != r.sum.h || std::fgetc(f) != EOF)
        return done(NBODY_EIO);
    for (int q = 0; q < kClasses; q++)
        if (!force_shape_supported(shape[q]) || grid[q] < 0)
            return done(NBODY_EIO);
    std::fclose(f);

    // everything read and checked: only now overwrite the caller's state
    State &st = c->st;
    double *dst[13] = {st.x, st.y, st.z, st.vx, st.vy, st.vz, st.ax, st.ay, st.az,
                       st.jx, st.jy, st.jz, st.m};
    NB_TRY(hipStreamSynchronize(c->stream));
    for (int q = 0; q < 13; q++)
        NB_TRY(hipMemcpy(dst[q], buf.data() + q * N, N * sizeof(double), hipMemcpyHostToDevice));
    NB_TRY(hipMemcpy(st.tick, tick.data(), N * sizeof(int64_t), hipMemcpyHostToDevice));
    NB_TRY(hipMemcpy(st.lev, lev.data(), N * sizeof(int8_t), hipMemcpyHostToDevice));
    NB_TRY(upload_cluster_scales(c, buf.data() + 12 * N, buf.data() + 3 * N, scales.data()));
    NB_TRY(upload_origins(c, buf.data(), origins.data()));
    DevCtl h;
    int rc = read_ctl(c, &h);
    if (rc != NBODY_OK)
        return rc;
    h.err = 0;
    h.steps = stats[0];
    h.updates = stats[1];
    h.clamps = stats[2];
    h.interactions = interactions;
    NB_TRY(hipMemcpy(c->ctl, &h, sizeof(h), hipMemcpyHostToDevice));
    for (int q = 0; q < kClasses; q++) {
        c->cls_shape[q] = shape[q];
        c->cls_grid[q] = grid[q];
    }
    std::memset(c->occ_cache, 0, sizeof(c->occ_cache));
    drop_graph(c);
    c->initialised = true;
    c->predicted = false;
    return NBODY_OK;
}

}  // extern "C"
