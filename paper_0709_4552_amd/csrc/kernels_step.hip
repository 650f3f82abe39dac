// Block-step kernels: selection, work planning, prediction, j-split
// reduction, Hermite correction and start-up.  All FP64 except the mixed
// j-particle buffer written by the predictor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "nbody_internal.h"

namespace nb {

namespace {

__device__ inline bool finite3(double a, double b, double c) {
    return isfinite(a) && isfinite(b) && isfinite(c);
}

__device__ inline double norm3(double a, double b, double c) {
    return sqrt(a * a + b * b + c * c);
}

__device__ inline int64_t dt_ticks(int lev_max, int lev) {
    return (int64_t)1 << (lev_max - lev);
}

// ---------------------------------------------------------------- fills
__global__ void k_fill_i64(int64_t *p, int64_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_f64(double *p, double v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_iota_i32(int32_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

// ---------------------------------------------------------------- predictor
// Prediction of particle i (of cluster c) to time T written to the
// j-particle buffer (the arithmetic is shared with the force kernels'
// in-kernel prediction).  False when a mixed record falls outside the exact
// range around the cluster's origin.
template <int MIXED>
__device__ inline bool predict_one(const State &st, const Params &pr, const JBuf &jb, int64_t i,
                                   int64_t T, int c) {
    if (MIXED) {
        float4 P, Q, V;
        float2 R;
        const bool ok = predict_mixed(st, pr.tick, pr.grid_q, pr.grid_inv, pr.origin[c], i, T, P,
                                      Q, R, V);
        jb.P[i] = P;
        jb.Q[i] = Q;
        jb.R[i] = R;
        jb.V[i] = V;
        return ok;
    } else {
        double2 A, B, C;
        double D;
        predict_fp64(st, pr.tick, i, T, A, B, C, D);
        jb.A[i] = A;
        jb.B[i] = B;
        jb.C[i] = C;
        jb.D[i] = D;
        return true;
    }
}

// Prediction of every particle, to the host's time or to its cluster's
// planned time (clusters with an empty block are skipped).
template <int MIXED>
__global__ __launch_bounds__(kWG) void k_predict(State st, Params pr, JBuf jb, const int32_t *cid,
                                                  const int64_t *t_cur, const int32_t *n_cur,
                                                  int64_t t_host, int use_host_t, DevCtl *ctl) {
    bool ok = true;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < pr.n_total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = pr.C > 1 ? cid[i] : 0;
        int64_t T = t_host;
        if (!use_host_t) {
            if (n_cur[c] == 0)
                continue;
            T = t_cur[c];
        }
        ok = predict_one<MIXED>(st, pr, jb, i, T, c) && ok;
    }
    if (!ok)
        atomicOr(&ctl->err, kErrExtent);
}

// The predicted positions and velocities in the caller's frame (the mixed
// records are relative to the cluster's origin).
__global__ void k_read_predicted(Params pr, JBuf jb, const int32_t *cid, double *pos, double *vel,
                                 int mixed) {
    const int64_t n = pr.n_total;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (mixed) {
            const float4 p = jb.P[i], q = jb.Q[i];
            const float2 r = jb.R[i];
            const double4 o = pr.origin[pr.C > 1 ? cid[i] : 0];
            pos[i] = ((double)p.x + (double)q.x) + o.x;
            pos[n + i] = ((double)p.y + (double)q.y) + o.y;
            pos[2 * n + i] = ((double)p.z + (double)q.z) + o.z;
            vel[i] = q.w;
            vel[n + i] = r.x;
            vel[2 * n + i] = r.y;
        } else {
            const double2 a = jb.A[i], b = jb.B[i], c = jb.C[i];
            pos[i] = a.x;
            pos[n + i] = a.y;
            pos[2 * n + i] = b.x;
            vel[i] = c.x;
            vel[n + i] = c.y;
            vel[2 * n + i] = jb.D[i];
        }
    }
}

// ---------------------------------------------------------------- selection
// Block-step scheme (section 4.1, steps 1-2).  A particle on level L (step
// dt_L = 2^-L) is stepped only at multiples of dt_L, and every particle was
// last stepped at or before its cluster's latest block time t_now.  So its
// last time is the latest multiple of dt_L not after t_now, and its next time
// the following multiple: all particles of one level share it.  The next block
// time is therefore the minimum of that over the occupied levels, and the block
// is every particle on a level whose step divides it.  The per-level counts of
// each cluster, kept up to date by the corrector, give both without a scan.
__device__ inline int64_t level_next(int64_t t_now, int shift) {
    return ((t_now >> shift) + 1) << shift;  // arithmetic shift: floor, also for t_now = -1
}

// Level L (lev_min <= L <= lev_max) is due at block time T when its step
// divides T.
__device__ inline bool level_due(const Params &pr, int L, int64_t T) {
    return (T & (dt_ticks(pr.lev_max, L) - 1)) == 0;
}

__device__ inline int32_t *list_at(const LevelLists &ll, int b, int L, int64_t cb) {
    return ll.idx + ((int64_t)b * ll.nlev + (L - ll.lev_min)) * ll.n_total + cb;
}

__device__ inline int32_t *list_cnt(const LevelLists &ll, int b, int c, int L) {
    return ll.cnt + ((int64_t)b * ll.C + c) * kLevels + L;
}

// Priming scan before a run of block steps: level counts, earliest next time
// and latest last time of each cluster.  A valid block-step state has every
// last time before every next time and each last time a multiple of the
// particle's step; anything else is flagged as not due.
__global__ __launch_bounds__(kWG) void k_prime(State st, Params pr, const int64_t *off,
                                               const int32_t *chunk_c, const int64_t *chunk_b,
                                               int32_t *lev_cnt, LevelLists ll, int64_t *t_min,
                                               int64_t *t_max, DevCtl *ctl) {
    __shared__ int32_t hist[kLevels];
    __shared__ int32_t lbase[kLevels];
    __shared__ unsigned long long rmin[kWG / 64], rmax[kWG / 64];
    if (threadIdx.x < kLevels)
        hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t k = blockIdx.x;
    const int c = uniform_i32(chunk_c[k]);
    const int64_t b = uniform_i64(chunk_b[k]);
    const int64_t e = min(uniform_i64(off[c + 1]), b + kChunk);
    const int64_t i = b + threadIdx.x;
    unsigned long long nmin = ULLONG_MAX, tmax = 0;
    int32_t err = 0;
    int lev = 0, rank = -1;
    if (i < e) {
        lev = st.lev[i];
        const int64_t tk = st.tick[i];
        if (lev < pr.lev_min || lev > pr.lev_max || tk < 0) {
            err = kErrNotDue;
        } else {
            const int64_t dtk = dt_ticks(pr.lev_max, lev);
            if (tk & (dtk - 1))
                err = kErrNotDue;
            rank = atomicAdd(&hist[lev], 1);
            nmin = (unsigned long long)(tk + dtk);
            tmax = (unsigned long long)tk;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long a = __shfl_xor(nmin, o), m = __shfl_xor(tmax, o);
        nmin = a < nmin ? a : nmin;
        tmax = m > tmax ? m : tmax;
    }
    if ((threadIdx.x & 63) == 0) {
        rmin[threadIdx.x >> 6] = nmin;
        rmax[threadIdx.x >> 6] = tmax;
    }
    if (err)
        atomicOr(&ctl->err, err);
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWG / 64; w++) {
            nmin = rmin[w] < nmin ? rmin[w] : nmin;
            tmax = rmax[w] > tmax ? rmax[w] : tmax;
        }
        atomicMin((unsigned long long *)&t_min[c], nmin);
        atomicMax((unsigned long long *)&t_max[c], tmax);
    }
    // level counts, and each particle into the list of its level (buffer 0)
    if (threadIdx.x < kLevels && hist[threadIdx.x] != 0) {
        atomicAdd(&lev_cnt[(int64_t)c * kLevels + threadIdx.x], hist[threadIdx.x]);
        lbase[threadIdx.x] = atomicAdd(list_cnt(ll, 0, c, threadIdx.x), hist[threadIdx.x]);
    }
    __syncthreads();
    if (rank >= 0)
        list_at(ll, 0, lev, uniform_i64(off[c]))[lbase[lev] + rank] = (int32_t)i;
}

// t_now = (earliest next time) - 1: every level's next time computed from it is
// then the true one, provided the state passed the checks above.
__global__ void k_prime_finish(Params pr, const int64_t *t_min, const int64_t *t_max,
                               int64_t *t_now, DevCtl *ctl) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < pr.C; c += gridDim.x * blockDim.x) {
        if (t_max[c] >= t_min[c])
            atomicOr(&ctl->err, kErrNotDue);
        t_now[c] = t_min[c] - 1;
    }
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP moves: row
// shifts by 1, 2, 4 and 8, then the row broadcasts of lanes 15 and 31.  Lanes
// whose shifted source lies outside their row add 0.  Every lane takes part.
__device__ inline int64_t wave_inclusive_scan(int64_t v) {
    v += __builtin_amdgcn_update_dpp((int64_t)0, v, 0x111, 0xF, 0xF, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp((int64_t)0, v, 0x112, 0xF, 0xF, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp((int64_t)0, v, 0x114, 0xF, 0xF, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp((int64_t)0, v, 0x118, 0xF, 0xF, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp((int64_t)0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp((int64_t)0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

// The block of cluster c at block time T in slot order: the lists of its due
// levels, levels ascending.  Wave 0 writes each level's buffer and the
// exclusive prefix of the due counts to LDS (s_pre[64] = total) and returns
// the total, which must equal the block size the level counts gave.
__device__ inline int64_t due_prefix(const Params &pr, const LevelLists &ll, int c, int64_t T,
                                     int32_t *s_buf, int32_t *s_pre) {
    const int L = threadIdx.x & 63;
    const bool in = L >= pr.lev_min && L <= pr.lev_max;
    const int b = in ? ll.buf[(int64_t)c * kLevels + L] : 0;
    const int32_t cnt = (in && level_due(pr, L, T)) ? *list_cnt(ll, b, c, L) : 0;
    const int64_t incl = wave_inclusive_scan((int64_t)cnt);
    s_buf[L] = b;
    s_pre[L] = (int32_t)(incl - cnt);
    if (L == 63)
        s_pre[kLevels] = (int32_t)incl;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)incl, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)incl >> 32), 63);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Particle in slot k of the block (0 <= k < total): the level whose prefix
// range holds k (the largest L with s_pre[L] <= k), then its place there.
__device__ inline int32_t gather_slot(const LevelLists &ll, int64_t cb, int64_t k,
                                      const int32_t *s_buf, const int32_t *s_pre) {
    int lo = 0, hi = kLevels - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= k)
            lo = mid;
        else
            hi = mid - 1;
    }
    return list_at(ll, s_buf[lo], lo, cb)[k - s_pre[lo]];
}

// One ensemble block step's scan (after the plan): predict every particle of
// a stepping cluster to its block time and gather the cluster's block from its
// level lists into the active list (slot of (c, k) = off[c] + k).  One
// workgroup per chunk, one particle and one slot per thread.
template <int MIXED>
__global__ __launch_bounds__(kWG) void k_predict_gather(State st, Params pr, JBuf jb,
                                                        const int64_t *off,
                                                        const int32_t *chunk_c,
                                                        const int64_t *chunk_b, PlanDev pl,
                                                        LevelLists ll, int32_t *i_list,
                                                        DevCtl *ctl) {
    static_assert(kChunk == kWG, "one particle per thread");
    __shared__ int32_t s_buf[kLevels], s_pre[kLevels + 1];
    const int64_t k = blockIdx.x;
    const int c = uniform_i32(chunk_c[k]);
    const int64_t n = uniform_i32(pl.n_cur[c]);
    if (n == 0)
        return;
    const int64_t T = uniform_i64(pl.t_cur[c]);
    const int64_t cb = uniform_i64(off[c]);
    const int64_t b = uniform_i64(chunk_b[k]);
    const int64_t e = min(uniform_i64(off[c + 1]), b + kChunk);
    if (threadIdx.x < 64) {
        const int64_t tot = due_prefix(pr, ll, c, T, s_buf, s_pre);
        if (b == cb && threadIdx.x == 0 && tot != n)
            atomicOr(&ctl->err, kErrPlan);
    }
    __syncthreads();
    const int64_t i = b + threadIdx.x;
    if (i < e) {
        if (!predict_one<MIXED>(st, pr, jb, i, T, c))
            atomicOr(&ctl->err, kErrExtent);
        // (a list total other than n has been flagged; gather no slot past it)
        if (i - cb < n && i - cb < s_pre[kLevels])
            i_list[i] = gather_slot(ll, cb, i - cb, s_buf, s_pre);
    }
}

// ---------------------------------------------------------------- planning
// Next block of cluster c from its level counts (one thread).  n = 0 when the
// cluster's next time lies beyond t_end; then the cluster's time stays.
__device__ inline int32_t block_from_levels(const Params &pr, const PlanDev &pl, int c,
                                            int64_t t_end, int64_t *T_out) {
    const int32_t *cnt = pl.lev_cnt + (int64_t)c * kLevels;
    const int64_t tnow = pl.t_now[c];
    int64_t T = INT64_MAX;
    for (int L = pr.lev_min; L <= pr.lev_max; L++)
        if (cnt[L] > 0) {
            const int64_t t = level_next(tnow, pr.lev_max - L);
            T = t < T ? t : T;
        }
    int32_t n = 0;
    if (T != INT64_MAX && T <= t_end)
        for (int L = pr.lev_min; L <= pr.lev_max; L++)
            if (cnt[L] > 0 && (T & (dt_ticks(pr.lev_max, L) - 1)) == 0)
                n += cnt[L];
    *T_out = n > 0 ? T : tnow;
    return n;
}

// Exclusive prefix sum over the kPlanThreads threads of the workgroup, and the
// total: wavefront scans, then a scan of the wave totals (two barriers; tmp
// needs 2 * kPlanThreads / 64 entries).
__device__ int64_t block_exclusive_scan(int64_t v, int64_t *tmp, int64_t *total) {
    constexpr int NW = kPlanThreads / 64;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t incl = wave_inclusive_scan(v);
    if (lane == 63)
        tmp[w] = incl;
    __syncthreads();
    if (w == 0) {
        const int64_t tot = wave_inclusive_scan(lane < NW ? tmp[lane] : 0);
        if (lane < NW)
            tmp[NW + lane] = tot;
    }
    __syncthreads();
    const int64_t before = w > 0 ? tmp[NW + w - 1] : 0;
    *total = tmp[2 * NW - 1];
    __syncthreads();
    return before + incl - v;
}

// Work list of one force evaluation of an ensemble (several clusters; one
// cluster is planned by plan_single_wave): cluster c gets ceil(n_c / ib)
// i-blocks times S_c j-slices.  The shape class (and so ib) follows the mean
// block size of the active clusters; S_c follows the cluster's share of the
// work so the whole evaluation has about 4*grid items, and the force kernel's
// work queue balances the rest.  One workgroup.
__global__ __launch_bounds__(kPlanThreads) void k_plan(Params pr, const int64_t *off, PlanDev pl,
                                                       int32_t *n_act, int64_t *t_next,
                                                       DevCtl *ctl, int64_t part_cap,
                                                       ClassTable ct,
                                                       int32_t host_n, int64_t host_t,
                                                       int32_t count_stats) {
    __shared__ int64_t tmp[kPlanThreads];
    __shared__ double dred[kPlanThreads];
    __shared__ int64_t carry_items, carry_parts;
    __shared__ int s_fallback;
    const int t = threadIdx.x;
    const int C = pr.C;
    const int64_t t_end = ctl->t_end_tick;
    if (t == 0)
        ctl->s_max = 0;
    // pass 1: take the block sizes of this step; total work
    double w_local = 0.0;
    int64_t n_local = 0, act_local = 0;
    for (int c = t; c < C; c += kPlanThreads) {
        int32_t n;
        if (host_n >= 0) {
            n = host_n;
            pl.t_cur[c] = host_t;
        } else if (host_n == kPlanFromLists) {
            n = n_act[c];
            pl.t_cur[c] = t_next[c];
            n_act[c] = 0;
            t_next[c] = LLONG_MAX;
        } else {
            int64_t T;
            n = block_from_levels(pr, pl, c, t_end, &T);
            pl.t_cur[c] = T;
            pl.t_now[c] = T;
        }
        pl.n_cur[c] = n;
        const double nc = (double)(off[c + 1] - off[c]);
        w_local += (double)n * nc;
        n_local += n;
        act_local += n > 0;
    }
    // totals over the workgroup: wavefront sums (DPP), then the 16 wave sums in
    // order by thread 0
    {
        constexpr int NW = kPlanThreads / 64;
        const int lane = t & 63, w = t >> 6;
        const double wsum = group_sum<64>(w_local);
        const int64_t nsum = wave_inclusive_scan(n_local);
        const int64_t asum = wave_inclusive_scan(act_local);
        if (lane == 63) {
            dred[w] = wsum;
            tmp[w] = nsum;
            tmp[NW + w] = asum;
        }
        __syncthreads();
        if (t == 0) {
            double wt = 0.0;
            int64_t nt = 0, at = 0;
            for (int q = 0; q < NW; q++) {
                wt += dred[q];
                nt += tmp[q];
                at += tmp[NW + q];
            }
            dred[NW] = wt;
            tmp[2 * NW] = nt;
            tmp[2 * NW + 1] = at;
        }
        __syncthreads();
    }
    const double W = dred[kPlanThreads / 64];
    const int64_t n_sum = tmp[2 * (kPlanThreads / 64)];
    const int64_t n_active_clusters = tmp[2 * (kPlanThreads / 64) + 1];
    __syncthreads();
    // shape class from the mean block size
    const int64_t n_mean = n_active_clusters > 0 ? n_sum / n_active_clusters : 0;
    int cls = kClasses - 1;
    for (int k = 0; k < kClasses; k++)
        if (n_mean >= ct.min_n[k]) {
            cls = k;
            break;
        }
    const int64_t ib_size = ct.ib[cls];
    const int64_t grid_res = ct.grid[cls];
    const int32_t j_tile = ct.jt[cls];
    if (t == 0)
        s_fallback = 0;
    __syncthreads();
    // pass 2 (repeated once with S = 1 if the partial-sum buffer would overflow)
    for (int attempt = 0; attempt < 2; attempt++) {
        if (t == 0) {
            carry_items = 0;
            carry_parts = 0;
        }
        __syncthreads();
        for (int c0 = 0; c0 < C; c0 += kPlanThreads) {
            const int c = c0 + t;
            int64_t items = 0, parts = 0;
            int32_t S = 0, jl = 0;
            if (c < C) {
                const int64_t n = pl.n_cur[c];
                const int64_t Nc = off[c + 1] - off[c];
                if (n > 0 && Nc > 0) {
                    const int64_t nib = (n + ib_size - 1) / ib_size;
                    const int64_t tiles = (Nc + j_tile - 1) / j_tile;
                    int64_t s = 1;
                    if (!uniform_i32(s_fallback)) {
                        if (W > 0.0) {
                            const double share = (double)n * (double)Nc / W;
                            s = (int64_t)ceil(4.0 * (double)grid_res * share / (double)nib);
                        }
                        s = s < 1 ? 1 : (s > tiles ? tiles : s);
                    }
                    const int64_t tiles_per = (tiles + s - 1) / s;
                    jl = (int32_t)(tiles_per * j_tile);
                    S = (int32_t)((Nc + jl - 1) / jl);
                    items = nib * S;
                    parts = S > 1 ? (int64_t)S * n : 0;
                }
                pl.S[c] = S;
                pl.jlen[c] = jl;
                if (S > 1)
                    atomicMax(&ctl->s_max, S);
            }
            int64_t tot_i, tot_p;
            const int64_t ex_i = block_exclusive_scan(items, tmp, &tot_i);
            const int64_t ex_p = block_exclusive_scan(parts, tmp, &tot_p);
            if (c < C) {
                pl.item_begin[c] = carry_items + ex_i;
                pl.part_begin[c] = carry_parts + ex_p;
            }
            __syncthreads();
            if (t == 0) {
                carry_items += tot_i;
                carry_parts += tot_p;
            }
            __syncthreads();
        }
        if (uniform_i64(carry_parts) <= part_cap)
            break;
        __syncthreads();
        if (t == 0)
            s_fallback = 1;
        __syncthreads();
    }
    if (t == 0) {
        pl.item_begin[C] = carry_items;
        ctl->total_items = carry_items;
        ctl->part_used = carry_parts;
        ctl->item_counter = 0;
        ctl->cls = cls;
        ctl->n_last = (int32_t)n_sum;
        ctl->any_active = n_sum > 0;
        if (carry_parts > part_cap)
            ctl->err |= kErrPlan;
        if (count_stats) {
            ctl->steps += (unsigned long long)n_active_clusters;
            ctl->updates += (unsigned long long)n_sum;
            ctl->interactions += W;
        }
    }
}

// One cluster, one wave (lane L looks at level L): the next block's time and
// size from the level counts; n = 0 (and the time unchanged) when the next
// time lies beyond t_end.  Every lane returns the same values.
// Minimum and sum over the 64 lanes of a wave with DPP moves (quad swaps,
// half-row and row mirrors, the row broadcasts of lanes 15 and 31; lanes a
// step leaves out take the identity), read back from lane 63 so every lane
// holds the result.
template <int CTRL, int ROW_MASK = 0xF>
__device__ inline int64_t dpp_min_step(int64_t v) {
    const int64_t o = __builtin_amdgcn_update_dpp((int64_t)INT64_MAX, v, CTRL, ROW_MASK, 0xF, false);
    return o < v ? o : v;
}

__device__ inline int64_t wave_min_i64(int64_t v) {
    v = dpp_min_step<0xB1>(v);
    v = dpp_min_step<0x4E>(v);
    v = dpp_min_step<0x141>(v);
    v = dpp_min_step<0x140>(v);
    v = dpp_min_step<0x142, 0xA>(v);
    v = dpp_min_step<0x143, 0xC>(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), 63);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ inline int32_t wave_sum_i32(int32_t v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ inline void next_block_wave(const Params &pr, const PlanDev &pl, int64_t t_end,
                                       int64_t *T_out, int64_t *n_out) {
    static_assert(kLevels == 64, "one level per lane");
    const int lane = threadIdx.x & 63;
    const bool in = lane >= pr.lev_min && lane <= pr.lev_max;
    const int32_t cnt = in ? pl.lev_cnt[lane] : 0;
    const int sh = in ? pr.lev_max - lane : 0;
    const int64_t tnow = uniform_i64(pl.t_now[0]);
    int64_t T = wave_min_i64(cnt > 0 ? level_next(tnow, sh) : INT64_MAX);
    const int32_t due = (cnt > 0 && T != INT64_MAX && (T & (((int64_t)1 << sh) - 1)) == 0) ? cnt : 0;
    int64_t n = wave_sum_i32(due);
    if (T == INT64_MAX || T > t_end) {
        n = 0;
        T = tnow;
    }
    *T_out = T;
    *n_out = n;
}

// One cluster, one wave: the plan of an evaluation of n particles at time
// tcur.  Lane l evaluates j-split counts S = l+1, l+65, ... (up to kMaxSlices)
// with the cost model above; a wave minimum picks the best (ties -> smaller
// S); lane 0 writes the plan.  No barriers and no early exit, so it can run
// inside a larger kernel.
__device__ inline void plan_single_wave(const int64_t *off, const PlanDev &pl, DevCtl *ctl,
                                        int64_t part_cap, const ClassTable &ct, int64_t n,
                                        int64_t tcur, int32_t count_stats) {
    const int lane = threadIdx.x & 63;
    const int64_t Nc = off[1] - off[0];
    const int cls = plan_class(ct, n);
    const int64_t ib_size = ct.ib[cls];
    const int64_t grid_res = ct.grid[cls];
    const int64_t j_tile = ct.jt[cls];
    const int64_t tiles = (Nc + j_tile - 1) / j_tile;
    const int64_t nib = (n + ib_size - 1) / ib_size;
    const int64_t grid = plan_grid(grid_res, nib, tiles);
    const uint32_t tiles32 = (uint32_t)tiles;
    const double nibd = (double)nib, inv_grid = 1.0 / (double)grid;
    int64_t key = INT64_MAX;
    for (uint32_t S = lane + 1; S <= (uint32_t)kMaxSlices && S <= tiles32; S += 64) {
        const int64_t k2 = plan_key(S, tiles32, nibd, inv_grid, grid, n, part_cap);
        key = k2 < key ? k2 : key;
    }
    key = wave_min_i64(key);
    if (lane == 0) {
        const PlanChoice pc = plan_from_key(key, cls, n, Nc, tiles, j_tile, nib);
        const int64_t items = pc.items, parts = pc.parts;
        const int32_t jl = pc.jl, Sfin = pc.S;
        pl.n_cur[0] = (int32_t)n;
        pl.t_cur[0] = tcur;
        pl.S[0] = Sfin;
        pl.jlen[0] = jl;
        pl.item_begin[0] = 0;
        pl.item_begin[1] = items;
        pl.part_begin[0] = 0;
        ctl->total_items = items;
        ctl->part_used = parts;
        ctl->item_counter = 0;
        ctl->cls = cls;
        ctl->s_max = Sfin > 1 ? Sfin : 0;
        ctl->n_last = (int32_t)n;
        ctl->any_active = n > 0;
        if (count_stats) {
            ctl->steps += n > 0 ? 1ull : 0ull;
            ctl->updates += (unsigned long long)n;
            ctl->interactions += (double)n * (double)Nc;
        }
    }
}

// One cluster, an explicit evaluation: n and t from the host, or from n_act /
// t_next (set by the host, reset here).
__global__ __launch_bounds__(64) void k_plan_one(Params pr, const int64_t *off, PlanDev pl,
                                                 int32_t *n_act, int64_t *t_next, DevCtl *ctl,
                                                 int64_t part_cap, ClassTable ct,
                                                 int32_t host_n, int64_t host_t,
                                                 int32_t count_stats) {
    int64_t n = host_n, tcur = host_t;
    if (host_n < 0) {
        n = uniform_i32(n_act[0]);
        tcur = uniform_i64(t_next[0]);
    }
    plan_single_wave(off, pl, ctl, part_cap, ct, n, tcur, count_stats);
    if (host_n < 0 && threadIdx.x == 0) {
        n_act[0] = 0;
        t_next[0] = LLONG_MAX;
    }
}

// One cluster, one block step's first kernel: every wave finds the next block
// from the level counts (so no workgroup waits for another), workgroup 0 also
// writes the plan, and every thread predicts one particle to the block time
// and gathers one slot of the block from the due levels' lists.  The
// cluster's time advances in the corrector, after every workgroup here has
// read it.
template <int MIXED>
__global__ __launch_bounds__(kWG) void k_plan_predict_gather(State st, Params pr, JBuf jb,
                                                             const int64_t *off, PlanDev pl,
                                                             LevelLists ll, int32_t *i_list,
                                                             DevCtl *ctl, int64_t part_cap,
                                                             ClassTable ct, int32_t fused_mask) {
    __shared__ int32_t s_buf[kLevels], s_pre[kLevels + 1];
    int64_t T, n;
    next_block_wave(pr, pl, uniform_i64(ctl->t_end_tick), &T, &n);
    if (blockIdx.x == 0 && threadIdx.x < 64)
        plan_single_wave(off, pl, ctl, part_cap, ct, n, T, 1);
    if (n == 0)  // the same in every wave: they all read the same counts
        return;
    if (threadIdx.x < 64) {
        const int64_t tot = due_prefix(pr, ll, 0, T, s_buf, s_pre);
        if (blockIdx.x == 0 && threadIdx.x == 0 && tot != n)
            atomicOr(&ctl->err, kErrPlan);
    }
    __syncthreads();
    // blocks of a class whose force kernel predicts in the kernel need no
    // prediction pass (the planner's class rule)
    int cls = kClasses - 1;
    for (int q = 0; q < kClasses; q++)
        if (n >= ct.min_n[q]) {
            cls = q;
            break;
        }
    const bool predict = ((fused_mask >> cls) & 1) == 0;
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i < pr.n_total && predict && !predict_one<MIXED>(st, pr, jb, i, T, 0))
        atomicOr(&ctl->err, kErrExtent);
    // (a list total other than n has been flagged; gather no slot past it)
    if (i < n && i < s_pre[kLevels])
        i_list[i] = gather_slot(ll, 0, i, s_buf, s_pre);
}

// ---------------------------------------------------------------- corrector
// Section 4.1, step 5: Hermite correction of particle i at time T from its new
// acceleration and jerk, and its next step level (Aarseth criterion, then the
// power-of-two quantisation).  Returns the new level, or -1 when the particle
// was not due at T (then nothing is written).  claimed: the caller has already
// moved the particle's tick to T itself (having checked that it was due).
__device__ inline int correct_particle(const State &st, const Params &pr, int64_t i, int64_t T,
                                       const double a1[3], const double j1[3], int32_t &err,
                                       unsigned long long &clamps, bool claimed = false) {
    const int lev = st.lev[i];
    const int64_t dtk = dt_ticks(pr.lev_max, lev);
    if (!claimed && st.tick[i] + dtk != T) {
        err |= kErrNotDue;
        return -1;
    }
    const double dt = ldexp(1.0, -lev);
    const double h = 0.5 * dt, s6 = dt * (1.0 / 6.0);
    const double x0[3] = {st.x[i], st.y[i], st.z[i]};
    const double v0[3] = {st.vx[i], st.vy[i], st.vz[i]};
    const double a0[3] = {st.ax[i], st.ay[i], st.az[i]};
    const double j0[3] = {st.jx[i], st.jy[i], st.jz[i]};
    double x1[3], v1[3], a2e[3], a3[3];
    const double dt2 = dt * dt, dt3 = dt2 * dt, dt4 = dt3 * dt, dt5 = dt4 * dt;
    const double idt2 = 1.0 / dt2, idt3 = 1.0 / dt3;  // exact: powers of two
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const double xp = fma(dt, fma(dt, fma(s6, j0[q], 0.5 * a0[q]), v0[q]), x0[q]);
        const double vp = fma(dt, fma(h, j0[q], a0[q]), v0[q]);
        const double da = a0[q] - a1[q];
        const double a2 = (-6.0 * da - dt * (4.0 * j0[q] + 2.0 * j1[q])) * idt2;
        const double a3q = (12.0 * da + 6.0 * dt * (j0[q] + j1[q])) * idt3;
        x1[q] = xp + a2 * dt4 / 24.0 + a3q * dt5 / 120.0;
        v1[q] = vp + a2 * dt3 / 6.0 + a3q * dt4 / 24.0;
        a2e[q] = a2 + dt * a3q;
        a3[q] = a3q;
    }
    if (!(finite3(x1[0], x1[1], x1[2]) && finite3(v1[0], v1[1], v1[2]) &&
          finite3(a1[0], a1[1], a1[2]) && finite3(j1[0], j1[1], j1[2])))
        err |= kErrNonFinite;
    // Aarseth criterion and block quantisation
    const double na = norm3(a1[0], a1[1], a1[2]), nj = norm3(j1[0], j1[1], j1[2]);
    const double na2 = norm3(a2e[0], a2e[1], a2e[2]), na3 = norm3(a3[0], a3[1], a3[2]);
    const double num = na * na2 + nj * nj;
    const double den = nj * na3 + na2 * na2;
    const double dt_raw = den > 0.0 ? sqrt(pr.eta * num / den) : INFINITY;
    int nlev = lev;
    if (dt_raw < dt) {
        while (nlev < pr.lev_max && ldexp(1.0, -nlev) > dt_raw)
            nlev++;
        if (ldexp(1.0, -nlev) > dt_raw)
            clamps++;
    } else if (dt_raw >= 2.0 * dt && lev > pr.lev_min && (T % (2 * dtk)) == 0) {
        nlev = lev - 1;
    }
    st.x[i] = x1[0];
    st.y[i] = x1[1];
    st.z[i] = x1[2];
    st.vx[i] = v1[0];
    st.vy[i] = v1[1];
    st.vz[i] = v1[2];
    st.ax[i] = a1[0];
    st.ay[i] = a1[1];
    st.az[i] = a1[2];
    st.jx[i] = j1[0];
    st.jy[i] = j1[1];
    st.jz[i] = j1[2];
    st.tick[i] = T;
    st.lev[i] = (int8_t)nlev;
    return nlev;
}

// Correction of a caller-given list (the explicit entry point).
__global__ __launch_bounds__(kWG) void k_correct(State st, Params pr, const int32_t *i_list,
                                                 int32_t slots_at_offsets, const int64_t *off,
                                                 const int32_t *cid, const int32_t *n_cur,
                                                 const int64_t *t_cur, int64_t slot_space,
                                                 const double *an, const double *jn,
                                                 int64_t in_stride, DevCtl *ctl) {
    unsigned long long clamps = 0;
    int32_t err = 0;
    const int64_t bound = pr.C == 1 ? min(slot_space, (int64_t)n_cur[0]) : slot_space;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < bound;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int c = pr.C > 1 ? cid[s] : 0;
        const int64_t cb = off[c];
        const int64_t k = slots_at_offsets ? s - cb : s;
        if (k >= n_cur[c])
            continue;
        const int64_t i = i_list[s];
        if (i < cb || i >= off[c + 1]) {
            err |= kErrRange;
            continue;
        }
        // a caller's list may name a particle twice: the first slot to move
        // its tick from the last step's time to T corrects it, any other
        // finds it no longer due
        const int64_t T = t_cur[c];
        const int64_t due_from = T - dt_ticks(pr.lev_max, st.lev[i]);
        if (atomicCAS(reinterpret_cast<unsigned long long *>(st.tick + i),
                      (unsigned long long)due_from, (unsigned long long)T) !=
            (unsigned long long)due_from) {
            err |= kErrNotDue;
            continue;
        }
        double a1[3], j1[3];
#pragma unroll
        for (int q = 0; q < 3; q++) {
            a1[q] = an[q * in_stride + s];
            j1[q] = jn[q * in_stride + s];
        }
        (void)correct_particle(st, pr, i, T, a1, j1, err, clamps, true);
    }
    if (err)
        atomicOr(&ctl->err, err);
    if (clamps)
        atomicAdd(&ctl->clamps, clamps);
}

// ---------------------------------------------------------------- reduction
// Sums the per-slice partial results of every slot whose cluster was split
// into S > 1 j-slices.  Slots are taken by groups of L lanes (L a power of two
// up to 64, the same for the whole launch): lane l of a group adds slices l,
// l+L, ... in order, a fixed DPP tree adds the group's lanes, and the group's
// last lane stores the slot.  L is the smallest width that leaves each lane at
// most four slices, widened (up to S) while the slots times L come to fewer
// than kReduceLanes lanes, so that small blocks still spread over the chip;
// loads of one slice are consecutive over the slots.  Splits wider than 64
// of blocks of at most kWgSlots slots take a workgroup per slot instead
// (thread t adds slices t, t+256, ..., then DPP trees and the four wave sums in
// order).  Every order is fixed and follows from the plan alone (never from the
// launch's grid), so results are bitwise reproducible for a given plan, and an
// explicit evaluation of a block sums it as the block step does.  With one
// cluster only the n live slots are visited.
//
// CORR (a block step): instead of storing a slot's sums, correct its particle
// with them right away (slots of clusters that were not split take the force
// kernel's direct output), and keep the per-level counts of the block-step
// scheme current: level changes are gathered per workgroup in LDS (one
// cluster) or added to the cluster's row directly (several).
constexpr int64_t kReduceLanes = 1 << 17;
constexpr int64_t kTileMin = 256;  // blocks of at least this many slots use slot tiles
constexpr int64_t kWgSlots = 1024;  // wide splits of blocks up to this size: a workgroup per slot

struct CorrArgs {
    State st;
    Params pr;
    const int64_t *t_cur;
    int64_t *t_now;
    int32_t *lev_cnt;
    LevelLists ll;
    DevCtl *ctl;
};

// Append each lane's corrected particle i (new level nl >= 0, cluster c) to
// the current list of its new level (the force launch of the step has given
// the due levels fresh, empty lists).  One atomic per (cluster, level) per
// wave; every lane of the wave that is running must call it.
__device__ inline void list_append(const CorrArgs &ca, const int64_t *off, int c, int nl,
                                   int64_t i) {
    const int lane = threadIdx.x & 63;
    const bool has = nl >= 0;
    // group the lanes by (cluster, level) first (no memory access), so that the
    // groups' leaders then reserve their places all at once
    uint64_t pending = __ballot(has);
    uint64_t mine = 0;
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int kc = __builtin_amdgcn_readlane(c, leader);
        const int kl = __builtin_amdgcn_readlane(nl, leader);
        const uint64_t m = __ballot(has && c == kc && nl == kl) & pending;
        if ((m >> lane) & 1ull)
            mine = m;
        pending &= ~m;
    }
    const int leader = has ? __ffsll((unsigned long long)mine) - 1 : lane;
    int base = 0, tb = 0;
    if (has && lane == leader) {
        tb = ca.ll.buf[(int64_t)c * kLevels + nl];
        base = atomicAdd(list_cnt(ca.ll, tb, c, nl), (int)__popcll(mine));
    }
    base = __shfl(base, leader);
    tb = __shfl(tb, leader);
    if (has) {
        const int rank = (int)__popcll(mine & ((1ull << lane) - 1ull));
        list_at(ca.ll, tb, nl, off[c])[base + rank] = (int32_t)i;
    }
}

template <bool CORR>
__global__ __launch_bounds__(kWG) void k_reduce_t(ForceArgs fa, const int32_t *cid,
                                                  int64_t slot_space, const int32_t *s_max,
                                                  CorrArgs ca) {
    __shared__ double red[7][kWG / 64];
    __shared__ double tred[kWG / 64][7][64];  // slot tiles: each wave's quarter sums
    __shared__ int32_t dlev[kLevels];
    // one cluster: the workgroup's list appends, staged in LDS and written at
    // the end with one atomic per level (particle; level << 16 | rank)
    constexpr int kStage = CORR ? 1024 : 1;
    __shared__ int32_t s_si[kStage], s_sr[kStage];
    __shared__ int32_t s_lcnt[kLevels], s_lbase[kLevels];
    __shared__ int32_t s_ns;
    // the force kernel's work queue back to zero: every evaluation ends here,
    // so the next one finds it empty whether a plan kernel resets it (device
    // plans) or not (plans made on the host)
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *fa.item_counter = 0;
    const bool hplan = fa.host_plan != 0;  // plan values from the host
    const int smax = hplan ? (fa.hp.S > 1 ? fa.hp.S : 0) : uniform_i32(*s_max);
    if (!CORR && smax <= 1)
        return;
    // cluster c's block size, j-split and first partial-sum slot
    auto plan_n = [&](int c) -> int64_t { return hplan ? (int64_t)fa.hp_n : fa.n_cur[c]; };
    auto plan_S = [&](int c) -> int { return hplan ? fa.hp.S : fa.S[c]; };
    auto plan_pb = [&](int c) -> int64_t { return hplan ? 0 : fa.part_begin[c]; };
    if (CORR) {
        if (threadIdx.x < kLevels) {
            dlev[threadIdx.x] = 0;
            s_lcnt[threadIdx.x] = 0;
        }
        if (threadIdx.x == 0)
            s_ns = 0;
        __syncthreads();
    }
    int32_t err = 0;
    unsigned long long clamps = 0;
    // a corrected particle of a single cluster into the LDS stage (beyond its
    // capacity straight into its list)
    auto stage = [&](int nl, int64_t i) {
        const int q = atomicAdd(&s_ns, 1);
        if (q < kStage) {
            const int r = atomicAdd(&s_lcnt[nl], 1);
            s_si[q] = (int32_t)i;
            s_sr[q] = (nl << 16) | r;
        } else {
            const int b = ca.ll.buf[nl];
            const int pos = atomicAdd(list_cnt(ca.ll, b, 0, nl), 1);
            list_at(ca.ll, b, nl, 0)[pos] = (int32_t)i;
        }
    };
    // store a slot's sums, or (CORR) correct its particle; returns the new
    // level (-1: nothing corrected) and the particle in *ip
    auto emit = [&](int64_t s, int c, const double *v, int64_t *ip) -> int {
        if (!CORR) {
            fa.out_acc[s] = v[0];
            fa.out_acc[fa.out_stride + s] = v[1];
            fa.out_acc[2 * fa.out_stride + s] = v[2];
            fa.out_jerk[s] = v[3];
            fa.out_jerk[fa.out_stride + s] = v[4];
            fa.out_jerk[2 * fa.out_stride + s] = v[5];
            if (fa.out_pot)
                fa.out_pot[s] = v[6];
            return -1;
        }
        const int64_t i = fa.i_list[s];
        if (i < fa.off[c] || i >= fa.off[c + 1]) {
            err |= kErrRange;
            return -1;
        }
        const int old = ca.st.lev[i];
        const int nl = correct_particle(ca.st, ca.pr, i, ca.t_cur[c], v, v + 3, err, clamps);
        if (nl >= 0 && nl != old) {
            if (fa.C == 1) {
                atomicAdd(&dlev[old], -1);
                atomicAdd(&dlev[nl], 1);
            } else {
                atomicAdd(&ca.lev_cnt[(int64_t)c * kLevels + old], -1);
                atomicAdd(&ca.lev_cnt[(int64_t)c * kLevels + nl], 1);
            }
        }
        *ip = i;
        return nl;
    };
    // the force kernel's own output for a slot of a cluster that was not split
    auto direct = [&](int64_t s, double *v) {
#pragma unroll
        for (int q = 0; q < 3; q++) {
            v[q] = fa.out_acc[q * fa.out_stride + s];
            v[3 + q] = fa.out_jerk[q * fa.out_stride + s];
        }
        v[6] = 0.0;
    };
    int64_t bound = slot_space;
    if (fa.C == 1)
        bound = min(bound, uniform_i64(plan_n(0)));
    int64_t n_tot = -1;  // active slots of the plan, where known
    if (fa.C == 1)
        n_tot = bound;
    else if (CORR)
        n_tot = uniform_i32(ca.ctl->n_last);
    const bool wg_mode = smax > 64 && (n_tot < 0 || n_tot <= kWgSlots);
    // Large split blocks: a workgroup takes 64 consecutive slots (lane = slot,
    // so a slice's loads are contiguous), wave w sums the slices of the w-th
    // quarter in order, and the quarters are added in wave order through LDS.
    const bool tile_mode = !wg_mode && smax > 4 && n_tot >= kTileMin;
    if (tile_mode) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        for (int64_t s0 = (int64_t)blockIdx.x * 64; s0 < bound; s0 += (int64_t)gridDim.x * 64) {
            const int64_t s = s0 + lane;
            int c = 0, S = 0;
            int64_t k = 0, n = 0;
            bool live = false;
            if (s < bound) {
                c = fa.C > 1 ? cid[s] : 0;
                k = fa.slots_at_offsets ? s - fa.off[c] : s;
                n = plan_n(c);
                S = plan_S(c);
                live = k < n && (CORR || S > 1);
            }
            double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            if (live && S > 1) {
                const int per = (S + 3) >> 2;
                const int j0 = w * per, j1 = min(S, j0 + per);
                const int64_t base = plan_pb(c) + k;
                // four slices' loads go out together, then their sums in slice
                // order (the same order as one slice at a time)
                int js = j0;
                for (; js + 3 < j1; js += 4) {
                    double u[4][7];
#pragma unroll
                    for (int r = 0; r < 4; r++)
#pragma unroll
                        for (int q = 0; q < 7; q++)
                            u[r][q] = fa.part[q * fa.part_cap + base + (int64_t)(js + r) * n];
#pragma unroll
                    for (int r = 0; r < 4; r++)
#pragma unroll
                        for (int q = 0; q < 7; q++)
                            v[q] += u[r][q];
                }
                for (; js < j1; js++) {
#pragma unroll
                    for (int q = 0; q < 7; q++)
                        v[q] += fa.part[q * fa.part_cap + base + (int64_t)js * n];
                }
            }
#pragma unroll
            for (int q = 0; q < 7; q++)
                tred[w][q][lane] = v[q];
            __syncthreads();
            int nl = -1;
            int64_t ip = 0;
            if (w == 0 && live) {
                if (S > 1) {
#pragma unroll
                    for (int q = 0; q < 7; q++)
                        v[q] = ((tred[0][q][lane] + tred[1][q][lane]) + tred[2][q][lane]) +
                               tred[3][q][lane];
                } else {
                    direct(s, v);
                }
                nl = emit(s, c, v, &ip);
            }
            if (CORR) {
                if (fa.C == 1) {
                    if (nl >= 0)
                        stage(nl, ip);
                } else if (w == 0) {
                    list_append(ca, fa.off, c, nl, ip);
                }
            }
            __syncthreads();
        }
    } else if (wg_mode) {
        const int t = threadIdx.x, lane = t & 63, w = t >> 6;
        for (int64_t s = blockIdx.x; s < bound; s += gridDim.x) {
            const int c = fa.C > 1 ? uniform_i32(cid[s]) : 0;
            const int64_t k = fa.slots_at_offsets ? s - uniform_i64(fa.off[c]) : s;
            const int64_t n = uniform_i64(plan_n(c));
            const int S = uniform_i32(plan_S(c));
            if (k >= n)
                continue;
            if (S <= 1) {
                int nl = -1;
                int64_t ip = 0;
                if (CORR && t == 0) {
                    double v[7];
                    direct(s, v);
                    nl = emit(s, c, v, &ip);
                }
                if (CORR) {
                    if (fa.C == 1) {
                        if (nl >= 0)
                            stage(nl, ip);
                    } else if (w == 0) {
                        list_append(ca, fa.off, c, nl, ip);
                    }
                }
                continue;
            }
            const int64_t base = uniform_i64(plan_pb(c)) + k;
            // all seven components' loads of a slice together, then the sums
            double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            for (int js = t; js < S; js += kWG) {
#pragma unroll
                for (int q = 0; q < 7; q++)
                    v[q] += fa.part[q * fa.part_cap + base + (int64_t)js * n];
            }
#pragma unroll
            for (int q = 0; q < 7; q++)
                v[q] = group_sum<64>(v[q]);
            if (lane == 63) {
#pragma unroll
                for (int q = 0; q < 7; q++)
                    red[q][w] = v[q];
            }
            __syncthreads();
            int nl = -1;
            int64_t ip = 0;
            if (t == 0) {
#pragma unroll
                for (int q = 0; q < 7; q++)
                    v[q] = ((red[q][0] + red[q][1]) + red[q][2]) + red[q][3];
                nl = emit(s, c, v, &ip);
            }
            if (CORR) {
                if (fa.C == 1) {
                    if (nl >= 0)
                        stage(nl, ip);
                } else if (w == 0) {
                    list_append(ca, fa.off, c, nl, ip);
                }
            }
            __syncthreads();
        }
    } else {
        int L = 1;
        while (L < 64 && L < smax && (4 * L < smax || (n_tot >= 0 && n_tot * L < kReduceLanes)))
            L <<= 1;
        const int lane = threadIdx.x & 63, l = lane & (L - 1);
        const int64_t gpw = 64 / L;  // slot groups per wave
        const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
        const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
        for (int64_t s0 = wave * gpw; s0 < bound; s0 += nwaves * gpw) {
            const int64_t s = s0 + lane / L;
            int c = 0, S = 0;
            bool live = false;
            int64_t k = 0, n = 0;
            if (s < bound) {
                c = fa.C > 1 ? cid[s] : 0;
                k = fa.slots_at_offsets ? s - fa.off[c] : s;
                n = plan_n(c);
                S = plan_S(c);
                live = k < n && (CORR || S > 1);
            }
            double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            if (live && S > 1) {
                const int64_t base = plan_pb(c) + k;
                for (int js = l; js < S; js += L) {
#pragma unroll
                    for (int q = 0; q < 7; q++)
                        v[q] += fa.part[q * fa.part_cap + base + (int64_t)js * n];
                }
            }
            if (L > 1) {
#pragma unroll
                for (int q = 0; q < 7; q++)
                    v[q] = group_sum_rt(v[q], L);
            }
            int nl = -1;
            int64_t ip = 0;
            if (live && l == L - 1) {
                if (S <= 1)
                    direct(s, v);
                nl = emit(s, c, v, &ip);
            }
            if (CORR) {
                if (fa.C == 1) {
                    if (nl >= 0)
                        stage(nl, ip);
                } else {
                    list_append(ca, fa.off, c, nl, ip);
                }
            }
        }
    }
    if (CORR) {
        __syncthreads();
        if (threadIdx.x < kLevels && dlev[threadIdx.x] != 0)
            atomicAdd(&ca.lev_cnt[threadIdx.x], dlev[threadIdx.x]);
        if (err)
            atomicOr(&ca.ctl->err, err);
        if (clamps)
            atomicAdd(&ca.ctl->clamps, clamps);
        if (fa.C == 1 && s_ns > 0) {
            // the staged appends: one atomic per level reserves the workgroup's
            // places in each list
            if (threadIdx.x < kLevels && s_lcnt[threadIdx.x] > 0)
                s_lbase[threadIdx.x] = atomicAdd(
                    list_cnt(ca.ll, ca.ll.buf[threadIdx.x], 0, threadIdx.x), s_lcnt[threadIdx.x]);
            __syncthreads();
            const int ns = min(s_ns, kStage);
            for (int q = threadIdx.x; q < ns; q += kWG) {
                const int L = s_sr[q] >> 16, r = s_sr[q] & 0xffff;
                list_at(ca.ll, ca.ll.buf[L], L, 0)[s_lbase[L] + r] = s_si[q];
            }
        }
        if (fa.C == 1 && blockIdx.x == 0 && threadIdx.x == 0 && fa.n_cur[0] > 0)
            ca.t_now[0] = ca.t_cur[0];  // one cluster: its time advances
    }
}

// Start-up: store the first force sweep, t_i = 0 and the start-up step.
__global__ __launch_bounds__(kWG) void k_init_finish(State st, Params pr, const double *an,
                                                     const double *jn, int64_t stride,
                                                     DevCtl *ctl) {
    unsigned long long clamps = 0;
    int32_t err = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < pr.n_total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double ax = an[i], ay = an[stride + i], az = an[2 * stride + i];
        const double jx = jn[i], jy = jn[stride + i], jz = jn[2 * stride + i];
        if (!finite3(ax, ay, az) || !finite3(jx, jy, jz) || !finite3(st.x[i], st.y[i], st.z[i]) ||
            !finite3(st.vx[i], st.vy[i], st.vz[i]))
            err |= kErrNonFinite;
        const double na = norm3(ax, ay, az), nj = norm3(jx, jy, jz);
        const double want = nj > 0.0 ? pr.eta_init * na / nj : INFINITY;
        int lev = pr.lev_min;
        while (lev < pr.lev_max && ldexp(1.0, -lev) > want)
            lev++;
        if (ldexp(1.0, -lev) > want)
            clamps++;
        st.ax[i] = ax;
        st.ay[i] = ay;
        st.az[i] = az;
        st.jx[i] = jx;
        st.jy[i] = jy;
        st.jz[i] = jz;
        st.tick[i] = 0;
        st.lev[i] = (int8_t)lev;
    }
    if (err)
        atomicOr(&ctl->err, err);
    if (clamps)
        atomicAdd(&ctl->clamps, clamps);
}

// The polled fields of the control block into the host's mapped mirror.
__global__ void k_mirror(const DevCtl *ctl, HostMirror *m) {
    if (threadIdx.x == 0) {
        m->err = ctl->err;
        m->any_active = ctl->any_active;
        __threadfence_system();
    }
}

int grid_for(int64_t n) {
    int64_t g = (n + kWG - 1) / kWG;
    if (g < 1)
        g = 1;
    if (g > 4096)
        g = 4096;
    return (int)g;
}

}  // namespace

hipError_t launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n)), dim3(kWG), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(kWG), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(kWG), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t launch_iota_i32(int32_t *p, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_iota_i32, dim3(grid_for(n)), dim3(kWG), 0, s, p, n);
    return hipGetLastError();
}
hipError_t launch_set_i64(int64_t *p, int64_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, s, p, v, (int64_t)1);
    return hipGetLastError();
}

hipError_t launch_predict(const State &st, const Params &pr, const JBuf &jb, const int32_t *cid,
                          const int64_t *t_cur, const int32_t *n_cur, int64_t t_host,
                          int use_host_t, DevCtl *ctl, hipStream_t s) {
    const int g = grid_for(pr.n_total);
    if (pr.precision == NBODY_PREC_MIXED)
        hipLaunchKernelGGL(k_predict<1>, dim3(g), dim3(kWG), 0, s, st, pr, jb, cid, t_cur, n_cur,
                           t_host, use_host_t, ctl);
    else
        hipLaunchKernelGGL(k_predict<0>, dim3(g), dim3(kWG), 0, s, st, pr, jb, cid, t_cur, n_cur,
                           t_host, use_host_t, ctl);
    return hipGetLastError();
}

hipError_t launch_read_predicted(const Params &pr, const JBuf &jb, const int32_t *cid,
                                 double *pos, double *vel, hipStream_t s) {
    hipLaunchKernelGGL(k_read_predicted, dim3(grid_for(pr.n_total)), dim3(kWG), 0, s, pr, jb, cid,
                       pos, vel, (int)(pr.precision == NBODY_PREC_MIXED));
    return hipGetLastError();
}

hipError_t launch_prime(const State &st, const Params &pr, const int64_t *off,
                        const int32_t *chunk_c, const int64_t *chunk_b, int64_t n_chunks,
                        const PlanDev &pl, const LevelLists &ll, int64_t *t_min, int64_t *t_max,
                        DevCtl *ctl, hipStream_t s) {
    hipError_t e;
    if ((e = launch_fill_i32(pl.lev_cnt, 0, (int64_t)pr.C * kLevels, s)) != hipSuccess ||
        (e = launch_fill_i32(ll.cnt, 0, 2 * (int64_t)pr.C * kLevels, s)) != hipSuccess ||
        (e = launch_fill_i32(ll.buf, 0, (int64_t)pr.C * kLevels, s)) != hipSuccess ||
        (e = launch_fill_i64(t_min, LLONG_MAX, pr.C, s)) != hipSuccess ||
        (e = launch_fill_i64(t_max, 0, pr.C, s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_prime, dim3((unsigned)n_chunks), dim3(kWG), 0, s, st, pr, off, chunk_c,
                       chunk_b, pl.lev_cnt, ll, t_min, t_max, ctl);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_prime_finish, dim3(grid_for(pr.C)), dim3(kWG), 0, s, pr, t_min, t_max,
                       pl.t_now, ctl);
    return hipGetLastError();
}

hipError_t launch_predict_gather(const State &st, const Params &pr, const JBuf &jb,
                                 const int64_t *off, const int32_t *chunk_c,
                                 const int64_t *chunk_b, int64_t n_chunks, const PlanDev &pl,
                                 const LevelLists &ll, int32_t *i_list, DevCtl *ctl, hipStream_t s) {
    if (pr.precision == NBODY_PREC_MIXED)
        hipLaunchKernelGGL(k_predict_gather<1>, dim3((unsigned)n_chunks), dim3(kWG), 0, s, st, pr,
                           jb, off, chunk_c, chunk_b, pl, ll, i_list, ctl);
    else
        hipLaunchKernelGGL(k_predict_gather<0>, dim3((unsigned)n_chunks), dim3(kWG), 0, s, st, pr,
                           jb, off, chunk_c, chunk_b, pl, ll, i_list, ctl);
    return hipGetLastError();
}

hipError_t launch_plan(const Params &pr, const int64_t *off, const PlanDev &pl, int32_t *n_act,
                       int64_t *t_next, DevCtl *ctl, int64_t part_cap, const ClassTable &ct,
                       int32_t host_n, int64_t host_t, int32_t count_stats, hipStream_t s) {
    if (pr.C == 1) {
        // a single cluster's block steps plan inside k_plan_predict_gather
        if (host_n == kPlanFromLevels)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_plan_one, dim3(1), dim3(64), 0, s, pr, off, pl, n_act, t_next, ctl,
                           part_cap, ct, host_n, host_t, count_stats);
    } else {
        hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanThreads), 0, s, pr, off, pl, n_act, t_next,
                           ctl, part_cap, ct, host_n, host_t, count_stats);
    }
    return hipGetLastError();
}

hipError_t launch_plan_predict_gather(const State &st, const Params &pr, const JBuf &jb,
                                      const int64_t *off, const PlanDev &pl, const LevelLists &ll,
                                      int32_t *i_list, DevCtl *ctl, int64_t part_cap,
                                      const ClassTable &ct, int32_t fused_mask, hipStream_t s) {
    if (pr.C != 1)
        return hipErrorInvalidValue;
    const unsigned g = (unsigned)((pr.n_total + kWG - 1) / kWG);
    if (pr.precision == NBODY_PREC_MIXED)
        hipLaunchKernelGGL(k_plan_predict_gather<1>, dim3(g), dim3(kWG), 0, s, st, pr, jb, off, pl,
                           ll, i_list, ctl, part_cap, ct, fused_mask);
    else
        hipLaunchKernelGGL(k_plan_predict_gather<0>, dim3(g), dim3(kWG), 0, s, st, pr, jb, off, pl,
                           ll, i_list, ctl, part_cap, ct, fused_mask);
    return hipGetLastError();
}

hipError_t launch_reduce(const ForceArgs &fa, const int32_t *cid, int64_t slot_space,
                         const int32_t *s_max, hipStream_t s) {
    // enough waves for one per slot up to 4096 workgroups (grid-stride
    // beyond), and a workgroup per slot up to kWgSlots slots, so wide splits
    // of small blocks are summed a workgroup per slot
    const int64_t g = std::max<int64_t>(grid_for(slot_space * 64), std::min<int64_t>(slot_space, kWgSlots));
    hipLaunchKernelGGL(k_reduce_t<false>, dim3((unsigned)g), dim3(kWG), 0, s, fa,
                       cid, slot_space, s_max, CorrArgs{});
    return hipGetLastError();
}

hipError_t launch_reduce_correct(const ForceArgs &fa, const State &st, const Params &pr,
                                 const int32_t *cid, const PlanDev &pl, const LevelLists &ll,
                                 const int32_t *s_max, DevCtl *ctl, hipStream_t s) {
    // the grid is fixed when a step is captured: one thread per particle for
    // unsplit and narrow splits, grid-stride waves / workgroups for wider ones
    const int64_t n = pr.n_total;
    const int64_t g = std::min<int64_t>(4096, std::max<int64_t>((n + kWG - 1) / kWG,
                                                                std::min<int64_t>(n, kWgSlots)));
    const CorrArgs ca{st, pr, pl.t_cur, pl.t_now, pl.lev_cnt, ll, ctl};
    hipLaunchKernelGGL(k_reduce_t<true>, dim3((unsigned)g), dim3(kWG), 0, s, fa, cid, n, s_max,
                       ca);
    return hipGetLastError();
}

hipError_t launch_correct(const State &st, const Params &pr, const int32_t *i_list,
                          int32_t slots_at_offsets, const int64_t *off, const int32_t *cid,
                          const int32_t *n_cur, const int64_t *t_cur, int64_t slot_space,
                          const double *acc_new, const double *jerk_new, int64_t in_stride,
                          DevCtl *ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_correct, dim3(grid_for(slot_space)), dim3(kWG), 0, s, st, pr, i_list,
                       slots_at_offsets, off, cid, n_cur, t_cur, slot_space, acc_new, jerk_new,
                       in_stride, ctl);
    return hipGetLastError();
}

hipError_t launch_mirror(const DevCtl *ctl, HostMirror *mirror_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_mirror, dim3(1), dim3(64), 0, s, ctl, mirror_dev);
    return hipGetLastError();
}

hipError_t launch_init_finish(const State &st, const Params &pr, const double *acc_new,
                              const double *jerk_new, int64_t stride, DevCtl *ctl,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_init_finish, dim3(grid_for(pr.n_total)), dim3(kWG), 0, s, st, pr,
                       acc_new, jerk_new, stride, ctl);
    return hipGetLastError();
}

}  // namespace nb
