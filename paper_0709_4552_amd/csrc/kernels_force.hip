// Force + jerk (+ potential) on the active block from all particles of its
// cluster (section 4.1, step 4; the sum GRAPE-6 pipelines evaluate in
// section 4.4).  For each listed i and every j of i's cluster:
//   r = x_j - x_i, w = v_j - v_i, s = |r|^2 + eps^2
//   a_i += m_j r s^{-3/2}
//   jerk_i += m_j [w s^{-3/2} - 3 (r.w) r s^{-5/2}]
//   pot_i -= m_j s^{-1/2}
//
// Work decomposition.  A persistent grid walks a list of work items built on
// the device (k_plan): item = (cluster, i-block, j-slice).  Inside a 256-thread
// workgroup, lane groups of J_LANES consecutive lanes share one i-particle and
// split each LDS j-tile between them; every lane holds I_PER_LANE i-particles
// in registers.  j-particles are staged in LDS from coalesced structure-of-
// arrays loads and read back as broadcasts (J_LANES = 1) or as consecutive
// addresses (J_LANES > 1).  Lane groups are reduced with cross-lane shuffles,
// and workgroups of one i-block (j-slices) through partial sums that k_reduce
// adds in slice order, so every result is bitwise deterministic.
//
// Arithmetic.  MIXED: positions are double-single pairs whose hi part lies
// on a fixed grid (hi = q rint(x/q), lo = fl32(x - hi)), so hi_j - hi_i is
// exact and r = (x_j^hi - x_i^hi) + (x_j^lo - x_i^lo) has one rounding that
// does not depend on i's low bits (with hi = fl32(x) that rounding repeats for
// every far j and shifts i's position systematically).  After r everything is
// FP32 with the hardware reciprocal square root; per-lane FP32 partial sums
// are flushed to FP64 accumulators every 128 j.  The jerk is kept as two sums,
// sum m s^{-3/2} w and sum m s^{-5/2} (r.w) r, combined in FP64 as the first
// minus three times the second (one multiply less per interaction).
// Near field: a pair whose term can exceed near_frac*|a_i| (|a_i| from the
// particle's stored acceleration) can be comparable to the whole force, where
// FP32 rounding would exceed the error budget; such pairs are masked out of
// the FP32 sums, recorded, and evaluated in FP64 after the tile.  With equal
// masses the test is m_max/s > near_frac*|a_i|, asked once per group of j on
// the smallest s (per-pair flags and masks only when a lane of the wave has a
// near pair); with a mass spectrum (PM) it is m_j/s > near_frac*|a_i| per pair,
// one multiply more, since m_max would flag nearly every pair.  A lane records at most kNearCap pairs
// per tile; masking stops while a whole group of pairs still fits, so every
// masked pair is recorded and none is lost.
// FP64: every operation in double precision; s^{-1/2} from the hardware
// estimate refined by one third-order Newton step.
//
// The self term (j = i) gives r = w = 0 and so adds nothing to a and jerk;
// its potential contribution m_i eps^{-1} is removed once per i (same
// arithmetic as in the loop).  With eps = 0 the self term is skipped instead.
#include <hip/hip_runtime.h>

#include "nbody_internal.h"

namespace nb {

namespace {

// s^{-1/2} in FP64: v_rsq_f64 (about 2^-23 relative) plus one Newton step of
// third order: y <- y + y e (1/2 + 3/8 e), e = 1 - s y^2.
__device__ inline double rsqrt_f64(double s) {
    const double y = __builtin_amdgcn_rsq(s);
    const double e = fma(-s * y, y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}

struct Acc64 {
    double ax, ay, az, jx, jy, jz, p;
};

// Occupancy target: the mixed one-lane-per-i shape holds 5 waves per SIMD
// (at most 102 VGPRs); the potential sum would otherwise push it to 4.
template <int I, int LJ, bool MIXED>
struct ForceOcc {
    static constexpr int kMinBlocks = (MIXED && I == 1 && LJ == 1) ? 5 : 1;
};

template <int I, int LJ, int JT, bool MIXED, bool POT, bool EXCL, bool PM, bool FUSE>
__device__ __forceinline__ void force_body(const ForceArgs &fa) {
    static_assert(MIXED || !PM, "per-pair near test only in the mixed form");
    static_assert(LJ == 1 || LJ == 4 || LJ == 16 || LJ == 64 || LJ == 256, "J_LANES");
    static_assert(LJ == 1 || I == 1, "several i per lane only without lane groups");
    constexpr int NI = kWG / LJ;  // i-slots per workgroup
    constexpr int IB = NI * I;    // i-particles per work item
    // DIRECT: with 64 or more lanes per i-particle a j is used by at most four
    // i-slots, so lanes read j straight from global memory (consecutive lanes,
    // consecutive j) instead of staging tiles in LDS: no barriers in the j loop
    // and four j per lane in flight per iteration.
    constexpr bool DIRECT = LJ >= 64;
    constexpr int JTX = DIRECT ? (JT > 4 * LJ ? JT : 4 * LJ) : JT;  // j per tile step
    constexpr int JPL = JTX / LJ;  // j per lane per tile step
    static_assert(JT % LJ == 0 && JT % kWG == 0 && JTX % kWG == 0, "tile");
    // FP32 partial sums are flushed after kFlushJ j per lane
    constexpr int kFlushJ = 128;
    constexpr int CHJ = JPL < kFlushJ ? JPL : kFlushJ;   // j per lane per chunk
    constexpr int NCH = JPL / CHJ;                       // chunks per tile
    constexpr int FLUSH_TILES = NCH > 1 ? 1 : kFlushJ / JPL;

    constexpr int LT = DIRECT ? 1 : JT;  // LDS tile entries
    __shared__ float4 sP[MIXED ? LT : 1];
    __shared__ float4 sQ[MIXED ? LT : 1];
    __shared__ float2 sR[MIXED ? LT : 1];
    __shared__ double2 sA[MIXED ? 1 : LT];
    __shared__ double2 sB[MIXED ? 1 : LT];
    __shared__ double2 sC[MIXED ? 1 : LT];
    __shared__ double sD[MIXED ? 1 : LT];
    __shared__ double sRed[LJ == 256 ? 4 * 7 : 1];
    // per-lane list of near pairs found in the current tile step (offset in it)
    constexpr int kNearCap = 8;
    __shared__ uint16_t sNear[MIXED ? I * kNearCap * kWG : 1];
    // Particle j's record: from the j-buffer, or (fused) predicted here from
    // the state to tick T with the prediction pass's own arithmetic.
    bool fused = false;
    auto fetch_m = [&](int64_t j, int64_t T, float4 &P, float4 &Q, float2 &R) {
        if (FUSE && fused) {
            float4 V;
            if (!predict_mixed(fa.st, fa.tick, fa.grid_q, fa.grid_inv, fa.origin[0], j, T, P, Q,
                               R, V))
                atomicOr(fa.err, kErrExtent);
        } else {
            P = fa.jb.P[j];
            Q = fa.jb.Q[j];
            R = fa.jb.R[j];
        }
    };
    // low parts of particle j's FP32 velocity (the near field's FP64 velocities)
    auto fetch_vlo = [&](int64_t j, int64_t T) -> float4 {
        if (FUSE && fused) {
            float4 P, Q, V;
            float2 R;
            (void)predict_mixed(fa.st, fa.tick, fa.grid_q, fa.grid_inv, fa.origin[0], j, T, P, Q,
                                R, V);
            return V;
        }
        return fa.jb.V[j];
    };
    auto fetch_d = [&](int64_t j, int64_t T, double2 &A, double2 &B, double2 &C, double &D) {
        if (FUSE && fused) {
            predict_fp64(fa.st, fa.tick, j, T, A, B, C, D);
        } else {
            A = fa.jb.A[j];
            B = fa.jb.B[j];
            C = fa.jb.C[j];
            D = fa.jb.D[j];
        }
    };
    // j-particle t of the current tile step: from LDS, or (DIRECT) fetched per
    // lane, with massless far-away padding past the end of the slice
    auto jPQR = [&](int64_t tb, int64_t j1, int t, int64_t T, float4 &p, float4 &q, float2 &r) {
        if (!DIRECT) {
            p = sP[t];
            q = sQ[t];
            r = sR[t];
        } else if (tb + t < j1) {
            fetch_m(tb + t, T, p, q, r);
        } else {
            p = make_float4(1e18f, 1e18f, 1e18f, 0.f);
            q = make_float4(0.f, 0.f, 0.f, 0.f);
            r = make_float2(0.f, 0.f);
        }
    };

    const int tid = threadIdx.x;
    int lj, li;
    if (LJ <= 64) {
        const int lane = tid & 63, w = tid >> 6;
        lj = lane % LJ;
        li = w * (64 / LJ) + lane / LJ;
    } else {
        lj = tid;
        li = 0;
    }

    __shared__ int64_t s_item;
    // the plan picks one class; a launch serves every class sharing its shape
    const bool hplan = fa.host_plan != 0;  // a single cluster planned on the host
    const int cls_now = hplan ? fa.hp.cls : uniform_i32(*fa.cls);
    if (((fa.cls_mask >> cls_now) & 1) == 0)
        return;
    if (FUSE)
        fused = ((fa.fused_mask >> cls_now) & 1) != 0;
    if (fa.flip_lists) {
        // block step: the block has been gathered from the due levels' lists
        // and the corrector has not started, so nothing else touches the lists
        // now: each due level changes to its other buffer, emptied, which the
        // corrector then fills with the particles stepped onto that level
        for (int64_t q = (int64_t)blockIdx.x * kWG + tid; q < (int64_t)fa.C * kLevels;
             q += (int64_t)gridDim.x * kWG) {
            const int cq = (int)(q / kLevels), L = (int)(q % kLevels);
            if (L >= fa.ll.lev_min && L <= fa.lev_max && fa.n_cur[cq] > 0 &&
                (fa.t_cur[cq] & ((int64_t(1) << (fa.lev_max - L)) - 1)) == 0) {
                const int b = 1 - fa.ll.buf[q];
                fa.ll.buf[q] = b;
                fa.ll.cnt[((int64_t)b * fa.C + cq) * kLevels + L] = 0;
            }
        }
    }
    const int64_t total = hplan ? fa.hp.items : uniform_i64(*fa.total_items);
    // first round static (item = workgroup index); only when there are more
    // items than workgroups do finished workgroups pop further items from the
    // queue (items gridDim.x, gridDim.x+1, ...).  Small launches thus take no
    // atomics at all: same-address atomics from every workgroup serialise in L2
    // and cost tens of microseconds.
    int64_t item = blockIdx.x;
    for (;;) {
        if (item >= total)
            break;
        // locate the cluster of this item (largest c with item_begin[c] <= item)
        int c = 0;
        if (fa.C > 1) {
            int lo = 0, hi = fa.C - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (fa.item_begin[mid] <= item)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            c = lo;
        }
        c = uniform_i32(c);
        const int64_t local = hplan ? item : item - uniform_i64(fa.item_begin[c]);
        const int S = hplan ? fa.hp.S : uniform_i32(fa.S[c]);
        // slice-major order: consecutive items share a j-slice, so workgroups on
        // all eight XCDs work on the same slice at once and each XCD's L2 fetches
        // it about once instead of once per i-block
        const int64_t n_c = hplan ? (int64_t)fa.hp_n : uniform_i32(fa.n_cur[c]);
        const int64_t nib_c = (n_c + IB - 1) / IB;
        const int js = (int)(local / nib_c);
        const int64_t ib = local - (int64_t)js * nib_c;
        const int64_t cb = uniform_i64(fa.off[c]), ce = uniform_i64(fa.off[c + 1]);
        const int64_t jl = hplan ? (int64_t)fa.hp.jl : uniform_i32(fa.jlen[c]);
        const int64_t j0 = cb + (int64_t)js * jl;
        const int64_t j1 = min(ce, j0 + jl);
        const int64_t slot0 = fa.slots_at_offsets ? cb : 0;
        const int64_t Tc = (FUSE && fused) ? uniform_i64(fa.t_cur[c]) : 0;

        // ---- i-particles into registers
        bool valid[I];
        int64_t kk[I];
        int64_t gi[I];
        float xh[I], yh[I], zh[I], xl[I], yl[I], zl[I], vxi[I], vyi[I], vzi[I], mi[I];
        float scrit[I];
        double X[I], Y[I], Z[I], VX[I], VY[I], VZ[I], M[I];
#pragma unroll
        for (int ii = 0; ii < I; ii++) {
            kk[ii] = ib * IB + ii * NI + li;
            valid[ii] = kk[ii] < n_c;
            int64_t i = valid[ii] ? (int64_t)fa.i_list[slot0 + kk[ii]] : cb;
            if (valid[ii] && (i < cb || i >= ce)) {
                atomicOr(fa.err, kErrRange);
                i = cb;
            }
            gi[ii] = i;
            if (MIXED) {
                float4 p, q;
                float2 r;
                fetch_m(i, Tc, p, q, r);
                xh[ii] = p.x; yh[ii] = p.y; zh[ii] = p.z; mi[ii] = p.w;
                xl[ii] = q.x; yl[ii] = q.y; zl[ii] = q.z; vxi[ii] = q.w;
                vyi[ii] = r.x; vzi[ii] = r.y;
                // near-field threshold on s from |a_i| and |jerk_i| (0 = none):
                // per unit of m_j with PM, else for m_max
                float sc = 0.f;
                if (fa.near_frac > 0.f) {
                    const float4 ns = fa.nscale[c];
                    const double ha = sqrt(fa.hax[i] * fa.hax[i] + fa.hay[i] * fa.hay[i] +
                                           fa.haz[i] * fa.haz[i]);
                    double v = (PM ? 1.0 : (double)ns.x) / ((double)fa.near_frac * ha);
                    if (fa.near_frac_jerk > 0.f) {
                        // m V s^{-3/2} > f |jerk_i|  <=>  s < (m V / (f |jerk_i|))^{2/3};
                        // with PM scaled per unit of m_j from the smallest mass,
                        // which covers every heavier j with room to spare
                        const double hj = sqrt(fa.hjx[i] * fa.hjx[i] + fa.hjy[i] * fa.hjy[i] +
                                               fa.hjz[i] * fa.hjz[i]);
                        const double V = sqrt((double)vxi[ii] * vxi[ii] + (double)vyi[ii] * vyi[ii] +
                                              (double)vzi[ii] * vzi[ii]) + (double)ns.z;
                        const double mref = PM ? (double)ns.y : (double)ns.x;
                        const double q = mref * V / ((double)fa.near_frac_jerk * hj);
                        // q^{2/3} from the hardware log2 / exp2 (a threshold needs
                        // no more precision than that)
                        const float qf = (float)fmin(q, 1.0e30);
                        double sj = (hj > 0.0 && mref > 0.0) ? (double)__builtin_amdgcn_exp2f(
                                                   __builtin_amdgcn_logf(qf) * (2.0f / 3.0f))
                                             : 0.0;
                        if (PM)
                            sj /= mref;
                        v = fmax(v, fmin(sj, 1.0e30));
                    }
                    sc = (ha > 0.0 && v < 3.0e38) ? (float)v : 0.f;
                }
                scrit[ii] = sc;
            } else {
                double2 a, b, cc;
                double dd;
                fetch_d(i, Tc, a, b, cc, dd);
                X[ii] = a.x; Y[ii] = a.y; Z[ii] = b.x; M[ii] = b.y;
                VX[ii] = cc.x; VY[ii] = cc.y; VZ[ii] = dd;
            }
        }

        Acc64 acc[I];
        float fax[I], fay[I], faz[I], f1x[I], f1y[I], f1z[I], f2x[I], f2y[I], f2z[I], fp[I];
#pragma unroll
        for (int ii = 0; ii < I; ii++) {
            acc[ii] = Acc64{0, 0, 0, 0, 0, 0, 0};
            fax[ii] = fay[ii] = faz[ii] = 0.f;
            f1x[ii] = f1y[ii] = f1z[ii] = 0.f;
            f2x[ii] = f2y[ii] = f2z[ii] = 0.f;
            fp[ii] = 0.f;
        }
        // FP64 form keeps the second jerk sum separately too
        double d2x[I], d2y[I], d2z[I];
#pragma unroll
        for (int ii = 0; ii < I; ii++)
            d2x[ii] = d2y[ii] = d2z[ii] = 0.0;

        int tcount = 0;
        for (int64_t tb = j0; tb < j1; tb += JTX) {
            int ncnt[I];
            float sc_eff[I];
#pragma unroll
            for (int ii = 0; ii < I; ii++) {
                ncnt[ii] = 0;
                sc_eff[ii] = MIXED ? scrit[ii] : 0.f;
            }
            if (!DIRECT) {
            __syncthreads();
#pragma unroll
            for (int t = tid; t < JT; t += kWG) {
                const int64_t j = tb + t;
                if (MIXED) {
                    if (j < j1) {
                        fetch_m(j, Tc, sP[t], sQ[t], sR[t]);
                    } else {  // massless padding far away: contributes exactly 0
                        sP[t] = make_float4(1e18f, 1e18f, 1e18f, 0.f);
                        sQ[t] = make_float4(0.f, 0.f, 0.f, 0.f);
                        sR[t] = make_float2(0.f, 0.f);
                    }
                } else {
                    if (j < j1) {
                        fetch_d(j, Tc, sA[t], sB[t], sC[t], sD[t]);
                    } else {
                        sA[t] = make_double2(1e18, 1e18);
                        sB[t] = make_double2(1e18, 0.0);
                        sC[t] = make_double2(0.0, 0.0);
                        sD[t] = 0.0;
                    }
                }
            }
            __syncthreads();
            }

            if (MIXED) {
#pragma unroll
                for (int ch = 0; ch < NCH; ch++) {
                    // groups of G j: all LDS reads first, then the arithmetic, then one
                    // wave-uniform test for near pairs (recorded in a rare branch).
                    // G = 2 keeps the kernel near 94 VGPRs (5 waves per SIMD); larger
                    // groups cost occupancy and measured slower on gfx950.
                    constexpr int G = CHJ < 2 ? CHJ : 2;
#pragma unroll 1
                    for (int u = 0; u < CHJ; u += G) {
                        float4 p[G], q[G];
                        float2 r[G];
#pragma unroll
                        for (int g = 0; g < G; g++) {
                            const int t = lj + (ch * CHJ + u + g) * LJ;
                            jPQR(tb, j1, t, Tc, p[g], q[g], r[g]);
                        }
                        float dx[G][I], dy[G][I], dz[G][I], wx[G][I], wy[G][I], wz[G][I];
                        float sq[G][I], rw[G][I], rinv[G][I];
#pragma unroll
                        for (int g = 0; g < G; g++) {
#pragma unroll
                            for (int ii = 0; ii < I; ii++) {
                                dx[g][ii] = (p[g].x - xh[ii]) + (q[g].x - xl[ii]);
                                dy[g][ii] = (p[g].y - yh[ii]) + (q[g].y - yl[ii]);
                                dz[g][ii] = (p[g].z - zh[ii]) + (q[g].z - zl[ii]);
                                wx[g][ii] = q[g].w - vxi[ii];
                                wy[g][ii] = r[g].x - vyi[ii];
                                wz[g][ii] = r[g].y - vzi[ii];
                                sq[g][ii] = __builtin_fmaf(dz[g][ii], dz[g][ii],
                                            __builtin_fmaf(dy[g][ii], dy[g][ii],
                                            __builtin_fmaf(dx[g][ii], dx[g][ii], fa.eps2f)));
                                rw[g][ii] = __builtin_fmaf(dz[g][ii], wz[g][ii],
                                            __builtin_fmaf(dy[g][ii], wy[g][ii], dx[g][ii] * wx[g][ii]));
                                rinv[g][ii] = __builtin_amdgcn_rsqf(sq[g][ii]);
                                if (EXCL)
                                    rinv[g][ii] = sq[g][ii] > 0.f ? rinv[g][ii] : 0.f;
                            }
                        }
                        // Is any pair of the group near?  With one threshold per i
                        // the smallest s decides (one compare per group); the per-pair
                        // flags and masks are only needed when the answer is yes.
                        bool any = false;
#pragma unroll
                        for (int ii = 0; ii < I; ii++) {
                            if (PM) {
#pragma unroll
                                for (int g = 0; g < G; g++)
                                    any = any || sq[g][ii] < p[g].w * sc_eff[ii];
                            } else {
                                float smin = sq[0][ii];
#pragma unroll
                                for (int g = 1; g < G; g++)
                                    smin = __builtin_fminf(smin, sq[g][ii]);
                                any = any || smin < sc_eff[ii];
                            }
                        }
                        // The hint keeps this block inside the loop: rare with equal
                        // masses, it is frequent around heavy stars, and moved out of
                        // line it slowed the sweep of a Salpeter cluster by 6%.
                        if (__builtin_expect(__ballot(any) != 0ull, 1)) {
                            // mask the near pairs out of the FP32 sums and remember
                            // them for the FP64 pass after the tile.  Masking stops
                            // once fewer than G slots are free, so the pairs of one
                            // group always fit: every masked pair is kept.
                            bool nr[G][I];
#pragma unroll
                            for (int g = 0; g < G; g++) {
#pragma unroll
                                for (int ii = 0; ii < I; ii++) {
                                    nr[g][ii] = sq[g][ii] < (PM ? p[g].w * sc_eff[ii] : sc_eff[ii]);
                                    rinv[g][ii] = nr[g][ii] ? 0.f : rinv[g][ii];
                                }
                            }
#pragma unroll
                            for (int g = 0; g < G; g++) {
#pragma unroll
                                for (int ii = 0; ii < I; ii++) {
                                    if (nr[g][ii] && ncnt[ii] < kNearCap) {
                                        const int t = lj + (ch * CHJ + u + g) * LJ;
                                        sNear[(ii * kNearCap + ncnt[ii]) * kWG + tid] = (uint16_t)t;
                                        if (++ncnt[ii] > kNearCap - G)
                                            sc_eff[ii] = 0.f;
                                    }
                                }
                            }
                        }
#pragma unroll
                        for (int g = 0; g < G; g++) {
#pragma unroll
                            for (int ii = 0; ii < I; ii++) {
                                const float rinv2 = rinv[g][ii] * rinv[g][ii];
                                const float mr = p[g].w * rinv[g][ii];
                                const float mr3 = mr * rinv2;
                                const float al = rw[g][ii] * rinv2;
                                const float be = mr3 * al;
                                if (POT)
                                    fp[ii] += mr;
                                fax[ii] = __builtin_fmaf(mr3, dx[g][ii], fax[ii]);
                                fay[ii] = __builtin_fmaf(mr3, dy[g][ii], fay[ii]);
                                faz[ii] = __builtin_fmaf(mr3, dz[g][ii], faz[ii]);
                                f1x[ii] = __builtin_fmaf(mr3, wx[g][ii], f1x[ii]);
                                f1y[ii] = __builtin_fmaf(mr3, wy[g][ii], f1y[ii]);
                                f1z[ii] = __builtin_fmaf(mr3, wz[g][ii], f1z[ii]);
                                f2x[ii] = __builtin_fmaf(be, dx[g][ii], f2x[ii]);
                                f2y[ii] = __builtin_fmaf(be, dy[g][ii], f2y[ii]);
                                f2z[ii] = __builtin_fmaf(be, dz[g][ii], f2z[ii]);
                            }
                        }
                    }
                    ++tcount;
                    if (tcount == FLUSH_TILES || (ch == NCH - 1 && tb + JTX >= j1)) {
                        tcount = 0;
#pragma unroll
                        for (int ii = 0; ii < I; ii++) {
                            acc[ii].ax += (double)fax[ii];
                            acc[ii].ay += (double)fay[ii];
                            acc[ii].az += (double)faz[ii];
                            acc[ii].jx += (double)f1x[ii] - 3.0 * (double)f2x[ii];
                            acc[ii].jy += (double)f1y[ii] - 3.0 * (double)f2y[ii];
                            acc[ii].jz += (double)f1z[ii] - 3.0 * (double)f2z[ii];
                            if (POT)
                                acc[ii].p += (double)fp[ii];
                            fax[ii] = fay[ii] = faz[ii] = 0.f;
                            f1x[ii] = f1y[ii] = f1z[ii] = 0.f;
                            f2x[ii] = f2y[ii] = f2z[ii] = 0.f;
                            fp[ii] = 0.f;
                        }
                    }
                }
                // FP64 pass over the near pairs of this tile (double-single positions
                // and velocities, FP64 masses)
#pragma unroll
                for (int ii = 0; ii < I; ii++) {
                    #pragma unroll 1
                    for (int k = 0; k < ncnt[ii]; k++) {
                        const int t = sNear[(ii * kNearCap + k) * kWG + tid];
                        const int64_t j = tb + t;
                        if (j == gi[ii]) {
                            // the self pair was masked: put back the FP32 self term the
                            // writer removes, so it is removed exactly once whichever
                            // lane of the group met it
                            if (POT && !EXCL)
                                acc[ii].p += (double)(mi[ii] * __builtin_amdgcn_rsqf(fa.eps2f));
                            continue;
                        }
                        if (j >= j1)
                            continue;
                        float4 p, q;
                        float2 r;
                        jPQR(tb, j1, t, Tc, p, q, r);
                        const double ex = ((double)p.x - (double)xh[ii]) + ((double)q.x - (double)xl[ii]);
                        const double ey = ((double)p.y - (double)yh[ii]) + ((double)q.y - (double)yl[ii]);
                        const double ez = ((double)p.z - (double)zh[ii]) + ((double)q.z - (double)zl[ii]);
                        // velocity difference from the double-single velocities
                        const float4 vlj = fetch_vlo(j, Tc), vli = fetch_vlo(gi[ii], Tc);
                        const double ux = ((double)q.w - (double)vxi[ii]) + (double)(vlj.x - vli.x);
                        const double uy = ((double)r.x - (double)vyi[ii]) + (double)(vlj.y - vli.y);
                        const double uz = ((double)r.y - (double)vzi[ii]) + (double)(vlj.z - vli.z);
                        const double sd = fma(ez, ez, fma(ey, ey, fma(ex, ex, fa.eps2)));
                        const double ri = rsqrt_f64(sd);
                        const double ri2 = ri * ri;
                        const double m1 = fa.m64[j] * ri;
                        const double m3 = m1 * ri2;
                        const double b3 = 3.0 * m3 * (fma(ez, uz, fma(ey, uy, ex * ux)) * ri2);
                        acc[ii].ax = fma(m3, ex, acc[ii].ax);
                        acc[ii].ay = fma(m3, ey, acc[ii].ay);
                        acc[ii].az = fma(m3, ez, acc[ii].az);
                        acc[ii].jx += m3 * ux - b3 * ex;
                        acc[ii].jy += m3 * uy - b3 * ey;
                        acc[ii].jz += m3 * uz - b3 * ez;
                        if (POT)
                            acc[ii].p += m1;
                    }
                }
            } else {
#pragma unroll 2
                for (int t = lj; t < JTX; t += LJ) {
                    double2 a, b, cv;
                    double vz;
                    if (DIRECT) {
                        const int64_t j = tb + t;
                        if (j < j1) {
                            fetch_d(j, Tc, a, b, cv, vz);
                        } else {
                            a = make_double2(1e18, 1e18);
                            b = make_double2(1e18, 0.0);
                            cv = make_double2(0.0, 0.0);
                            vz = 0.0;
                        }
                    } else {
                        a = sA[t];
                        b = sB[t];
                        cv = sC[t];
                        vz = sD[t];
                    }
#pragma unroll
                    for (int ii = 0; ii < I; ii++) {
                        const double dx = a.x - X[ii];
                        const double dy = a.y - Y[ii];
                        const double dz = b.x - Z[ii];
                        const double wx = cv.x - VX[ii];
                        const double wy = cv.y - VY[ii];
                        const double wz = vz - VZ[ii];
                        const double s = fma(dz, dz, fma(dy, dy, fma(dx, dx, fa.eps2)));
                        const double rw = fma(dz, wz, fma(dy, wy, dx * wx));
                        double rinv = rsqrt_f64(s);
                        if (EXCL)
                            rinv = s > 0.0 ? rinv : 0.0;
                        const double rinv2 = rinv * rinv;
                        const double mr = b.y * rinv;
                        const double mr3 = mr * rinv2;
                        const double be = mr3 * (rw * rinv2);
                        if (POT)
                            acc[ii].p += mr;
                        acc[ii].ax = fma(mr3, dx, acc[ii].ax);
                        acc[ii].ay = fma(mr3, dy, acc[ii].ay);
                        acc[ii].az = fma(mr3, dz, acc[ii].az);
                        acc[ii].jx = fma(mr3, wx, acc[ii].jx);
                        acc[ii].jy = fma(mr3, wy, acc[ii].jy);
                        acc[ii].jz = fma(mr3, wz, acc[ii].jz);
                        d2x[ii] = fma(be, dx, d2x[ii]);
                        d2y[ii] = fma(be, dy, d2y[ii]);
                        d2z[ii] = fma(be, dz, d2z[ii]);
                    }
                }
            }
        }
        if (!MIXED) {
#pragma unroll
            for (int ii = 0; ii < I; ii++) {
                acc[ii].jx -= 3.0 * d2x[ii];
                acc[ii].jy -= 3.0 * d2y[ii];
                acc[ii].jz -= 3.0 * d2z[ii];
            }
        }

        // ---- reduce the lane group (J_LANES > 1)
        bool writer = true;
        if constexpr (LJ > 1 && LJ <= 64) {
            acc[0].ax = group_sum<LJ>(acc[0].ax);
            acc[0].ay = group_sum<LJ>(acc[0].ay);
            acc[0].az = group_sum<LJ>(acc[0].az);
            acc[0].jx = group_sum<LJ>(acc[0].jx);
            acc[0].jy = group_sum<LJ>(acc[0].jy);
            acc[0].jz = group_sum<LJ>(acc[0].jz);
            if (POT)
                acc[0].p = group_sum<LJ>(acc[0].p);
            writer = lj == LJ - 1;
        } else if constexpr (LJ == 256) {
            double v[7] = {acc[0].ax, acc[0].ay, acc[0].az, acc[0].jx, acc[0].jy, acc[0].jz, acc[0].p};
#pragma unroll
            for (int q = 0; q < 7; q++)
                v[q] = group_sum<64>(v[q]);
            __syncthreads();
            if ((tid & 63) == 63) {
#pragma unroll
                for (int q = 0; q < 7; q++)
                    sRed[(tid >> 6) * 7 + q] = v[q];
            }
            __syncthreads();
            if (tid == 0) {
                double r[7];
#pragma unroll
                for (int q = 0; q < 7; q++)
                    r[q] = ((sRed[q] + sRed[7 + q]) + sRed[14 + q]) + sRed[21 + q];
                acc[0] = Acc64{r[0], r[1], r[2], r[3], r[4], r[5], r[6]};
            }
            writer = tid == 0;
        }

        // ---- write results or partial sums
        if (writer) {
#pragma unroll
            for (int ii = 0; ii < I; ii++) {
                if (!valid[ii])
                    continue;
                double pot = -acc[ii].p;
                if (POT && !EXCL && gi[ii] >= j0 && gi[ii] < j1) {
                    // remove the self term m_i eps^{-1}, evaluated as in the loop, in
                    // the item whose j-slice holds i (mixed: if the FP32 loop masked
                    // it, the near-field pass has put the same value back)
                    if (MIXED) {
                        pot += (double)(mi[ii] * __builtin_amdgcn_rsqf(fa.eps2f));
                    } else {
                        pot += M[ii] * rsqrt_f64(fa.eps2);
                    }
                }
                if (S == 1) {
                    const int64_t o = slot0 + kk[ii];
                    const int64_t st = fa.out_stride;
                    fa.out_acc[o] = acc[ii].ax;
                    fa.out_acc[st + o] = acc[ii].ay;
                    fa.out_acc[2 * st + o] = acc[ii].az;
                    fa.out_jerk[o] = acc[ii].jx;
                    fa.out_jerk[st + o] = acc[ii].jy;
                    fa.out_jerk[2 * st + o] = acc[ii].jz;
                    if (POT)
                        fa.out_pot[o] = pot;
                } else {
                    const int64_t o = (hplan ? 0 : fa.part_begin[c]) + (int64_t)js * n_c + kk[ii];
                    const int64_t cap = fa.part_cap;
                    fa.part[o] = acc[ii].ax;
                    fa.part[cap + o] = acc[ii].ay;
                    fa.part[2 * cap + o] = acc[ii].az;
                    fa.part[3 * cap + o] = acc[ii].jx;
                    fa.part[4 * cap + o] = acc[ii].jy;
                    fa.part[5 * cap + o] = acc[ii].jz;
                    fa.part[6 * cap + o] = POT ? pot : 0.0;
                }
            }
        }
        if (total <= (int64_t)gridDim.x)
            break;
        if (tid == fa.fetch_lane)
            s_item = (int64_t)gridDim.x + (int64_t)atomicAdd(fa.item_counter, 1ull);
        __syncthreads();
        item = uniform_i64(s_item);
        __syncthreads();
    }
}

// One lane per i-particle (one or two per lane): a launch of its own.
template <int I, int LJ, int JT, bool MIXED, bool POT, bool EXCL, bool PM>
__global__ __launch_bounds__(kWG, (ForceOcc<I, LJ, MIXED>::kMinBlocks)) void k_force(ForceArgs fa) {
    force_body<I, LJ, JT, MIXED, POT, EXCL, PM, false>(fa);
}

// Lane groups of 4, 16, 64 or 256 per i-particle: one launch serves every
// class that uses any of them, with the group width of the class the plan
// picked (log2 in fa.cls_lj), so a block step needs at most two force
// launches whatever shapes the classes were tuned to.  The FUSE instance,
// launched only when fa.fused_mask is not empty, lets the classes in it
// predict their particles in the kernel (the other instance carries no code
// for that).
template <int JT, bool MIXED, bool POT, bool EXCL, bool PM, bool FUSE>
__global__ __launch_bounds__(kWG) void k_force_groups(ForceArgs fa) {
    const int cls = fa.host_plan ? fa.hp.cls : uniform_i32(*fa.cls);
    if (((fa.cls_mask >> cls) & 1) == 0)
        return;
    switch ((fa.cls_lj >> (4 * cls)) & 15u) {
        case 2: force_body<1, 4, JT, MIXED, POT, EXCL, PM, FUSE>(fa); break;
        case 4: force_body<1, 16, JT, MIXED, POT, EXCL, PM, FUSE>(fa); break;
        case 6: force_body<1, 64, JT, MIXED, POT, EXCL, PM, FUSE>(fa); break;
        case 8: force_body<1, 256, JT, MIXED, POT, EXCL, PM, FUSE>(fa); break;
        default: atomicOr(fa.err, kErrPlan); break;
    }
}

using KernelFn = void (*)(ForceArgs);

template <int I, int LJ, int JT>
KernelFn pick(int mixed, int pot, int excl, int pm) {
    const int key = mixed ? 4 + (pm ? 4 : 0) + pot * 2 + excl : pot * 2 + excl;
    switch (key) {
        case 0: return k_force<I, LJ, JT, false, false, false, false>;
        case 1: return k_force<I, LJ, JT, false, false, true, false>;
        case 2: return k_force<I, LJ, JT, false, true, false, false>;
        case 3: return k_force<I, LJ, JT, false, true, true, false>;
        case 4: return k_force<I, LJ, JT, true, false, false, false>;
        case 5: return k_force<I, LJ, JT, true, false, true, false>;
        case 6: return k_force<I, LJ, JT, true, true, false, false>;
        case 7: return k_force<I, LJ, JT, true, true, true, false>;
        case 8: return k_force<I, LJ, JT, true, false, false, true>;
        case 9: return k_force<I, LJ, JT, true, false, true, true>;
        case 10: return k_force<I, LJ, JT, true, true, false, true>;
        default: return k_force<I, LJ, JT, true, true, true, true>;
    }
}

template <int JT, bool FUSE>
KernelFn pick_groups(int mixed, int pot, int excl, int pm) {
    const int key = mixed ? 4 + (pm ? 4 : 0) + pot * 2 + excl : pot * 2 + excl;
    switch (key) {
        case 0: return k_force_groups<JT, false, false, false, false, FUSE>;
        case 1: return k_force_groups<JT, false, false, true, false, FUSE>;
        case 2: return k_force_groups<JT, false, true, false, false, FUSE>;
        case 3: return k_force_groups<JT, false, true, true, false, FUSE>;
        case 4: return k_force_groups<JT, true, false, false, false, FUSE>;
        case 5: return k_force_groups<JT, true, false, true, false, FUSE>;
        case 6: return k_force_groups<JT, true, true, false, false, FUSE>;
        case 7: return k_force_groups<JT, true, true, true, false, FUSE>;
        case 8: return k_force_groups<JT, true, false, false, true, FUSE>;
        case 9: return k_force_groups<JT, true, false, true, true, FUSE>;
        case 10: return k_force_groups<JT, true, true, false, true, FUSE>;
        default: return k_force_groups<JT, true, true, true, true, FUSE>;
    }
}

KernelFn lookup(const Shape &sh, int mixed, int pot, int excl, int pm, int fuse = 0) {
    if (sh.j_tile != 256)
        return nullptr;
    if (sh.j_lanes == 1 && sh.i_per_lane == 1) return pick<1, 1, 256>(mixed, pot, excl, pm);
    if (sh.j_lanes == 1 && sh.i_per_lane == 2) return pick<2, 1, 256>(mixed, pot, excl, pm);
    if (force_shape_grouped(sh))
        return fuse ? pick_groups<256, true>(mixed, pot, excl, pm)
                    : pick_groups<256, false>(mixed, pot, excl, pm);
    return nullptr;
}

}  // namespace

bool force_shape_grouped(const Shape &sh) {
    return sh.i_per_lane == 1 && sh.j_tile == 256 &&
           (sh.j_lanes == 4 || sh.j_lanes == 16 || sh.j_lanes == 64 || sh.j_lanes == 256);
}

bool force_shape_supported(const Shape &sh) { return lookup(sh, 1, 0, 0, 0) != nullptr; }

int force_j_step(const Shape &sh) {
    // must match JTX of k_force
    if (sh.j_lanes >= 64)
        return sh.j_tile > 4 * sh.j_lanes ? sh.j_tile : 4 * sh.j_lanes;
    return sh.j_tile;
}

int force_occupancy(const Shape &sh, int mixed, int want_pot, int exclude_self, int pair_mass) {
    KernelFn fn = lookup(sh, mixed, want_pot, exclude_self, pair_mass);
    if (!fn)
        return 0;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void *>(fn),
                                                     kWG, 0) != hipSuccess)
        return 0;
    return blocks;
}

hipError_t launch_force(const Shape &sh, int mixed, int want_pot, int exclude_self, int pair_mass,
                        const ForceArgs &fa, int grid, hipStream_t s) {
    KernelFn fn = lookup(sh, mixed, want_pot, exclude_self, pair_mass, fa.fused_mask != 0);
    if (!fn)
        return hipErrorInvalidValue;
    ForceArgs a = fa;
    void *args[] = {&a};
    return hipLaunchKernel(reinterpret_cast<const void *>(fn), dim3(grid), dim3(kWG), args, 0, s);
}

}  // namespace nb
