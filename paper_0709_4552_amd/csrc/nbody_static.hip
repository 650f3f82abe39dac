// Allocation-free force evaluation (nbody_force_jerk_static): the force,
// jerk and potential sum of nbody_force_jerk (section 4.1, step 4) on
// caller-given particles, with every buffer the kernels need beyond the
// inputs and outputs in one file-scope device array.  For callers that cannot
// allocate device memory: code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc.
//
// The array (`scratch`) is a host-side stand-in in host code: its device
// address on each GPU comes from hipGetSymbolAddress on the first call made
// with that GPU current, and only that address is ever handed to a kernel.
// Every call on a GPU shares that GPU's array and leaves its contents behind;
// each call clears what must start at zero with a fill kernel (no memset, so
// the call can be captured into a graph).  Calls that overlap on one GPU (two
// streams, two threads) race on the array.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "nbody.h"
#include "nbody_internal.h"

using namespace nb;

namespace {

// ---- layout of the scratch array (byte offsets, 256-byte aligned) ----------
constexpr int64_t kMaxJ = NBODY_STATIC_MAX_PARTICLES;
constexpr int64_t kPartSlots = 1 << 17;  // j-split partial sums (7 doubles each)

constexpr int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

// j-particle buffer: mixed P, Q (float4), R (float2), V (float4) = 56 B; FP64
// A, B, C (double2), D (double) = 56 B; the two forms share the region
constexpr int64_t kOffJ0 = 0;                                  // P or A
constexpr int64_t kOffJ1 = kOffJ0 + align256(16 * kMaxJ);      // Q or B
constexpr int64_t kOffJ2 = kOffJ1 + align256(16 * kMaxJ);      // R (float2) or C (double2)
constexpr int64_t kOffJ3 = kOffJ2 + align256(16 * kMaxJ);      // V (float4) or D (double)
constexpr int64_t kOffHint = kOffJ3 + align256(16 * kMaxJ);    // 6 x kMaxJ doubles (a, jerk)
constexpr int64_t kOffPart = kOffHint + align256(6 * 8 * kMaxJ);
constexpr int64_t kOffSmall = kOffPart + align256(7 * 8 * kPartSlots);
// small region: cluster offsets, scales, bounding box, plan, control block
constexpr int64_t kOffOff = kOffSmall;                    // int64[2]
constexpr int64_t kOffScale = kOffOff + 256;              // float4 (as 4 x uint32 for atomics)
constexpr int64_t kOffBox = kOffScale + 256;              // 6 x uint64 ordered keys, double4 origin
constexpr int64_t kOffPlan = kOffBox + 256;               // plan arrays, 64 B each
constexpr int64_t kOffCtl = kOffPlan + 8 * 64;            // DevCtl
constexpr int64_t kScratchBytes = align256(kOffCtl + (int64_t)sizeof(DevCtl));

static_assert(sizeof(DevCtl) <= 256, "control block");

}  // namespace

// The allocation-free entry point's device memory: about 35 MB per GPU,
// held until the process ends.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
std::atomic<unsigned char *> g_ptr[kMaxDevices];
std::atomic<int> g_cus[kMaxDevices];
std::atomic<int> g_err[kMaxDevices];

// Device address of `scratch` on the current device, looked up once.
unsigned char *scratch_ptr(int dev, int *cus, hipError_t *err) {
    std::call_once(g_once[dev], [dev] {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        int n = 0;
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
        g_err[dev].store((int)e);
        g_cus[dev].store(n > 0 ? n : 256);
        g_ptr[dev].store(e == hipSuccess ? static_cast<unsigned char *>(p) : nullptr);
    });
    *err = (hipError_t)g_err[dev].load();
    *cus = g_cus[dev].load();
    return g_ptr[dev].load();
}

// ---- kernels ----------------------------------------------------------------

// Order-preserving integer keys of finite doubles (for atomic min / max).
__device__ inline unsigned long long order_key(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | (1ull << 63));
}
__device__ inline double from_order_key(unsigned long long k) {
    return __longlong_as_double((long long)((k >> 63) ? (k & ~(1ull << 63)) : ~k));
}

// Reset the control block, the cluster offsets, the scale accumulators and
// the bounding box.
__global__ void k_static_clear(DevCtl *ctl, int64_t *off, unsigned *scale,
                               unsigned long long *box, int64_t n_j) {
    const int t = threadIdx.x;
    unsigned *c = reinterpret_cast<unsigned *>(ctl);
    for (int q = t; q < (int)(sizeof(DevCtl) / 4); q += blockDim.x)
        c[q] = 0u;
    if (t == 0) {
        ctl->t_end_tick = INT64_MAX;
        off[0] = 0;
        off[1] = n_j;
        scale[0] = 0u;            // largest |m| (float bits; values >= 0)
        scale[1] = 0x7f800000u;   // smallest |m| (+inf)
        scale[2] = 0u;            // largest speed
        scale[3] = 0u;
    }
    if (t < 3) {
        box[t] = ~0ull;      // smallest coordinate on axis t
        box[3 + t] = 0ull;   // largest
    }
}

// Mixed form: the bounding box of the finite positions, whose centre rounded
// to a multiple of 64 is the origin of the j-records (as a context's cluster).
__global__ __launch_bounds__(kWG) void k_static_bounds(State st, int64_t n,
                                                       unsigned long long *box) {
    unsigned long long lo[3] = {~0ull, ~0ull, ~0ull}, hi[3] = {0ull, 0ull, 0ull};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double x[3] = {st.x[i], st.y[i], st.z[i]};
        for (int q = 0; q < 3; q++)
            if (isfinite(x[q])) {
                const unsigned long long k = order_key(x[q]);
                lo[q] = min(lo[q], k);
                hi[q] = max(hi[q], k);
            }
    }
    for (int q = 0; q < 3; q++)
        for (int o = 32; o > 0; o >>= 1) {
            lo[q] = min(lo[q], (unsigned long long)__shfl_xor((long long)lo[q], o));
            hi[q] = max(hi[q], (unsigned long long)__shfl_xor((long long)hi[q], o));
        }
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 3; q++) {
            atomicMin(&box[q], lo[q]);
            atomicMax(&box[3 + q], hi[q]);
        }
}

__device__ inline float wave_max_f(float v) {
    for (int o = 32; o > 0; o >>= 1)
        v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
__device__ inline float wave_min_f(float v) {
    for (int o = 32; o > 0; o >>= 1)
        v = fminf(v, __shfl_xor(v, o));
    return v;
}

// The j-particle records of the caller's particles (taken as they are: the
// evaluation time is theirs), and in the mixed form the cluster's largest and
// smallest mass and largest speed, which size the near field.
template <int MIXED>
__global__ __launch_bounds__(kWG) void k_static_stage(State st, int64_t n, JBuf jb, double grid_q,
                                                      double grid_inv, unsigned *scale,
                                                      const unsigned long long *box,
                                                      double4 *origin_out) {
    float mx = 0.f, mn = INFINITY, vx = 0.f;
    double o[3] = {0.0, 0.0, 0.0};
    if (MIXED)
        for (int q = 0; q < 3; q++)
            if (box[q] <= box[3 + q])  // some finite coordinate
                o[q] = 64.0 * rint((0.5 * from_order_key(box[q]) +
                                    0.5 * from_order_key(box[3 + q])) * (1.0 / 64.0));
    if (MIXED && blockIdx.x == 0 && threadIdx.x == 0)
        *origin_out = make_double4(o[0], o[1], o[2], 0.0);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double x = st.x[i], y = st.y[i], z = st.z[i];
        const double u = st.vx[i], v = st.vy[i], w = st.vz[i];
        const double m = st.m[i];
        if (MIXED) {
            float4 P, Q, V;
            float2 R;
            split_mixed(x - o[0], y - o[1], z - o[2], u, v, w, m, grid_q, grid_inv, P, Q, R, V);
            jb.P[i] = P;
            jb.Q[i] = Q;
            jb.R[i] = R;
            jb.V[i] = V;
            const float am = (float)fabs(m);
            mx = fmaxf(mx, am);
            if (am > 0.f)  // the smallest mass that attracts
                mn = fminf(mn, am);
            vx = fmaxf(vx, (float)sqrt(u * u + v * v + w * w));
        } else {
            jb.A[i] = make_double2(x, y);
            jb.B[i] = make_double2(z, m);
            jb.C[i] = make_double2(u, v);
            jb.D[i] = w;
        }
    }
    if (MIXED) {
        __shared__ float red[3][kWG / 64];
        mx = wave_max_f(mx);
        mn = wave_min_f(mn);
        vx = wave_max_f(vx);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        if (lane == 0) {
            red[0][wv] = mx;
            red[1][wv] = mn;
            red[2][wv] = vx;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = 1; q < kWG / 64; q++) {
                mx = fmaxf(mx, red[0][q]);
                mn = fminf(mn, red[1][q]);
                vx = fmaxf(vx, red[2][q]);
            }
            // non-negative floats order like their bit patterns
            atomicMax(&scale[0], __float_as_uint(mx));
            atomicMin(&scale[1], __float_as_uint(mn));
            atomicMax(&scale[2], __float_as_uint(vx));
        }
    }
}

// Near-field hints from a first pass: the acceleration and jerk of each listed
// particle, stored at its particle index (the force kernel reads them there).
__global__ void k_static_hints(const int32_t *i_list, int64_t n, int64_t n_j, const double *acc,
                               const double *jerk, double *hint) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = i_list[k];
        if (i < 0 || i >= n_j)
            continue;  // the force kernel flags it
        for (int q = 0; q < 3; q++) {
            hint[q * n_j + i] = acc[q * n + k];
            hint[(3 + q) * n_j + i] = jerk[q * n + k];
        }
    }
}

int grid_for_n(int64_t n) {
    int64_t g = (n + kWG - 1) / kWG;
    return (int)(g < 1 ? 1 : (g > 2048 ? 2048 : g));
}

// Default launch shapes by block size (the same classes as a new context).
const Shape kShapes[kClasses] = {{1, 1, 256}, {1, 4, 256}, {1, 16, 256}, {1, 64, 256},
                                 {1, 256, 256}};
const int32_t kMinN[kClasses] = {2048, 256, 32, 4, 0};

// One force evaluation: the plan (made here), the planned class's force
// launch (the one-lane shape or the lane-group launch), j-split reduction.
hipError_t evaluate(ForceArgs fa, DevCtl *ctl, int mixed, int want_pot, int excl, int cus,
                    int64_t n, hipStream_t s) {
    const int pm = mixed;  // the per-pair near test: masses are not known on the host
    ClassTable ct{};
    int grid[kClasses];
    for (int k = 0; k < kClasses; k++) {
        const int occ = force_occupancy(kShapes[k], mixed, want_pot, excl, pm);
        grid[k] = (occ > 0 ? occ : 1) * cus;
        ct.min_n[k] = kMinN[k];
        ct.ib[k] = (kWG / kShapes[k].j_lanes) * kShapes[k].i_per_lane;
        ct.grid[k] = grid[k];
        ct.jt[k] = force_j_step(kShapes[k]);
    }
    // the plan, made here: only the planned class's kernel is launched
    fa.host_plan = 1;
    fa.hp = plan_on_host(ct, n, fa.n_total, fa.part_cap);
    fa.hp_n = (int32_t)n;
    fa.cls_lj = 0;
    for (int k = 0; k < kClasses; k++) {
        int lg = 0;
        while ((1 << lg) < kShapes[k].j_lanes)
            lg++;
        fa.cls_lj |= (uint32_t)lg << (4 * k);
    }
    // class 0: one lane per i; classes 1-4: the lane-group launch
    const int k = fa.hp.cls;
    fa.cls_mask = 1 << k;
    hipError_t e = launch_force(kShapes[k], mixed, want_pot, excl, pm, fa, grid[k], s);
    if (e != hipSuccess)
        return e;
    return launch_reduce(fa, nullptr, n, &ctl->s_max, s);
}

}  // namespace

extern "C" int nbody_force_jerk_static(const nbody_direct *in, const int32_t *i_list, int64_t n,
                                       double *acc, double *jerk, double *pot, void *stream) {
    if (!in || !i_list || !acc || !jerk)
        return NBODY_EINVAL;
    for (int q = 0; q < 3; q++)
        if (!in->pos[q] || !in->vel[q])
            return NBODY_EINVAL;
    if (!in->mass)
        return NBODY_EINVAL;
    if (in->precision != NBODY_PREC_FP64 && in->precision != NBODY_PREC_MIXED)
        return NBODY_EINVAL;
    if (!(in->eps >= 0.0) || !std::isfinite(in->eps))
        return NBODY_EINVAL;
    const int hints_a = in->acc_hint[0] && in->acc_hint[1] && in->acc_hint[2];
    const int hints_j = in->jerk_hint[0] && in->jerk_hint[1] && in->jerk_hint[2];
    const int any_hint = in->acc_hint[0] || in->acc_hint[1] || in->acc_hint[2] ||
                         in->jerk_hint[0] || in->jerk_hint[1] || in->jerk_hint[2];
    if (any_hint && !(hints_a && hints_j))
        return NBODY_EINVAL;  // all six hint arrays or none
    if (in->n_j < 1 || n < 1)
        return NBODY_EINVAL;
    if (in->n_j > kMaxJ || n > kMaxJ)
        return NBODY_ESCRATCH;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return NBODY_EDEVICE;
    if (dev < 0 || dev >= kMaxDevices)
        return NBODY_EUNSUPPORTED;
    int cus = 256;
    hipError_t e = hipSuccess;
    unsigned char *base = scratch_ptr(dev, &cus, &e);
    if (!base || e != hipSuccess)
        return NBODY_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);

    const int mixed = in->precision == NBODY_PREC_MIXED;
    const int64_t N = in->n_j;
    const double eps2 = in->eps * in->eps;
    const int excl = eps2 == 0.0;
    const int want_pot = pot != nullptr;
    const double grid_q = std::ldexp(1.0, kGridQLog2), grid_inv = std::ldexp(1.0, -kGridQLog2);

    JBuf jb;
    if (mixed) {
        jb.P = reinterpret_cast<float4 *>(base + kOffJ0);
        jb.Q = reinterpret_cast<float4 *>(base + kOffJ1);
        jb.R = reinterpret_cast<float2 *>(base + kOffJ2);
        jb.V = reinterpret_cast<float4 *>(base + kOffJ3);
    } else {
        jb.A = reinterpret_cast<double2 *>(base + kOffJ0);
        jb.B = reinterpret_cast<double2 *>(base + kOffJ1);
        jb.C = reinterpret_cast<double2 *>(base + kOffJ2);
        jb.D = reinterpret_cast<double *>(base + kOffJ3);
    }
    double *hint = reinterpret_cast<double *>(base + kOffHint);
    double *part = reinterpret_cast<double *>(base + kOffPart);
    int64_t *off = reinterpret_cast<int64_t *>(base + kOffOff);
    unsigned *scale = reinterpret_cast<unsigned *>(base + kOffScale);
    unsigned long long *box = reinterpret_cast<unsigned long long *>(base + kOffBox);
    double4 *origin = reinterpret_cast<double4 *>(base + kOffBox + 64);
    DevCtl *ctl = reinterpret_cast<DevCtl *>(base + kOffCtl);
    unsigned char *pb = base + kOffPlan;
    PlanDev pl{};
    pl.item_begin = reinterpret_cast<int64_t *>(pb + 0 * 64);
    pl.S = reinterpret_cast<int32_t *>(pb + 1 * 64);
    pl.jlen = reinterpret_cast<int32_t *>(pb + 2 * 64);
    pl.part_begin = reinterpret_cast<int64_t *>(pb + 3 * 64);
    pl.n_cur = reinterpret_cast<int32_t *>(pb + 4 * 64);
    pl.t_cur = reinterpret_cast<int64_t *>(pb + 5 * 64);
    pl.t_now = reinterpret_cast<int64_t *>(pb + 6 * 64);
    pl.lev_cnt = nullptr;

    State st{};
    st.x = const_cast<double *>(in->pos[0]);
    st.y = const_cast<double *>(in->pos[1]);
    st.z = const_cast<double *>(in->pos[2]);
    st.vx = const_cast<double *>(in->vel[0]);
    st.vy = const_cast<double *>(in->vel[1]);
    st.vz = const_cast<double *>(in->vel[2]);
    st.m = const_cast<double *>(in->mass);

    hipLaunchKernelGGL(k_static_clear, dim3(1), dim3(64), 0, s, ctl, off, scale, box, N);
    if ((e = hipGetLastError()) != hipSuccess)
        return NBODY_EDEVICE;
    if (mixed) {
        hipLaunchKernelGGL(k_static_bounds, dim3(grid_for_n(N)), dim3(kWG), 0, s, st, N, box);
        if ((e = hipGetLastError()) != hipSuccess)
            return NBODY_EDEVICE;
        hipLaunchKernelGGL(k_static_stage<1>, dim3(grid_for_n(N)), dim3(kWG), 0, s, st, N, jb,
                           grid_q, grid_inv, scale, box, origin);
    } else {
        hipLaunchKernelGGL(k_static_stage<0>, dim3(grid_for_n(N)), dim3(kWG), 0, s, st, N, jb,
                           grid_q, grid_inv, scale, box, origin);
    }
    if ((e = hipGetLastError()) != hipSuccess)
        return NBODY_EDEVICE;

    ForceArgs fa{};
    fa.jb = jb;
    fa.off = off;
    fa.C = 1;
    fa.item_begin = pl.item_begin;
    fa.S = pl.S;
    fa.jlen = pl.jlen;
    fa.part_begin = pl.part_begin;
    fa.n_cur = pl.n_cur;
    fa.total_items = reinterpret_cast<const int64_t *>(&ctl->total_items);
    fa.i_list = i_list;
    fa.slots_at_offsets = 0;
    fa.out_acc = acc;
    fa.out_jerk = jerk;
    fa.out_pot = pot;
    fa.out_stride = n;
    fa.part = part;
    fa.part_cap = kPartSlots;
    fa.err = &ctl->err;
    fa.item_counter = &ctl->item_counter;
    fa.cls = &ctl->cls;
    fa.fetch_lane = 0;
    fa.n_total = N;
    fa.eps2 = eps2;
    fa.eps2f = (float)eps2;
    fa.m64 = in->mass;
    fa.nscale = reinterpret_cast<const float4 *>(scale);
    fa.fused_mask = 0;
    fa.st = st;
    fa.t_cur = pl.t_cur;
    fa.tick = 1.0;
    fa.grid_q = grid_q;
    fa.grid_inv = grid_inv;
    fa.origin = origin;
    fa.near_frac = 0.f;
    fa.near_frac_jerk = 0.f;

    if (mixed) {
        const double *ha[3], *hj[3];
        if (hints_a) {
            for (int q = 0; q < 3; q++) {
                ha[q] = in->acc_hint[q];
                hj[q] = in->jerk_hint[q];
            }
        } else {
            // a first pass without the near field gives the hints (the start-up
            // sweep of nbody_init does the same); its outputs are overwritten
            fa.hax = fa.hay = fa.haz = nullptr;
            fa.hjx = fa.hjy = fa.hjz = nullptr;
            fa.out_pot = nullptr;
            if ((e = evaluate(fa, ctl, mixed, 0, excl, cus, n, s)) != hipSuccess)
                return NBODY_EDEVICE;
            hipLaunchKernelGGL(k_static_hints, dim3(grid_for_n(n)), dim3(kWG), 0, s, i_list, n, N,
                               acc, jerk, hint);
            if ((e = hipGetLastError()) != hipSuccess)
                return NBODY_EDEVICE;
            for (int q = 0; q < 3; q++) {
                ha[q] = hint + q * N;
                hj[q] = hint + (3 + q) * N;
            }
            fa.out_pot = pot;
        }
        fa.hax = ha[0];
        fa.hay = ha[1];
        fa.haz = ha[2];
        fa.hjx = hj[0];
        fa.hjy = hj[1];
        fa.hjz = hj[2];
        fa.near_frac = kNearFrac;
        fa.near_frac_jerk = kNearFracJerk;
    }
    if ((e = evaluate(fa, ctl, mixed, want_pot, excl, cus, n, s)) != hipSuccess)
        return NBODY_EDEVICE;
    return NBODY_OK;
}
