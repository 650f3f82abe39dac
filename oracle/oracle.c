/*
 * Plain FP64 CPU oracle for the direct N-body hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path (the
 * HIP library under paper_0709_4552_amd/) never calls into it, and the two
 * share no code, header, table or helper.
 *
 * What it computes (Groen, Portegies Zwart, McMillan & Makino, "Distributed
 * N-body Simulation on the Grid Using Dedicated Hardware"):
 *
 *   Section 4.1, step list: select the block of active particles at the next
 *   system time, predict all N particles to that time, compute the forces and
 *   their time derivatives between the n active particles and all N, correct
 *   the n active particles and update their time steps, repeat until one
 *   N-body time unit has passed.
 *   Section 2: 4th-order Hermite scheme (Makino & Aarseth 1992) with block
 *   time steps quantised to powers of two between 2^-22 and 2^-3, Plummer
 *   softening 2^-8 (both are parameters here).
 *
 * The paper prints none of the formulas; the ones below are the standard
 * published Hermite-4 and block-step mathematics of the methods it cites.
 * Readings where the paper is silent:
 *   - softening enters as s = r^2 + eps^2, G = 1;
 *   - the potential is returned beside acceleration and jerk;
 *   - the time-step criterion is Aarseth's, with parameter eta; the start-up
 *     step is eta_init*|a|/|j|;
 *   - one predict-evaluate-correct pass per step (no iteration), and the
 *     active particles use predicted values like every other particle;
 *   - a step may be halved freely, and doubled (at most once per step) only
 *     when the new time is a multiple of the doubled step.
 *
 * Layout: positions, velocities, accelerations and jerks are (N,3) row-major
 * float64 arrays (array of structures), times t_i and steps dt_i are float64.
 * Powers of two up to 2^-30 added to times below 2^20 are exact in binary
 * floating point, so times need no integer representation here.
 *
 * Built with gcc -O3 -fopenmp, without -ffast-math, so the arithmetic is the
 * plain IEEE arithmetic written below.  Force sums run over j in ascending
 * order; OpenMP splits only the independent i (or particle) loops.
 *
 * Every function below names the part of the method it follows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double eps2;      /* square of the softening length */
    double eta;       /* accuracy parameter of the Aarseth step criterion */
    double eta_init;  /* accuracy parameter of the start-up step |a|/|j| */
    double dt_min;    /* smallest block step (a power of two) */
    double dt_max;    /* largest block step (a power of two) */
} oracle_params;

/*
 * Force, jerk and potential on each listed particle i from all other
 * particles j (section 4.1, step 4: forces and their time derivatives between
 * the n active particles and all N particles):
 *
 *   r = x_j - x_i,  w = v_j - v_i,  s = |r|^2 + eps^2
 *   a_i    =  sum_{j != i} m_j r s^{-3/2}
 *   jerk_i =  sum_{j != i} m_j [ w s^{-3/2} - 3 (r.w) r s^{-5/2} ]
 *   pot_i  = -sum_{j != i} m_j s^{-1/2}
 *
 * The sum runs over j in ascending index order.  pot may be NULL.
 */
void oracle_force(int64_t N, const double *x, const double *v, const double *m,
                  double eps2, int64_t n_i, const int64_t *i_list,
                  double *acc, double *jerk, double *pot)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n_i; k++) {
        const int64_t i = i_list[k];
        double ax = 0.0, ay = 0.0, az = 0.0;
        double jx = 0.0, jy = 0.0, jz = 0.0;
        double p = 0.0;
        for (int64_t j = 0; j < N; j++) {
            if (j == i)
                continue;
            const double rx = x[3 * j + 0] - x[3 * i + 0];
            const double ry = x[3 * j + 1] - x[3 * i + 1];
            const double rz = x[3 * j + 2] - x[3 * i + 2];
            const double wx = v[3 * j + 0] - v[3 * i + 0];
            const double wy = v[3 * j + 1] - v[3 * i + 1];
            const double wz = v[3 * j + 2] - v[3 * i + 2];
            const double s = rx * rx + ry * ry + rz * rz + eps2;
            const double s_m12 = 1.0 / sqrt(s);          /* s^{-1/2} */
            const double s_m32 = s_m12 / s;              /* s^{-3/2} */
            const double s_m52 = s_m32 / s;              /* s^{-5/2} */
            const double rw = rx * wx + ry * wy + rz * wz;
            ax += m[j] * rx * s_m32;
            ay += m[j] * ry * s_m32;
            az += m[j] * rz * s_m32;
            jx += m[j] * (wx * s_m32 - 3.0 * rw * rx * s_m52);
            jy += m[j] * (wy * s_m32 - 3.0 * rw * ry * s_m52);
            jz += m[j] * (wz * s_m32 - 3.0 * rw * rz * s_m52);
            p -= m[j] * s_m12;
        }
        acc[3 * k + 0] = ax;
        acc[3 * k + 1] = ay;
        acc[3 * k + 2] = az;
        jerk[3 * k + 0] = jx;
        jerk[3 * k + 1] = jy;
        jerk[3 * k + 2] = jz;
        if (pot)
            pot[k] = p;
    }
}

/*
 * Predictor (section 4.1, step 3: predict positions and velocities of all N
 * particles to time t): third-order Taylor series from each particle's own
 * time t_i, using its acceleration and jerk at t_i.
 *   d = t - t_i
 *   xp = x + v d + a d^2/2 + jerk d^3/6
 *   vp = v + a d + jerk d^2/2
 */
void oracle_predict(int64_t N, double t, const double *t_i, const double *x,
                    const double *v, const double *a, const double *jk,
                    double *xp, double *vp)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        const double d = t - t_i[i];
        for (int c = 0; c < 3; c++) {
            const int64_t q = 3 * i + c;
            xp[q] = x[q] + v[q] * d + a[q] * d * d / 2.0 + jk[q] * d * d * d / 6.0;
            vp[q] = v[q] + a[q] * d + jk[q] * d * d / 2.0;
        }
    }
}

/*
 * Hermite corrector for one particle over a step of length dt (section 4.1,
 * step 5: correct positions, velocities and velocity derivatives).  From the
 * old (a0, j0) and new (a1, j1) values the cubic a(t) through both ends gives
 * the second and third derivatives at the start of the step:
 *   a2 = [-6 (a0 - a1) - dt (4 j0 + 2 j1)] / dt^2
 *   a3 = [12 (a0 - a1) + 6 dt (j0 + j1)]   / dt^3
 * and the corrected state
 *   x1 = xp + a2 dt^4/24 + a3 dt^5/120
 *   v1 = vp + a2 dt^3/6  + a3 dt^4/24.
 * a2_out receives a2 at the END of the step (a2 + dt a3), a3_out receives a3.
 */
void oracle_correct_one(double dt, const double xp[3], const double vp[3],
                        const double a0[3], const double j0[3],
                        const double a1[3], const double j1[3],
                        double x1[3], double v1[3], double a2_out[3],
                        double a3_out[3])
{
    for (int c = 0; c < 3; c++) {
        const double a2 = (-6.0 * (a0[c] - a1[c]) - dt * (4.0 * j0[c] + 2.0 * j1[c])) / (dt * dt);
        const double a3 = (12.0 * (a0[c] - a1[c]) + 6.0 * dt * (j0[c] + j1[c])) / (dt * dt * dt);
        x1[c] = xp[c] + a2 * dt * dt * dt * dt / 24.0 + a3 * dt * dt * dt * dt * dt / 120.0;
        v1[c] = vp[c] + a2 * dt * dt * dt / 6.0 + a3 * dt * dt * dt * dt / 24.0;
        a2_out[c] = a2 + dt * a3;
        a3_out[c] = a3;
    }
}

static double norm3(const double *u)
{
    return sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
}

/*
 * Aarseth's time-step criterion evaluated at the end of a step (section 2
 * says the correction also yields each particle's next block step but does
 * not name the criterion; this one is the reading chosen here):
 *   dt = sqrt( eta (|a||a2| + |j|^2) / (|j||a3| + |a2|^2) )
 * A zero denominator means no constraint (+infinity).
 */
double oracle_aarseth_dt(const double a[3], const double j[3], const double a2[3],
                         const double a3[3], double eta)
{
    const double na = norm3(a), nj = norm3(j), na2 = norm3(a2), na3 = norm3(a3);
    const double num = na * na2 + nj * nj;
    const double den = nj * na3 + na2 * na2;
    if (den > 0.0)
        return sqrt(eta * num / den);
    return INFINITY;
}

/*
 * Block-step quantisation (section 2: steps blocked in powers of two between
 * a minimum and a maximum).  Starting from the particle's current step dt_old
 * at its new time t_new:
 *   - if the criterion asks for less than dt_old, halve until dt <= dt_raw
 *     (stopping at dt_min; *clamped is set when dt_min is still too long);
 *   - else if it allows at least 2 dt_old, and t_new is a multiple of
 *     2 dt_old, and 2 dt_old <= dt_max, double once;
 *   - otherwise keep dt_old.
 */
double oracle_block_dt(double dt_old, double t_new, double dt_raw,
                       const oracle_params *p, int *clamped)
{
    double dt = dt_old;
    if (dt_raw < dt) {
        while (dt > dt_raw && dt > p->dt_min)
            dt *= 0.5;
        if (dt > dt_raw && clamped)
            *clamped = 1;
    } else if (dt_raw >= 2.0 * dt && 2.0 * dt <= p->dt_max &&
               fmod(t_new, 2.0 * dt) == 0.0) {
        dt *= 2.0;
    }
    return dt;
}

/*
 * Start-up step: the largest power of two not above eta_init |a|/|j|, inside
 * [dt_min, dt_max].  |j| = 0 puts no constraint on the step.
 */
double oracle_initial_dt(const double a[3], const double j[3], const oracle_params *p,
                         int *clamped)
{
    const double na = norm3(a), nj = norm3(j);
    const double want = nj > 0.0 ? p->eta_init * na / nj : INFINITY;
    double dt = p->dt_max;
    while (dt > want && dt > p->dt_min)
        dt *= 0.5;
    if (dt > want && clamped)
        *clamped = 1;
    return dt;
}

/*
 * Initialisation (section 4.1, step 1): all particles at time t0, a full force
 * sweep for every particle, then the start-up step of each particle.
 */
void oracle_init(int64_t N, const oracle_params *p, const double *x, const double *v,
                 const double *m, double t0, double *a, double *jk, double *t_i,
                 double *dt_i, int64_t *n_clamped)
{
    int64_t *all = (int64_t *)calloc((size_t)(N > 0 ? N : 1), sizeof(int64_t));
    for (int64_t i = 0; i < N; i++)
        all[i] = i;
    oracle_force(N, x, v, m, p->eps2, N, all, a, jk, NULL);
    free(all);
    int64_t clamps = 0;
    for (int64_t i = 0; i < N; i++) {
        int c = 0;
        t_i[i] = t0;
        dt_i[i] = oracle_initial_dt(&a[3 * i], &jk[3 * i], p, &c);
        clamps += c;
    }
    if (n_clamped)
        *n_clamped = clamps;
}

/*
 * One block step (section 4.1, steps 2 to 5):
 *   2. t = min_i (t_i + dt_i); the block is every i with t_i + dt_i = t,
 *      taken in ascending index order;
 *   3. predict all N particles to t;
 *   4. force, jerk (and potential) on the block from all N predicted particles;
 *   5. correct each particle of the block, set t_i = t, store the new a and
 *      jerk, and give it its next block step.
 * Returns the block size n; *t_out receives t.  If i_out is not NULL it
 * receives the block (ascending).  pot_out (length N, may be NULL) receives
 * the potential of the block particles at their index.
 */
int64_t oracle_block_step(int64_t N, const oracle_params *p, double *x, double *v,
                          double *a, double *jk, const double *m, double *t_i,
                          double *dt_i, double *t_out, int64_t *i_out,
                          int64_t *n_clamped, double *pot_out)
{
    double t = INFINITY;
    for (int64_t i = 0; i < N; i++) {
        const double ti = t_i[i] + dt_i[i];
        if (ti < t)
            t = ti;
    }
    int64_t *act = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    int64_t n = 0;
    for (int64_t i = 0; i < N; i++)
        if (t_i[i] + dt_i[i] == t)
            act[n++] = i;

    double *xp = (double *)malloc((size_t)N * 3 * sizeof(double));
    double *vp = (double *)malloc((size_t)N * 3 * sizeof(double));
    oracle_predict(N, t, t_i, x, v, a, jk, xp, vp);

    double *a1 = (double *)malloc((size_t)n * 3 * sizeof(double));
    double *j1 = (double *)malloc((size_t)n * 3 * sizeof(double));
    double *pt = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    oracle_force(N, xp, vp, m, p->eps2, n, act, a1, j1, pt);

    int64_t clamps = 0;
    for (int64_t k = 0; k < n; k++) {
        const int64_t i = act[k];
        const double dt = dt_i[i];
        double x1[3], v1[3], a2[3], a3[3];
        oracle_correct_one(dt, &xp[3 * i], &vp[3 * i], &a[3 * i], &jk[3 * i],
                           &a1[3 * k], &j1[3 * k], x1, v1, a2, a3);
        for (int c = 0; c < 3; c++) {
            x[3 * i + c] = x1[c];
            v[3 * i + c] = v1[c];
            a[3 * i + c] = a1[3 * k + c];
            jk[3 * i + c] = j1[3 * k + c];
        }
        t_i[i] = t;
        const double dt_raw = oracle_aarseth_dt(&a1[3 * k], &j1[3 * k], a2, a3, p->eta);
        int cl = 0;
        dt_i[i] = oracle_block_dt(dt, t, dt_raw, p, &cl);
        clamps += cl;
        if (pot_out)
            pot_out[i] = pt[k];
        if (i_out)
            i_out[k] = i;
    }
    if (n_clamped)
        *n_clamped += clamps;
    if (t_out)
        *t_out = t;
    free(act);
    free(xp);
    free(vp);
    free(a1);
    free(j1);
    free(pt);
    return n;
}

/*
 * Repeat block steps while the next block time does not exceed t_end
 * (section 4.1, step 6).  Returns the number of block steps; *n_updates
 * receives the total number of particle updates (sum of block sizes).
 */
int64_t oracle_run(int64_t N, const oracle_params *p, double *x, double *v, double *a,
                   double *jk, const double *m, double *t_i, double *dt_i,
                   double t_end, int64_t max_steps, int64_t *n_updates,
                   int64_t *n_clamped)
{
    int64_t steps = 0, updates = 0;
    while (steps < max_steps) {
        double t = INFINITY;
        for (int64_t i = 0; i < N; i++)
            if (t_i[i] + dt_i[i] < t)
                t = t_i[i] + dt_i[i];
        if (!(t <= t_end))
            break;
        double tt;
        updates += oracle_block_step(N, p, x, v, a, jk, m, t_i, dt_i, &tt, NULL,
                                     n_clamped, NULL);
        steps++;
    }
    if (n_updates)
        *n_updates = updates;
    return steps;
}

/*
 * Total energy of the softened system and its parts:
 *   T = sum_i m_i |v_i|^2 / 2,   U = -sum_{i<j} m_i m_j (|x_i-x_j|^2 + eps^2)^{-1/2}.
 * The per-i partial sums are added in ascending i so the result does not
 * depend on the thread count.
 */
void oracle_energy(int64_t N, const double *x, const double *v, const double *m,
                   double eps2, double *ekin, double *epot)
{
    double *row = (double *)malloc((size_t)(N > 0 ? N : 1) * sizeof(double));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < N; i++) {
        double u = 0.0;
        for (int64_t j = i + 1; j < N; j++) {
            const double rx = x[3 * j + 0] - x[3 * i + 0];
            const double ry = x[3 * j + 1] - x[3 * i + 1];
            const double rz = x[3 * j + 2] - x[3 * i + 2];
            u -= m[i] * m[j] / sqrt(rx * rx + ry * ry + rz * rz + eps2);
        }
        row[i] = u;
    }
    double t = 0.0, u = 0.0;
    for (int64_t i = 0; i < N; i++) {
        t += 0.5 * m[i] * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] +
                           v[3 * i + 2] * v[3 * i + 2]);
        u += row[i];
    }
    free(row);
    *ekin = t;
    *epot = u;
}

/* Number of OpenMP threads the oracle will use (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int oracle_threads(void) { return omp_get_max_threads(); }
void oracle_set_threads(int n) { omp_set_num_threads(n); }
#else
int oracle_threads(void) { return 1; }
void oracle_set_threads(int n) { (void)n; }
#endif
