/*
 * TEST INFRASTRUCTURE ONLY -- plain FP64 CPU oracle of the batched
 * driving-physics control step.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg use it; the HIP product path never does, and
 * the two share no code.
 *
 * The paper (SceneFactory, arXiv 2605.08528) fixes the problem: W worlds of
 * up to M vehicles stepped at 120 Hz with 4 substeps per 30 Hz control tick
 * (Sec. "Experimental Setup", Algorithm "SceneFactory Pipeline"), steering
 * by a PD loop (Eq. steer PD), front-wheel drive and four-wheel brakes
 * (Sec. "Action Space Details"), friction from surface and water film
 * (Sec. "Weather-to-Friction Module"), the three-circle vehicle shape and
 * swept-circle TTC (Sec. "Neighbor vehicles"), sparse event rewards and
 * termination (Sec. "Reward Design Details"), teleport resets (Sec.
 * "Teleport-only reset").  The paper's own physics is a closed solver; the
 * vehicle model here (raycast wheels, massless spring-damper suspension,
 * linear-saturated tire inside a friction circle, implicit wheel spin with a
 * Coulomb brake, semi-implicit rigid chassis, frictionless Jacobi contact
 * between vehicle circles) is the reading the design notes list, written out
 * plainly.  Discrete decisions (contact pairs, goal / drift / fall / tilt,
 * nearest-neighbour order) are integer predicates on quantised positions so
 * that any implementation evaluating them on the same floats agrees exactly.
 */
#include "sf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NW 4
#define KEY_CAP ((int64_t)1 << 43) /* saturation of kNN squared distances */

struct or_sim {
    or_params p;
    int W, N, S;
    int *aoff, *roff, *toff, *soff;
    double *road_xy; uint8_t *road_type;
    double *road_dir;   /* [P][2] polyline direction per point (0 if not given) */
    double *tri; uint8_t *tri_surf;
    double *mu;      /* [W][S] effective */
    double *film;    /* [W] water film depth [mm] */
    int *pav;        /* [W] pavement (0 AC, 1 SMA, 2 OGFC) */
    double *spawn;   /* [E][5] */
    uint64_t seed;
    int *world_of;   /* [N] */
    double *f;       /* [OR_NF][N] */
    int32_t *k;      /* [OR_NK][N] */
    /* derived constants */
    double Iw, ell, cr, cd, z_ride;
    /* learned tire surrogate (optional) */
    int sur_on;
    float *sur;                 /* flat parameters, OR_SUR_PARAMS floats */
    float env_lo[OR_SUR_IN], env_hi[OR_SUR_IN];
    long long sur_used, sur_fallback;
    float *sample_rec;          /* [N][4][OR_SAMPLE] of the last substep, or NULL */
    int dynamics;               /* OR_DYN_PHYSICS or OR_DYN_BICYCLE */
    int shaping;                /* dense rewards and the lane-forbidden event */
    double *tri_mu_scale;       /* [T] friction factor per road triangle, or NULL */
};

#define F(s, fld, i) ((s)->f[(size_t)(fld) * (s)->N + (i)])
#define K(s, fld, i) ((s)->k[(size_t)(fld) * (s)->N + (i)])

/* ---------------------------------------------------------------- vectors */
static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
/* rotation matrix of unit quaternion q = (w, x, y, z) */
static void quat_to_R(const double *q, double R[3][3]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z); R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z); R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y); R[2][1] = 2 * (y * z + w * x); R[2][2] = 1 - 2 * (x * x + y * y);
}
static void matvec(double R[3][3], const double *a, double *b) {
    for (int r = 0; r < 3; ++r) b[r] = R[r][0] * a[0] + R[r][1] * a[1] + R[r][2] * a[2];
}
static void matTvec(double R[3][3], const double *a, double *b) {
    for (int r = 0; r < 3; ++r) b[r] = R[0][r] * a[0] + R[1][r] * a[1] + R[2][r] * a[2];
}

/* ------------------------------------------------------------ quantisers */
/* positions in units of 2^-10 m, round half to even, saturating at 2^29 */
static int64_t Qp(double x) {
    double y = x * 1024.0;
    if (isnan(y)) return 0;
    if (y >= 536870912.0) return 536870912;
    if (y <= -536870912.0) return -536870912;
    return (int64_t)rint(y);
}
/* quaternion components in units of 2^-14 */
static int64_t Qq(double x) {
    double y = x * 16384.0;
    if (isnan(y)) return 0;
    if (y >= 32768.0) return 32768;
    if (y <= -32768.0) return -32768;
    return (int64_t)rint(y);
}
/* floor(sqrt(v)) for v >= 0, digit by digit */
static uint64_t isqrt_u64(uint64_t v) {
    uint64_t res = 0, bit = (uint64_t)1 << 62;
    while (bit > v) bit >>= 2;
    while (bit) {
        if (v >= res + bit) { v -= res + bit; res = (res >> 1) + bit; }
        else res >>= 1;
        bit >>= 2;
    }
    return res;
}

/* ------------------------------------------------------------------ rng */
/* SplitMix64 (Steele, Lea, Flood 2014) */
static uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------ weather -> mu  */
/* Effective static mu vs water film at 13.89 m/s for the three pavements,
 * read from the paper's figure of mu against film depth (0..0.8 mm). */
static const double MU_CURVE[3][9] = {
    {1.1048, 1.0657, 1.0161, 0.9593, 0.9039, 0.8595, 0.8302, 0.8134, 0.8044},
    {1.2043, 1.1618, 1.1078, 1.0461, 0.9857, 0.9374, 0.9056, 0.8874, 0.8776},
    {1.3368, 1.2898, 1.2301, 1.1617, 1.0948, 1.0413, 1.0061, 0.9860, 0.9753}};

static double curve_at(int pav, double h) {
    const double *c = MU_CURVE[(pav >= 0 && pav < 3) ? pav : 0];
    if (!(h > 0.0)) return c[0];
    if (h >= 1.0) return 0.0; /* full hydroplaning at >= 1 mm */
    if (h > 0.8) return c[8] * (1.0 - h) / 0.2; /* to zero at 1 mm */
    double x = h / 0.1;
    int i = (int)floor(x);
    if (i >= 8) return c[8];
    double a = x - i;
    return c[i] * (1.0 - a) + c[i + 1] * a;
}

double or_weather_mu(double mu_class, double film_mm, int pavement) {
    double mu = mu_class * curve_at(pavement, film_mm) / curve_at(pavement, 0.0);
    return mu < 1e-3 ? 1e-3 : mu; /* friction floor */
}

void or_circle_model(const or_params *p, double *r, double *d) {
    double rr = 0.55 * p->width;
    if (rr < 0.45) rr = 0.45;
    double dd = 0.5 * p->length - 0.8 * rr;
    if (dd < 0.0) dd = 0.0;
    if (dd > 0.5 * p->wheelbase) dd = 0.5 * p->wheelbase;
    *r = rr;
    *d = dd;
}

/* ------------------------------------------------------------ lifecycle */
static void spawn_agent(or_sim *s, int i);

void or_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

or_sim *or_create(const or_world_desc *d, const or_params *prm) {
    or_sim *s = (or_sim *)calloc(1, sizeof(or_sim));
    s->p = *prm;
    s->W = d->num_worlds;
    s->S = d->num_surfaces;
    s->seed = d->seed;
    int W = s->W;
    s->aoff = (int *)malloc(sizeof(int) * (W + 1));
    s->roff = (int *)malloc(sizeof(int) * (W + 1));
    s->toff = (int *)malloc(sizeof(int) * (W + 1));
    s->soff = (int *)malloc(sizeof(int) * (W + 1));
    for (int w = 0; w <= W; ++w) {
        s->aoff[w] = d->agent_offsets[w];
        s->roff[w] = d->road_offsets[w];
        s->toff[w] = d->tri_offsets[w];
        s->soff[w] = d->spawn_offsets[w];
    }
    s->N = s->aoff[W];
    int P = s->roff[W], T = s->toff[W], E = s->soff[W];
    s->road_xy = (double *)malloc(sizeof(double) * 2 * (P + 1));
    s->road_type = (uint8_t *)malloc(P + 1);
    for (int i = 0; i < 2 * P; ++i) s->road_xy[i] = d->road_xy[i];
    for (int i = 0; i < P; ++i) s->road_type[i] = d->road_type[i];
    s->road_dir = (double *)malloc(sizeof(double) * 2 * (P + 1));
    for (int i = 0; i < 2 * P; ++i) s->road_dir[i] = d->road_dir ? d->road_dir[i] : 0.0;
    s->tri = (double *)malloc(sizeof(double) * 9 * (T + 1));
    s->tri_surf = (uint8_t *)malloc(T + 1);
    for (int i = 0; i < 9 * T; ++i) s->tri[i] = d->tri_verts[i];
    for (int i = 0; i < T; ++i) s->tri_surf[i] = d->tri_surface[i];
    s->film = (double *)malloc(sizeof(double) * (W + 1));
    s->pav = (int *)malloc(sizeof(int) * (W + 1));
    for (int w = 0; w < W; ++w) {
        s->film[w] = d->film_mm ? d->film_mm[w] : 0.0;
        s->pav[w] = d->pavement ? d->pavement[w] : 0;
    }
    s->mu = (double *)malloc(sizeof(double) * W * s->S);
    for (int w = 0; w < W; ++w)
        for (int j = 0; j < s->S; ++j) {
            double film = d->film_mm ? d->film_mm[w] : 0.0;
            int pav = d->pavement ? d->pavement[w] : 0;
            double mc = d->mu_class[(size_t)w * s->S + j];
            s->mu[(size_t)w * s->S + j] = film > 0.0 ? or_weather_mu(mc, film, pav) : mc;
        }
    s->spawn = (double *)malloc(sizeof(double) * 5 * (E + 1));
    for (int i = 0; i < 5 * E; ++i) s->spawn[i] = d->spawn[i];
    s->world_of = (int *)malloc(sizeof(int) * (s->N + 1));
    for (int w = 0; w < W; ++w)
        for (int i = s->aoff[w]; i < s->aoff[w + 1]; ++i) s->world_of[i] = w;
    s->f = (double *)calloc((size_t)OR_NF * (s->N + 1), sizeof(double));
    s->k = (int32_t *)calloc((size_t)OR_NK * (s->N + 1), sizeof(int32_t));

    const or_params *p = &s->p;
    s->Iw = p->wheel_inertia > 0 ? p->wheel_inertia
                                 : 0.5 * p->wheel_mass * p->wheel_radius * p->wheel_radius;
    s->ell = p->susp_rest + p->wheel_radius;
    or_circle_model(p, &s->cr, &s->cd);
    /* ride height: level chassis whose four springs each carry m g / 4 */
    s->z_ride = s->ell - p->mass * p->gravity / (4.0 * p->susp_k) - p->mount[0][2];
    for (int i = 0; i < s->N; ++i) spawn_agent(s, i);
    return s;
}

void or_destroy(or_sim *s) {
    if (!s) return;
    free(s->aoff); free(s->roff); free(s->toff); free(s->soff);
    free(s->road_xy); free(s->road_type); free(s->road_dir); free(s->film); free(s->pav); free(s->tri); free(s->tri_surf);
    free(s->tri_mu_scale);
    free(s->mu); free(s->spawn); free(s->world_of); free(s->f); free(s->k);
    free(s->sur);
    free(s);
}

int or_num_agents(const or_sim *s) { return s->N; }

void or_get_state(const or_sim *s, double *f, int32_t *k) {
    memcpy(f, s->f, sizeof(double) * OR_NF * s->N);
    memcpy(k, s->k, sizeof(int32_t) * OR_NK * s->N);
}
void or_set_state(or_sim *s, const double *f, const int32_t *k) {
    memcpy(s->f, f, sizeof(double) * OR_NF * s->N);
    memcpy(s->k, k, sizeof(int32_t) * OR_NK * s->N);
}
void or_get_mu(const or_sim *s, double *mu) {
    memcpy(mu, s->mu, sizeof(double) * s->W * s->S);
}

/* Teleport to a spawn entry (Sec. "Teleport-only reset"): the world's entry
 * table is rotated by an offset drawn from SplitMix64 keyed by (seed, world,
 * episode), so agents of one world reset together take distinct entries. */
static void spawn_agent(or_sim *s, int i) {
    int w = s->world_of[i];
    int j = i - s->aoff[w];
    int M = s->soff[w + 1] - s->soff[w];
    uint64_t e = (uint64_t)(uint32_t)K(s, OR_EPISODE, i);
    uint64_t key = s->seed ^ ((uint64_t)(uint32_t)w << 32) ^ e;
    int off = (int)(splitmix64(key) % (uint64_t)M);
    const double *sp = s->spawn + 5 * (size_t)(s->soff[w] + (j + off) % M);
    double yaw = sp[2];
    F(s, OR_PX, i) = sp[0];
    F(s, OR_PY, i) = sp[1];
    F(s, OR_PZ, i) = s->z_ride;
    F(s, OR_QW, i) = cos(0.5 * yaw);
    F(s, OR_QX, i) = 0.0;
    F(s, OR_QY, i) = 0.0;
    F(s, OR_QZ, i) = sin(0.5 * yaw);
    for (int c = OR_VX; c <= OR_MU; ++c) F(s, c, i) = 0.0;
    F(s, OR_GX, i) = sp[3];
    F(s, OR_GY, i) = sp[4];
    F(s, OR_SX, i) = sp[0];
    F(s, OR_SY, i) = sp[1];
    K(s, OR_ACTIVE, i) = 1;
    K(s, OR_EPSTEP, i) = 0;
    K(s, OR_SINCE, i) = 0;
}

/* Terminated agents leave the scene at x = 1000 m at rest (Sec. "Termination
 * and time-out") and take no further part until reset. */
static void park_agent(or_sim *s, int i) {
    F(s, OR_PX, i) = 1000.0;
    F(s, OR_PY, i) = 0.0;
    F(s, OR_PZ, i) = s->z_ride;
    F(s, OR_QW, i) = 1.0;
    F(s, OR_QX, i) = F(s, OR_QY, i) = F(s, OR_QZ, i) = 0.0;
    for (int c = OR_VX; c <= OR_MU; ++c) F(s, c, i) = 0.0;
    K(s, OR_ACTIVE, i) = 0;
}

void or_reset(or_sim *s, const uint8_t *mask) {
    for (int i = 0; i < s->N; ++i)
        if (mask[i]) {
            K(s, OR_EPISODE, i) += 1;
            spawn_agent(s, i);
        }
}

/* -------------------------------------------------------------- raycast */
/* Nearest hit of the wheel ray (mount point m, direction u, length ell)
 * against the ground plane z = 0 and every road triangle of the world
 * (two-sided Moller-Trumbore, closed barycentric bounds).  Hits whose
 * distance lies within 0.1 mm of the nearest are the same surface point:
 * among them a road triangle wins over the ground, the lowest index first. */
static int raycast(const or_sim *s, int w, const double *m, const double *u,
                   double *t_out, double *n_out, int *surf, int *tri_id) {
    const double ell = s->ell;
    double tmin = INFINITY;
    double tg = INFINITY;
    if (u[2] < 0.0) {
        double t = m[2] / (-u[2]);
        if (t >= 0.0 && t <= ell) { tg = t; tmin = t; }
    }
    int t0 = s->toff[w], t1 = s->toff[w + 1];
    double *ts = (double *)malloc(sizeof(double) * (t1 - t0 + 1));
    for (int k = t0; k < t1; ++k) {
        ts[k - t0] = INFINITY;
        const double *v = s->tri + 9 * (size_t)k;
        double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
        double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
        double pv[3]; cross3(u, e2, pv);
        double det = dot3(e1, pv);
        if (fabs(det) < 1e-12) continue;
        double inv = 1.0 / det;
        double tv[3] = {m[0] - v[0], m[1] - v[1], m[2] - v[2]};
        double bu = dot3(tv, pv) * inv;
        if (bu < 0.0 || bu > 1.0) continue;
        double qv[3]; cross3(tv, e1, qv);
        double bv = dot3(u, qv) * inv;
        if (bv < 0.0 || bu + bv > 1.0) continue;
        double t = dot3(e2, qv) * inv;
        if (t < 0.0 || t > ell) continue;
        ts[k - t0] = t;
        if (t < tmin) tmin = t;
    }
    int hit = 0;
    if (tmin < INFINITY) {
        hit = 1;
        int chosen = -1;
        for (int k = t0; k < t1; ++k)
            if (ts[k - t0] <= tmin + 1e-4) { chosen = k; break; }
        if (chosen >= 0) {
            const double *v = s->tri + 9 * (size_t)chosen;
            double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
            double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
            double nn[3]; cross3(e1, e2, nn);
            double L = sqrt(dot3(nn, nn));
            for (int c = 0; c < 3; ++c) nn[c] /= L;
            if (dot3(nn, u) > 0.0) for (int c = 0; c < 3; ++c) nn[c] = -nn[c];
            *t_out = ts[chosen - t0];
            n_out[0] = nn[0]; n_out[1] = nn[1]; n_out[2] = nn[2];
            *surf = s->tri_surf[chosen];
            *tri_id = chosen - t0;
        } else {
            *t_out = tg;
            n_out[0] = 0.0; n_out[1] = 0.0; n_out[2] = 1.0;
            *surf = 0;
            *tri_id = -1;
        }
    }
    free(ts);
    return hit;
}

static void agent_pose(const or_sim *s, int i, double *p, double *q, double R[3][3]) {
    p[0] = F(s, OR_PX, i); p[1] = F(s, OR_PY, i); p[2] = F(s, OR_PZ, i);
    q[0] = F(s, OR_QW, i); q[1] = F(s, OR_QX, i); q[2] = F(s, OR_QY, i); q[3] = F(s, OR_QZ, i);
    quat_to_R(q, R);
}

int or_raycast(const or_sim *s, int i, int wh, double *t, double *n, int *surf, int *tri) {
    double p[3], q[4], R[3][3];
    agent_pose(s, i, p, q, R);
    double rm[3], m[3], u[3];
    matvec(R, s->p.mount[wh], rm);
    for (int c = 0; c < 3; ++c) { m[c] = p[c] + rm[c]; u[c] = -R[c][2]; }
    return raycast(s, s->world_of[i], m, u, t, n, surf, tri);
}

/* ------------------------------------------------------- tire surrogate */
/* Inputs of the learned tire model for one wheel, each scaled to order one:
 * slip ratio, slip angle, load, friction, rim speed, camber, then the
 * longitudinal and lateral contact speeds, the wheel's steer angle, spring
 * compression and rate, drive and brake torque fractions, the slip vector
 * over the friction coefficient (slip ratio / mu, tan(slip angle) / mu)
 * shortened to length 2 if longer, and the yaw rate.  The outputs are forces
 * over mu F_z, so that pair is the scale on which they vary at any mu.
 * Rounded to float (the form in which both the logged training samples and
 * the inference inputs exist). */
static void sur_features(const or_sim *s, double Fz, double mu, double vx, double vy, double Om,
                         double td, double tb, double x, double xd, double delta, double gamma,
                         const double *om, float *f) {
    const or_params *p = &s->p;
    double D = fabs(vx) > p->v_eps ? fabs(vx) : p->v_eps;
    const double kap = (p->wheel_radius * Om - vx) / D;
    double sx = 0.0, sy = 0.0;
    if (mu > 0.0) {
        sx = kap / mu;
        sy = vy / D / mu;
        const double L = sqrt(sx * sx + sy * sy);
        if (L > 2.0) { sx *= 2.0 / L; sy *= 2.0 / L; }
    }
    double v[OR_SUR_IN] = {
        kap, atan(vy / D), Fz / 4000.0, mu, p->wheel_radius * Om / 30.0,
        gamma, vx / 30.0, vy / 5.0, delta, x / 0.2, xd / 2.0, td / p->tau_drive,
        tb / p->tau_brake_front, sx, sy, om[2] / 2.0};
    for (int k = 0; k < OR_SUR_IN; ++k) f[k] = (float)v[k];
}

static void sur_forward(const or_sim *s, const float *f, double *y);

/* ---------------------------------------------------------------- tire */
/* Linear-saturated tire inside the friction circle with an implicit wheel
 * spin update and a Coulomb brake, in closed form.  K = c_kappa Fz / D is
 * the longitudinal slip stiffness (per m/s of slip speed), D = max(|vx|,
 * v_eps).  The spin solve is implicit in the slip force; when the force
 * leaves the friction circle both components scale back onto it and the
 * spin integrates with the saturated force. */
void or_tire(const or_params *p, double h, double Fz, double mu, double vx,
             double vy, double omega, double tau_d, double tau_b, double *Fx,
             double *Fy, double *Mz, double *omega_new) {
    double rw = p->wheel_radius;
    double Iw = p->wheel_inertia > 0 ? p->wheel_inertia : 0.5 * p->wheel_mass * rw * rw;
    double D = fabs(vx) > p->v_eps ? fabs(vx) : p->v_eps;
    double Kx = p->c_kappa * Fz / D;
    double Fy0 = -p->c_alpha * Fz * vy / D;
    double a = h / Iw;
    double B = omega + a * (tau_d + rw * Kx * vx);
    double A = 1.0 + a * rw * rw * Kx;
    double bb = a * tau_b;
    double om;
    if (B > bb) om = (B - bb) / A;
    else if (B < -bb) om = (B + bb) / A;
    else om = 0.0;
    double Fx0 = Kx * (rw * om - vx);
    double lim = mu * Fz;
    if (Fx0 * Fx0 + Fy0 * Fy0 <= lim * lim) {
        *Fx = Fx0;
        *Fy = Fy0;
        *omega_new = om;
    } else {
        double sc = lim / sqrt(Fx0 * Fx0 + Fy0 * Fy0);
        *Fx = sc * Fx0;
        *Fy = sc * Fy0;
        double Bs = omega + a * (tau_d - rw * (*Fx));
        double mag = fabs(Bs) - bb;
        if (mag < 0.0) mag = 0.0;
        *omega_new = Bs > 0 ? mag : (Bs < 0 ? -mag : 0.0);
    }
    *Mz = -p->trail * (*Fy);
}

/* --------------------------------------------------------- circle model */
/* integer three-circle centres from the quantised pose (bit-exact contract) */
static void circle_centres_q(const or_sim *s, int i, int64_t C[3][2]) {
    int64_t X = Qp(F(s, OR_PX, i)), Y = Qp(F(s, OR_PY, i));
    int64_t qw = Qq(F(s, OR_QW, i)), qx = Qq(F(s, OR_QX, i));
    int64_t qy = Qq(F(s, OR_QY, i)), qz = Qq(F(s, OR_QZ, i));
    int64_t hx = ((int64_t)1 << 28) - 2 * (qy * qy + qz * qz);
    int64_t hy = 2 * (qx * qy + qw * qz);
    int64_t nh = (int64_t)isqrt_u64((uint64_t)(hx * hx + hy * hy));
    int64_t Qd = Qp(s->cd);
    int64_t ox = 0, oy = 0;
    if (nh > 0) { ox = Qd * hx / nh; oy = Qd * hy / nh; }
    for (int a = 0; a < 3; ++a) {
        C[a][0] = X + (a - 1) * ox;
        C[a][1] = Y + (a - 1) * oy;
    }
}

/* planar heading unit vector from the float pose, (1, 0) if degenerate */
static void heading_fp(const or_sim *s, int i, double *hx, double *hy) {
    double qw = F(s, OR_QW, i), qx = F(s, OR_QX, i), qy = F(s, OR_QY, i), qz = F(s, OR_QZ, i);
    double x = 1 - 2 * (qy * qy + qz * qz), y = 2 * (qx * qy + qw * qz);
    double L = sqrt(x * x + y * y);
    if (L < 1e-12) { *hx = 1.0; *hy = 0.0; return; }
    *hx = x / L;
    *hy = y / L;
}

/* All overlapping circle pairs of active agents i < j of world w, in (i, j)
 * order, packed as i | j << 8 | mask << 16 with mask bit 3a + b for circle
 * a of i (0 rear, 1 centre, 2 front) against circle b of j. */
int or_detect_pairs(const or_sim *s, int w, uint32_t *pairs, int cap) {
    int a0 = s->aoff[w], a1 = s->aoff[w + 1];
    int64_t R2 = 2 * Qp(s->cr);
    R2 = R2 * R2;
    int n = 0;
    for (int i = a0; i < a1; ++i) {
        if (!K(s, OR_ACTIVE, i)) continue;
        int64_t Ci[3][2];
        circle_centres_q(s, i, Ci);
        for (int j = i + 1; j < a1; ++j) {
            if (!K(s, OR_ACTIVE, j)) continue;
            int64_t Cj[3][2];
            circle_centres_q(s, j, Cj);
            uint32_t mask = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    int64_t dx = Ci[a][0] - Cj[b][0], dy = Ci[a][1] - Cj[b][1];
                    if (dx * dx + dy * dy < R2) mask |= 1u << (3 * a + b);
                }
            if (mask) {
                if (n < cap && pairs)
                    pairs[n] = (uint32_t)(i - a0) | ((uint32_t)(j - a0) << 8) | (mask << 16);
                ++n;
            }
        }
    }
    return n;
}

/* ------------------------------------------------------------ substep */
typedef struct {
    double n[2], pc[3], ri[3], rj[3], keff, bias, lam;
    int i, j;
} contact_t;

static void inv_inertia_apply(const or_sim *s, double R[3][3], const double *x, double *y) {
    double b[3], c[3];
    matTvec(R, x, b);
    for (int k = 0; k < 3; ++k) c[k] = b[k] / s->p.inertia[k];
    matvec(R, c, y);
}

static void substep_world(or_sim *s, int w, const float *actions, double h,
                          uint8_t *nan_act, uint8_t *collided, int last,
                          uint32_t *rec, int32_t *rec_cnt, int rec_cap) {
    const or_params *p = &s->p;
    int a0 = s->aoff[w], a1 = s->aoff[w + 1], A = a1 - a0;
    double *vs = (double *)malloc(sizeof(double) * 6 * (A + 1));  /* v*, w* */
    double *Rs = (double *)malloc(sizeof(double) * 9 * (A + 1));
    for (int i = a0; i < a1; ++i) {
        int li = i - a0;
        if (!K(s, OR_ACTIVE, i)) continue;
        double pos[3], q[4], R[3][3];
        agent_pose(s, i, pos, q, R);
        memcpy(Rs + 9 * li, R, sizeof(double) * 9);
        double v[3] = {F(s, OR_VX, i), F(s, OR_VY, i), F(s, OR_VZ, i)};
        double om[3] = {F(s, OR_WX, i), F(s, OR_WY, i), F(s, OR_WZ, i)};
        /* action decode (Sec. "Action Space Details"): positive longitudinal
         * command drives the front wheels, negative brakes all four;
         * commands are clamped to range, NaN counts as zero */
        double al = actions[2 * i], st = actions[2 * i + 1];
        if (isnan(al)) { al = 0.0; nan_act[li] = 1; }
        if (isnan(st)) { st = 0.0; nan_act[li] = 1; }
        if (al > 1.0) al = 1.0;
        if (al < -1.0) al = -1.0;
        double tau_d = al > 0 ? al * p->tau_drive : 0.0;
        double brk = al < 0 ? -al : 0.0;
        /* steering PD (Eq. steer PD), implicit in the steering rate; the
         * torque clamp falls back to the explicit rate update */
        double th = F(s, OR_TH, i), thd = F(s, OR_THD, i);
        double tgt = st;
        if (tgt > p->steer_max) tgt = p->steer_max;
        if (tgt < -p->steer_max) tgt = -p->steer_max;
        double g = h / p->steer_inertia;
        double thd1 = (thd + g * p->steer_kp * (tgt - th)) / (1.0 + g * (p->steer_kd + h * p->steer_kp));
        double tau = p->steer_kp * (tgt - th - h * thd1) - p->steer_kd * thd1;
        if (fabs(tau) > p->steer_tau_max) {
            tau = tau > 0 ? p->steer_tau_max : -p->steer_tau_max;
            thd1 = thd + g * tau;
        }
        double th1 = th + h * thd1;
        F(s, OR_TH, i) = th1;
        F(s, OR_THD, i) = thd1;

        double Fsum[3] = {0, 0, -p->mass * p->gravity};
        double Tsum[3] = {0, 0, -p->yaw_damping * om[2]};
        double mu_acc = 0.0;
        for (int wh = 0; wh < NW; ++wh) {
            double rm[3], m[3], u[3];
            matvec(R, p->mount[wh], rm);
            for (int c = 0; c < 3; ++c) { m[c] = pos[c] + rm[c]; u[c] = -R[c][2]; }
            double t, n[3];
            int surf, tri;
            int hit = raycast(s, w, m, u, &t, n, &surf, &tri);
            double Omega = F(s, OR_OM0 + wh, i);
            double td = wh < 2 ? tau_d : 0.0;
            double tb = brk * (wh < 2 ? p->tau_brake_front : p->tau_brake_rear);
            double Fz = 0.0, Fx = 0.0, Fy = 0.0, Mz = 0.0, om_new;
            double rc[3] = {0, 0, 0}, ex[3] = {0, 0, 0}, ey[3] = {0, 0, 0};
            double mu = 0.0;
            int tire = 0;
            if (hit) {
                mu = s->mu[(size_t)w * s->S + surf];
                /* spatially varying friction: the hit triangle's own factor */
                if (tri >= 0 && s->tri_mu_scale) mu *= s->tri_mu_scale[s->toff[w] + tri];
                mu_acc += mu;
                /* suspension: massless spring-damper along the ray */
                double x = s->ell - t;
                double vm[3], wr[3];
                cross3(om, rm, wr);
                for (int c = 0; c < 3; ++c) vm[c] = v[c] + wr[c];
                double xd = -dot3(n, vm) / (-dot3(n, u));
                Fz = p->susp_k * x + p->susp_c * xd;
                if (Fz < 0.0) Fz = 0.0;
                for (int c = 0; c < 3; ++c) rc[c] = rm[c] + t * u[c];
                /* tire frame: wheel heading projected onto the contact plane */
                double dl = wh < 2 ? th1 : 0.0;
                double hb[3] = {cos(dl), sin(dl), 0.0}, hw[3];
                matvec(R, hb, hw);
                double hn = dot3(hw, n);
                for (int c = 0; c < 3; ++c) ex[c] = hw[c] - hn * n[c];
                double L = sqrt(dot3(ex, ex));
                if (L > 1e-9) {
                    for (int c = 0; c < 3; ++c) ex[c] /= L;
                    cross3(n, ex, ey);
                    double vc[3], wc[3];
                    cross3(om, rc, wc);
                    for (int c = 0; c < 3; ++c) vc[c] = v[c] + wc[c];
                    double vx = dot3(vc, ex), vy = dot3(vc, ey);
                    int used = 0;
                    float feat[OR_SUR_IN];
                    int in_domain = Fz > 0.0 && fabs(vx) >= 3.0;
                    if (in_domain && (s->sur_on || s->sample_rec)) {
                        double ab[3] = {-sin(dl), cos(dl), 0.0}, axle[3];
                        matvec(R, ab, axle);
                        double g = dot3(axle, n);
                        if (g > 1.0) g = 1.0;
                        if (g < -1.0) g = -1.0;
                        sur_features(s, Fz, mu, vx, vy, Omega, td, tb, x, xd, dl, asin(g), om, feat);
                    }
                    if (in_domain && s->sur_on) {
                        int inside = 1;
                        for (int q = 0; q < OR_SUR_IN; ++q)
                            if (!(feat[q] >= s->env_lo[q] && feat[q] <= s->env_hi[q])) inside = 0;
                        if (inside) {
                            double y[3];
                            sur_forward(s, feat, y);
                            double lim = mu * Fz;
                            double Fxs = lim * y[0], Fys = lim * y[1];
                            double kap = (p->wheel_radius * Omega - vx) / fabs(vx);
                            /* physical residual checks: inside the friction
                             * circle (2 % slack) and force along the slip */
                            if (sqrt(Fxs * Fxs + Fys * Fys) <= 1.02 * lim &&
                                (fabs(kap) <= 0.02 || ((Fxs > 0.0) == (kap > 0.0)))) {
                                double a = h / s->Iw, Bs = Omega + a * (td - p->wheel_radius * Fxs);
                                double mag = fabs(Bs) - a * tb;
                                if (mag < 0.0) mag = 0.0;
                                Fx = Fxs;
                                Fy = Fys;
                                Mz = p->trail * lim * y[2];
                                om_new = Bs > 0 ? mag : (Bs < 0 ? -mag : 0.0);
                                used = 1;
                            }
                        }
                    }
                    if (!used) or_tire(p, h, Fz, mu, vx, vy, Omega, td, tb, &Fx, &Fy, &Mz, &om_new);
                    if (s->sur_on && in_domain) {
                        /* worlds run on several threads */
                        if (used) {
#pragma omp atomic
                            s->sur_used++;
                        } else {
#pragma omp atomic
                            s->sur_fallback++;
                        }
                    }
                    if (s->sample_rec && last) {
                        float *r = s->sample_rec + ((size_t)i * NW + wh) * OR_SAMPLE;
                        for (int q = 0; q < OR_SAMPLE; ++q) r[q] = 0.0f;
                        if (in_domain) {
                            double Fxp, Fyp, Mzp, omp, lim = mu * Fz;
                            or_tire(p, h, Fz, mu, vx, vy, Omega, td, tb, &Fxp, &Fyp, &Mzp, &omp);
                            for (int q = 0; q < OR_SUR_IN; ++q) r[q] = feat[q];
                            r[OR_SUR_IN] = (float)(lim > 0 ? Fxp / lim : 0.0);
                            r[OR_SUR_IN + 1] = (float)(lim > 0 ? Fyp / lim : 0.0);
                            r[OR_SUR_IN + 2] = (float)(lim > 0 ? Mzp / (p->trail * lim) : 0.0);
                            r[OR_SUR_IN + 3] = 1.0f;
                        }
                    }
                    tire = 1;
                }
                if (!tire) or_tire(p, h, 0.0, mu, 0.0, 0.0, Omega, td, tb, &Fx, &Fy, &Mz, &om_new);
                double f[3], tq[3];
                for (int c = 0; c < 3; ++c) f[c] = Fz * n[c] + Fx * ex[c] + Fy * ey[c];
                cross3(rc, f, tq);
                for (int c = 0; c < 3; ++c) {
                    Fsum[c] += f[c];
                    Tsum[c] += tq[c] + Mz * n[c];
                }
            } else {
                /* airborne wheel: no load, free spin under drive and brake */
                or_tire(p, h, 0.0, 0.0, 0.0, 0.0, Omega, td, tb, &Fx, &Fy, &Mz, &om_new);
            }
            F(s, OR_OM0 + wh, i) = om_new;
        }
        if (last) F(s, OR_MU, i) = mu_acc / NW;
        /* chassis: semi-implicit Euler, gyroscopic term explicit in body frame */
        double *out = vs + 6 * li;
        for (int c = 0; c < 3; ++c) out[c] = v[c] + h * Fsum[c] / p->mass;
        double wb[3], Tb[3], Lb[3], gy[3];
        matTvec(R, om, wb);
        matTvec(R, Tsum, Tb);
        for (int c = 0; c < 3; ++c) Lb[c] = p->inertia[c] * wb[c];
        cross3(wb, Lb, gy);
        double wb1[3];
        for (int c = 0; c < 3; ++c) wb1[c] = wb[c] + h * (Tb[c] - gy[c]) / p->inertia[c];
        matvec(R, wb1, out + 3);
    }

    /* vehicle-vehicle contact on the substep's input poses */
    int cap = A * (A - 1) / 2 + 1;
    uint32_t *pairs = (uint32_t *)malloc(sizeof(uint32_t) * cap);
    int np = or_detect_pairs(s, w, pairs, cap);
    if (rec) {
        for (int k = 0; k < np && k < rec_cap; ++k) rec[k] = pairs[k];
        *rec_cnt = np;
    }
    contact_t *cs = (contact_t *)malloc(sizeof(contact_t) * (9 * np + 1));
    int *ncon = (int *)calloc(A + 1, sizeof(int));
    int nc = 0;
    for (int k = 0; k < np; ++k) {
        int li = pairs[k] & 0xFF, lj = (pairs[k] >> 8) & 0xFF;
        uint32_t mask = pairs[k] >> 16;
        collided[li] = 1;
        collided[lj] = 1;
        int i = a0 + li, j = a0 + lj;
        double hix, hiy, hjx, hjy;
        heading_fp(s, i, &hix, &hiy);
        heading_fp(s, j, &hjx, &hjy);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                if (!(mask & (1u << (3 * a + b)))) continue;
                double cix = F(s, OR_PX, i) + (a - 1) * s->cd * hix;
                double ciy = F(s, OR_PY, i) + (a - 1) * s->cd * hiy;
                double cjx = F(s, OR_PX, j) + (b - 1) * s->cd * hjx;
                double cjy = F(s, OR_PY, j) + (b - 1) * s->cd * hjy;
                double dx = cjx - cix, dy = cjy - ciy;
                double L = sqrt(dx * dx + dy * dy);
                contact_t *c = &cs[nc++];
                if (L > 0) { c->n[0] = dx / L; c->n[1] = dy / L; }
                else { c->n[0] = 1.0; c->n[1] = 0.0; }
                double phi = 2.0 * s->cr - L;
                c->pc[0] = 0.5 * (cix + cjx);
                c->pc[1] = 0.5 * (ciy + cjy);
                c->pc[2] = 0.5 * (F(s, OR_PZ, i) + F(s, OR_PZ, j));
                c->ri[0] = c->pc[0] - F(s, OR_PX, i);
                c->ri[1] = c->pc[1] - F(s, OR_PY, i);
                c->ri[2] = c->pc[2] - F(s, OR_PZ, i);
                c->rj[0] = c->pc[0] - F(s, OR_PX, j);
                c->rj[1] = c->pc[1] - F(s, OR_PY, j);
                c->rj[2] = c->pc[2] - F(s, OR_PZ, j);
                c->i = li;
                c->j = lj;
                c->lam = 0.0;
                double pen = phi - p->slop;
                c->bias = pen > 0 ? (p->baumgarte / h) * pen : 0.0;
                ncon[li]++;
                ncon[lj]++;
            }
    }
    for (int k = 0; k < nc; ++k) {
        contact_t *c = &cs[k];
        double n3[3] = {c->n[0], c->n[1], 0.0}, x[3], y[3];
        double keff = 2.0 / p->mass;
        cross3(c->ri, n3, x);
        inv_inertia_apply(s, (double(*)[3])(Rs + 9 * c->i), x, y);
        keff += dot3(x, y);
        cross3(c->rj, n3, x);
        inv_inertia_apply(s, (double(*)[3])(Rs + 9 * c->j), x, y);
        keff += dot3(x, y);
        c->keff = keff;
    }
    /* Jacobi: every contact sees the velocities of the previous sweep */
    double *dl = (double *)malloc(sizeof(double) * (nc + 1));
    for (int it = 0; it < p->jacobi_iters && nc > 0; ++it) {
        for (int k = 0; k < nc; ++k) {
            contact_t *c = &cs[k];
            const double *vi = vs + 6 * c->i, *vj = vs + 6 * c->j;
            double wi[3], wj[3];
            cross3(vi + 3, c->ri, wi);
            cross3(vj + 3, c->rj, wj);
            double vn = 0.0;
            for (int d = 0; d < 2; ++d) vn += ((vj[d] + wj[d]) - (vi[d] + wi[d])) * c->n[d];
            int nmax = ncon[c->i] > ncon[c->j] ? ncon[c->i] : ncon[c->j];
            double delta = (1.0 / nmax) * (-vn + c->bias) / c->keff;
            double lam1 = c->lam + delta;
            if (lam1 < 0.0) lam1 = 0.0;
            dl[k] = lam1 - c->lam;
            c->lam = lam1;
        }
        for (int k = 0; k < nc; ++k) {
            contact_t *c = &cs[k];
            double J[3] = {dl[k] * c->n[0], dl[k] * c->n[1], 0.0};
            for (int side = 0; side < 2; ++side) {
                int b = side ? c->j : c->i;
                double sg = side ? 1.0 : -1.0;
                double Jb[3] = {sg * J[0], sg * J[1], 0.0}, x[3], y[3];
                double *vb = vs + 6 * b;
                for (int d = 0; d < 3; ++d) vb[d] += Jb[d] / p->mass;
                cross3(side ? c->rj : c->ri, Jb, x);
                inv_inertia_apply(s, (double(*)[3])(Rs + 9 * b), x, y);
                for (int d = 0; d < 3; ++d) vb[3 + d] += y[d];
            }
        }
    }
    /* positions and orientations */
    for (int i = a0; i < a1; ++i) {
        if (!K(s, OR_ACTIVE, i)) continue;
        const double *o = vs + 6 * (i - a0);
        F(s, OR_VX, i) = o[0]; F(s, OR_VY, i) = o[1]; F(s, OR_VZ, i) = o[2];
        F(s, OR_WX, i) = o[3]; F(s, OR_WY, i) = o[4]; F(s, OR_WZ, i) = o[5];
        F(s, OR_PX, i) += h * o[0];
        F(s, OR_PY, i) += h * o[1];
        F(s, OR_PZ, i) += h * o[2];
        double qw = F(s, OR_QW, i), qx = F(s, OR_QX, i), qy = F(s, OR_QY, i), qz = F(s, OR_QZ, i);
        double wx = o[3], wy = o[4], wz = o[5];
        /* dq = 1/2 (0, w) * q */
        double dw = -(wx * qx + wy * qy + wz * qz);
        double dx = wx * qw + (wy * qz - wz * qy);
        double dy = wy * qw + (wz * qx - wx * qz);
        double dz = wz * qw + (wx * qy - wy * qx);
        qw += 0.5 * h * dw; qx += 0.5 * h * dx; qy += 0.5 * h * dy; qz += 0.5 * h * dz;
        double L = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        F(s, OR_QW, i) = qw / L; F(s, OR_QX, i) = qx / L;
        F(s, OR_QY, i) = qy / L; F(s, OR_QZ, i) = qz / L;
    }
    free(dl); free(cs); free(ncon); free(pairs); free(vs); free(Rs);
}

/* ----------------------------------------------------------- events */
/* Sparse events on the quantised final pose (Sec. "Sparse event rewards"):
 * goal within 3 m, crash on falling below the ground, drifting more than
 * 100 m from the start or tilting (body up-axis z below 0.15), collision
 * after the 24-step spawn warm-up, plus a numeric-fault crash. */
static uint32_t agent_events(const or_sim *s, int i, int collided) {
    uint32_t ev = 0;
    for (int c = 0; c < OR_NDYN; ++c)
        if (!isfinite(F(s, c, i))) return OR_EV_CRASH | OR_EV_NUMERIC;
    int64_t X = Qp(F(s, OR_PX, i)), Y = Qp(F(s, OR_PY, i)), Z = Qp(F(s, OR_PZ, i));
    int64_t gx = X - Qp(F(s, OR_GX, i)), gy = Y - Qp(F(s, OR_GY, i));
    if (gx * gx + gy * gy <= (int64_t)3072 * 3072) ev |= OR_EV_GOAL;
    if (collided && K(s, OR_SINCE, i) >= s->p.collision_warmup) ev |= OR_EV_COLLISION;
    int64_t sx = X - Qp(F(s, OR_SX, i)), sy = Y - Qp(F(s, OR_SY, i));
    int crash = 0;
    if (sx * sx + sy * sy > (int64_t)102400 * 102400) crash = 1;
    if (Z < 0) crash = 1;
    int64_t qx = Qq(F(s, OR_QX, i)), qy = Qq(F(s, OR_QY, i));
    if (((int64_t)1 << 28) - 2 * (qx * qx + qy * qy) < 40265318) crash = 1;
    if (crash) ev |= OR_EV_CRASH;
    return ev;
}

void or_events(const or_sim *s, const uint8_t *collided, uint8_t *events) {
    for (int i = 0; i < s->N; ++i)
        events[i] = K(s, OR_ACTIVE, i) ? (uint8_t)agent_events(s, i, collided[i]) : 0;
}

/* ------------------------------------------------- kinematic bicycle */
/* The lightweight backend of Sec. "Vehicle Dynamics Ablation": the same
 * actions drive a kinematic single-track ("bicycle") model, advanced once
 * per control tick by forward Euler, without suspension, tires or contact
 * forces.  Its state (x, y, yaw psi, speed v >= 0) lives in the shared
 * state: position at ride height, yaw-only orientation, planar velocity
 * along the direction of travel psi + beta, yaw rate, wheels rolling at
 * v / r_w, steering angle equal to the clamped command.  With l_f, l_r the
 * axle distances from the centre of mass, the slip angle at the centre of
 * mass is beta = atan(l_r / (l_f + l_r) tan delta) and the yaw rate
 * v sin(beta) / l_r.  A positive command gives the front wheels' drive
 * force 2 tau_drive a / r_w, a negative one the four brakes' force
 * 2 (tau_brake_front + tau_brake_rear) |a| / r_w (divided by the mass);
 * braking stops the vehicle at v = 0, it never reverses.  No wheel touches
 * a surface, so the friction seen is 0. */
static void bicycle_world(or_sim *s, int w, const float *actions, double dt, uint8_t *nan_act) {
    const or_params *p = &s->p;
    const int a0 = s->aoff[w], a1 = s->aoff[w + 1];
    const double lf = p->mount[0][0], lr = -p->mount[2][0];
    for (int i = a0; i < a1; ++i) {
        const int li = i - a0;
        if (!K(s, OR_ACTIVE, i)) continue;
        double al = actions[2 * i], st = actions[2 * i + 1];
        if (isnan(al)) { al = 0.0; nan_act[li] = 1; }
        if (isnan(st)) { st = 0.0; nan_act[li] = 1; }
        if (al > 1.0) al = 1.0;
        if (al < -1.0) al = -1.0;
        double delta = st;
        if (delta > p->steer_max) delta = p->steer_max;
        if (delta < -p->steer_max) delta = -p->steer_max;
        const double qw = F(s, OR_QW, i), qx = F(s, OR_QX, i), qy = F(s, OR_QY, i), qz = F(s, OR_QZ, i);
        const double psi = atan2(2.0 * (qw * qz + qx * qy), 1.0 - 2.0 * (qy * qy + qz * qz));
        const double v = hypot(F(s, OR_VX, i), F(s, OR_VY, i));
        const double beta = atan(lr / (lf + lr) * tan(delta));
        double acc = 0.0;
        if (al > 0.0) acc = 2.0 * p->tau_drive * al / (p->wheel_radius * p->mass);
        else if (al < 0.0) acc = -2.0 * (p->tau_brake_front + p->tau_brake_rear) * (-al) / (p->wheel_radius * p->mass);
        const double x1 = F(s, OR_PX, i) + v * cos(psi + beta) * dt;
        const double y1 = F(s, OR_PY, i) + v * sin(psi + beta) * dt;
        const double psi1 = psi + v * sin(beta) / lr * dt;
        double v1 = v + acc * dt;
        if (v1 < 0.0) v1 = 0.0;
        F(s, OR_PX, i) = x1;
        F(s, OR_PY, i) = y1;
        F(s, OR_PZ, i) = s->z_ride;
        F(s, OR_QW, i) = cos(0.5 * psi1);
        F(s, OR_QX, i) = 0.0;
        F(s, OR_QY, i) = 0.0;
        F(s, OR_QZ, i) = sin(0.5 * psi1);
        F(s, OR_VX, i) = v1 * cos(psi1 + beta);
        F(s, OR_VY, i) = v1 * sin(psi1 + beta);
        F(s, OR_VZ, i) = 0.0;
        F(s, OR_WX, i) = 0.0;
        F(s, OR_WY, i) = 0.0;
        F(s, OR_WZ, i) = v1 * sin(beta) / lr;
        for (int wh = 0; wh < NW; ++wh) F(s, OR_OM0 + wh, i) = v1 / p->wheel_radius;
        F(s, OR_TH, i) = delta;
        F(s, OR_THD, i) = 0.0;
        F(s, OR_MU, i) = 0.0;
    }
}

void or_set_dynamics(or_sim *s, int mode) { s->dynamics = mode == OR_DYN_BICYCLE ? OR_DYN_BICYCLE : OR_DYN_PHYSICS; }

int or_set_tri_friction(or_sim *s, const float *scale) {
    const int T = s->toff[s->W];
    if (!scale) {
        free(s->tri_mu_scale);
        s->tri_mu_scale = NULL;
        return 0;
    }
    for (int k = 0; k < T; ++k)
        if (!(scale[k] >= 0.0f) || !isfinite(scale[k])) return -1;
    if (!s->tri_mu_scale) s->tri_mu_scale = (double *)malloc(sizeof(double) * (T + 1));
    for (int k = 0; k < T; ++k) s->tri_mu_scale[k] = scale[k];
    return 0;
}

/* ------------------------------------------------- shaping rewards */
/* Appendix "Reward Design Details": six dense terms at every active step
 * and the lane-forbidden event.  Readings: the road context of both is the
 * observation's 64 nearest road points; every road point stands for the
 * 0.5 m segment of its polyline centred on it along its direction; the
 * decisions (which point is nearest, which side, off-road, idle, which
 * edges lie ahead, overlap) are integer predicates on quantised values
 * (positions 2^-10 m, directions and headings 2^-14). */
void or_set_shaping(or_sim *s, int on) { s->shaping = on != 0; }

static int64_t sat_key(int64_t d2);
static double ttc_pair(const or_sim *s, int i, int j);

/* circle of quantised centre (cx, cy) and radius r against the segment of
 * global road point q: exact squared distance from the centre to the
 * segment below r^2 */
static int circle_hits_segment(const or_sim *s, int64_t cx, int64_t cy, int q) {
    const int64_t px = Qp(s->road_xy[2 * q]), py = Qp(s->road_xy[2 * q + 1]);
    const int64_t hx = Qp(0.25 * s->road_dir[2 * q]), hy = Qp(0.25 * s->road_dir[2 * q + 1]);
    const int64_t ax = px - hx, ay = py - hy, vx = 2 * hx, vy = 2 * hy;
    const int64_t wx = cx - ax, wy = cy - ay;
    if (wx > 4096 || wx < -4096 || wy > 4096 || wy < -4096) return 0;   /* farther than 4 m: no overlap */
    const int64_t R = Qp(s->cr), R2 = R * R;
    const int64_t len2 = vx * vx + vy * vy, t = wx * vx + wy * vy;
    if (len2 == 0 || t <= 0) return wx * wx + wy * wy < R2;
    if (t >= len2) {
        const int64_t ex = wx - vx, ey = wy - vy;
        return ex * ex + ey * ey < R2;
    }
    return (wx * wx + wy * wy) * len2 - t * t < R2 * len2;
}

static int is_edge(int type) { return type == 15 || type == 16; }
static int is_lane(int type) { return type == 1 || type == 2; }

int or_lane_forbidden(const or_sim *s, int i) {
    int32_t idx[OR_ROAD_K];
    or_knn_road(s, i, idx);
    int64_t C[3][2];
    circle_centres_q(s, i, C);
    const int r0 = s->roff[s->world_of[i]];
    for (int k = 0; k < OR_ROAD_K; ++k) {
        if (idx[k] < 0) break;
        const int q = r0 + idx[k];
        if (!is_edge(s->road_type[q])) continue;
        for (int a = 0; a < 3; ++a)
            if (circle_hits_segment(s, C[a][0], C[a][1], q)) return 1;
    }
    return 0;
}

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

void or_shaping_terms(const or_sim *s, int i, double dx, double dy, double *terms) {
    const or_params *p = &s->p;
    for (int k = 0; k < 6; ++k) terms[k] = 0.0;
    const int w = s->world_of[i], r0 = s->roff[w];
    int32_t idx[OR_ROAD_K];
    or_knn_road(s, i, idx);
    const double px = F(s, OR_PX, i), py = F(s, OR_PY, i);
    const int64_t X = Qp(px), Y = Qp(py);
    double hx, hy;
    heading_fp(s, i, &hx, &hy);
    /* the nearest driving-lane point (types 1-2) among the 64 */
    int best = -1;
    int64_t bkey = 0;
    for (int k = 0; k < OR_ROAD_K; ++k) {
        if (idx[k] < 0) break;
        const int q = r0 + idx[k];
        if (!is_lane(s->road_type[q])) continue;
        const int64_t ex = Qp(s->road_xy[2 * q]) - X, ey = Qp(s->road_xy[2 * q + 1]) - Y;
        const int64_t key = sat_key(ex * ex + ey * ey);
        if (best < 0 || key < bkey) { best = q; bkey = key; }   /* index order: ties keep the lower */
    }
    int off = 1;
    if (best >= 0) {
        /* lane tangent oriented toward the goal (integer sign; 0 keeps it) */
        double tx = s->road_dir[2 * best], ty = s->road_dir[2 * best + 1];
        const int64_t gdx = Qp(F(s, OR_GX, i)) - X, gdy = Qp(F(s, OR_GY, i)) - Y;
        if (Qq(tx) * gdx + Qq(ty) * gdy < 0) { tx = -tx; ty = -ty; }
        /* route progress: displacement along the tangent, clamped to +-2 m */
        terms[0] = 2.0 * clampd(dx * tx + dy * ty, -2.0, 2.0);
        /* lane keeping: lateral offset and heading alignment */
        const double qx = s->road_xy[2 * best], qy = s->road_xy[2 * best + 1];
        const double lat = (px - qx) * (-ty) + (py - qy) * tx;
        const double align = hx * tx + hy * ty;
        terms[1] = 0.08 * exp(-(lat / 1.75) * (lat / 1.75)) * (0.2 + 0.8 * (align > 0.0 ? align : 0.0));
        /* off the road: lateral offset beyond 3.25 m or the lane point
         * farther than 6 m (integers: lateral in 2^-24 m) */
        const int64_t ox = X - Qp(qx), oy = Y - Qp(qy);
        int64_t latq = ox * (-Qq(ty)) + oy * Qq(tx);
        if (latq < 0) latq = -latq;
        off = latq > (int64_t)(3.25 * 16777216.0) || bkey > (int64_t)6144 * 6144;
    }
    if (off) terms[2] = -0.5;
    /* idle: speed below 1 m/s (quantised velocity) */
    {
        const int64_t vx = Qp(F(s, OR_VX, i)), vy = Qp(F(s, OR_VY, i));
        if (vx * vx + vy * vy < (int64_t)1024 * 1024) terms[3] = -0.05;
    }
    /* inter-vehicle TTC: the smallest over the observation's neighbours */
    {
        int32_t nidx[OR_NEIGH_K];
        or_knn_neigh(s, i, nidx);
        double tau = 10.0;
        const int a0 = s->aoff[w];
        for (int k = 0; k < OR_NEIGH_K; ++k) {
            if (nidx[k] < 0) break;
            const int j = a0 + nidx[k];
            const double bx = hx * (F(s, OR_PX, j) - px) + hy * (F(s, OR_PY, j) - py);
            const double t = bx < 0.0 ? 10.0 : ttc_pair(s, i, j);
            if (t < tau) tau = t;
        }
        const double pen = 0.10 / (tau > 0.5 ? tau : 0.5);
        terms[4] = -(pen < 0.35 ? pen : 0.35);
    }
    /* road-edge TTC: edge points ahead in the vehicle's corridor (|lateral|
     * <= W / 2 + r), reached by the front circle at the forward speed; the
     * side decisions use the planar heading of the quantised quaternion
     * (unnormalised, exact integers, as the circle model does) */
    {
        const double vf = hx * F(s, OR_VX, i) + hy * F(s, OR_VY, i);
        const int64_t qw = Qq(F(s, OR_QW, i)), qx = Qq(F(s, OR_QX, i));
        const int64_t qy = Qq(F(s, OR_QY, i)), qz = Qq(F(s, OR_QZ, i));
        const int64_t ihx = ((int64_t)1 << 28) - 2 * (qy * qy + qz * qz), ihy = 2 * (qx * qy + qw * qz);
        const int64_t nh = (int64_t)isqrt_u64((uint64_t)(ihx * ihx + ihy * ihy));
        const int64_t half = (int64_t)nearbyint((0.5 * p->width + s->cr) * 1024.0);
        double tau = INFINITY;
        for (int k = 0; k < OR_ROAD_K && vf > 0.0; ++k) {
            if (idx[k] < 0) break;
            const int q = r0 + idx[k];
            if (!is_edge(s->road_type[q])) continue;
            const int64_t ex = Qp(s->road_xy[2 * q]) - X, ey = Qp(s->road_xy[2 * q + 1]) - Y;
            if (ex > (1 << 20) || ex < -(1 << 20) || ey > (1 << 20) || ey < -(1 << 20)) continue;
            const int64_t along = ex * ihx + ey * ihy, side = -ex * ihy + ey * ihx;
            if (along <= 0 || side > half * nh || side < -half * nh) continue;
            const double xb = hx * (s->road_xy[2 * q] - px) + hy * (s->road_xy[2 * q + 1] - py);
            const double gap = xb - (s->cd + s->cr);
            const double t = (gap > 0.0 ? gap : 0.0) / vf;
            if (t < tau) tau = t;
        }
        if (tau < INFINITY) {
            const double pen = 0.07 / (tau > 0.5 ? tau : 0.5);
            terms[5] = -(pen < 0.40 ? pen : 0.40);
        }
    }
}

void or_step(or_sim *s, const float *actions, double dt, int S, float *reward,
             uint8_t *done, uint8_t *events, uint32_t *pair_rec, int32_t *pair_cnt,
             int pair_cap) {
    double h = dt / S;
    const or_params *p = &s->p;
    int W = s->W;
    /* a wheel without a tire frame in the last substep records nothing */
    if (s->sample_rec) memset(s->sample_rec, 0, sizeof(float) * (size_t)s->N * NW * OR_SAMPLE);
#pragma omp parallel for schedule(dynamic, 1)
    for (int w = 0; w < W; ++w) {
        int a0 = s->aoff[w], a1 = s->aoff[w + 1], A = a1 - a0;
        uint8_t *nan_act = (uint8_t *)calloc(A + 1, 1);
        uint8_t *coll = (uint8_t *)calloc(A + 1, 1);
        uint8_t *was_active = (uint8_t *)calloc(A + 1, 1);
        uint8_t *forbid = (uint8_t *)calloc(A + 1, 1);
        double *p0 = (double *)calloc(2 * (A + 1), sizeof(double));
        double *sparse = (double *)calloc(A + 1, sizeof(double));
        uint8_t *carry = (uint8_t *)calloc(A + 1, 1);
        for (int i = a0; i < a1; ++i) {
            was_active[i - a0] = (uint8_t)K(s, OR_ACTIVE, i);
            /* lane-forbidden is decided on the control step's input pose */
            if (s->shaping && was_active[i - a0]) forbid[i - a0] = (uint8_t)or_lane_forbidden(s, i);
            p0[2 * (i - a0)] = F(s, OR_PX, i);
            p0[2 * (i - a0) + 1] = F(s, OR_PY, i);
        }
        if (s->dynamics == OR_DYN_BICYCLE) {
            /* one update per control tick; collisions from the circle pairs
             * of the tick's input poses (as the articulated step takes them
             * on each substep's input poses) */
            const int cap = A * (A - 1) / 2 + 1;
            uint32_t *pairs = (uint32_t *)malloc(sizeof(uint32_t) * cap);
            const int np = or_detect_pairs(s, w, pairs, cap);
            for (int k = 0; k < np; ++k) {
                coll[pairs[k] & 0xFF] = 1;
                coll[(pairs[k] >> 8) & 0xFF] = 1;
            }
            if (pair_rec) {
                for (int k = 0; k < np && k < pair_cap; ++k) pair_rec[(size_t)w * pair_cap + k] = pairs[k];
                pair_cnt[w] = np;
            }
            free(pairs);
            bicycle_world(s, w, actions, dt, nan_act);
        } else {
            for (int sub = 0; sub < S; ++sub) {
                uint32_t *rec = pair_rec ? pair_rec + ((size_t)sub * W + w) * pair_cap : NULL;
                int32_t *rc = pair_cnt ? pair_cnt + (size_t)sub * W + w : NULL;
                substep_world(s, w, actions, h, nan_act, coll, sub == S - 1, rec, rc, pair_cap);
            }
        }
        for (int i = a0; i < a1; ++i) {
            int li = i - a0;
            if (!was_active[li]) {
                reward[i] = 0.0f;
                done[i] = 0;
                events[i] = 0;
                continue;
            }
            uint32_t ev = agent_events(s, i, coll[li]);
            if (forbid[li] && !(ev & OR_EV_NUMERIC)) ev |= OR_EV_LANE_FORBIDDEN;
            if (nan_act[li]) ev |= OR_EV_NAN_ACTION;
            K(s, OR_EPSTEP, i) += 1;
            K(s, OR_SINCE, i) += 1;
            if (K(s, OR_EPSTEP, i) >= p->max_episode_steps) ev |= OR_EV_TIMEOUT;
            double r = 0.0;
            if (ev & OR_EV_GOAL) r = 45.0;
            else if (ev & OR_EV_COLLISION) r = -6.0;
            else if (ev & OR_EV_CRASH) r = -10.0;
            else if (ev & OR_EV_LANE_FORBIDDEN) r = -20.0;
            int term = (ev & (OR_EV_GOAL | OR_EV_COLLISION | OR_EV_CRASH | OR_EV_LANE_FORBIDDEN)) != 0;
            int dn = (term && !p->invincible) || (ev & (OR_EV_TIMEOUT | OR_EV_NUMERIC)) != 0;
            sparse[li] = r;
            carry[li] = !dn;
            reward[i] = (float)r;
            done[i] = (uint8_t)dn;
            events[i] = (uint8_t)ev;
            if (dn) {
                if (p->auto_reset) {
                    K(s, OR_EPISODE, i) += 1;
                    spawn_agent(s, i);
                } else {
                    park_agent(s, i);
                }
            }
        }
        /* dense terms on the new pose of every agent that carries on (a
         * terminating step delivers its sparse reward only), with the world
         * as the step leaves it: agents that ended this step are already at
         * their new spawn or parked */
        if (s->shaping)
            for (int i = a0; i < a1; ++i) {
                const int li = i - a0;
                if (!was_active[li] || !carry[li]) continue;
                double terms[6];
                or_shaping_terms(s, i, F(s, OR_PX, i) - p0[2 * li], F(s, OR_PY, i) - p0[2 * li + 1], terms);
                double r = sparse[li];
                for (int k = 0; k < 6; ++k) r += terms[k];
                reward[i] = (float)r;
            }
        free(nan_act); free(coll); free(was_active); free(forbid); free(p0); free(sparse); free(carry);
    }
}

/* ------------------------------------------------------ observations */
typedef struct { int64_t key; int idx; } kv_t;
static int kv_cmp(const void *a, const void *b) {
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}
static int int_cmp(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return x < y ? -1 : (x > y);
}
static int64_t sat_key(int64_t d2) { return d2 < KEY_CAP ? d2 : KEY_CAP - 1; }

/* the 64 road points with the smallest quantised distance (ties: lower
 * index), returned in point-index order (the paper keeps polyline order) */
void or_knn_road(const or_sim *s, int i, int32_t *out) {
    int w = s->world_of[i];
    int r0 = s->roff[w], P = s->roff[w + 1] - r0;
    kv_t *kv = (kv_t *)malloc(sizeof(kv_t) * (P + 1));
    int64_t X = Qp(F(s, OR_PX, i)), Y = Qp(F(s, OR_PY, i));
    for (int k = 0; k < P; ++k) {
        int64_t dx = Qp(s->road_xy[2 * (r0 + k)]) - X, dy = Qp(s->road_xy[2 * (r0 + k) + 1]) - Y;
        kv[k].key = sat_key(dx * dx + dy * dy);
        kv[k].idx = k;
    }
    qsort(kv, P, sizeof(kv_t), kv_cmp);
    int n = P < OR_ROAD_K ? P : OR_ROAD_K;
    int sel[OR_ROAD_K];
    for (int k = 0; k < n; ++k) sel[k] = kv[k].idx;
    qsort(sel, n, sizeof(int), int_cmp);
    for (int k = 0; k < OR_ROAD_K; ++k) out[k] = k < n ? sel[k] : -1;
    free(kv);
}

/* the 8 nearest other active agents of the world, ascending */
void or_knn_neigh(const or_sim *s, int i, int32_t *out) {
    int w = s->world_of[i];
    int a0 = s->aoff[w], A = s->aoff[w + 1] - a0;
    kv_t *kv = (kv_t *)malloc(sizeof(kv_t) * (A + 1));
    int64_t X = Qp(F(s, OR_PX, i)), Y = Qp(F(s, OR_PY, i));
    int n = 0;
    for (int j = a0; j < a0 + A; ++j) {
        if (j == i || !K(s, OR_ACTIVE, j)) continue;
        int64_t dx = Qp(F(s, OR_PX, j)) - X, dy = Qp(F(s, OR_PY, j)) - Y;
        kv[n].key = sat_key(dx * dx + dy * dy);
        kv[n].idx = j - a0;
        ++n;
    }
    qsort(kv, n, sizeof(kv_t), kv_cmp);
    for (int k = 0; k < OR_NEIGH_K; ++k) out[k] = k < n ? kv[k].idx : -1;
    free(kv);
}

/* swept-circle time to collision between agents i and j (Sec. "Neighbor
 * vehicles"): smallest t >= 0 at which any of the 3 x 3 circle pairs touch
 * under constant planar velocities; 0 if touching, 10 s cap */
static double ttc_pair(const or_sim *s, int i, int j) {
    double hix, hiy, hjx, hjy;
    heading_fp(s, i, &hix, &hiy);
    heading_fp(s, j, &hjx, &hjy);
    double dvx = F(s, OR_VX, j) - F(s, OR_VX, i), dvy = F(s, OR_VY, j) - F(s, OR_VY, i);
    double best = 10.0;
    double R = 2.0 * s->cr;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double cx = (F(s, OR_PX, j) + (b - 1) * s->cd * hjx) - (F(s, OR_PX, i) + (a - 1) * s->cd * hix);
            double cy = (F(s, OR_PY, j) + (b - 1) * s->cd * hjy) - (F(s, OR_PY, i) + (a - 1) * s->cd * hiy);
            double c = cx * cx + cy * cy - R * R;
            double t;
            if (c <= 0.0) t = 0.0;
            else {
                double bq = 2.0 * (cx * dvx + cy * dvy);
                if (bq >= 0.0) continue;
                double aq = dvx * dvx + dvy * dvy;
                double disc = bq * bq - 4.0 * aq * c;
                if (disc < 0.0) continue;
                t = (-bq - sqrt(disc)) / (2.0 * aq);
            }
            if (t < best) best = t;
        }
    return best;
}

void or_observe(const or_sim *s, float *obs) {
    const or_params *p = &s->p;
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < s->N; ++i) {
        float *o = obs + (size_t)OR_OBS_DIM * i;
        for (int k = 0; k < OR_OBS_DIM; ++k) o[k] = 0.0f;
        if (!K(s, OR_ACTIVE, i)) continue;
        int w = s->world_of[i];
        double hx, hy;
        heading_fp(s, i, &hx, &hy);
        double px = F(s, OR_PX, i), py = F(s, OR_PY, i);
        /* ego: goal in the body frame, heading error, distance, body velocity, mu */
        double gx = F(s, OR_GX, i) - px, gy = F(s, OR_GY, i) - py;
        double gbx = hx * gx + hy * gy, gby = -hy * gx + hx * gy;
        double dist = sqrt(gx * gx + gy * gy);
        double vx = F(s, OR_VX, i), vy = F(s, OR_VY, i);
        o[0] = (float)(gbx / 100.0);
        o[1] = (float)(gby / 100.0);
        o[2] = (float)(dist > 0 ? gby / dist : 0.0);
        o[3] = (float)(dist > 0 ? gbx / dist : 1.0);
        o[4] = (float)(dist / 100.0);
        o[5] = (float)((hx * vx + hy * vy) / 10.0);
        o[6] = (float)((-hy * vx + hx * vy) / 10.0);
        o[7] = (float)F(s, OR_MU, i);
        /* road context */
        int32_t ridx[OR_ROAD_K];
        or_knn_road(s, i, ridx);
        int r0 = s->roff[w];
        for (int k = 0; k < OR_ROAD_K; ++k) {
            if (ridx[k] < 0) break;
            double dx = s->road_xy[2 * (r0 + ridx[k])] - px, dy = s->road_xy[2 * (r0 + ridx[k]) + 1] - py;
            o[8 + 3 * k] = (float)((hx * dx + hy * dy) / 10.0);
            o[8 + 3 * k + 1] = (float)((-hy * dx + hx * dy) / 10.0);
            o[8 + 3 * k + 2] = (float)(s->road_type[r0 + ridx[k]] / 20.0);
        }
        /* neighbour context */
        int32_t nidx[OR_NEIGH_K];
        or_knn_neigh(s, i, nidx);
        int a0 = s->aoff[w];
        for (int k = 0; k < OR_NEIGH_K; ++k) {
            if (nidx[k] < 0) break;
            int j = a0 + nidx[k];
            double dx = F(s, OR_PX, j) - px, dy = F(s, OR_PY, j) - py;
            double bx = hx * dx + hy * dy, by = -hy * dx + hx * dy;
            double hjx, hjy;
            heading_fp(s, j, &hjx, &hjy);
            double dpsi = atan2(hx * hjy - hy * hjx, hx * hjx + hy * hjy);
            if (dpsi == -M_PI) dpsi = M_PI;
            double ttc = bx < 0.0 ? 10.0 : ttc_pair(s, i, j);
            double vjx = F(s, OR_VX, j), vjy = F(s, OR_VY, j);
            float *q = o + 200 + 7 * k;
            q[0] = (float)(bx / 100.0);
            q[1] = (float)(by / 100.0);
            q[2] = (float)(p->length / 100.0);
            q[3] = (float)(p->width / 100.0);
            q[4] = (float)(dpsi / M_PI);
            q[5] = (float)(sqrt(vjx * vjx + vjy * vjy) / 10.0);
            q[6] = (float)(ttc / 10.0);
        }
    }
}

/* ------------------------------------------- the paper's observation */
/* Appendix "Observation Space Details", at the paper's shape: per agent
 * OR_FULL_DIM = 11 + 350 x 5 + 24 x 7 = 1929 floats, zero where a slot is
 * empty, and the numbers of valid road and neighbour slots (the slots the
 * network's masked max-pool reads).
 *   ego 11: goal in the body frame / 100 (2), sin and cos of the goal
 *     bearing, goal distance / 100, body-frame velocity / 10 (2), then the
 *     weather token of Eq. weather_obs: film depth / 1 mm and the one-hot
 *     pavement (AC, SMA, OGFC);
 *   road 350 x 5: every road point within 10 m (quantised squared distance,
 *     inclusive), in point-index order, the first 350: body-frame offset / 10
 *     (2), type / 20, body-frame polyline direction (2);
 *   neighbours 24 x 7: the 24 nearest other active agents (quantised key,
 *     ties by lower index), ascending, with the features of the
 *     8-neighbour observation. */
void or_knn_neigh_k(const or_sim *s, int i, int K, int32_t *out) {
    int w = s->world_of[i];
    int a0 = s->aoff[w], A = s->aoff[w + 1] - a0;
    kv_t *kv = (kv_t *)malloc(sizeof(kv_t) * (A + 1));
    int64_t X = Qp(F(s, OR_PX, i)), Y = Qp(F(s, OR_PY, i));
    int n = 0;
    for (int j = a0; j < a0 + A; ++j) {
        if (j == i || !K(s, OR_ACTIVE, j)) continue;
        int64_t dx = Qp(F(s, OR_PX, j)) - X, dy = Qp(F(s, OR_PY, j)) - Y;
        kv[n].key = sat_key(dx * dx + dy * dy);
        kv[n].idx = j - a0;
        ++n;
    }
    qsort(kv, n, sizeof(kv_t), kv_cmp);
    for (int k = 0; k < K; ++k) out[k] = k < n ? kv[k].idx : -1;
    free(kv);
}

int or_road_within(const or_sim *s, int i, int K, int32_t *out) {
    int w = s->world_of[i];
    int r0 = s->roff[w], P = s->roff[w + 1] - r0;
    int64_t X = Qp(F(s, OR_PX, i)), Y = Qp(F(s, OR_PY, i));
    const int64_t R = (int64_t)10 * 1024;
    int n = 0;
    for (int k = 0; k < P && n < K; ++k) {
        int64_t dx = Qp(s->road_xy[2 * (r0 + k)]) - X, dy = Qp(s->road_xy[2 * (r0 + k) + 1]) - Y;
        if (dx * dx + dy * dy <= R * R) out[n++] = k;
    }
    for (int k = n; k < K; ++k) out[k] = -1;
    return n;
}

void or_observe_full(const or_sim *s, float *obs, int32_t *counts) {
    const or_params *p = &s->p;
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < s->N; ++i) {
        float *o = obs + (size_t)OR_FULL_DIM * i;
        for (int k = 0; k < OR_FULL_DIM; ++k) o[k] = 0.0f;
        counts[2 * i] = counts[2 * i + 1] = 0;
        if (!K(s, OR_ACTIVE, i)) continue;
        int w = s->world_of[i];
        double hx, hy;
        heading_fp(s, i, &hx, &hy);
        double px = F(s, OR_PX, i), py = F(s, OR_PY, i);
        double gx = F(s, OR_GX, i) - px, gy = F(s, OR_GY, i) - py;
        double gbx = hx * gx + hy * gy, gby = -hy * gx + hx * gy;
        double dist = sqrt(gx * gx + gy * gy);
        double vx = F(s, OR_VX, i), vy = F(s, OR_VY, i);
        o[0] = (float)(gbx / 100.0);
        o[1] = (float)(gby / 100.0);
        o[2] = (float)(dist > 0 ? gby / dist : 0.0);
        o[3] = (float)(dist > 0 ? gbx / dist : 1.0);
        o[4] = (float)(dist / 100.0);
        o[5] = (float)((hx * vx + hy * vy) / 10.0);
        o[6] = (float)((-hy * vx + hx * vy) / 10.0);
        o[7] = (float)(s->film[w] / 1.0);
        o[8 + (s->pav[w] >= 0 && s->pav[w] <= 2 ? s->pav[w] : 0)] = 1.0f;
        int32_t ridx[OR_FULL_ROAD_K];
        const int nr = or_road_within(s, i, OR_FULL_ROAD_K, ridx);
        int r0 = s->roff[w];
        for (int k = 0; k < nr; ++k) {
            const int q = r0 + ridx[k];
            double dx = s->road_xy[2 * q] - px, dy = s->road_xy[2 * q + 1] - py;
            double ux = s->road_dir[2 * q], uy = s->road_dir[2 * q + 1];
            float *r = o + OR_FULL_EGO + 5 * k;
            r[0] = (float)((hx * dx + hy * dy) / 10.0);
            r[1] = (float)((-hy * dx + hx * dy) / 10.0);
            r[2] = (float)(s->road_type[q] / 20.0);
            r[3] = (float)(hx * ux + hy * uy);
            r[4] = (float)(-hy * ux + hx * uy);
        }
        int32_t nidx[OR_FULL_NEIGH_K];
        or_knn_neigh_k(s, i, OR_FULL_NEIGH_K, nidx);
        int a0 = s->aoff[w], nv = 0;
        for (int k = 0; k < OR_FULL_NEIGH_K; ++k) {
            if (nidx[k] < 0) break;
            int j = a0 + nidx[k];
            double dx = F(s, OR_PX, j) - px, dy = F(s, OR_PY, j) - py;
            double bx = hx * dx + hy * dy, by = -hy * dx + hx * dy;
            double hjx, hjy;
            heading_fp(s, j, &hjx, &hjy);
            double dpsi = atan2(hx * hjy - hy * hjx, hx * hjx + hy * hjy);
            if (dpsi == -M_PI) dpsi = M_PI;
            double ttc = bx < 0.0 ? 10.0 : ttc_pair(s, i, j);
            double vjx = F(s, OR_VX, j), vjy = F(s, OR_VY, j);
            float *q = o + OR_FULL_EGO + 5 * OR_FULL_ROAD_K + 7 * k;
            q[0] = (float)(bx / 100.0);
            q[1] = (float)(by / 100.0);
            q[2] = (float)(p->length / 100.0);
            q[3] = (float)(p->width / 100.0);
            q[4] = (float)(dpsi / M_PI);
            q[5] = (float)(sqrt(vjx * vjx + vjy * vjy) / 10.0);
            q[6] = (float)(ttc / 10.0);
            ++nv;
        }
        counts[2 * i] = nr;
        counts[2 * i + 1] = nv;
    }
}

/* ----------------------------------------------------------- networks */
/* round to bfloat16 (8 significant bits), nearest-even, from the value;
 * switched off only for finite-difference checks of the gradients */
static int g_bf16 = 1;
void or_set_bf16(int on) { g_bf16 = on; }
static double bf16r(double x) {
    if (!g_bf16 || x == 0.0 || !isfinite(x)) return x;
    int e;
    double m = frexp(x, &e); /* x = m 2^e, 0.5 <= |m| < 1 */
    double r = nearbyint(ldexp(m, 8));
    return ldexp(r, e - 8);
}

static double elu(double x) { return x > 0 ? x : expm1(x); }

/* forward pass keeping the bf16-rounded activations of every layer */
static void mlp_fwd_keep(int L, const int *sz, const float *const *W, const float *const *b,
                         int act, const float *x, double **a, double **z) {
    for (int k = 0; k < sz[0]; ++k) a[0][k] = bf16r(x[k]);
    for (int l = 0; l < L; ++l) {
        for (int o = 0; o < sz[l + 1]; ++o) {
            double acc = b[l][o];
            for (int k = 0; k < sz[l]; ++k) acc += bf16r(W[l][(size_t)o * sz[l] + k]) * a[l][k];
            z[l][o] = acc;
            if (l < L - 1) {
                double y = act == 0 ? elu(acc) : (acc > 0 ? acc : 0.0);
                a[l + 1][o] = bf16r(y);
            } else {
                a[l + 1][o] = acc;
            }
        }
    }
}

void or_mlp_forward(int L, const int *sz, const float *const *W, const float *const *b,
                    int act, int M, const float *x, double *y) {
    int mx = 0;
    for (int l = 0; l <= L; ++l) if (sz[l] > mx) mx = sz[l];
    for (int r = 0; r < M; ++r) {
        double *a[16], *z[16];
        for (int l = 0; l <= L; ++l) { a[l] = (double *)malloc(sizeof(double) * mx); z[l] = (double *)malloc(sizeof(double) * mx); }
        mlp_fwd_keep(L, sz, W, b, act, x + (size_t)r * sz[0], a, z);
        for (int o = 0; o < sz[L]; ++o) y[(size_t)r * sz[L] + o] = a[L][o];
        for (int l = 0; l <= L; ++l) { free(a[l]); free(z[l]); }
    }
}

/* The late-fusion actor-critic of appendix "Network Architecture Details"
 * on the paper's observation: per network (actor, then critic; no shared
 * weights) an ego encoder 11 -> 64 -> 64, a road encoder 5 -> 96 -> 96 on
 * every valid road slot and a vehicle encoder 7 -> 96 -> 96 on every valid
 * neighbour slot, each followed by a max over its valid slots (the masked
 * max-pool; an empty set pools to 0), the 64 + 96 + 96 embedding through a
 * trunk 256 -> 128 -> 64, ELU after every hidden layer, then the actor's
 * 3-dim mean or the critic's value.  bf16 rounding points as in the other
 * networks: the layers' inputs, weights and hidden activations.
 * Parameter block (float32): for each network, ego W1[64][11] b1 W2[64][64]
 * b2, road W1[96][5] b1 W2[96][96] b2, vehicle W1[96][7] b1 W2[96][96] b2,
 * trunk W1[128][256] b1 W2[64][128] b2, then the actor's head W[3][64] b[3]
 * and log sigma[3], or the critic's W[1][64] b[1]. */
static const float *ac_dense(const float *P, int in, int out, double *xin, double *y, int act) {
    const float *W = P, *b = P + (size_t)in * out;
    for (int o = 0; o < out; ++o) {
        double acc = b[o];
        for (int k = 0; k < in; ++k) acc += bf16r(W[(size_t)o * in + k]) * xin[k];
        y[o] = act ? bf16r(elu(acc)) : acc;
    }
    return b + out;
}

static const float *ac_encoder_pool(const float *P, int in, int rows, const float *x, int stride, double *pool) {
    double h[96], z[96], xin[16];
    const float *end = P;
    for (int c = 0; c < 96; ++c) pool[c] = rows > 0 ? -INFINITY : 0.0;
    for (int r = 0; r < rows; ++r) {
        for (int k = 0; k < in; ++k) xin[k] = bf16r(x[(size_t)r * stride + k]);
        const float *P2 = ac_dense(P, in, 96, xin, h, 1);
        end = ac_dense(P2, 96, 96, h, z, 1);
        for (int c = 0; c < 96; ++c) if (z[c] > pool[c]) pool[c] = z[c];
    }
    if (rows == 0) end = P + (size_t)in * 96 + 96 + 96 * 96 + 96;
    return end;
}

/* one network on one agent's observation; returns the parameters after it */
static const float *ac_net(const float *P, const float *o, int nr, int nv, int nout, double *out) {
    double xin[OR_FULL_EGO], e1[64], emb[256], t1[128], t2[64];
    for (int k = 0; k < OR_FULL_EGO; ++k) xin[k] = bf16r(o[k]);
    P = ac_dense(P, OR_FULL_EGO, 64, xin, e1, 1);
    P = ac_dense(P, 64, 64, e1, emb, 1);
    P = ac_encoder_pool(P, 5, nr, o + OR_FULL_EGO, 5, emb + 64);
    P = ac_encoder_pool(P, 7, nv, o + OR_FULL_EGO + 5 * OR_FULL_ROAD_K, 7, emb + 160);
    P = ac_dense(P, 256, 128, emb, t1, 1);
    P = ac_dense(P, 128, 64, t1, t2, 1);
    return ac_dense(P, 64, nout, t2, out, 0);
}

void or_actor_critic(const float *params, int M, const float *obs, const int32_t *counts, double *mean,
                     double *value) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int r = 0; r < M; ++r) {
        const float *o = obs + (size_t)OR_FULL_DIM * r;
        const int nr = counts[2 * r], nv = counts[2 * r + 1];
        const float *critic = ac_net(params, o, nr, nv, 3, mean + 3 * (size_t)r) + 3;   /* skip log sigma */
        ac_net(critic, o, nr, nv, 1, value + r);
    }
}

void or_policy(int M, const float *obs, const float *const *W, const float *const *b,
               double steer_max, double *act) {
    int sz[4] = {OR_OBS_DIM, 256, 256, 2};
    double *y = (double *)malloc(sizeof(double) * 2 * M);
    or_mlp_forward(3, sz, W, b, 0, M, obs, y);
    for (int r = 0; r < M; ++r) {
        act[2 * r] = tanh(y[2 * r]);
        act[2 * r + 1] = steer_max * tanh(y[2 * r + 1]);
    }
    free(y);
}

double or_mlp_mse_grad(int L, const int *sz, const float *const *W, const float *const *b,
                       int M, const float *x, const float *target, const double *row_weight,
                       double *const *gW, double *const *gb) {
    int mx = 0;
    for (int l = 0; l <= L; ++l) if (sz[l] > mx) mx = sz[l];
    for (int l = 0; l < L; ++l) {
        memset(gW[l], 0, sizeof(double) * sz[l] * sz[l + 1]);
        memset(gb[l], 0, sizeof(double) * sz[l + 1]);
    }
    double loss = 0.0;
    double scale = 1.0 / ((double)M * sz[L]);
    double *a[16], *z[16], *d0 = (double *)malloc(sizeof(double) * mx), *d1 = (double *)malloc(sizeof(double) * mx);
    for (int l = 0; l <= L; ++l) { a[l] = (double *)malloc(sizeof(double) * mx); z[l] = (double *)malloc(sizeof(double) * mx); }
    for (int r = 0; r < M; ++r) {
        mlp_fwd_keep(L, sz, W, b, 1, x + (size_t)r * sz[0], a, z);
        const double wr = row_weight ? row_weight[r] : 1.0;
        for (int o = 0; o < sz[L]; ++o) {
            double e = a[L][o] - target[(size_t)r * sz[L] + o];
            loss += wr * e * e * scale;
            d0[o] = 2.0 * wr * e * scale;
        }
        for (int l = L - 1; l >= 0; --l) {
            for (int o = 0; o < sz[l + 1]; ++o) {
                gb[l][o] += d0[o];
                for (int k = 0; k < sz[l]; ++k) gW[l][(size_t)o * sz[l] + k] += d0[o] * a[l][k];
            }
            if (l > 0) {
                for (int k = 0; k < sz[l]; ++k) {
                    double acc = 0.0;
                    for (int o = 0; o < sz[l + 1]; ++o) acc += bf16r(W[l][(size_t)o * sz[l] + k]) * d0[o];
                    d1[k] = z[l - 1][k] > 0 ? acc : 0.0;
                }
                double *t = d0; d0 = d1; d1 = t;
            }
        }
    }
    for (int l = 0; l <= L; ++l) { free(a[l]); free(z[l]); }
    free(d0); free(d1);
    return loss;
}

/* surrogate forward in FP64 with the bf16 rounding points */
static void sur_forward(const or_sim *s, const float *f, double *y) {
    int sz[5] = {OR_SUR_IN, OR_SUR_HID, OR_SUR_HID, OR_SUR_HID, 3};
    const float *Wp[4], *bp[4];
    const float *q = s->sur;
    for (int l = 0; l < 4; ++l) {
        Wp[l] = q;
        q += sz[l] * sz[l + 1];
        bp[l] = q;
        q += sz[l + 1];
    }
    or_mlp_forward(4, sz, Wp, bp, 1, 1, f, y);
}

void or_set_surrogate(or_sim *s, const float *params, const float *env_lo, const float *env_hi,
                      int enable) {
    if (!s->sur) s->sur = (float *)malloc(sizeof(float) * OR_SUR_PARAMS);
    if (params) memcpy(s->sur, params, sizeof(float) * OR_SUR_PARAMS);
    if (env_lo) memcpy(s->env_lo, env_lo, sizeof(float) * OR_SUR_IN);
    if (env_hi) memcpy(s->env_hi, env_hi, sizeof(float) * OR_SUR_IN);
    s->sur_on = enable;
    s->sur_used = s->sur_fallback = 0;
}

void or_surrogate_counts(const or_sim *s, long long *used, long long *fallback) {
    *used = s->sur_used;
    *fallback = s->sur_fallback;
}

void or_record_samples(or_sim *s, float *rec) { s->sample_rec = rec; }

/* Adam (Kingma and Ba 2015) with bias correction */
void or_adam(int n, float *w, const double *g, double *m, double *v, int step, double lr,
             double b1, double b2, double eps) {
    double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
    for (int k = 0; k < n; ++k) {
        m[k] = b1 * m[k] + (1.0 - b1) * g[k];
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
        double mh = m[k] / c1, vh = v[k] / c2;
        w[k] = (float)(w[k] - lr * mh / (sqrt(vh) + eps));
    }
}
