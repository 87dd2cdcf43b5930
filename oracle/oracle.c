/*
 * FP64 CPU oracle of the per-ray image-generation pipeline of Rajendran, Bane & Vlachos,
 * "PIV/BOS synthetic image generation in variable density environments" (arXiv 1812.05902).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load this file:
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark use it.  It shares
 * no code, header, table or constant with the GPU library; the two meet only through the
 * seeded input generators (density grids and source lists).
 *
 * Plain and slow on purpose: world coordinates in double precision, one ray at a time, every
 * step written in the order the paper states it.  Readings taken where the paper is silent
 * are marked READING.
 *
 * Pipeline (section 3, four steps):
 *   1. light field (sec. 3.1): a ray joins a source point to a sampled point of the lens
 *      aperture; its direction is the unit vector between them.
 *   2. density gradients (sec. 3.2): Gladstone-Dale n = K rho + 1 (eq. 1); the ray equation
 *      d/dxi(n dx/dxi) = grad n (eq. 2) advanced by the Runge-Kutta scheme of eqs. 3-6.
 *   3. optical elements (sec. 3.3): aperture (selective transmission), then refraction by
 *      Snell's law (eq. 7) at each spherical surface of the lens in turn, with total internal
 *      reflection possible.
 *   4. sensor (sec. 3.4): line-plane intersection; Gaussian approximation of the Airy spot
 *      with diameter from eq. 8, integrated over each pixel with the error function; intensities
 *      summed over all rays.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- public structs (ctypes) */

enum { ORC_GRID = 0, ORC_LINEAR_N = 1, ORC_N2_LINEAR = 2, ORC_BUMP = 3 };

enum {
    ORC_DEPOSITED = 0, ORC_OFF_SENSOR = 1, ORC_BLOCKED_APERTURE = 2, ORC_BLOCKED_LENS = 3,
    ORC_TIR = 4, ORC_STEP_LIMIT = 5, ORC_MISSED = 6
};

typedef struct {
    /* field */
    int32_t nx, ny, nz, field_mode;
    double origin[3], spacing[3];
    double K, rho_inf;
    double ana[10];              /* analytic field parameters (field_mode != ORC_GRID) */
    /* optics */
    double z_lens, focal_length, f_number, n_glass, thickness, clear_radius, z_focus;
    /* sensor */
    int32_t width, height, dtau_with_pi, pad0;
    double pitch, z_sensor, wavelength, sigma_px;
    /* integration */
    double ds;
    uint64_t seed;
    int32_t max_steps, pad1;     /* max_steps <= 0: 4 * ceil(box diagonal / ds) + 64 */
} orc_cfg;

typedef struct {
    int64_t ray_id;
    int32_t status, n_steps;
    int32_t entered, pad;
    double lens_point[2];        /* sampled aperture point, lens frame (x, y) */
    double dir0[3];              /* initial unit direction */
    double vol_exit_pos[3];      /* where the ray left the density box (or the source) */
    double vol_exit_dir[3];      /* unit direction there */
    double sensor_px[2];         /* sensor hit in pixel coordinates */
} orc_ray;

/* One surface of a general optical chain (sec. 3.3), rotationally symmetric about the axis. */
enum { ORC_SURF_REFRACT = 0, ORC_SURF_MIRROR = 1, ORC_SURF_APERTURE = 2, ORC_SURF_LENSLETS = 3 };
typedef struct {
    int32_t type, reserved;
    double z;          /* vertex on the axis */
    double radius;     /* signed radius of curvature (centre at z + radius); 0 = plane */
    double clear;      /* rays meeting the surface farther than this from the axis are blocked */
    double n_after;    /* index after a refracting surface; <= 0 = ambient */
    double pitch;      /* lenslet pitch (square grid centred on the axis) */
} orc_surface;
#define ORC_MAX_SURFACES 16

typedef struct {
    orc_cfg c;
    double *dn, *gx, *gy, *gz;   /* node values: n - 1 and grad n (grid mode) */
    double lo[3], hi[3];         /* box corners */
    double n_inf;                /* ambient refractive index */
    double h;                    /* RKN step in the parameter t of dR/dt = T */
    double a;                    /* aperture radius */
    double R;                    /* lens surface radius (symmetric biconvex) */
    double t;                    /* lens thickness */
    double clear;                /* clear radius of each surface */
    double z_sensor;             /* sensor plane */
    double M;                    /* lateral magnification (signed, < 0 = inverted) */
    double sigma_px;             /* Gaussian spot sigma in pixels */
    int r_fp;                    /* footprint half-width in pixels */
    int max_steps;
    orc_surface chain[ORC_MAX_SURFACES];  /* general optical chain (n_chain > 0) replacing the singlet */
    int n_chain;
    double aim_z, aim_r;         /* with a chain: rays aim at this disk (sec. 3.1) */
    double *mie;                 /* Mie intensity table at theta_k = k pi / (mie_n - 1), or NULL */
    int mie_n;
    double laser[3];             /* unit propagation direction of the laser light */
} orc_scene;

/* ---------------------------------------------------------------- counter-based RNG */

/* k-th output (k = 0, 1, ...) of SplitMix64 seeded with `seed` (Steele, Lea & Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014): the state advances by the
 * odd constant 0x9E3779B97F4A7C15 and each state is passed through the variant-13 mixer. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Two uniforms in [0,1) for ray j of source s: 24-bit fields of one SplitMix64 output at
 * counter (s << 32) | j.  24 bits so that both sides hold them exactly. */
void orc_ray_uniforms(uint64_t seed, int64_t s, int64_t j, double u[2])
{
    uint64_t hsh = orc_splitmix64(seed, ((uint64_t)s << 32) | (uint64_t)(uint32_t)j);
    u[0] = (double)(hsh >> 40) * (1.0 / 16777216.0);
    u[1] = (double)((hsh >> 16) & 0xFFFFFFu) * (1.0 / 16777216.0);
}

/* ---------------------------------------------------------------- field */

static size_t nidx(const orc_scene *S, int i, int j, int k)
{
    return ((size_t)k * S->c.ny + (size_t)j) * S->c.nx + (size_t)i;
}

/* d rho / d(index) along one axis at node m of a line of n samples spaced `stride` apart:
 * central difference inside, second-order one-sided difference on the two end nodes,
 * first-order difference when the line has only two nodes.  READING: the paper says only
 * that the update uses the local refractive-index gradient (sec. 3.2). */
static double diff_index(const float *rho, size_t base, size_t stride, int m, int n)
{
#define RHO(q) ((double)rho[base + (size_t)(q) * stride])
    if (n == 2) return RHO(1) - RHO(0);
    if (m == 0) return 0.5 * (-3.0 * RHO(0) + 4.0 * RHO(1) - RHO(2));
    if (m == n - 1) return 0.5 * (3.0 * RHO(n - 1) - 4.0 * RHO(n - 2) + RHO(n - 3));
    return 0.5 * (RHO(m + 1) - RHO(m - 1));
#undef RHO
}

/* Gladstone-Dale, eq. 1: n = K rho + 1, so n - 1 = K rho and grad n = K grad rho. */
static void field_prepare(orc_scene *S, const float *rho)
{
    const int nx = S->c.nx, ny = S->c.ny, nz = S->c.nz;
    const double K = S->c.K;
    size_t N = (size_t)nx * ny * nz;
    S->dn = (double *)malloc(N * sizeof(double));
    S->gx = (double *)malloc(N * sizeof(double));
    S->gy = (double *)malloc(N * sizeof(double));
    S->gz = (double *)malloc(N * sizeof(double));
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t q = nidx(S, i, j, k);
                S->dn[q] = K * (double)rho[q];
                S->gx[q] = K * diff_index(rho, nidx(S, 0, j, k), 1, i, nx) / S->c.spacing[0];
                S->gy[q] = K * diff_index(rho, nidx(S, i, 0, k), (size_t)nx, j, ny) / S->c.spacing[1];
                S->gz[q] = K * diff_index(rho, nidx(S, i, j, 0), (size_t)nx * ny, k, nz) / S->c.spacing[2];
            }
}

/* n and grad n at a point.  Grid mode: trilinear interpolation of (n - 1, grad n) in the cell
 * holding the point; a point outside the box is first moved onto the box (edge extension).
 * Analytic modes: the formula itself. */
void orc_field_eval(const orc_scene *S, const double R[3], double out[4])
{
    const double *p = S->c.ana;
    if (S->c.field_mode == ORC_LINEAR_N) {
        /* n = n0 + G . (R - R0) */
        double n = p[0] + p[1] * (R[0] - p[4]) + p[2] * (R[1] - p[5]) + p[3] * (R[2] - p[6]);
        out[0] = n - 1.0; out[1] = p[1]; out[2] = p[2]; out[3] = p[3];
        return;
    }
    if (S->c.field_mode == ORC_N2_LINEAR) {
        /* n^2 = n0^2 + 2 g . (R - R0), so grad n = g / n */
        double n2 = p[0] * p[0] + 2.0 * (p[1] * (R[0] - p[4]) + p[2] * (R[1] - p[5]) + p[3] * (R[2] - p[6]));
        double n = sqrt(n2);
        out[0] = n - 1.0; out[1] = p[1] / n; out[2] = p[2] / n; out[3] = p[3] / n;
        return;
    }
    if (S->c.field_mode == ORC_BUMP) {
        /* rho = rho0 (1 + A exp(-|R - c|^2 / (2 s^2))), n = 1 + K rho */
        double dx = R[0] - p[3], dy = R[1] - p[4], dz = R[2] - p[5];
        double e = exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * p[2] * p[2]));
        double rho = p[0] * (1.0 + p[1] * e);
        double g = -S->c.K * p[0] * p[1] * e / (p[2] * p[2]);
        out[0] = S->c.K * rho; out[1] = g * dx; out[2] = g * dy; out[3] = g * dz;
        return;
    }
    const int n3[3] = {S->c.nx, S->c.ny, S->c.nz};
    int c[3];
    double w[3];
    for (int a = 0; a < 3; ++a) {
        double f = (R[a] - S->c.origin[a]) / S->c.spacing[a];
        if (f < 0.0) f = 0.0;
        if (f > (double)(n3[a] - 1)) f = (double)(n3[a] - 1);
        int i = (int)floor(f);
        if (i > n3[a] - 2) i = n3[a] - 2;
        c[a] = i;
        w[a] = f - (double)i;
    }
    const double *arr[4] = {S->dn, S->gx, S->gy, S->gz};
    for (int q = 0; q < 4; ++q) {
        double v = 0.0;
        for (int dk = 0; dk < 2; ++dk)
            for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di) {
                    double wt = (di ? w[0] : 1.0 - w[0]) * (dj ? w[1] : 1.0 - w[1]) * (dk ? w[2] : 1.0 - w[2]);
                    v += wt * arr[q][nidx(S, c[0] + di, c[1] + dj, c[2] + dk)];
                }
        out[q] = v;
    }
}

/* D = n grad n (eq. 6), from the interpolated n and grad n. */
static void field_D(const orc_scene *S, const double R[3], double D[3])
{
    double f[4];
    orc_field_eval(S, R, f);
    double n = 1.0 + f[0];
    D[0] = n * f[1]; D[1] = n * f[2]; D[2] = n * f[3];
}

/* One step of eqs. 3 and 5 with step h of the ray parameter t (dR/dt = T, dT/dt = D):
 *   A = h D(R),  B = h D(R + h (T/2 + A/8)),  C = h D(R + h (T + B/2)),
 *   R <- R + h (T + (A + 2B)/6),  T <- T + (A + 4B + C)/6.
 * READING: the T_n of eq. 5 is the T_i of eq. 3 (the index letter is garbled). */
void orc_rkn_step(const orc_scene *S, double R[3], double T[3], double h)
{
    double A[3], B[3], C[3], P[3], D[3];
    field_D(S, R, D);
    for (int a = 0; a < 3; ++a) A[a] = h * D[a];
    for (int a = 0; a < 3; ++a) P[a] = R[a] + h * (0.5 * T[a] + 0.125 * A[a]);
    field_D(S, P, D);
    for (int a = 0; a < 3; ++a) B[a] = h * D[a];
    for (int a = 0; a < 3; ++a) P[a] = R[a] + h * (T[a] + 0.5 * B[a]);
    field_D(S, P, D);
    for (int a = 0; a < 3; ++a) C[a] = h * D[a];
    for (int a = 0; a < 3; ++a) {
        R[a] = R[a] + h * (T[a] + (A[a] + 2.0 * B[a]) / 6.0);
        T[a] = T[a] + (A[a] + 4.0 * B[a] + C[a]) / 6.0;
    }
}

/* Advance `nsteps` fixed steps with no box test (analytic-field pins). */
void orc_rkn_integrate(const orc_scene *S, double R[3], double T[3], double h, int64_t nsteps)
{
    for (int64_t s = 0; s < nsteps; ++s) orc_rkn_step(S, R, T, h);
}

/* Trace through the box from R (inside) with T = n u.  READING (exit rule; the paper does not
 * say how a ray leaves the grid): before each step, find the smallest straight-line parameter
 * lam at which R + lam T reaches a face it moves towards; if lam <= h, take one step of length
 * lam (if lam > 0), then move straight along the new T onto that face and stop.
 * Returns the number of steps, or -1 when max_steps is exceeded. */
static int trace_volume(const orc_scene *S, double R[3], double T[3])
{
    int steps = 0;
    for (;;) {
        double lam = INFINITY;
        int ax = -1;
        double face = 0.0;
        for (int a = 0; a < 3; ++a) {
            double l;
            if (T[a] > 0.0) l = (S->hi[a] - R[a]) / T[a];
            else if (T[a] < 0.0) l = (S->lo[a] - R[a]) / T[a];
            else continue;
            if (l < lam) { lam = l; ax = a; face = T[a] > 0.0 ? S->hi[a] : S->lo[a]; }
        }
        if (ax < 0) return steps; /* T == 0: cannot happen for a unit-speed ray */
        if (lam <= S->h) {
            double sgn = T[ax];
            if (lam > 0.0) { orc_rkn_step(S, R, T, lam); ++steps; }
            if ((sgn > 0.0 && T[ax] > 0.0) || (sgn < 0.0 && T[ax] < 0.0)) {
                double l2 = (face - R[ax]) / T[ax];
                for (int a = 0; a < 3; ++a) R[a] += l2 * T[a];
                R[ax] = face;
                return steps;
            }
            /* turned back by the field inside the last step: keep integrating */
            if (steps > S->max_steps) return -1;
            continue;
        }
        orc_rkn_step(S, R, T, S->h);
        if (++steps > S->max_steps) return -1;
    }
}

/* ---------------------------------------------------------------- optics (sec. 3.3) */

/* Snell's law (eq. 7) in vector form at a surface with unit normal N facing the incoming
 * unit direction u; n1 -> n2.  Returns 0 on success, 1 on total internal reflection. */
int orc_refract(const double u[3], const double N[3], double n1, double n2, double out[3])
{
    double eta = n1 / n2;
    double ci = -(u[0] * N[0] + u[1] * N[1] + u[2] * N[2]);
    double k = 1.0 - eta * eta * (1.0 - ci * ci);
    if (k < 0.0) return 1;
    double b = eta * ci - sqrt(k);
    for (int a = 0; a < 3; ++a) out[a] = eta * u[a] + b * N[a];
    return 0;
}

/* Intersection of the ray P + s u with the spherical surface whose vertex is at z = zv on the
 * axis and whose signed radius is Rs (centre at zv + Rs): the root on the cap around the
 * vertex.  Writes the hit point and the unit normal oriented against +z.  Returns 0 on hit. */
static int sphere_hit(const double P[3], const double u[3], double zv, double Rs,
                      double H[3], double N[3])
{
    double q0 = P[0], q1 = P[1], q2 = P[2] - zv;          /* vertex-local point */
    double b = q0 * u[0] + q1 * u[1] + q2 * u[2] - Rs * u[2];
    double c = q0 * q0 + q1 * q1 + q2 * q2 - 2.0 * Rs * q2;
    double disc = b * b - c;
    if (disc < 0.0) return 1;
    double q = -(b + (b >= 0.0 ? sqrt(disc) : -sqrt(disc)));
    if (q == 0.0) return 1;
    double s = c / q;                                      /* root nearer the vertex */
    H[0] = P[0] + s * u[0]; H[1] = P[1] + s * u[1]; H[2] = P[2] + s * u[2];
    N[0] = H[0] / Rs; N[1] = H[1] / Rs; N[2] = (H[2] - zv - Rs) / Rs;
    return 0;
}

/* Ambient straight line from P (world) along unit u through the aperture stop (disk of radius
 * a in the plane of the front vertex), both lens surfaces and onto the sensor plane.
 * READING: the lens prescription is absent from the paper; a symmetric biconvex singlet of
 * index n_glass and centre thickness t is used, radii from the thick-lens lensmaker equation.
 * Rays leaving a surface outside its clear radius, or missing it, are blocked; total internal
 * reflection drops the ray. */
int orc_lens_to_sensor(const orc_scene *S, const double P[3], const double u[3], double px[2])
{
    const double zl = S->c.z_lens;
    if (u[2] <= 0.0) return ORC_MISSED;
    double s = (zl - P[2]) / u[2];
    double A[3] = {P[0] + s * u[0], P[1] + s * u[1], zl};
    if (A[0] * A[0] + A[1] * A[1] > S->a * S->a) return ORC_BLOCKED_APERTURE;
    double H[3], N[3], v[3], w[3];
    if (sphere_hit(A, u, zl, S->R, H, N)) return ORC_BLOCKED_LENS;
    if (H[0] * H[0] + H[1] * H[1] > S->clear * S->clear) return ORC_BLOCKED_LENS;
    if (orc_refract(u, N, S->n_inf, S->c.n_glass, v)) return ORC_TIR;
    double H2[3];
    if (sphere_hit(H, v, zl + S->t, -S->R, H2, N)) return ORC_BLOCKED_LENS;
    if (H2[0] * H2[0] + H2[1] * H2[1] > S->clear * S->clear) return ORC_BLOCKED_LENS;
    if (orc_refract(v, N, S->c.n_glass, S->n_inf, w)) return ORC_TIR;
    if (w[2] <= 0.0) return ORC_MISSED;
    /* sec. 3.4: line-plane intersection with the sensor */
    double s2 = (S->z_sensor - H2[2]) / w[2];
    double xs = H2[0] + s2 * w[0], ys = H2[1] + s2 * w[1];
    /* READING: pixel (i, j) covers [i, i+1) x [j, j+1); the axis meets the sensor centre */
    px[0] = xs / S->c.pitch + 0.5 * S->c.width;
    px[1] = ys / S->c.pitch + 0.5 * S->c.height;
    return ORC_DEPOSITED;
}

/* ---------------------------------------------------------------- general optical chain (sec. 3.3) */

/* First intersection, at s > 1e-12 along P + s u, of the ray with the sphere of signed radius Rs
 * whose vertex is (cx, cy, zv), on the cap around the vertex (the half of the sphere facing its
 * vertex); Rs = 0 is the plane z = zv.  Writes the hit and the geometric normal (H - C) / Rs
 * ((0, 0, -1) for a plane), which faces -z at the vertex.  Returns 0 on a hit. */
static int chain_hit(const double P[3], const double u[3], double cx, double cy, double zv, double Rs,
                     double H[3], double N[3])
{
    const double eps = 1e-12;
    if (Rs == 0.0) {
        if (u[2] == 0.0) return 1;
        const double s = (zv - P[2]) / u[2];
        if (!(s > eps)) return 1;
        H[0] = P[0] + s * u[0]; H[1] = P[1] + s * u[1]; H[2] = zv;
        N[0] = 0.0; N[1] = 0.0; N[2] = -1.0;
        return 0;
    }
    const double C[3] = {cx, cy, zv + Rs};
    const double d[3] = {P[0] - C[0], P[1] - C[1], P[2] - C[2]};
    const double b = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
    const double c = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] - Rs * Rs;
    const double disc = b * b - c;
    if (disc < 0.0) return 1;
    const double sq = sqrt(disc);
    const double q = -(b + (b >= 0.0 ? sq : -sq));     /* stable pair of roots: q and c / q */
    double r1 = q, r2 = (q != 0.0) ? c / q : q;
    if (r1 > r2) { double t = r1; r1 = r2; r2 = t; }
    const double roots[2] = {r1, r2};
    for (int k = 0; k < 2; ++k) {
        const double s = roots[k];
        if (!(s > eps)) continue;
        const double h[3] = {P[0] + s * u[0], P[1] + s * u[1], P[2] + s * u[2]};
        if ((h[2] - C[2]) * Rs > 0.0) continue;        /* far half of the sphere */
        for (int a = 0; a < 3; ++a) { H[a] = h[a]; N[a] = (h[a] - C[a]) / Rs; }
        return 0;
    }
    return 1;
}

/* The ray from P (world) along unit u through the surfaces of the chain in order, then onto the
 * sensor plane.  Refraction by Snell's law (eq. 7) with total internal reflection, reflection by
 * the law of reflection about the local normal, apertures and surface rims block (sec. 3.3, items
 * 1-3); a lenslet array refracts at the spherical cap of the lenslet whose square cell the ray
 * meets (crossing into a neighbouring cell blocks it).  READING: sequential tracing; a ray that
 * would have to travel backwards to reach the next surface is blocked. */
int orc_chain_to_sensor(const orc_scene *S, const double P0[3], const double u0[3], double px[2])
{
    double P[3] = {P0[0], P0[1], P0[2]}, u[3] = {u0[0], u0[1], u0[2]};
    double n_cur = S->n_inf;
    for (int k = 0; k < S->n_chain; ++k) {
        const orc_surface *f = &S->chain[k];
        double H[3], N[3];
        double cx = 0.0, cy = 0.0, Rs = f->radius;
        if (f->type == ORC_SURF_APERTURE) Rs = 0.0;
        if (f->type == ORC_SURF_LENSLETS) {
            double A[3], NA[3];                           /* cell from the plane of the array */
            if (chain_hit(P, u, 0.0, 0.0, f->z, 0.0, A, NA)) return ORC_BLOCKED_LENS;
            cx = f->pitch * floor(A[0] / f->pitch + 0.5);
            cy = f->pitch * floor(A[1] / f->pitch + 0.5);
        }
        if (chain_hit(P, u, cx, cy, f->z, Rs, H, N))
            return f->type == ORC_SURF_APERTURE ? ORC_BLOCKED_APERTURE : ORC_BLOCKED_LENS;
        if (H[0] * H[0] + H[1] * H[1] > f->clear * f->clear)
            return f->type == ORC_SURF_APERTURE ? ORC_BLOCKED_APERTURE : ORC_BLOCKED_LENS;
        if (f->type == ORC_SURF_LENSLETS &&
            (fabs(H[0] - cx) > 0.5 * f->pitch || fabs(H[1] - cy) > 0.5 * f->pitch))
            return ORC_BLOCKED_LENS;
        const double un = u[0] * N[0] + u[1] * N[1] + u[2] * N[2];
        if (un > 0.0) for (int a = 0; a < 3; ++a) N[a] = -N[a];   /* normal against the ray */
        if (f->type == ORC_SURF_MIRROR) {
            const double d = u[0] * N[0] + u[1] * N[1] + u[2] * N[2];
            for (int a = 0; a < 3; ++a) u[a] = u[a] - 2.0 * d * N[a];
        } else if (f->type == ORC_SURF_REFRACT || f->type == ORC_SURF_LENSLETS) {
            const double n_next = f->n_after > 0.0 ? f->n_after : S->n_inf;
            double v[3];
            if (orc_refract(u, N, n_cur, n_next, v)) return ORC_TIR;
            const double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            for (int a = 0; a < 3; ++a) u[a] = v[a] / vn;
            n_cur = n_next;
        }
        for (int a = 0; a < 3; ++a) P[a] = H[a];
    }
    if (u[2] == 0.0) return ORC_MISSED;
    const double s = (S->z_sensor - P[2]) / u[2];
    if (!(s > 0.0)) return ORC_MISSED;
    px[0] = (P[0] + s * u[0]) / S->c.pitch + 0.5 * S->c.width;
    px[1] = (P[1] + s * u[1]) / S->c.pitch + 0.5 * S->c.height;
    return ORC_DEPOSITED;
}

/* Sets (n >= 1) or clears (n = 0) the general chain; rays then aim at the disk of radius aim_r in
 * the plane z = aim_z. */
void orc_set_chain(orc_scene *S, const orc_surface *surf, int n, double aim_z, double aim_r)
{
    S->n_chain = n < 0 ? 0 : (n > ORC_MAX_SURFACES ? ORC_MAX_SURFACES : n);
    for (int k = 0; k < S->n_chain; ++k) S->chain[k] = surf[k];
    S->aim_z = aim_z;
    S->aim_r = aim_r;
}

/* Paraxial marginal-ray trace (y, n*u) from the on-axis object point z_obj through the two
 * surfaces: gives the image plane and the lateral magnification M = (n u)_obj / (n u)_img. */
static void paraxial_image(const orc_scene *S, double z_obj, double *z_img, double *M)
{
    const double ng = S->c.n_glass, na = S->n_inf, R1 = S->R, R2 = -S->R;
    double u0 = 1.0;
    double y = u0 * (S->c.z_lens - z_obj);
    double nu = na * u0;
    nu = nu - y * (ng - na) / R1;          /* refraction at surface 1 */
    y = y + S->t * nu / ng;                /* transfer through the glass */
    nu = nu - y * (na - ng) / R2;          /* refraction at surface 2 */
    double ui = nu / na;
    *z_img = S->c.z_lens + S->t - y / ui;
    *M = (na * u0) / (na * ui);
}

/* ---------------------------------------------------------------- scene set-up */

orc_scene *orc_create(const orc_cfg *cfg, const float *rho)
{
    orc_scene *S = (orc_scene *)calloc(1, sizeof(orc_scene));
    S->c = *cfg;
    const int n3[3] = {cfg->nx, cfg->ny, cfg->nz};
    double diag2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        S->lo[a] = cfg->origin[a];
        S->hi[a] = cfg->origin[a] + (double)(n3[a] - 1) * cfg->spacing[a];
        diag2 += (S->hi[a] - S->lo[a]) * (S->hi[a] - S->lo[a]);
    }
    if (cfg->field_mode == ORC_GRID) field_prepare(S, rho);
    S->n_inf = 1.0 + cfg->K * cfg->rho_inf;                 /* eq. 1 outside the box */
    /* READING: the step variable of eqs. 3-5 is the parameter t with dt = ds / n (so that
     * dR/dt = T); a fixed arc length ds per step in the ambient medium gives h = ds / n_inf. */
    S->h = cfg->ds / S->n_inf;
    S->max_steps = cfg->max_steps > 0 ? cfg->max_steps : 4 * (int)ceil(sqrt(diag2) / cfg->ds) + 64;
    S->a = cfg->focal_length / (2.0 * cfg->f_number);
    S->t = cfg->thickness > 0.0 ? cfg->thickness : 0.1 * cfg->focal_length;
    S->clear = cfg->clear_radius > 0.0 ? cfg->clear_radius : 1.5 * S->a;
    /* thick lensmaker equation for R1 = -R2 = R (lens designed in vacuum):
     * 1/f = (n-1) [2/R - (n-1) t / (n R^2)]  =>  R = f (n-1) [1 + sqrt(1 - t / (n f))] */
    {
        double n = cfg->n_glass, f = cfg->focal_length;
        S->R = f * (n - 1.0) * (1.0 + sqrt(1.0 - S->t / (n * f)));
    }
    double zi, M;
    paraxial_image(S, cfg->z_focus, &zi, &M);
    S->z_sensor = isnan(cfg->z_sensor) ? zi : cfg->z_sensor;
    S->M = M;
    /* eq. 8 diffraction diameter.  READING: the factor pi printed in eq. 8 is taken out by
     * default (the Airy diameter of the cited references has none); sigma = d / 4, i.e. d read
     * as the 1/e^2 diameter of the Gaussian. */
    if (cfg->sigma_px > 0.0) {
        S->sigma_px = cfg->sigma_px;
    } else {
        double d = 2.44 * cfg->f_number * (fabs(M) + 1.0) * cfg->wavelength;
        if (cfg->dtau_with_pi) d *= M_PI;
        S->sigma_px = d / 4.0 / cfg->pitch;
    }
    S->r_fp = (int)ceil(3.0 * S->sigma_px);
    if (S->r_fp < 1) S->r_fp = 1;
    return S;
}

void orc_destroy(orc_scene *S)
{
    if (!S) return;
    free(S->dn); free(S->gx); free(S->gy); free(S->gz); free(S->mie);
    free(S);
}

/* derived quantities: R, z_sensor, M, sigma_px, n_inf, h, a, r_fp, t, clear, max_steps */
void orc_derived(const orc_scene *S, double out[11])
{
    out[0] = S->R; out[1] = S->z_sensor; out[2] = S->M; out[3] = S->sigma_px;
    out[4] = S->n_inf; out[5] = S->h; out[6] = S->a; out[7] = (double)S->r_fp;
    out[8] = S->t; out[9] = S->clear; out[10] = (double)S->max_steps;
}

/* ---------------------------------------------------------------- one ray */

/* Ray j of source src (x, y, z, w) with index s: steps 1-3 and the sensor hit. */
int orc_trace_ray(const orc_scene *S, const float src[4], int64_t s, int32_t j, orc_ray *out)
{
    memset(out, 0, sizeof(*out));
    out->ray_id = -1;
    double P0[3] = {src[0], src[1], src[2]};
    /* sec. 3.1: aperture point sampled uniformly by area on the disk of radius a */
    double uu[2];
    orc_ray_uniforms(S->c.seed, s, j, uu);
    const double aim_r = S->n_chain ? S->aim_r : S->a, aim_z = S->n_chain ? S->aim_z : S->c.z_lens;
    double r = aim_r * sqrt(uu[0]), phi = 2.0 * M_PI * uu[1];
    double L[3] = {r * cos(phi), r * sin(phi), aim_z};
    out->lens_point[0] = L[0]; out->lens_point[1] = L[1];
    double u[3] = {L[0] - P0[0], L[1] - P0[1], L[2] - P0[2]};
    double nu = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int a = 0; a < 3; ++a) u[a] /= nu;
    for (int a = 0; a < 3; ++a) out->dir0[a] = u[a];

    /* box entry: slab test; a source inside the box starts there */
    double R[3] = {P0[0], P0[1], P0[2]};
    int inside = 1;
    for (int a = 0; a < 3; ++a) if (P0[a] < S->lo[a] || P0[a] > S->hi[a]) inside = 0;
    int entered = inside;
    if (!inside) {
        double t0 = -INFINITY, t1 = INFINITY;
        int ax = -1, ok = 1;
        for (int a = 0; a < 3; ++a) {
            if (u[a] != 0.0) {
                double ta = (S->lo[a] - P0[a]) / u[a], tb = (S->hi[a] - P0[a]) / u[a];
                double tn = ta < tb ? ta : tb, tf = ta < tb ? tb : ta;
                if (tn > t0) { t0 = tn; ax = a; }
                if (tf < t1) t1 = tf;
            } else if (P0[a] < S->lo[a] || P0[a] > S->hi[a]) ok = 0;
        }
        if (ok && ax >= 0 && t0 <= t1 && t0 >= 0.0) {
            entered = 1;
            for (int a = 0; a < 3; ++a) R[a] = P0[a] + t0 * u[a];
            R[ax] = u[ax] > 0.0 ? S->lo[ax] : S->hi[ax];
            for (int a = 0; a < 3; ++a) {           /* rounding may leave a hair outside */
                if (R[a] < S->lo[a]) R[a] = S->lo[a];
                if (R[a] > S->hi[a]) R[a] = S->hi[a];
            }
        }
    }
    out->entered = entered;
    double dir[3] = {u[0], u[1], u[2]};
    if (entered) {
        /* inside: T = n dR/ds = n u (eq. 4) */
        double f[4];
        orc_field_eval(S, R, f);
        double n = 1.0 + f[0];
        double T[3] = {n * u[0], n * u[1], n * u[2]};
        int st = trace_volume(S, R, T);
        if (st < 0) { out->status = ORC_STEP_LIMIT; out->n_steps = S->max_steps; return out->status; }
        out->n_steps = st;
        double tn = sqrt(T[0] * T[0] + T[1] * T[1] + T[2] * T[2]);
        for (int a = 0; a < 3; ++a) dir[a] = T[a] / tn;
    }
    for (int a = 0; a < 3; ++a) { out->vol_exit_pos[a] = R[a]; out->vol_exit_dir[a] = dir[a]; }
    out->status = S->n_chain ? orc_chain_to_sensor(S, R, dir, out->sensor_px)
                             : orc_lens_to_sensor(S, R, dir, out->sensor_px);
    if (out->status == ORC_DEPOSITED) {
        int i0 = (int)floor(out->sensor_px[0]), j0 = (int)floor(out->sensor_px[1]);
        if (out->sensor_px[0] < 0.0 || out->sensor_px[1] < 0.0 ||
            i0 >= S->c.width || j0 >= S->c.height)
            out->status = ORC_OFF_SENSOR;
    }
    return out->status;
}

/* Fraction of a unit Gaussian spot (sigma in pixels) centred at x that falls in the pixel
 * column [i, i+1): (erf((i+1-x)/(sqrt2 sigma)) - erf((i-x)/(sqrt2 sigma))) / 2 (sec. 3.4). */
double orc_pixel_fraction(double x, int i, double sigma)
{
    double s = M_SQRT2 * sigma;
    return 0.5 * (erf(((double)i + 1.0 - x) / s) - erf(((double)i - x) / s));
}

/* ---------------------------------------------------------------- Mie radiance (sec. 3.1) */

/* Sets (n >= 2) or clears (n = 0) the Mie weighting of rays: a ray leaving its source along the
 * unit direction u is weighted by the table's intensity at the scattering angle
 * theta = acos(u . k) between u and the laser direction k, linearly interpolated between
 * theta_k = k pi / (n - 1).  READING: the paper weights by the Mie intensity at that angle
 * (sec. 3.1) without naming a polarisation; the table holds the unpolarised intensity. */
void orc_set_mie(orc_scene *S, const double *table, int n, const double laser[3])
{
    free(S->mie);
    S->mie = NULL;
    S->mie_n = 0;
    if (n < 2) return;
    S->mie = (double *)malloc((size_t)n * sizeof(double));
    memcpy(S->mie, table, (size_t)n * sizeof(double));
    S->mie_n = n;
    const double k = sqrt(laser[0] * laser[0] + laser[1] * laser[1] + laser[2] * laser[2]);
    for (int a = 0; a < 3; ++a) S->laser[a] = laser[a] / k;
}

/* Mie factor of a ray whose initial unit direction is u (1 without a table). */
double orc_mie_weight(const orc_scene *S, const double u[3])
{
    if (!S->mie) return 1.0;
    double c = u[0] * S->laser[0] + u[1] * S->laser[1] + u[2] * S->laser[2];
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    const double t = acos(c) / M_PI * (double)(S->mie_n - 1);
    int i = (int)floor(t);
    if (i > S->mie_n - 2) i = S->mie_n - 2;
    const double f = t - (double)i;
    return S->mie[i] * (1.0 - f) + S->mie[i + 1] * f;
}

/* ---------------------------------------------------------------- whole image */

/* Weight of a source's rays.  READING: the paper weights rays by the source's brightness without
 * bounds; here a weight is a fraction in [0, 1] (ray intensities then stay within one unit of the
 * fixed-point sensor), a weight beyond the range counts as the nearer end and a NaN weight as 0. */
static double source_weight(float w)
{
    return w > 0.0f ? (w < 1.0f ? (double)w : 1.0) : 0.0;
}

/* Deposits every ray of every source.  img_q: uint64 Q32.32 image (+=), img_f: double image
 * (+=), counts[8]: per-status ray counts (+=) then total RKN steps at counts[7].
 * Per-thread images are summed in thread order, so the result is deterministic for a given
 * thread count (the integer image is deterministic for any). */
int orc_render(const orc_scene *S, const float *src, int64_t n_src, int32_t rays_per_src,
               uint64_t *img_q, double *img_f, uint64_t *counts, int n_threads)
{
    const int W = S->c.width, H = S->c.height, rfp = S->r_fp;
    const size_t npx = (size_t)W * H;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#else
    n_threads = 1;
#endif
    uint64_t **tq = (uint64_t **)calloc((size_t)n_threads, sizeof(void *));
    double **tf = (double **)calloc((size_t)n_threads, sizeof(void *));
    uint64_t (*tc)[8] = calloc((size_t)n_threads, sizeof(*tc));
#pragma omp parallel num_threads(n_threads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        uint64_t *q = (uint64_t *)calloc(npx, sizeof(uint64_t));
        double *f = img_f ? (double *)calloc(npx, sizeof(double)) : NULL;
        double ex[64], ey[64];
        tq[tid] = q; tf[tid] = f;
#pragma omp for schedule(static, 4)
        for (int64_t s = 0; s < n_src; ++s) {
            const float *sp = src + 4 * s;
            for (int32_t j = 0; j < rays_per_src; ++j) {
                orc_ray ry;
                int st = orc_trace_ray(S, sp, s, j, &ry);
                tc[tid][st] += 1;
                tc[tid][7] += (uint64_t)ry.n_steps;
                if (st != ORC_DEPOSITED) continue;
                const double w = source_weight(sp[3]) * orc_mie_weight(S, ry.dir0);
                const double x = ry.sensor_px[0], y = ry.sensor_px[1];
                const int i0 = (int)floor(x), j0 = (int)floor(y);
                for (int d = -rfp; d <= rfp; ++d) {
                    ex[d + rfp] = orc_pixel_fraction(x, i0 + d, S->sigma_px);
                    ey[d + rfp] = orc_pixel_fraction(y, j0 + d, S->sigma_px);
                }
                for (int dj = -rfp; dj <= rfp; ++dj) {
                    int jj = j0 + dj;
                    if (jj < 0 || jj >= H) continue;
                    for (int di = -rfp; di <= rfp; ++di) {
                        int ii = i0 + di;
                        if (ii < 0 || ii >= W) continue;
                        double c = w * ex[di + rfp] * ey[dj + rfp];
                        q[(size_t)jj * W + ii] += (uint64_t)rint(c * 4294967296.0);
                        if (f) f[(size_t)jj * W + ii] += c;
                    }
                }
            }
        }
    }
    for (int t = 0; t < n_threads; ++t) {
        for (size_t p = 0; p < npx; ++p) {
            img_q[p] += tq[t][p];
            if (img_f) img_f[p] += tf[t][p];
        }
        if (counts) for (int k = 0; k < 8; ++k) counts[k] += tc[t][k];
        free(tq[t]); free(tf[t]);
    }
    free(tq); free(tf); free(tc);
    return 0;
}

/* Records for a list of ray ids (id = s * rays_per_src + j). */
int orc_trace_ids(const orc_scene *S, const float *src, int32_t rays_per_src,
                  const int64_t *ids, int64_t n, orc_ray *out, int n_threads)
{
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#endif
#pragma omp parallel for schedule(dynamic, 16) num_threads(n_threads)
    for (int64_t k = 0; k < n; ++k) {
        int64_t s = ids[k] / rays_per_src;
        int32_t j = (int32_t)(ids[k] % rays_per_src);
        orc_trace_ray(S, src + 4 * s, s, j, &out[k]);
        out[k].ray_id = ids[k];
    }
    return 0;
}

/* 16-bit readout of a Q32.32 image: v = q 2^-32, out = min(65535, round_half_even(v gain)),
 * gain = 65535 / max(v) when gain <= 0 (sec. 3.4: about 1e4 rays per source give 16 bits). */
void orc_readout_u16(const uint64_t *q, int64_t n, double gain, uint16_t *out)
{
    if (!(gain > 0.0)) {
        uint64_t mx = 0;
        for (int64_t p = 0; p < n; ++p) if (q[p] > mx) mx = q[p];
        double vmax = (double)mx / 4294967296.0;
        gain = vmax > 0.0 ? 65535.0 / vmax : 0.0;
    }
    for (int64_t p = 0; p < n; ++p) {
        double r = rint((double)q[p] / 4294967296.0 * gain);
        out[p] = (uint16_t)(r < 65535.0 ? r : 65535.0);
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- BOS theory (sec. 4, eq. 9) */

/* Paraxial image plane and lateral magnification of the object plane z_obj: out = (z, M). */
void orc_paraxial(const orc_scene *S, double z_obj, double out[2])
{
    paraxial_image(S, z_obj, &out[0], &out[1]);
}

/* Eq. 9 on a regular grid of the dot plane z = z_dots, node (i, j) at (x0 + i dx, y0 + j dy):
 * the image displacement, in pixels, of a dot seen through the density box,
 *     dX = |M| Z_D / n0 * integral over the box depth of (dn/dx, dn/dy) dz,
 * taken along the chief ray from the node to the centre of the aperture stop (the front vertex
 * on the axis).  M: magnification of the dot plane; Z_D: distance from the dot plane to the mid
 * plane of the box; n0: ambient index.  The sign is that of the unflipped sensor: a ray bent
 * towards +x seems to come from a point at -x on the dot plane, whose inverted image lies at +x.
 * READING: the integral is the midpoint rule with `samples` points over [z_min, z_max] of the
 * box; points of the chief ray beyond the box's x-y extent lie in the ambient medium and add
 * nothing.  out: [ny][nx][2]. */
void orc_bos_theory_map(const orc_scene *S, double x0, double y0, double dx, double dy, int nx,
                        int ny, double z_dots, int samples, double *out)
{
    double zi, M;
    paraxial_image(S, z_dots, &zi, &M);
    const double zc = 0.5 * (S->lo[2] + S->hi[2]);
    const double scale = fabs(M) * (zc - z_dots) / (S->n_inf * S->c.pitch);
    const double dz = (S->hi[2] - S->lo[2]) / (double)samples;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const double X = x0 + (double)i * dx, Y = y0 + (double)j * dy;
            double sx = 0.0, sy = 0.0;
            for (int k = 0; k < samples; ++k) {
                const double z = S->lo[2] + ((double)k + 0.5) * dz;
                const double f = (z - z_dots) / (S->c.z_lens - z_dots);
                const double R[3] = {X * (1.0 - f), Y * (1.0 - f), z};
                if (R[0] < S->lo[0] || R[0] > S->hi[0] || R[1] < S->lo[1] || R[1] > S->hi[1]) continue;
                double g[4];
                orc_field_eval(S, R, g);
                sx += g[1];
                sy += g[2];
            }
            out[2 * ((size_t)j * nx + i)] = scale * sx * dz;
            out[2 * ((size_t)j * nx + i) + 1] = scale * sy * dz;
        }
}

/* ---------------------------------------------------------------- PIV frame pairs (sec. 1) */

/* Velocity at x from float32 node values vel[(k ny + j) nx + i][3]: trilinear in the cell holding
 * the point, a point outside the grid first moved onto it (edge extension). */
static void velocity_at(const float *vel, int nx, int ny, int nz, const double org[3], const double sp[3],
                        const double x[3], double u[3])
{
    const int n3[3] = {nx, ny, nz};
    int c[3];
    double w[3];
    for (int a = 0; a < 3; ++a) {
        double f = (x[a] - org[a]) / sp[a];
        if (f < 0.0) f = 0.0;
        if (f > (double)(n3[a] - 1)) f = (double)(n3[a] - 1);
        int i = (int)floor(f);
        if (i > n3[a] - 2) i = n3[a] - 2;
        c[a] = i;
        w[a] = f - (double)i;
    }
    for (int q = 0; q < 3; ++q) {
        double v = 0.0;
        for (int dk = 0; dk < 2; ++dk)
            for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di) {
                    const double wt = (di ? w[0] : 1.0 - w[0]) * (dj ? w[1] : 1.0 - w[1]) * (dk ? w[2] : 1.0 - w[2]);
                    const size_t node = ((size_t)(c[2] + dk) * ny + (size_t)(c[1] + dj)) * nx + (size_t)(c[0] + di);
                    v += wt * (double)vel[3 * node + q];
                }
        u[q] = v;
    }
}

/* Second frame of a PIV pair: every particle x advanced by dx/dt = u(x) over dt with `substeps`
 * classical fourth-order Runge-Kutta steps (k1 = u(x), k2 = u(x + h k1/2), k3 = u(x + h k2/2),
 * k4 = u(x + h k3), x += h (k1 + 2 k2 + 2 k3 + k4) / 6).  READING: the paper names the use (sec. 1:
 * velocity from the particle displacement between two frames) but no displacement rule; a
 * prescribed field integrated over the frame interval is the plain definition.  out: [n][4] with
 * the weight copied. */
void orc_displace_sources(const float *src, int64_t n, const float *vel, int nx, int ny, int nz,
                          const double org[3], const double sp[3], double dt, int substeps, double *out)
{
    const double h = dt / (double)substeps;
    for (int64_t s = 0; s < n; ++s) {
        double x[3] = {src[4 * s], src[4 * s + 1], src[4 * s + 2]};
        for (int m = 0; m < substeps; ++m) {
            double k1[3], k2[3], k3[3], k4[3], p[3];
            velocity_at(vel, nx, ny, nz, org, sp, x, k1);
            for (int a = 0; a < 3; ++a) p[a] = x[a] + 0.5 * h * k1[a];
            velocity_at(vel, nx, ny, nz, org, sp, p, k2);
            for (int a = 0; a < 3; ++a) p[a] = x[a] + 0.5 * h * k2[a];
            velocity_at(vel, nx, ny, nz, org, sp, p, k3);
            for (int a = 0; a < 3; ++a) p[a] = x[a] + h * k3[a];
            velocity_at(vel, nx, ny, nz, org, sp, p, k4);
            for (int a = 0; a < 3; ++a) x[a] += h * (k1[a] + 2.0 * k2[a] + 2.0 * k3[a] + k4[a]) / 6.0;
        }
        out[4 * s] = x[0]; out[4 * s + 1] = x[1]; out[4 * s + 2] = x[2];
        out[4 * s + 3] = (double)src[4 * s + 3];
    }
}
