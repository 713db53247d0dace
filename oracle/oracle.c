/*
 * oracle.c -- plain FP64 CPU oracle for the full-3D SPARKLING energy,
 * gradient and projection path (arXiv 2108.02991).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark call it.  It shares no code, header, table or
 * constant with the HIP library, and it never reads anything the HIP path
 * produced.  Every quantity is computed straight from its definition in the
 * paper, in double precision, with Neumaier-compensated sums and OpenMP over
 * independent targets/shots only (each target's sum runs in one fixed order).
 *
 * Definitions followed (all from the paper's Theory section):
 *   - objective F = F^a - F^r ("3D SPARKLING formulation": attraction term
 *     F^a = (1/p) sum_i integral H(x - K[i]) rho(x) dx, repulsion term
 *     F^r = 1/(2p^2) sum_{i,j} H(K[i] - K[j]), H = Euclidean norm, or the
 *     logarithm of the norm that the same section names as an alternative,
 *     regularised by eps > 0);
 *   - the attraction integral taken over the discretised density (Sec.
 *     "Evaluating F^a and its gradient": rho sampled on a grid), evaluated as
 *     the direct weighted sum over grid cells;
 *   - gradients (same section, attraction derivative; Sec. "Evaluating F^r
 *     and its gradient", repulsion derivative with the factor read as H'(r));
 *   - constraint set Q (Sec. "3D K-space sampling", rotation-invariant speed
 *     and slew bounds, box, echo-time point) and the normalised bounds
 *     alpha, beta of the same section;
 *   - the per-shot projection (supplement, "Multi-shot projection step"),
 *     solved by accelerated proximal gradient on the dual problem;
 *   - one projected gradient step with fixed then Barzilai-Borwein step sizes
 *     (Sec. "Choice of step size").
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - H(0) = 0 and grad H(0) = 0 (minimum-norm subgradient) for coincident
 *     samples; with a regularised kernel H = sqrt(r^2 + eps^2) both follow
 *     from the formula;
 *   - rho is a cell-centred G^3 grid over [-L, L]^3, x fastest, weights as
 *     given (the caller normalises them);
 *   - the projection's dual iteration, step 1/20 and cold start are fixed
 *     below; its speed/slew feasibility after finitely many iterations is
 *     approximate, box and echo-time constraints are exact.
 *
 * Status codes: 0 ok, -1 invalid argument.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Neumaier-compensated running sum.                                   */
/* ------------------------------------------------------------------ */
typedef struct {
    double s, c;
} csum;

static void cs_add(csum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double cs_get(const csum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* Kernel H and its gradient.                                          */
/* kern = 0 (distance): H(d) = |d|_2 (eps = 0) or sqrt(|d|^2 + eps^2)  */
/*   (regularised kernel of Sec. "Choice of step size");               */
/*   grad H(d) = d / H(d), and 0 at d = 0.                             */
/* kern = 1 (logarithmic, the alternative kernel the "3D SPARKLING      */
/*   formulation" mentions), regularised: H(d) = log sqrt(|d|^2 + eps^2) */
/*   = log(|d|^2 + eps^2) / 2, grad H(d) = d / (|d|^2 + eps^2); eps > 0. */
/* ------------------------------------------------------------------ */
static int bad_kernel(double eps, int kern)
{
    if (!(eps >= 0.0))
        return 1;
    if (kern == 0)
        return 0;
    return kern != 1 || !(eps > 0.0);
}

static double kernel_h(double dx, double dy, double dz, double eps, int kern)
{
    double s = dx * dx + dy * dy + dz * dz + eps * eps;
    return kern == 1 ? 0.5 * log(s) : sqrt(s);
}

static void kernel_grad(double dx, double dy, double dz, double eps, int kern, double out[3])
{
    double den;
    if (kern == 1)
        den = dx * dx + dy * dy + dz * dz + eps * eps;
    else
        den = kernel_h(dx, dy, dz, eps, kern);
    if (den == 0.0) {
        out[0] = out[1] = out[2] = 0.0;
    } else {
        out[0] = dx / den;
        out[1] = dy / den;
        out[2] = dz / den;
    }
}

/* Centre of grid cell `idx` along one axis: -L + (idx + 1/2) * (2L / G). */
static double cell_centre(int64_t idx, int64_t G, double L)
{
    return -L + ((double)idx + 0.5) * (2.0 * L / (double)G);
}

/* ------------------------------------------------------------------ */
/* Per-target sums.  For each requested target i:                       */
/*   ua[t]  = sum_v rho_v H(K[i] - x_v)                                  */
/*   ga[t]  = sum_v rho_v grad H(K[i] - x_v)          (3 components)     */
/*   ur[t]  = sum_j H(K[i] - K[j])        (all j, j = i gives H(0))      */
/*   gr[t]  = sum_j grad H(K[i] - K[j])   (3 components; j = i gives 0)  */
/* Component c of target t is stored at [c * n_t + t].                   */
/* ------------------------------------------------------------------ */
static void target_sums(int64_t p, const double *kx, const double *ky, const double *kz,
                        int64_t G, double L, const double *rho, double eps, int kern,
                        int64_t i, double *ua, double ga[3], double *ur, double gr[3])
{
    csum sa = {0, 0}, sr = {0, 0};
    csum a3[3] = {{0, 0}, {0, 0}, {0, 0}}, r3[3] = {{0, 0}, {0, 0}, {0, 0}};
    double xi = kx[i], yi = ky[i], zi = kz[i];
    double g[3];

    for (int64_t iz = 0; iz < G; ++iz) {
        double zv = cell_centre(iz, G, L);
        for (int64_t iy = 0; iy < G; ++iy) {
            double yv = cell_centre(iy, G, L);
            for (int64_t ix = 0; ix < G; ++ix) {
                double xv = cell_centre(ix, G, L);
                double w = rho[ix + G * (iy + G * iz)];
                double dx = xi - xv, dy = yi - yv, dz = zi - zv;
                cs_add(&sa, w * kernel_h(dx, dy, dz, eps, kern));
                kernel_grad(dx, dy, dz, eps, kern, g);
                for (int c = 0; c < 3; ++c)
                    cs_add(&a3[c], w * g[c]);
            }
        }
    }
    for (int64_t j = 0; j < p; ++j) {
        double dx = xi - kx[j], dy = yi - ky[j], dz = zi - kz[j];
        cs_add(&sr, kernel_h(dx, dy, dz, eps, kern));
        kernel_grad(dx, dy, dz, eps, kern, g);
        for (int c = 0; c < 3; ++c)
            cs_add(&r3[c], g[c]);
    }
    *ua = cs_get(&sa);
    *ur = cs_get(&sr);
    for (int c = 0; c < 3; ++c) {
        ga[c] = cs_get(&a3[c]);
        gr[c] = cs_get(&r3[c]);
    }
}

/*
 * Gradient of F at a list of targets (attraction derivative of Sec.
 * "Evaluating F^a and its gradient", repulsion derivative of Sec.
 * "Evaluating F^r and its gradient"):
 *   dFa[i] = (1/p)   sum_v rho_v grad H(K[i] - x_v)
 *   dFr[i] = (1/p^2) sum_j grad H(K[i] - K[j])
 *   dF[i]  = dFa[i] - dFr[i]
 * Also returns the per-target potentials ua, ur (unscaled sums of H).
 * Any output pointer may be NULL.  Layout: component c of target t at
 * [c * n_t + t].
 */
int orc_grad(int64_t p, const double *kx, const double *ky, const double *kz,
             int64_t G, double L, const double *rho, double eps, int kern,
             int64_t n_t, const int64_t *targets,
             double *dF, double *dFa, double *dFr, double *ua, double *ur)
{
    if (p < 1 || G < 1 || n_t < 0 || !kx || !ky || !kz || !rho || !targets || bad_kernel(eps, kern))
        return -1;
    for (int64_t t = 0; t < n_t; ++t)
        if (targets[t] < 0 || targets[t] >= p)
            return -1;
    double inv_p = 1.0 / (double)p;
    double inv_p2 = inv_p * inv_p;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < n_t; ++t) {
        double a, r, ga[3], gr[3];
        target_sums(p, kx, ky, kz, G, L, rho, eps, kern, targets[t], &a, ga, &r, gr);
        for (int c = 0; c < 3; ++c) {
            double fa = ga[c] * inv_p, fr = gr[c] * inv_p2;
            if (dFa) dFa[c * n_t + t] = fa;
            if (dFr) dFr[c * n_t + t] = fr;
            if (dF) dF[c * n_t + t] = fa - fr;
        }
        if (ua) ua[t] = a;
        if (ur) ur[t] = r;
    }
    return 0;
}

/*
 * Energies of the objective ("3D SPARKLING formulation"):
 *   Fa = (1/p) sum_i sum_v rho_v H(K[i] - x_v)
 *   Fr = 1/(2 p^2) sum_{i,j} H(K[i] - K[j])
 *   F  = Fa - Fr
 * out[0..2] = F, Fa, Fr.
 */
int orc_energy(int64_t p, const double *kx, const double *ky, const double *kz,
               int64_t G, double L, const double *rho, double eps, int kern, double out[3])
{
    if (p < 1 || G < 1 || !kx || !ky || !kz || !rho || !out || bad_kernel(eps, kern))
        return -1;
    double *ua = malloc(sizeof(double) * p), *ur = malloc(sizeof(double) * p);
    int64_t *idx = malloc(sizeof(int64_t) * p);
    if (!ua || !ur || !idx) {
        free(ua); free(ur); free(idx);
        return -1;
    }
    for (int64_t i = 0; i < p; ++i)
        idx[i] = i;
    orc_grad(p, kx, ky, kz, G, L, rho, eps, kern, p, idx, NULL, NULL, NULL, ua, ur);
    csum sa = {0, 0}, sr = {0, 0};
    for (int64_t i = 0; i < p; ++i) {
        cs_add(&sa, ua[i]);
        cs_add(&sr, ur[i]);
    }
    double fa = cs_get(&sa) / (double)p;
    double fr = cs_get(&sr) / (2.0 * (double)p * (double)p);
    out[0] = fa - fr;
    out[1] = fa;
    out[2] = fr;
    free(ua); free(ur); free(idx);
    return 0;
}

/*
 * Self-energy of the discretised density, E_rho = 1/2 sum_{u,v} rho_u rho_v
 * H(x_u - x_v).  F - E_rho is the non-negative discrepancy between the
 * sample measure and rho (H = |.| is conditionally negative definite).
 */
int orc_rho_self_energy(int64_t G, double L, const double *rho, double eps, int kern, double *out)
{
    if (G < 1 || !rho || !out || bad_kernel(eps, kern))
        return -1;
    int64_t M = G * G * G;
    double *row = malloc(sizeof(double) * M);
    if (!row)
        return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t u = 0; u < M; ++u) {
        double xu = cell_centre(u % G, G, L);
        double yu = cell_centre((u / G) % G, G, L);
        double zu = cell_centre(u / (G * G), G, L);
        csum s = {0, 0};
        for (int64_t v = 0; v < M; ++v) {
            double xv = cell_centre(v % G, G, L);
            double yv = cell_centre((v / G) % G, G, L);
            double zv = cell_centre(v / (G * G), G, L);
            cs_add(&s, rho[v] * kernel_h(xu - xv, yu - yv, zu - zv, eps, kern));
        }
        row[u] = rho[u] * cs_get(&s);
    }
    csum tot = {0, 0};
    for (int64_t u = 0; u < M; ++u)
        cs_add(&tot, row[u]);
    *out = 0.5 * cs_get(&tot);
    free(row);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Normalised speed and slew bounds (Sec. "3D K-space sampling"):       */
/*   alpha = min(gamma_bar G_max, 1/(FOV dwell)) / K_max                */
/*   beta  = gamma_bar S_max / K_max                                    */
/* in units where K_max maps to 1 per second (resp. second^2).  One     */
/* raster step of a trajectory living in [-L, L]^3 may then move at     */
/* most a = alpha * raster * L and change speed by b = beta raster^2 L. */
/* gamma_bar is the gyromagnetic ratio already divided by 2 pi.         */
/* ------------------------------------------------------------------ */
int orc_alpha_beta(double gmax, double smax, double raster_dt, double dwell_dt,
                   double fov, double kmax, double gamma_bar, double half_width,
                   double *a, double *b)
{
    if (!(gmax > 0) || !(smax > 0) || !(raster_dt > 0) || !(dwell_dt > 0) || !(fov > 0) ||
        !(kmax > 0) || !(gamma_bar > 0) || !(half_width > 0) || !a || !b)
        return -1;
    double grad_rate = gamma_bar * gmax;
    double nyquist_rate = 1.0 / (fov * dwell_dt);
    double alpha = (grad_rate < nyquist_rate ? grad_rate : nyquist_rate) / kmax;
    double beta = gamma_bar * smax / kmax;
    *a = alpha * raster_dt * half_width;
    *b = beta * raster_dt * raster_dt * half_width;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Per-shot projection onto the constraint set (supplement, "Multi-shot */
/* projection step"): s* = argmin_{s in Q} 1/2 |s - k|^2 with           */
/*   Q = { |s|_inf <= L, s[te] = 0, max_n |s[n+1]-s[n]| <= a,           */
/*         max_n |s[n+2]-2s[n+1]+s[n]| <= b }                           */
/* (norms over the 3 coordinates of one sample: the rotation-invariant  */
/* mixed norm).  Accelerated proximal gradient (FISTA) on the dual:     */
/*   s(q, r) = P0(k - D1^T q - D2^T r),  P0 = box clamp then s[te] = 0;  */
/*   q+ = shrink(qh + tau D1 s, tau a),  r+ = shrink(rh + tau D2 s, tau b) */
/*   t+ = (1 + sqrt(1 + 4 t^2)) / 2,  qh = q+ + ((t-1)/t+)(q+ - q), ...  */
/* with tau = 1/20 (|D1|^2 + |D2|^2 <= 4 + 16), q = qh = r = rh = 0 and */
/* t = 1 at the start; the result is P0(k - D1^T q - D2^T r) of the     */
/* last (non-extrapolated) dual iterate.                                */
/* Every operation below is written in one fixed order.                 */
/* ------------------------------------------------------------------ */
static double clamp_box(double z, double L)
{
    if (z < -L) return -L;
    if (z > L) return L;
    return z;    /* NaN stays NaN */
}

/* s[m] = P0(k[m] - (D1^T q)[m] - (D2^T r)[m]) for one coordinate.
 * (D1^T q)[m] = q[m-1] - q[m],  (D2^T r)[m] = r[m-2] - 2 r[m-1] + r[m],
 * entries outside q[0..Ns-2], r[0..Ns-3] read as 0. */
static double primal_coord(const double *k, const double *q, const double *r,
                           int64_t Ns, int64_t m, double L)
{
    double qa = (m >= 1) ? q[m - 1] : 0.0;
    double qb = (m <= Ns - 2) ? q[m] : 0.0;
    double ra = (m >= 2) ? r[m - 2] : 0.0;
    double rb = (m >= 1 && m - 1 <= Ns - 3) ? r[m - 1] : 0.0;
    double rc = (m <= Ns - 3) ? r[m] : 0.0;
    double d1t = qa - qb;
    double d2t = (ra - 2.0 * rb) + rc;
    return clamp_box((k[m] - d1t) - d2t, L);
}

static void shrink3(double z[3], double thr)
{
    double nrm = sqrt((z[0] * z[0] + z[1] * z[1]) + z[2] * z[2]);
    double f = (nrm > thr) ? (1.0 - thr / nrm) : 0.0;
    z[0] = z[0] * f;
    z[1] = z[1] * f;
    z[2] = z[2] * f;
}

/* Rotation-variant bounds (per-axis |.| <= bound, the l_inf form noted in
 * Sec. "3D K-space sampling"): the dual prox is soft-thresholding of each
 * coordinate on its own, z * max(0, 1 - thr/|z|). */
static void shrink_each(double z[3], double thr)
{
    for (int c = 0; c < 3; ++c) {
        double m = fabs(z[c]);
        double f = (m > thr) ? (1.0 - thr / m) : 0.0;
        z[c] = z[c] * f;
    }
}

/* duals: NULL (every dual variable starts at 0), or this shot's 6*Ns doubles,
 * q then r, [c * Ns + n] each (q for n < Ns-1, r for n < Ns-2, the rest 0):
 * the iteration starts from them (warm start) and leaves its last dual
 * iterate there. */
static void project_shot(int64_t Ns, double *xyz[3], double L, double a, double b,
                         int64_t te, int n_pit, int rv, double *buf, double *duals)
{
    /* buf holds k[3][Ns], s[3][Ns], q,qh,qn[3][Ns], r,rh,rn[3][Ns] */
    double *k = buf, *s = k + 3 * Ns;
    double *q = s + 3 * Ns, *qh = q + 3 * Ns, *qn = qh + 3 * Ns;
    double *r = qn + 3 * Ns, *rh = r + 3 * Ns, *rn = rh + 3 * Ns;
    const double tau = 1.0 / 20.0;
    const double thr_a = tau * a, thr_b = tau * b;

    for (int c = 0; c < 3; ++c)
        for (int64_t m = 0; m < Ns; ++m) {
            k[c * Ns + m] = xyz[c][m];
            double q0 = 0.0, r0 = 0.0;
            if (duals) {
                q0 = (m + 1 < Ns) ? duals[c * Ns + m] : 0.0;
                r0 = (m + 2 < Ns) ? duals[(3 + c) * Ns + m] : 0.0;
            }
            q[c * Ns + m] = qh[c * Ns + m] = q0;
            r[c * Ns + m] = rh[c * Ns + m] = r0;
        }
    double t = 1.0;
    for (int it = 0; it < n_pit; ++it) {
        for (int c = 0; c < 3; ++c)
            for (int64_t m = 0; m < Ns; ++m)
                s[c * Ns + m] = primal_coord(k + c * Ns, qh + c * Ns, rh + c * Ns, Ns, m, L);
        if (te >= 0)
            for (int c = 0; c < 3; ++c)
                s[c * Ns + te] = 0.0;
        for (int64_t n = 0; n + 1 < Ns; ++n) {
            double z[3];
            for (int c = 0; c < 3; ++c) {
                const double *sc = s + c * Ns;
                z[c] = qh[c * Ns + n] + tau * (sc[n + 1] - sc[n]);
            }
            if (rv)
                shrink_each(z, thr_a);
            else
                shrink3(z, thr_a);
            for (int c = 0; c < 3; ++c)
                qn[c * Ns + n] = z[c];
        }
        for (int64_t n = 0; n + 2 < Ns; ++n) {
            double z[3];
            for (int c = 0; c < 3; ++c) {
                const double *sc = s + c * Ns;
                z[c] = rh[c * Ns + n] + tau * ((sc[n + 2] - 2.0 * sc[n + 1]) + sc[n]);
            }
            if (rv)
                shrink_each(z, thr_b);
            else
                shrink3(z, thr_b);
            for (int c = 0; c < 3; ++c)
                rn[c * Ns + n] = z[c];
        }
        double tn = (1.0 + sqrt(1.0 + 4.0 * t * t)) / 2.0;
        double mom = (t - 1.0) / tn;
        for (int c = 0; c < 3; ++c) {
            for (int64_t n = 0; n + 1 < Ns; ++n) {
                int64_t o = c * Ns + n;
                qh[o] = qn[o] + mom * (qn[o] - q[o]);
                q[o] = qn[o];
            }
            for (int64_t n = 0; n + 2 < Ns; ++n) {
                int64_t o = c * Ns + n;
                rh[o] = rn[o] + mom * (rn[o] - r[o]);
                r[o] = rn[o];
            }
        }
        t = tn;
    }
    for (int c = 0; c < 3; ++c)
        for (int64_t m = 0; m < Ns; ++m)
            xyz[c][m] = primal_coord(k + c * Ns, q + c * Ns, r + c * Ns, Ns, m, L);
    if (te >= 0)
        for (int c = 0; c < 3; ++c)
            xyz[c][te] = 0.0;
    if (duals)
        for (int c = 0; c < 3; ++c)
            for (int64_t m = 0; m < Ns; ++m) {
                duals[c * Ns + m] = (m + 1 < Ns) ? q[c * Ns + m] : 0.0;
                duals[(3 + c) * Ns + m] = (m + 2 < Ns) ? r[c * Ns + m] : 0.0;
            }
}

/* Project every shot of K (3 arrays of Nc*Ns, shot-lexicographic) in place.
 * rv = 0: rotation-invariant bounds on |.|_2 per sample; rv = 1: per-axis bounds.
 * duals: NULL (cold start), or Nc * 6 * Ns doubles, shot c's at c * 6 * Ns
 * (warm start in, last dual iterate out; see project_shot). */
int orc_project(int64_t Nc, int64_t Ns, double *kx, double *ky, double *kz,
                double L, double a, double b, int64_t te, int n_pit, int rv, double *duals)
{
    if (Nc < 1 || Ns < 2 || !kx || !ky || !kz || !(L > 0) || !(a > 0) || !(b > 0) ||
        te < -1 || te >= Ns || n_pit < 0)
        return -1;
    int fail = 0;
#pragma omp parallel
    {
        double *buf = malloc(sizeof(double) * 24 * (size_t)Ns);
        if (!buf) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t c = 0; c < Nc; ++c) {
                double *xyz[3] = {kx + c * Ns, ky + c * Ns, kz + c * Ns};
                project_shot(Ns, xyz, L, a, b, te, n_pit, rv, buf,
                             duals ? duals + c * 6 * Ns : NULL);
            }
            free(buf);
        }
    }
    return fail ? -1 : 0;
}

/* NaN-propagating maximum: once NaN, stays NaN. */
static double vmax(double m, double x)
{
    if (m != m) return m;
    if (x != x || x > m) return x;
    return m;
}

/*
 * Normalised constraint violations of K (Sec. "3D K-space sampling"):
 *   out[0] = max |s[n+1] - s[n]| / a          (speed; <= 1 is feasible)
 *   out[1] = max |s[n+2] - 2 s[n+1] + s[n]| / b  (slew)
 * with |.| the Euclidean norm of the 3 coordinates (rv = 0) or their
 * largest magnitude (rv = 1, per-axis bounds);
 *   out[2] = max |s|_inf / L                  (box)
 *   out[3] = max over shots |s[te]|           (echo-time point; 0 if te < 0)
 */
static double norm3(double dx, double dy, double dz, int rv)
{
    if (rv)
        return vmax(vmax(fabs(dx), fabs(dy)), fabs(dz));
    return sqrt((dx * dx + dy * dy) + dz * dz);
}

int orc_constraint_check(int64_t Nc, int64_t Ns, const double *kx, const double *ky,
                         const double *kz, double L, double a, double b, int64_t te, int rv,
                         double out[4])
{
    if (Nc < 1 || Ns < 2 || !kx || !ky || !kz || !(L > 0) || !(a > 0) || !(b > 0) ||
        te < -1 || te >= Ns || !out)
        return -1;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    for (int64_t c = 0; c < Nc; ++c) {
        const double *x = kx + c * Ns, *y = ky + c * Ns, *z = kz + c * Ns;
        for (int64_t n = 0; n + 1 < Ns; ++n) {
            double dx = x[n + 1] - x[n], dy = y[n + 1] - y[n], dz = z[n + 1] - z[n];
            m0 = vmax(m0, norm3(dx, dy, dz, rv) / a);
        }
        for (int64_t n = 0; n + 2 < Ns; ++n) {
            double dx = (x[n + 2] - 2.0 * x[n + 1]) + x[n];
            double dy = (y[n + 2] - 2.0 * y[n + 1]) + y[n];
            double dz = (z[n + 2] - 2.0 * z[n + 1]) + z[n];
            m1 = vmax(m1, norm3(dx, dy, dz, rv) / b);
        }
        for (int64_t n = 0; n < Ns; ++n) {
            m2 = vmax(m2, fabs(x[n]) / L);
            m2 = vmax(m2, fabs(y[n]) / L);
            m2 = vmax(m2, fabs(z[n]) / L);
        }
        if (te >= 0)
            m3 = vmax(m3, sqrt((x[te] * x[te] + y[te] * y[te]) + z[te] * z[te]));
    }
    out[0] = m0; out[1] = m1; out[2] = m2; out[3] = m3;
    return 0;
}

/*
 * One projected gradient step (projected gradient descent equation of the
 * "3D SPARKLING formulation" section; step-size policy of Sec. "Choice of
 * step size"):
 *   g = grad F(K);  eta = eta_fixed for iter < 20, afterwards
 *   eta = (s.s)/(s.y) with s = K - K_prev, y = g - g_prev over all 3p
 *   coordinates, clamped to [0.1, 10] eta_fixed, and eta_fixed if s.y <= 0;
 *   K_prev = K, g_prev = g, K = P_Q(K - eta g).
 * K, k_prev, g_prev are 3 arrays of p each, laid out [c * p + i].
 * info_out[0..9] = eta, F, Fa, Fr, viol[0..3], bb_used, and the quotient s.s/s.y
 * before the clamp (NaN below iteration 20).
 */
int orc_step(int64_t Nc, int64_t Ns, double *K, int64_t G, double L, const double *rho,
             double eps, int kern, double a, double b, int64_t te, int n_pit, int rv,
             double *k_prev, double *g_prev, int64_t iter, double eta_fixed,
             double info_out[10], double *duals)
{
    int64_t p = Nc * Ns;
    if (Nc < 1 || Ns < 2 || !K || !rho || !k_prev || !g_prev || !info_out || !(eta_fixed > 0) ||
        iter < 0)
        return -1;
    double *g = malloc(sizeof(double) * 3 * p);
    int64_t *idx = calloc((size_t)p, sizeof(int64_t));
    double *ua = malloc(sizeof(double) * p), *ur = malloc(sizeof(double) * p);
    if (!g || !idx || !ua || !ur) {
        free(g); free(idx); free(ua); free(ur);
        return -1;
    }
    for (int64_t i = 0; i < p; ++i)
        idx[i] = i;
    int rc = orc_grad(p, K, K + p, K + 2 * p, G, L, rho, eps, kern, p, idx, g, NULL, NULL, ua, ur);
    if (rc) {
        free(g); free(idx); free(ua); free(ur);
        return rc;
    }
    csum sa = {0, 0}, sr = {0, 0};
    for (int64_t i = 0; i < p; ++i) {
        cs_add(&sa, ua[i]);
        cs_add(&sr, ur[i]);
    }
    double fa = cs_get(&sa) / (double)p;
    double fr = cs_get(&sr) / (2.0 * (double)p * (double)p);

    double eta = eta_fixed, bb_used = 0.0, quotient = NAN;
    if (iter >= 20) {
        csum ss = {0, 0}, sy = {0, 0};
        for (int64_t e = 0; e < 3 * p; ++e) {
            double sv = K[e] - k_prev[e], yv = g[e] - g_prev[e];
            cs_add(&ss, sv * sv);
            cs_add(&sy, sv * yv);
        }
        double vss = cs_get(&ss), vsy = cs_get(&sy);
        quotient = vss / vsy;
        if (vsy > 0.0 && isfinite(vss / vsy)) {
            eta = vss / vsy;
            if (eta < 0.1 * eta_fixed) eta = 0.1 * eta_fixed;
            if (eta > 10.0 * eta_fixed) eta = 10.0 * eta_fixed;
            bb_used = 1.0;
        }
    }
    for (int64_t e = 0; e < 3 * p; ++e) {
        k_prev[e] = K[e];
        g_prev[e] = g[e];
        K[e] = K[e] - eta * g[e];
    }
    double viol[4];
    rc = orc_project(Nc, Ns, K, K + p, K + 2 * p, L, a, b, te, n_pit, rv, duals);
    if (!rc)
        rc = orc_constraint_check(Nc, Ns, K, K + p, K + 2 * p, L, a, b, te, rv, viol);
    info_out[0] = eta;
    info_out[1] = fa - fr;
    info_out[2] = fa;
    info_out[3] = fr;
    for (int c = 0; c < 4; ++c)
        info_out[4 + c] = rc ? NAN : viol[c];
    info_out[8] = bb_used;
    info_out[9] = quotient;
    free(g); free(idx); free(ua); free(ur);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Central finite difference of F along a direction delta, without      */
/* cancellation:  H(d + h D) - H(d - h D) = 4 h (d . D) /               */
/* (H(d + h D) + H(d - h D)), exact algebra for H = sqrt(|.|^2 + eps^2), */
/* and the log1p form below for the logarithmic kernel.                 */
/* Returns (F(K + h delta) - F(K - h delta)) / (2h).  Pairs in which     */
/* neither sample moves contribute exactly 0 and are skipped; the       */
/* repulsion double sum is symmetric in (i, j), so an ordered pair with  */
/* one moving end is counted twice from that end.                        */
/* ------------------------------------------------------------------ */
static double pair_diff(double dx, double dy, double dz, double ex, double ey, double ez,
                        double h, double eps, int kern)
{
    double num = 4.0 * h * ((dx * ex + dy * ey) + dz * ez);
    if (kern == 1) {
        /* log kernel: with A = |d + hD|^2 + eps^2 and B = |d - hD|^2 + eps^2,
         * A - B = 4 h (d . D), so H(+) - H(-) = log1p((A - B) / B) / 2. */
        double mx = dx - h * ex, my = dy - h * ey, mz = dz - h * ez;
        double B = mx * mx + my * my + mz * mz + eps * eps;
        return 0.5 * log1p(num / B);
    }
    double hp = kernel_h(dx + h * ex, dy + h * ey, dz + h * ez, eps, kern);
    double hm = kernel_h(dx - h * ex, dy - h * ey, dz - h * ez, eps, kern);
    double den = hp + hm;
    if (den == 0.0)
        return 0.0;
    return num / den;
}

int orc_fd_directional(int64_t p, const double *kx, const double *ky, const double *kz,
                       int64_t G, double L, const double *rho, double eps, int kern,
                       const double *delta /* [3][p] */, double h, double *out)
{
    if (p < 1 || G < 1 || !kx || !ky || !kz || !rho || !delta || !out || !(h > 0) || bad_kernel(eps, kern))
        return -1;
    const double *ex = delta, *ey = delta + p, *ez = delta + 2 * p;
    double *ta = calloc((size_t)p, sizeof(double)), *tr = calloc((size_t)p, sizeof(double));
    if (!ta || !tr) {
        free(ta); free(tr);
        return -1;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < p; ++i) {
        int moves_i = (ex[i] != 0.0 || ey[i] != 0.0 || ez[i] != 0.0);
        if (!moves_i)
            continue;
        csum sa = {0, 0}, sr = {0, 0};
        for (int64_t iz = 0; iz < G; ++iz)
            for (int64_t iy = 0; iy < G; ++iy)
                for (int64_t ix = 0; ix < G; ++ix) {
                    double w = rho[ix + G * (iy + G * iz)];
                    cs_add(&sa, w * pair_diff(kx[i] - cell_centre(ix, G, L),
                                              ky[i] - cell_centre(iy, G, L),
                                              kz[i] - cell_centre(iz, G, L),
                                              ex[i], ey[i], ez[i], h, eps, kern));
                }
        for (int64_t j = 0; j < p; ++j) {
            int moves_j = (ex[j] != 0.0 || ey[j] != 0.0 || ez[j] != 0.0);
            double dterm = pair_diff(kx[i] - kx[j], ky[i] - ky[j], kz[i] - kz[j],
                                     ex[i] - ex[j], ey[i] - ey[j], ez[i] - ez[j], h, eps, kern);
            cs_add(&sr, moves_j ? dterm : 2.0 * dterm);
        }
        ta[i] = cs_get(&sa);
        tr[i] = cs_get(&sr);
    }
    csum A = {0, 0}, R = {0, 0};
    for (int64_t i = 0; i < p; ++i) {
        cs_add(&A, ta[i]);
        cs_add(&R, tr[i]);
    }
    double dfa = cs_get(&A) / (double)p;
    double dfr = cs_get(&R) / (2.0 * (double)p * (double)p);
    *out = (dfa - dfr) / (2.0 * h);
    free(ta); free(tr);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Grid attraction (Sec. "Evaluating F^a and its gradient"): the        */
/* potential U(x) = sum_v rho_v H(x - x_v) and the field                 */
/* dU(x) = sum_v rho_v grad H(x - x_v) are sampled once on a node grid   */
/* (the discrete convolution of the sampled kernel with the sampled      */
/* density) and evaluated off the grid by the trilinear interpolant.     */
/* The node grid extends the cell centres by one node on each side:      */
/* X_k = -L + (k - 1/2) h, k = 0..G+1, h = 2L/G, so every point of       */
/* [-L, L]^3 lies inside it.  Node (kx, ky, kz) has index                */
/* kx + (G+2)(ky + (G+2) kz).                                            */
/* ------------------------------------------------------------------ */
static double node_coord(int64_t k, int64_t G, double L)
{
    return -L + ((double)k - 0.5) * (2.0 * L / (double)G);
}

/* U and dU at one point by direct summation over the G^3 cells. */
static void attraction_at(double x, double y, double z, int64_t G, double L, const double *rho,
                          double eps, int kern, double out[4])
{
    csum u = {0, 0}, d[3] = {{0, 0}, {0, 0}, {0, 0}};
    double g[3];
    for (int64_t iz = 0; iz < G; ++iz)
        for (int64_t iy = 0; iy < G; ++iy)
            for (int64_t ix = 0; ix < G; ++ix) {
                double w = rho[ix + G * (iy + G * iz)];
                double dx = x - cell_centre(ix, G, L), dy = y - cell_centre(iy, G, L),
                       dz = z - cell_centre(iz, G, L);
                cs_add(&u, w * kernel_h(dx, dy, dz, eps, kern));
                kernel_grad(dx, dy, dz, eps, kern, g);
                for (int c = 0; c < 3; ++c)
                    cs_add(&d[c], w * g[c]);
            }
    out[0] = cs_get(&u);
    for (int c = 0; c < 3; ++c)
        out[1 + c] = cs_get(&d[c]);
}

/* Field at every node of the extended grid: out[(node)*4 + {U, Ux, Uy, Uz}]. */
int orc_field(int64_t G, double L, const double *rho, double eps, int kern, double *out)
{
    if (G < 1 || !rho || !out || bad_kernel(eps, kern))
        return -1;
    int64_t Gn = G + 2, Mn = Gn * Gn * Gn;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t n = 0; n < Mn; ++n) {
        int64_t kx = n % Gn, ky = (n / Gn) % Gn, kz = n / (Gn * Gn);
        attraction_at(node_coord(kx, G, L), node_coord(ky, G, L), node_coord(kz, G, L), G, L,
                      rho, eps, kern, out + 4 * n);
    }
    return 0;
}

/* Lower node index and weight of the upper node along one axis:
 * t = (x - X_0)/h, k0 = floor(t) clamped to [0, G], f = t - k0. */
static void axis_weight(double x, int64_t G, double L, int64_t *k0, double *f)
{
    double h = 2.0 * L / (double)G;
    double t = (x - node_coord(0, G, L)) / h;
    double k = floor(t);
    if (!(k >= 0.0)) k = 0.0;          /* NaN and -inf: node 0, the weight carries it */
    if (k > (double)G) k = (double)G;
    *k0 = (int64_t)k;
    *f = t - k;
}

/* Trilinear interpolant of the 4 node fields at one point (x fastest). */
static void trilinear(const double *field, int64_t G, double L, double x, double y, double z,
                      double out[4])
{
    int64_t Gn = G + 2, k[3];
    double f[3];
    axis_weight(x, G, L, &k[0], &f[0]);
    axis_weight(y, G, L, &k[1], &f[1]);
    axis_weight(z, G, L, &k[2], &f[2]);
    for (int c = 0; c < 4; ++c)
        out[c] = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *
                           (dz ? f[2] : 1.0 - f[2]);
                int64_t n = (k[0] + dx) + Gn * ((k[1] + dy) + Gn * (k[2] + dz));
                for (int c = 0; c < 4; ++c)
                    out[c] += w * field[4 * n + c];
            }
}

/* Trilinear interpolation of a given node field at n points (out [4][n]). */
int orc_interpolate(int64_t G, double L, const double *field, int64_t n, const double *px,
                    const double *py, const double *pz, double *out)
{
    if (G < 1 || !field || n < 0 || !px || !py || !pz || !out)
        return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double v[4];
        trilinear(field, G, L, px[i], py[i], pz[i], v);
        for (int c = 0; c < 4; ++c)
            out[c * n + i] = v[c];
    }
    return 0;
}

/*
 * Gradient with the grid attraction at a list of targets: the attraction of
 * target i is the trilinear interpolant of the node field (each of the 8
 * surrounding nodes summed directly over the G^3 cells), the repulsion is
 * the all-pairs sum.  Outputs as orc_grad (ua = interpolated potential).
 */
int orc_grad_field(int64_t p, const double *kx, const double *ky, const double *kz,
                   int64_t G, double L, const double *rho, double eps, int kern,
                   int64_t n_t, const int64_t *targets,
                   double *dF, double *dFa, double *dFr, double *ua, double *ur)
{
    if (p < 1 || G < 1 || n_t < 0 || !kx || !ky || !kz || !rho || !targets || bad_kernel(eps, kern))
        return -1;
    for (int64_t t = 0; t < n_t; ++t)
        if (targets[t] < 0 || targets[t] >= p)
            return -1;
    double inv_p = 1.0 / (double)p;
    double inv_p2 = inv_p * inv_p;
    int64_t Gn = G + 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < n_t; ++t) {
        int64_t i = targets[t], k[3];
        double f[3], att[4] = {0, 0, 0, 0};
        axis_weight(kx[i], G, L, &k[0], &f[0]);
        axis_weight(ky[i], G, L, &k[1], &f[1]);
        axis_weight(kz[i], G, L, &k[2], &f[2]);
        double local[8 * 4];
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx)
                    attraction_at(node_coord(k[0] + dx, G, L), node_coord(k[1] + dy, G, L),
                                  node_coord(k[2] + dz, G, L), G, L, rho, eps, kern,
                                  local + 4 * (dx + 2 * (dy + 2 * dz)));
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *
                               (dz ? f[2] : 1.0 - f[2]);
                    for (int c = 0; c < 4; ++c)
                        att[c] += w * local[4 * (dx + 2 * (dy + 2 * dz)) + c];
                }
        (void)Gn;
        csum sr = {0, 0}, r3[3] = {{0, 0}, {0, 0}, {0, 0}};
        double g[3];
        for (int64_t j = 0; j < p; ++j) {
            double dx = kx[i] - kx[j], dy = ky[i] - ky[j], dz = kz[i] - kz[j];
            cs_add(&sr, kernel_h(dx, dy, dz, eps, kern));
            kernel_grad(dx, dy, dz, eps, kern, g);
            for (int c = 0; c < 3; ++c)
                cs_add(&r3[c], g[c]);
        }
        for (int c = 0; c < 3; ++c) {
            double fa = att[1 + c] * inv_p, fr = cs_get(&r3[c]) * inv_p2;
            if (dFa) dFa[c * n_t + t] = fa;
            if (dFr) dFr[c * n_t + t] = fr;
            if (dF) dF[c * n_t + t] = fa - fr;
        }
        if (ua) ua[t] = att[0];
        if (ur) ur[t] = cs_get(&sr);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Dyadic up-sampling of shots by linear interpolation (Sec.            */
/* "Multi-resolution strategy for faster convergence", Algorithm 1):    */
/* a shot of N samples on a raster of 2 dt becomes 2N samples on dt.    */
/* Fine sample m sits at coarse position m/2: even m copy k[m/2], odd   */
/* m average k[(m-1)/2] and k[(m+1)/2]; the last fine sample, half a    */
/* coarse step past the end, continues the last coarse step linearly:   */
/* 1.5 k[N-1] - 0.5 k[N-2] (k[0] when N = 1).                            */
/* coarse: [3][Nc*N], fine: [3][Nc*2N], both shot-lexicographic.        */
/* ------------------------------------------------------------------ */
int orc_upsample(int64_t Nc, int64_t N, const double *coarse, double *fine)
{
    if (Nc < 1 || N < 1 || !coarse || !fine)
        return -1;
    int64_t pc = Nc * N, pf = 2 * pc;
    for (int c = 0; c < 3; ++c)
        for (int64_t s = 0; s < Nc; ++s) {
            const double *k = coarse + c * pc + s * N;
            double *f = fine + c * pf + s * 2 * N;
            for (int64_t m = 0; m < 2 * N; ++m) {
                int64_t n = m / 2;
                if (m % 2 == 0)
                    f[m] = k[n];
                else if (n + 1 < N)
                    f[m] = (k[n] + k[n + 1]) * 0.5;
                else
                    f[m] = N > 1 ? 1.5 * k[n] - 0.5 * k[n - 1] : k[n];
            }
        }
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
