/*
 * fd_oracle.c -- plain FP64 CPU oracle for the explicit finite-difference
 * wave-propagation step (test infrastructure only).
 *
 * This file is the checker, not the product.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it.  It shares no code,
 * header, table or constant with the GPU library: every weight, sponge value
 * and interpolation weight is recomputed here in double precision from the
 * definitions below.
 *
 * What it computes (paper: "Automated MPI-X code generation for scalable
 * finite-difference solvers", appendix "Isotropic acoustic", equation (acou)):
 *
 *     m u_tt + m*gamma*u_t - Lap u = delta(x_s) q(t),   d(t) = u(t, x_r),
 *
 * with m = 1/v^2, discretised by the centred second-order leapfrog in time
 * and a centred star stencil of even space order `so` (radius r = so/2) in
 * space.  The damping term is the absorbing layer of the problem-setup
 * section (40-point ABC); its profile is not printed in the paper and the
 * reading used here is a quadratic PML-like ramp (see or_sponge_gamma).
 *
 * Layout: every field is a dense array over DOMAIN plus a halo of width r on
 * each side of every active axis (the DATA/HALO regions of the
 * "Access alignment" paragraph), axis order (z, y, x), x fastest.  2-D grids
 * have ndim = 2, n[1] = 1 and no y halo.
 *
 * Parallelism is a plain `omp parallel for` over z planes; there is no
 * blocking, fusion or reordering beyond the formulas.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int ndim;        /* 2 or 3 */
    int64_t n[3];    /* DOMAIN points along (z, y, x); n[1] == 1 when ndim == 2 */
    double h[3];     /* grid spacing in metres along (z, y, x) */
    int so;          /* even space order, 2..16 */
    int nbl;         /* absorbing-layer width in points, inside DOMAIN (0 = none) */
    double dt;       /* time step in seconds */
    double vmax;     /* velocity that sets the sponge strength (m/s) */
    int bc;          /* 0: zero halo, 1: periodic halo via face pack/unpack,
                        2: halo left as the caller filled it (an exchange
                        between subdomains) */
} or_grid;

/* ------------------------------------------------------------------------ */
/* Layout helpers                                                            */
/* ------------------------------------------------------------------------ */

static int64_t halo_of(const or_grid *g, int axis)
{
    if (axis == 1 && g->ndim == 2) return 0;
    return g->so / 2;
}

static int64_t ext_of(const or_grid *g, int axis)
{
    return g->n[axis] + 2 * halo_of(g, axis);
}

/* number of doubles in one padded field */
int64_t or_field_elems(const or_grid *g)
{
    return ext_of(g, 0) * ext_of(g, 1) * ext_of(g, 2);
}

/* linear index of DOMAIN coordinate (z, y, x); halo coordinates are negative
 * or >= n */
static int64_t at(const or_grid *g, int64_t z, int64_t y, int64_t x)
{
    int64_t Y = ext_of(g, 1), X = ext_of(g, 2);
    return ((z + halo_of(g, 0)) * Y + (y + halo_of(g, 1))) * X + (x + halo_of(g, 2));
}

int64_t or_index(const or_grid *g, int64_t z, int64_t y, int64_t x)
{
    return at(g, z, y, x);
}

/* ------------------------------------------------------------------------ */
/* Finite-difference weights                                                 */
/* ------------------------------------------------------------------------ */

static double fact(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; i++) f *= i;
    return f;
}

/* Centred second-derivative weights of order so on the unit grid:
 *   w_k = 2 (-1)^(k+1) (r!)^2 / (k^2 (r-k)! (r+k)!),  k = 1..r,
 *   w_0 = -2 sum_k 1/k^2,
 * so that  d2u/dx2 ~ (w_0 u_0 + sum_k w_k (u_k + u_-k)) / h^2.
 * For so = 2 this is (-2, 1), the update printed in the generated-code
 * appendix (r3 = -2u plus the two neighbours, times 1/h^2).
 * w must hold r+1 doubles.  Returns 0, or -1 for an invalid order. */
int or_d2_weights(int so, double *w)
{
    if (so < 2 || so > 16 || so % 2) return -1;
    int r = so / 2;
    double rr = fact(r) * fact(r);
    w[0] = 0.0;
    for (int k = 1; k <= r; k++) {
        double sgn = (k % 2) ? 1.0 : -1.0;
        w[k] = 2.0 * sgn * rr / ((double)k * k * fact(r - k) * fact(r + k));
        w[0] -= 2.0 / ((double)k * k);
    }
    return 0;
}

/* Centred first-derivative weights of order so on the unit grid:
 *   a_k = (-1)^(k+1) (r!)^2 / (k (r-k)! (r+k)!),   k = 1..r,
 * so that du/dx ~ sum_k a_k (u_k - u_-k) / h.  a[k-1] holds a_k. */
int or_d1_weights(int so, double *a)
{
    if (so < 2 || so > 16 || so % 2) return -1;
    int r = so / 2;
    double rr = fact(r) * fact(r);
    for (int k = 1; k <= r; k++) {
        double sgn = (k % 2) ? 1.0 : -1.0;
        a[k - 1] = sgn * rr / ((double)k * fact(r - k) * fact(r + k));
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Absorbing layer                                                           */
/* ------------------------------------------------------------------------ */

/* Damping rate of the absorbing layer at DOMAIN index i along `axis`
 * (problem-setup section: a 40-point ABC; the profile is a reading):
 *   gamma_1 = gamma_max * xi^2,  xi in [0,1] the depth into the layer
 *   (0 at the inner edge, 1 at the outermost DOMAIN point),
 *   gamma_max = 3 vmax ln(1/R) / (2 nbl h),  R = 1e-3.
 * The total rate is the sum over the active axes. */
static double sponge_1d(const or_grid *g, int axis, int64_t i)
{
    int64_t n = g->n[axis];
    int nbl = g->nbl;
    if (nbl <= 0 || (axis == 1 && g->ndim == 2)) return 0.0;
    double xi = 0.0;
    if (i < nbl) xi = (double)(nbl - i) / nbl;
    else if (i > n - 1 - nbl) xi = (double)(i - (n - 1 - nbl)) / nbl;
    double gmax = 3.0 * g->vmax * log(1.0e3) / (2.0 * nbl * g->h[axis]);
    return gmax * xi * xi;
}

double or_sponge_gamma(const or_grid *g, int64_t z, int64_t y, int64_t x)
{
    return sponge_1d(g, 0, z) + sponge_1d(g, 1, y) + sponge_1d(g, 2, x);
}

/* ------------------------------------------------------------------------ */
/* Halo faces (the "basic" exchange pattern: one message per face)           */
/* ------------------------------------------------------------------------ */

/* Face f in 0..5 is (-z, +z, -y, +y, -x, +x).  The OWNED slab of face f is the
 * r layers of DOMAIN adjacent to that face, over the full DOMAIN extent of the
 * other two axes (no edges or corners: a star stencil never reads them).  The
 * buffer is that slab in field axis order, row-major.  Returns the number of
 * elements, 0 for an inactive face (y faces in 2-D). */
int64_t or_face_elems(const or_grid *g, int f)
{
    int axis = f / 2;
    int64_t r = halo_of(g, axis);
    if (r == 0) return 0;
    int64_t e = 1;
    for (int a = 0; a < 3; a++) e *= (a == axis) ? r : g->n[a];
    return e;
}

/* start of the slab along the face axis: OWNED (pack) or HALO (unpack) */
static int64_t slab_start(const or_grid *g, int f, int halo_side)
{
    int axis = f / 2, plus = f & 1;
    int64_t r = halo_of(g, axis), n = g->n[axis];
    if (!halo_side) return plus ? n - r : 0;
    return plus ? n : -r;
}

static void face_copy(const or_grid *g, int f, int halo_side, double *field,
                      double *buf, int to_buf)
{
    int axis = f / 2;
    int64_t r = halo_of(g, axis);
    int64_t lo[3] = {0, 0, 0}, cnt[3] = {g->n[0], g->n[1], g->n[2]};
    lo[axis] = slab_start(g, f, halo_side);
    cnt[axis] = r;
    int64_t k = 0;
    for (int64_t z = 0; z < cnt[0]; z++)
        for (int64_t y = 0; y < cnt[1]; y++)
            for (int64_t x = 0; x < cnt[2]; x++, k++) {
                int64_t p = at(g, lo[0] + z, lo[1] + y, lo[2] + x);
                if (to_buf) buf[k] = field[p];
                else field[p] = buf[k];
            }
}

/* pack: copy the OWNED slab of face f into buf */
int or_pack_face(const or_grid *g, const double *field, int f, double *buf)
{
    if (f < 0 || f > 5) return -1;
    if (or_face_elems(g, f) == 0) return 0;
    face_copy(g, f, 0, (double *)field, buf, 1);
    return 0;
}

/* unpack: copy buf (the data a neighbour on side f sent) into the HALO slab
 * beyond face f */
int or_unpack_face(const or_grid *g, double *field, int f, const double *buf)
{
    if (f < 0 || f > 5) return -1;
    if (or_face_elems(g, f) == 0) return 0;
    face_copy(g, f, 1, field, (double *)buf, 0);
    return 0;
}

/* Fill the halo of `u`: zero (bc 0), or periodic (bc 1) by packing every face
 * and unpacking it into the halo of the opposite face -- a rank that is its
 * own neighbour on a periodic Cartesian topology. */
void or_fill_halo(const or_grid *g, double *u)
{
    if (g->bc == 2) return;
    if (g->bc == 0) {
        int64_t Z = ext_of(g, 0), Y = ext_of(g, 1), X = ext_of(g, 2);
        for (int64_t z = 0; z < Z; z++)
            for (int64_t y = 0; y < Y; y++)
                for (int64_t x = 0; x < X; x++) {
                    int64_t dz = z - halo_of(g, 0), dy = y - halo_of(g, 1), dx = x - halo_of(g, 2);
                    int inside = dz >= 0 && dz < g->n[0] && dy >= 0 && dy < g->n[1] &&
                                 dx >= 0 && dx < g->n[2];
                    if (!inside) u[(z * Y + y) * X + x] = 0.0;
                }
        return;
    }
    for (int f = 0; f < 6; f++) {
        int64_t e = or_face_elems(g, f);
        if (e == 0) continue;
        double *buf = (double *)malloc(sizeof(double) * e);
        or_pack_face(g, u, f ^ 1, buf);   /* the opposite face's OWNED slab ... */
        or_unpack_face(g, u, f, buf);     /* ... becomes this face's HALO */
        free(buf);
    }
}

/* ------------------------------------------------------------------------ */
/* Laplacian                                                                  */
/* ------------------------------------------------------------------------ */

/* lap[DOMAIN] = sum over active axes of (w_0 u + sum_k w_k (u[+k] + u[-k])) / h^2,
 * reading the halo of u as it stands.  lap is DOMAIN-shaped (nz, ny, nx). */
void or_laplacian(const or_grid *g, const double *u, double *lap)
{
    int r = g->so / 2;
    double w[9];
    or_d2_weights(g->so, w);
    int64_t nz = g->n[0], ny = g->n[1], nx = g->n[2];
    int64_t sz = at(g, 1, 0, 0) - at(g, 0, 0, 0);
    int64_t sy = at(g, 0, 1, 0) - at(g, 0, 0, 0);
    double iz = 1.0 / (g->h[0] * g->h[0]), iy = 1.0 / (g->h[1] * g->h[1]),
           ix = 1.0 / (g->h[2] * g->h[2]);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; z++)
        for (int64_t y = 0; y < ny; y++)
            for (int64_t x = 0; x < nx; x++) {
                int64_t p = at(g, z, y, x);
                double dzz = w[0] * u[p], dyy = w[0] * u[p], dxx = w[0] * u[p];
                for (int k = 1; k <= r; k++) {
                    dzz += w[k] * (u[p + k * sz] + u[p - k * sz]);
                    dxx += w[k] * (u[p + k] + u[p - k]);
                    if (g->ndim == 3) dyy += w[k] * (u[p + k * sy] + u[p - k * sy]);
                }
                double s = dzz * iz + dxx * ix;
                if (g->ndim == 3) s += dyy * iy;
                lap[(z * ny + y) * nx + x] = s;
            }
}

/* ------------------------------------------------------------------------ */
/* Sparse points: multilinear injection / interpolation                     */
/* ------------------------------------------------------------------------ */

/* For npts points with coordinates coords[p][ndim] (metres from DOMAIN index 0,
 * axis order (z, [y,] x)), compute the 2^ndim surrounding DOMAIN nodes
 * (as padded linear indices) and their multilinear weights:
 *   base_a = floor(c_a / h_a), clamped to n_a - 2; frac_a = c_a/h_a - base_a;
 *   weight = prod_a (bit_a ? frac_a : 1 - frac_a).
 * Corner c uses bit (ndim-1-j) of c for the j-th listed axis.
 * Returns 0, or -1 if a point lies outside [0, (n_a - 1) h_a]. */
int or_sparse_weights(const or_grid *g, const double *coords, int npts,
                      int64_t *node, double *wt)
{
    int axes[3], na = 0;
    for (int a = 0; a < 3; a++)
        if (!(a == 1 && g->ndim == 2)) axes[na++] = a;
    int nc = 1 << na;
    for (int p = 0; p < npts; p++) {
        int64_t base[3] = {0, 0, 0};
        double frac[3] = {0, 0, 0};
        for (int j = 0; j < na; j++) {
            int a = axes[j];
            double c = coords[p * na + j];
            double s = c / g->h[a];
            if (!(s >= 0.0) || s > (double)(g->n[a] - 1)) return -1;
            int64_t b = (int64_t)floor(s);
            if (b > g->n[a] - 2) b = g->n[a] - 2;
            base[a] = b;
            frac[a] = s - (double)b;
        }
        for (int c = 0; c < nc; c++) {
            int64_t idx[3] = {base[0], base[1], base[2]};
            double w = 1.0;
            for (int j = 0; j < na; j++) {
                int a = axes[j];
                int bit = (c >> (na - 1 - j)) & 1;
                idx[a] += bit;
                w *= bit ? frac[a] : 1.0 - frac[a];
            }
            node[p * nc + c] = at(g, idx[0], idx[1], idx[2]);
            wt[p * nc + c] = w;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Time stepping                                                             */
/* ------------------------------------------------------------------------ */

static void domain_coords(const or_grid *g, int64_t q, int64_t *z, int64_t *y, int64_t *x)
{
    int64_t ny = g->n[1], nx = g->n[2];
    *x = q % nx;
    *y = (q / nx) % ny;
    *z = q / (nx * ny);
}

/* One leapfrog update on DOMAIN (equation (acou) with the damping term):
 *   u_new = [2 u - (1 - gamma dt/2) u_old + v^2 dt^2 (Lap u + f)] / (1 + gamma dt/2)
 * `f` is the DOMAIN-shaped forcing (may be NULL), lap the DOMAIN-shaped
 * Laplacian of u.  u_new may alias u_old (each point reads only itself). */
static void leapfrog(const or_grid *g, const double *v, const double *u,
                     const double *u_old, const double *lap, const double *f,
                     double *u_new)
{
    int64_t nd = g->n[0] * g->n[1] * g->n[2];
    double dt = g->dt;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nd; q++) {
        int64_t z, y, x;
        domain_coords(g, q, &z, &y, &x);
        int64_t p = at(g, z, y, x);
        double a = 0.5 * dt * or_sponge_gamma(g, z, y, x);
        double rhs = lap[q] + (f ? f[q] : 0.0);
        double c = v[q] * v[q] * dt * dt;
        u_new[p] = (2.0 * u[p] - (1.0 - a) * u_old[p] + c * rhs) / (1.0 + a);
    }
}

/* forcing f = h^-d * sum_s sum_corners w q_s spread onto DOMAIN nodes
 * (scale = h^-d for a physical point source, 1 for the adjoint's receiver
 * residual injection) */
static void spread(const or_grid *g, int npts, const int64_t *node, const double *wt,
                   const double *vals, double scale, double *f)
{
    int nc = 1 << (g->ndim);
    int64_t nd = g->n[0] * g->n[1] * g->n[2];
    memset(f, 0, sizeof(double) * nd);
    for (int p = 0; p < npts; p++)
        for (int c = 0; c < nc; c++) {
            /* convert padded index back to DOMAIN index */
            int64_t pi = node[p * nc + c];
            int64_t X = ext_of(g, 2), Y = ext_of(g, 1);
            int64_t x = pi % X - halo_of(g, 2);
            int64_t y = (pi / X) % Y - halo_of(g, 1);
            int64_t z = pi / (X * Y) - halo_of(g, 0);
            f[(z * g->n[1] + y) * g->n[2] + x] += scale * wt[p * nc + c] * vals[p];
        }
}

static void sample(const or_grid *g, int npts, const int64_t *node, const double *wt,
                   const double *u, double scale, double *out)
{
    int nc = 1 << (g->ndim);
    for (int p = 0; p < npts; p++) {
        double s = 0.0;
        for (int c = 0; c < nc; c++) s += wt[p * nc + c] * u[node[p * nc + c]];
        out[p] = scale * s;
    }
}

static double cell_volume(const or_grid *g)
{
    double hv = g->h[0] * g->h[2];
    if (g->ndim == 3) hv *= g->h[1];
    return hv;
}

/* Forward modelling, nt leapfrog updates.
 *   v         DOMAIN-shaped velocity (m/s)
 *   u, u_old  padded fields: on entry u^0 and u^-1, on exit u^nt and u^(nt-1)
 *   src       ns source coordinates, q[nt][ns] their signatures
 *   rec       nr receiver coordinates, d[nt][nr] the recorded traces
 *   hist      NULL, or (nt+2) DOMAIN-shaped slots receiving u^-1 .. u^nt
 * Update n uses q[n] to produce u^(n+1); d[n] is sampled from u^(n+1).
 * Returns 0, or -1 if a sparse point is outside the grid. */
int or_forward(const or_grid *g, const double *v, double *u, double *u_old,
               int ns, const double *src, const double *q,
               int nr, const double *rec, double *d, int nt, double *hist)
{
    int nc = 1 << g->ndim;
    int64_t nd = g->n[0] * g->n[1] * g->n[2];
    int64_t ne = or_field_elems(g);
    int64_t *snode = malloc(sizeof(int64_t) * (ns ? ns : 1) * nc);
    int64_t *rnode = malloc(sizeof(int64_t) * (nr ? nr : 1) * nc);
    double *sw = malloc(sizeof(double) * (ns ? ns : 1) * nc);
    double *rw = malloc(sizeof(double) * (nr ? nr : 1) * nc);
    double *lap = malloc(sizeof(double) * nd);
    double *f = malloc(sizeof(double) * nd);
    double *tmp = malloc(sizeof(double) * ne);
    int rc = 0;
    if (or_sparse_weights(g, src, ns, snode, sw) || or_sparse_weights(g, rec, nr, rnode, rw)) {
        rc = -1;
        goto done;
    }
    double hinv = 1.0 / cell_volume(g);
    if (hist) {
        for (int64_t k = 0; k < nd; k++) {
            int64_t z, y, x;
            domain_coords(g, k, &z, &y, &x);
            hist[k] = u_old[at(g, z, y, x)];
            hist[nd + k] = u[at(g, z, y, x)];
        }
    }
    for (int n = 0; n < nt; n++) {
        or_fill_halo(g, u);
        or_laplacian(g, u, lap);
        spread(g, ns, snode, sw, q + (int64_t)n * ns, hinv, f);
        /* u_old <- u^(n+1) in place; then swap roles */
        leapfrog(g, v, u, u_old, lap, f, u_old);
        double *t = u_old; u_old = u; u = t;
        if (nr) sample(g, nr, rnode, rw, u, 1.0, d + (int64_t)n * nr);
        if (hist) {
            double *hs = hist + (int64_t)(n + 2) * nd;
            for (int64_t k = 0; k < nd; k++) {
                int64_t z, y, x;
                domain_coords(g, k, &z, &y, &x);
                hs[k] = u[at(g, z, y, x)];
            }
        }
    }
    /* after an odd number of swaps the caller's buffers hold the states the
     * other way round: put u^nt back into the caller's `u` */
    if (nt % 2) {
        memcpy(tmp, u, sizeof(double) * ne);
        memcpy(u, u_old, sizeof(double) * ne);
        memcpy(u_old, tmp, sizeof(double) * ne);
    }
done:
    free(snode); free(rnode); free(sw); free(rw); free(lap); free(f); free(tmp);
    return rc;
}

/* Adjoint (transposed) modelling.  The forward scheme is the block
 * lower-triangular system, row n (n = 0..nt-1):
 *   M+ u^(n+1) - (M0 + L) u^n + M- u^(n-1) = f^n,
 *   M+ = m (1/dt^2 + gamma/(2dt)),  M0 = 2m/dt^2,  M- = m (1/dt^2 - gamma/(2dt)),
 * with d[n] = R u^(n+1).  Its transpose is the same recurrence run backwards
 * for the multipliers lambda_n of row n:
 *   lambda_n = [2 lambda_(n+1) - (1 - gamma dt/2) lambda_(n+2)
 *               + v^2 dt^2 (L lambda_(n+1) + R^T resid[n])] / (1 + gamma dt/2),
 * lambda_nt = lambda_(nt+1) = 0, and the adjoint source signature is
 *   qadj[n][s] = h^-d sum_corners w lambda_n.
 *   resid[nt][nr] receiver residuals; qadj[nt][ns] output (may be NULL)
 *   hist    NULL, or the (nt+2) forward states u^-1..u^nt from or_forward;
 *           then grad_m (DOMAIN) accumulates the zero-lag imaging condition
 *     dJ/dm += - sum_n lambda_n * [(1/dt^2 + gamma/(2dt)) u^(n+1) - (2/dt^2) u^n
 *                                  + (1/dt^2 - gamma/(2dt)) u^(n-1)].
 *   lam, lam_old  padded work fields, zero on entry (the terminal condition);
 *           on exit lambda_0 and lambda_1. */
int or_adjoint(const or_grid *g, const double *v, double *lam, double *lam_old,
               int nr, const double *rec, const double *resid,
               int ns, const double *src, double *qadj, int nt,
               const double *hist, double *grad_m)
{
    int nc = 1 << g->ndim;
    int64_t nd = g->n[0] * g->n[1] * g->n[2];
    int64_t ne = or_field_elems(g);
    int64_t *snode = malloc(sizeof(int64_t) * (ns ? ns : 1) * nc);
    int64_t *rnode = malloc(sizeof(int64_t) * (nr ? nr : 1) * nc);
    double *sw = malloc(sizeof(double) * (ns ? ns : 1) * nc);
    double *rw = malloc(sizeof(double) * (nr ? nr : 1) * nc);
    double *lap = malloc(sizeof(double) * nd);
    double *f = malloc(sizeof(double) * nd);
    double *tmp = malloc(sizeof(double) * ne);
    int rc = 0;
    if (or_sparse_weights(g, src, ns, snode, sw) || or_sparse_weights(g, rec, nr, rnode, rw)) {
        rc = -1;
        goto done;
    }
    double hinv = 1.0 / cell_volume(g);
    double dt = g->dt;
    for (int n = nt - 1; n >= 0; n--) {
        /* lam = lambda_(n+1), lam_old = lambda_(n+2) */
        or_fill_halo(g, lam);
        or_laplacian(g, lam, lap);
        spread(g, nr, rnode, rw, resid + (int64_t)n * nr, 1.0, f);
        leapfrog(g, v, lam, lam_old, lap, f, lam_old);
        double *t = lam_old; lam_old = lam; lam = t;   /* lam = lambda_n */
        if (qadj && ns) sample(g, ns, snode, sw, lam, hinv, qadj + (int64_t)n * ns);
        if (hist && grad_m) {
            const double *um = hist + (int64_t)n * nd;        /* u^(n-1) */
            const double *u0 = hist + (int64_t)(n + 1) * nd;  /* u^n     */
            const double *up = hist + (int64_t)(n + 2) * nd;  /* u^(n+1) */
#pragma omp parallel for schedule(static)
            for (int64_t k = 0; k < nd; k++) {
                int64_t z, y, x;
                domain_coords(g, k, &z, &y, &x);
                double gam = or_sponge_gamma(g, z, y, x);
                double cp = 1.0 / (dt * dt) + gam / (2.0 * dt);
                double cm = 1.0 / (dt * dt) - gam / (2.0 * dt);
                double dE = cp * up[k] - 2.0 / (dt * dt) * u0[k] + cm * um[k];
                grad_m[k] -= lam[at(g, z, y, x)] * dE;
            }
        }
    }
    if (nt % 2) {
        memcpy(tmp, lam, sizeof(double) * ne);
        memcpy(lam, lam_old, sizeof(double) * ne);
        memcpy(lam_old, tmp, sizeof(double) * ne);
    }
done:
    free(snode); free(rnode); free(sw); free(rw); free(lap); free(f); free(tmp);
    return rc;
}

/* Forward-Euler heat step u <- u + dt * Lap u, repeated nsteps times, with
 * the halo filled per g->bc before each step.  This is the diffusion operator
 * of the paper's introductory DSL example (Eq(u.dt, u.laplace)). */
void or_heat(const or_grid *g, double *u, int nsteps)
{
    int64_t nd = g->n[0] * g->n[1] * g->n[2];
    double *lap = malloc(sizeof(double) * nd);
    for (int s = 0; s < nsteps; s++) {
        or_fill_halo(g, u);
        or_laplacian(g, u, lap);
        for (int64_t k = 0; k < nd; k++) {
            int64_t z, y, x;
            domain_coords(g, k, &z, &y, &x);
            u[at(g, z, y, x)] += g->dt * lap[k];
        }
    }
    free(lap);
}
