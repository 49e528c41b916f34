/*
 * dect_oracle.c -- plain FP64 CPU oracle of the DECT reconstruction path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package's smoke check and
 * the benchmark's CPU-baseline leg load this library.  It shares no code,
 * header or table with the GPU library: it implements the same mathematics
 * from the paper (Li et al., "Efficient Image Reconstruction and Practical
 * Decomposition for Dual-energy CT") in the most direct form, slowly.
 *
 * Contents and the passage each follows:
 *   or_project / or_backproject  line integrals of the image and their literal
 *                                transpose (the linear model A x = m of Eq. 1;
 *                                A^T of the gradient G_f, Eq. 9), with either
 *                                Joseph's interpolating ray model or Siddon's
 *                                exact pixel intersection lengths, the model
 *                                Sec. 2.1 names
 *   or_fbp                       fan-beam filtered back-projection, the
 *                                analytic reconstruction the paper compares
 *                                with (Sec. 3)
 *   or_grad / or_gradT           backward differences of the TV norm (Eq. 2)
 *                                and their exact adjoint
 *   or_shrink                    the z-subproblem's closed form (Eq. 8, read as
 *                                isotropic shrinkage)
 *   or_adm                       the reconstruction procedure (Eq. 10) for one
 *                                energy block of Eq. 3, with the f-gradient of
 *                                Eq. 9 and a Barzilai-Borwein step
 *   or_dinv                      direct decomposition u = D^{-1} x (Eqs. 11-12)
 *   or_edges / or_edges3         Prewitt edge weights e_ik (after Eq. 14), the
 *                                gradient magnitude and threshold in FP64
 *   or_laplacian                 the Hessian of R(u) (Eq. 14), halved
 *   or_pcg                       Jacobi-preconditioned CG for Eq. 15
 *   or_pcg_att / or_pcg_att3     the attenuation-space variant |x - Du|^2 +
 *                                gamma R(u), both materials coupled (image and
 *                                volume)
 *
 * Readings of the paper taken here (each is also listed in the design notes):
 *   - separable TV per energy block, zero difference on the first row/column;
 *   - lambda has z's shape (two planes); xi is a free parameter;
 *   - the BB step is BB1 = <s,s>/<s,y> with y the change of the f-gradient
 *     at fixed (z, lambda), i.e. y = (mu A^T A + rho grad^T grad) s; the first
 *     step is the exact line-search (Cauchy) step along G; a non-positive
 *     <s,y> keeps the previous step;
 *   - Eq. 15 with grad R = 2L (L the edge-weighted graph Laplacian) reads
 *     (I + gamma L) u = D^{-1} x per material.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    int32_t nx, ny;
    double pixel;
    int32_t n_views;
    const double *angles; /* NULL: theta_v = 2*pi*v/n_views */
    int32_t n_bins;
    double bin, det_offset, sod, sdd;
    int32_t model; /* 0: Joseph, 1: Siddon */
} or_geom;

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Source position and (unnormalised) direction source -> centre of bin b. */
static void ray_of(const or_geom *g, int v, int b, double *sx, double *sy, double *dx, double *dy)
{
    double th = g->angles ? g->angles[v] : 2.0 * M_PI * v / g->n_views;
    double ct = cos(th), st = sin(th);
    double u = (b - (g->n_bins - 1) / 2.0) * g->bin + g->det_offset;
    double px = -(g->sdd - g->sod) * ct - u * st;
    double py = -(g->sdd - g->sod) * st + u * ct;
    *sx = g->sod * ct;
    *sy = g->sod * st;
    *dx = px - *sx;
    *dy = py - *sy;
}

/*
 * Walk one Joseph ray.  The driving axis is the one the ray is more aligned
 * with (ties go to x).  On every line of the driving axis the ray's crossing
 * is interpolated linearly between the two nearest pixel centres of that line;
 * pixels outside the grid are zero.  Each line's two weights are scaled by the
 * ray length per line, pixel / |cos| of the angle to the driving axis.
 * mode 0: return sum_lines weight * X.  mode 1: X += weight * y (transpose).
 */
static double joseph_walk(const or_geom *g, int v, int b, double *X, double y, int mode)
{
    const int nx = g->nx, ny = g->ny;
    const double dl = g->pixel;
    double sx, sy, dx, dy;
    ray_of(g, v, b, &sx, &sy, &dx, &dy);
    const double len = sqrt(dx * dx + dy * dy);
    double acc = 0.0;
    if (fabs(dx) >= fabs(dy)) {
        const double L = dl * len / fabs(dx);
        for (int c = 0; c < nx; ++c) {
            double xc = (c - (nx - 1) / 2.0) * dl;
            double yy = sy + (xc - sx) * dy / dx;
            double q = yy / dl + (ny - 1) / 2.0;
            double fq = floor(q);
            if (fq < -1.0 || fq > ny - 1.0) continue;
            int r0 = (int)fq;
            double w = q - fq;
            if (r0 >= 0) {
                if (mode == 0) acc += L * (1.0 - w) * X[(size_t)r0 * nx + c];
                else X[(size_t)r0 * nx + c] += L * (1.0 - w) * y;
            }
            if (r0 + 1 <= ny - 1) {
                if (mode == 0) acc += L * w * X[(size_t)(r0 + 1) * nx + c];
                else X[(size_t)(r0 + 1) * nx + c] += L * w * y;
            }
        }
    } else {
        const double L = dl * len / fabs(dy);
        for (int r = 0; r < ny; ++r) {
            double yr = (r - (ny - 1) / 2.0) * dl;
            double xx = sx + (yr - sy) * dx / dy;
            double q = xx / dl + (nx - 1) / 2.0;
            double fq = floor(q);
            if (fq < -1.0 || fq > nx - 1.0) continue;
            int c0 = (int)fq;
            double w = q - fq;
            if (c0 >= 0) {
                if (mode == 0) acc += L * (1.0 - w) * X[(size_t)r * nx + c0];
                else X[(size_t)r * nx + c0] += L * (1.0 - w) * y;
            }
            if (c0 + 1 <= nx - 1) {
                if (mode == 0) acc += L * w * X[(size_t)r * nx + c0 + 1];
                else X[(size_t)r * nx + c0 + 1] += L * w * y;
            }
        }
    }
    return acc;
}

/*
 * Walk one Siddon ray: the segment from the source to the bin centre, and
 * the exact length of its part inside every pixel (pixels are squares of side
 * `pixel` tiling the grid, which is centred on the isocentre).  Points on the
 * segment are s + t d, t in [0, 1].  The segment enters and leaves the grid
 * at t0 < t1 (slab clipping against the grid's four sides).  Its crossings
 * with the nx + 1 vertical and ny + 1 horizontal grid lines inside (t0, t1),
 * merged in increasing t together with t0 and t1, cut it into pieces that
 * each lie in one pixel, the pixel that contains the piece's midpoint; the
 * piece's length is its parameter interval times |d|.
 * mode 0: return sum over pieces of length * X.  mode 1: X += length * y.
 */
static double siddon_walk(const or_geom *g, int v, int b, double *X, double y, int mode)
{
    const int nx = g->nx, ny = g->ny;
    const double dl = g->pixel;
    double sx, sy, dx, dy;
    ray_of(g, v, b, &sx, &sy, &dx, &dy);
    const double len = sqrt(dx * dx + dy * dy);
    const double xmin = -0.5 * nx * dl, ymin = -0.5 * ny * dl;
    const double xmax = 0.5 * nx * dl, ymax = 0.5 * ny * dl;
    double t0 = 0.0, t1 = 1.0;
    if (dx != 0.0) {
        double ta = (xmin - sx) / dx, tb = (xmax - sx) / dx;
        t0 = fmax(t0, fmin(ta, tb));
        t1 = fmin(t1, fmax(ta, tb));
    } else if (!(sx > xmin && sx < xmax)) {
        return 0.0;
    }
    if (dy != 0.0) {
        double ta = (ymin - sy) / dy, tb = (ymax - sy) / dy;
        t0 = fmax(t0, fmin(ta, tb));
        t1 = fmin(t1, fmax(ta, tb));
    } else if (!(sy > ymin && sy < ymax)) {
        return 0.0;
    }
    if (!(t1 > t0)) return 0.0;
    /* grid-line crossings of each family in increasing t */
    double *tx = (double *)malloc((size_t)(nx + 1) * sizeof(double));
    double *ty = (double *)malloc((size_t)(ny + 1) * sizeof(double));
    int nxc = 0, nyc = 0;
    if (dx != 0.0)
        for (int j = 0; j <= nx; ++j) {
            int i = dx > 0.0 ? j : nx - j;
            double t = (xmin + i * dl - sx) / dx;
            if (t > t0 && t < t1) tx[nxc++] = t;
        }
    if (dy != 0.0)
        for (int j = 0; j <= ny; ++j) {
            int i = dy > 0.0 ? j : ny - j;
            double t = (ymin + i * dl - sy) / dy;
            if (t > t0 && t < t1) ty[nyc++] = t;
        }
    double acc = 0.0, prev = t0;
    int ix = 0, iy = 0;
    for (;;) {
        double next;
        if (ix < nxc && (iy >= nyc || tx[ix] <= ty[iy])) next = tx[ix++];
        else if (iy < nyc) next = ty[iy++];
        else next = t1;
        if (next > prev) {
            double tm = 0.5 * (prev + next);
            int c = (int)floor((sx + tm * dx - xmin) / dl);
            int r = (int)floor((sy + tm * dy - ymin) / dl);
            if (c >= 0 && c < nx && r >= 0 && r < ny) {
                double l = (next - prev) * len;
                if (mode == 0) acc += l * X[(size_t)r * nx + c];
                else X[(size_t)r * nx + c] += l * y;
            }
        }
        prev = next;
        if (next == t1 && ix >= nxc && iy >= nyc) break;
    }
    free(tx);
    free(ty);
    return acc;
}

static double ray_walk(const or_geom *g, int v, int b, double *X, double y, int mode)
{
    return g->model == 1 ? siddon_walk(g, v, b, X, y, mode) : joseph_walk(g, v, b, X, y, mode);
}

/* Number of (ray, driving line) samples whose crossing lies in (-1, n). */
int64_t or_count_samples(const or_geom *g)
{
    int64_t total = 0;
    for (int v = 0; v < g->n_views; ++v)
        for (int b = 0; b < g->n_bins; ++b) {
            double sx, sy, dx, dy;
            ray_of(g, v, b, &sx, &sy, &dx, &dy);
            int xmaj = fabs(dx) >= fabs(dy);
            int nl = xmaj ? g->nx : g->ny, nq = xmaj ? g->ny : g->nx;
            for (int i = 0; i < nl; ++i) {
                double q;
                if (xmaj) {
                    double xc = (i - (g->nx - 1) / 2.0) * g->pixel;
                    q = (sy + (xc - sx) * dy / dx) / g->pixel + (g->ny - 1) / 2.0;
                } else {
                    double yr = (i - (g->ny - 1) / 2.0) * g->pixel;
                    q = (sx + (yr - sy) * dx / dy) / g->pixel + (g->nx - 1) / 2.0;
                }
                if (q > -1.0 && q < nq) ++total;
            }
        }
    return total;
}

/* sino[v][b] = (A img)[v,b] */
void or_project(const or_geom *g, const double *img, double *sino)
{
    const int V = g->n_views, B = g->n_bins;
#pragma omp parallel for schedule(static)
    for (int v = 0; v < V; ++v)
        for (int b = 0; b < B; ++b)
            sino[(size_t)v * B + b] = ray_walk(g, v, b, (double *)img, 0.0, 0);
}

/* img = A^T sino: every ray scatters its weights back.  Views are split into
 * fixed contiguous chunks, one private image each, summed in chunk order, so
 * the result does not depend on thread timing. */
void or_backproject(const or_geom *g, const double *sino, double *img)
{
    const int V = g->n_views, B = g->n_bins;
    const size_t N = (size_t)g->nx * g->ny;
    int T = or_num_threads();
    if (T > V) T = V;
    if (T < 1) T = 1;
    double *buf = (double *)calloc((size_t)T * N, sizeof(double));
#pragma omp parallel for schedule(static, 1) num_threads(T)
    for (int t = 0; t < T; ++t) {
        int v0 = (int)((int64_t)V * t / T), v1 = (int)((int64_t)V * (t + 1) / T);
        double *mine = buf + (size_t)t * N;
        for (int v = v0; v < v1; ++v)
            for (int b = 0; b < B; ++b)
                ray_walk(g, v, b, mine, sino[(size_t)v * B + b], 1);
    }
    for (size_t i = 0; i < N; ++i) {
        double s = 0.0;
        for (int t = 0; t < T; ++t) s += buf[(size_t)t * N + i];
        img[i] = s;
    }
    free(buf);
}

/*
 * Filtered back-projection for the flat-detector fan beam over a full turn of
 * equally spaced views: the analytic reconstruction the paper compares its
 * method with (Sec. 3, Tables 1-2), in the textbook form for equally spaced
 * collinear detectors.
 *  1. Detector positions u_b are scaled to a virtual detector through the
 *     isocentre, s_b = u_b R / D (R = SOD, D = SDD), spacing ds = du R / D.
 *  2. Each sample is weighted by R / sqrt(R^2 + s_b^2).
 *  3. Each view is convolved with the band-limited ramp kernel of spacing ds
 *     (h(0) = 1 / (4 ds^2), h(k ds) = -1 / (pi^2 k^2 ds^2) for odd k, 0 for
 *     even k != 0) as the sum ds * sum_n p(n) h(b - n), and halved, since a
 *     full turn measures every line twice.
 *  4. Each pixel p sums, over the views, the filtered view at the virtual
 *     detector position s'(p) = R (p . e_u) / (R - p . e_s) where the ray from
 *     the source through p meets it (linear interpolation between bins, zero
 *     outside the detector), weighted by R^2 / (R - p . e_s)^2, times the
 *     view spacing 2 pi / V.  e_s = (cos t, sin t) points from the isocentre
 *     to the source, e_u = (-sin t, cos t) along the detector.
 * sino [V][B] -> img [ny][nx].
 */
void or_fbp(const or_geom *g, const double *sino, double *img)
{
    const int V = g->n_views, B = g->n_bins, nx = g->nx, ny = g->ny;
    const double R = g->sod, D = g->sdd;
    const double ds = g->bin * R / D;
    double *q = (double *)malloc((size_t)V * B * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int v = 0; v < V; ++v) {
        double *pw = (double *)malloc((size_t)B * sizeof(double));
        for (int b = 0; b < B; ++b) {
            double u = (b - (B - 1) / 2.0) * g->bin + g->det_offset;
            double s = u * R / D;
            pw[b] = sino[(size_t)v * B + b] * R / sqrt(R * R + s * s);
        }
        for (int b = 0; b < B; ++b) {
            double acc = 0.0;
            for (int n = 0; n < B; ++n) {
                int k = b - n;
                double h;
                if (k == 0) h = 1.0 / (4.0 * ds * ds);
                else if (k % 2 == 0) h = 0.0;
                else h = -1.0 / (M_PI * M_PI * (double)k * (double)k * ds * ds);
                acc += pw[n] * h;
            }
            q[(size_t)v * B + b] = 0.5 * ds * acc;
        }
        free(pw);
    }
#pragma omp parallel for schedule(static)
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c < nx; ++c) {
            double x = (c - (nx - 1) / 2.0) * g->pixel, y = (r - (ny - 1) / 2.0) * g->pixel;
            double acc = 0.0;
            for (int v = 0; v < V; ++v) {
                double th = g->angles ? g->angles[v] : 2.0 * M_PI * v / V;
                double ct = cos(th), st = sin(th);
                double dist = R - (x * ct + y * st);
                double sp = R * (-x * st + y * ct) / dist;
                double bf = (sp * D / R - g->det_offset) / g->bin + (B - 1) / 2.0;
                double f0 = floor(bf);
                int b0 = (int)f0;
                double w = bf - f0, val = 0.0;
                if (b0 >= 0 && b0 < B) val += (1.0 - w) * q[(size_t)v * B + b0];
                if (b0 + 1 >= 0 && b0 + 1 < B) val += w * q[(size_t)v * B + b0 + 1];
                acc += val * R * R / (dist * dist);
            }
            img[(size_t)r * nx + c] = acc * 2.0 * M_PI / V;
        }
    free(q);
}

/* Backward differences (Eq. 2): planes [0] = along x (columns), [1] = along y
 * (rows); the first column/row has zero difference. */
void or_grad(int nx, int ny, const double *x, double *gx, double *gy)
{
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c < nx; ++c) {
            size_t i = (size_t)r * nx + c;
            gx[i] = c >= 1 ? x[i] - x[i - 1] : 0.0;
            gy[i] = r >= 1 ? x[i] - x[i - nx] : 0.0;
        }
}

/* Exact adjoint of or_grad. */
void or_gradT(int nx, int ny, const double *px, const double *py, double *out)
{
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c < nx; ++c) {
            size_t i = (size_t)r * nx + c;
            double s = 0.0;
            if (c >= 1) s += px[i];
            if (c + 1 <= nx - 1) s -= px[i + 1];
            if (r >= 1) s += py[i];
            if (r + 1 <= ny - 1) s -= py[i + nx];
            out[i] = s;
        }
}

/* Isotropic shrinkage: argmin_z |z| + 1/(2t) |z - v|^2 = max(|v| - t, 0) v/|v|. */
void or_shrink(size_t n, const double *vx, const double *vy, double t, double *zx, double *zy)
{
    for (size_t i = 0; i < n; ++i) {
        double m = sqrt(vx[i] * vx[i] + vy[i] * vy[i]);
        double s = m > t ? (m - t) / m : 0.0;
        zx[i] = s * vx[i];
        zy[i] = s * vy[i];
    }
}

static double dot(size_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* TV norm of Eq. 2. */
double or_tv(int nx, int ny, const double *x)
{
    size_t N = (size_t)nx * ny;
    double *gx = malloc(N * sizeof(double)), *gy = malloc(N * sizeof(double));
    or_grad(nx, ny, x, gx, gy);
    double s = 0.0;
    for (size_t i = 0; i < N; ++i) s += sqrt(gx[i] * gx[i] + gy[i] * gy[i]);
    free(gx);
    free(gy);
    return s;
}

/*
 * ADM-TV for one energy block of Eq. 3 (the two blocks decouple because W is
 * block-diagonal and the TV is applied per block).
 *
 * In:  m [V][B] measured projections of this energy; beta the Eq. 3 weight;
 *      x0 [ny][nx] start image (NULL: zeros).
 * Out: x_out = f / beta after the last iteration; optional lam_out, z_out
 *      [2][ny][nx]; log [(K+1)][5] rows (J(f^k), alpha^k, |grad f^k - z^k|,
 *      |f^k - f^{k-1}|/|f^{k-1}|, |G^k|) -- the last row holds J(f^K).
 * nonneg != 0: every f-step is followed by the projection f = max(f, 0)
 * (images are attenuation maps, non-negative); the BB step is then taken
 * from the projected step s.
 * step_rule: 0 BB1 <s,s>/<s,y>; 1 BB2 <s,y>/<y,y>; 2 adaptive (BB2 where
 * BB2/BB1 < 1/2, else BB1).  A non-positive <s,y> keeps the step.
 * Returns the number of iterations run (stops early when tol > 0 and the
 * relative image change drops below tol).
 */
int or_adm(const or_geom *g, const double *m, double beta, double mu, double rho, double xi,
           int K, double tol, const double *x0, double *x_out, double *lam_out, double *z_out,
           double *log, int nonneg, int step_rule)
{
    const int nx = g->nx, ny = g->ny;
    const size_t N = (size_t)nx * ny, M = (size_t)g->n_views * g->n_bins;
    double *f = calloc(N, sizeof(double)), *fo = calloc(N, sizeof(double));
    double *G = calloc(N, sizeof(double)), *h = calloc(N, sizeof(double)), *ho = calloc(N, sizeof(double));
    double *lx = calloc(N, sizeof(double)), *ly = calloc(N, sizeof(double));
    double *zx = calloc(N, sizeof(double)), *zy = calloc(N, sizeof(double));
    double *dx = calloc(N, sizeof(double)), *dy = calloc(N, sizeof(double));
    double *wx = calloc(N, sizeof(double)), *wy = calloc(N, sizeof(double));
    double *t1 = calloc(N, sizeof(double)), *s = calloc(N, sizeof(double)), *y = calloc(N, sizeof(double));
    double *gs = calloc(M, sizeof(double)), *r = calloc(M, sizeof(double)), *p = calloc(M, sizeof(double));

    for (size_t j = 0; j < M; ++j) gs[j] = beta * m[j];
    if (x0)
        for (size_t i = 0; i < N; ++i) f[i] = beta * x0[i];
    /* r = A f - g ; h = mu A^T r */
    or_project(g, f, r);
    for (size_t j = 0; j < M; ++j) r[j] -= gs[j];
    or_backproject(g, r, h);
    for (size_t i = 0; i < N; ++i) h[i] *= mu;

    double alpha = 0.0, relchg = 0.0;
    int k;
    for (k = 0; k < K; ++k) {
        /* z-step (Eq. 8): z = shrink(grad f - lambda/rho, 1/rho) */
        or_grad(nx, ny, f, dx, dy);
        double tvf = 0.0;
        for (size_t i = 0; i < N; ++i) {
            tvf += sqrt(dx[i] * dx[i] + dy[i] * dy[i]);
            wx[i] = dx[i] - lx[i] / rho;
            wy[i] = dy[i] - ly[i] / rho;
        }
        or_shrink(N, wx, wy, 1.0 / rho, zx, zy);
        /* G = mu A^T (A f - g) + rho grad^T (grad f - z) - grad^T lambda (Eq. 9) */
        for (size_t i = 0; i < N; ++i) {
            wx[i] = rho * (dx[i] - zx[i]) - lx[i];
            wy[i] = rho * (dy[i] - zy[i]) - ly[i];
        }
        or_gradT(nx, ny, wx, wy, G);
        for (size_t i = 0; i < N; ++i) G[i] += h[i];
        double pres = 0.0;
        for (size_t i = 0; i < N; ++i)
            pres += (dx[i] - zx[i]) * (dx[i] - zx[i]) + (dy[i] - zy[i]) * (dy[i] - zy[i]);
        if (k == 0) {
            /* exact minimiser of the f-subproblem along -G */
            or_project(g, G, p);
            or_grad(nx, ny, G, wx, wy);
            double gg = dot(N, G, G);
            double den = mu * dot(M, p, p) + rho * (dot(N, wx, wx) + dot(N, wy, wy));
            alpha = den > 0.0 ? gg / den : 0.0;
        }
        if (log) {
            double *row = log + (size_t)k * 5;
            row[0] = tvf + 0.5 * mu * dot(M, r, r);
            row[1] = alpha;
            row[2] = sqrt(pres);
            row[3] = relchg;
            row[4] = sqrt(dot(N, G, G));
        }
        /* f-step (Eq. 9) and the new gradient's data part */
        memcpy(fo, f, N * sizeof(double));
        memcpy(ho, h, N * sizeof(double));
        for (size_t i = 0; i < N; ++i) f[i] -= alpha * G[i];
        if (nonneg)  /* projection onto the non-negative images */
            for (size_t i = 0; i < N; ++i) f[i] = f[i] > 0.0 ? f[i] : 0.0;
        or_project(g, f, r);
        for (size_t j = 0; j < M; ++j) r[j] -= gs[j];
        or_backproject(g, r, h);
        for (size_t i = 0; i < N; ++i) h[i] *= mu;
        /* BB step from s = f^{k+1} - f^k, y = change of the f-gradient */
        for (size_t i = 0; i < N; ++i) s[i] = f[i] - fo[i];
        or_grad(nx, ny, s, wx, wy);
        or_gradT(nx, ny, wx, wy, t1);
        for (size_t i = 0; i < N; ++i) y[i] = (h[i] - ho[i]) + rho * t1[i];
        double ss = dot(N, s, s), sy = dot(N, s, y), yy = dot(N, y, y);
        if (sy > 0.0) {
            const double bb1 = ss / sy, bb2 = yy > 0.0 ? sy / yy : bb1;
            if (step_rule == 1) alpha = bb2;
            else if (step_rule == 2) alpha = bb2 / bb1 < 0.5 ? bb2 : bb1;  /* adaptive */
            else alpha = bb1;
        }
        double fn = sqrt(dot(N, fo, fo));
        relchg = fn > 0.0 ? sqrt(ss) / fn : (ss > 0.0 ? INFINITY : 0.0);
        /* multiplier step (Eq. 7) */
        or_grad(nx, ny, f, dx, dy);
        for (size_t i = 0; i < N; ++i) {
            lx[i] -= xi * (dx[i] - zx[i]);
            ly[i] -= xi * (dy[i] - zy[i]);
        }
        if (tol > 0.0 && relchg < tol) {
            ++k;
            break;
        }
    }
    if (log) {
        or_grad(nx, ny, f, dx, dy);
        double tvf = 0.0;
        for (size_t i = 0; i < N; ++i) tvf += sqrt(dx[i] * dx[i] + dy[i] * dy[i]);
        double *row = log + (size_t)k * 5;
        row[0] = tvf + 0.5 * mu * dot(M, r, r);
        row[1] = alpha;
        row[2] = 0.0;
        row[3] = relchg;
        row[4] = 0.0;
    }
    for (size_t i = 0; i < N; ++i) x_out[i] = f[i] / beta;
    if (lam_out) {
        memcpy(lam_out, lx, N * sizeof(double));
        memcpy(lam_out + N, ly, N * sizeof(double));
    }
    if (z_out) {
        memcpy(z_out, zx, N * sizeof(double));
        memcpy(z_out + N, zy, N * sizeof(double));
    }
    free(f); free(fo); free(G); free(h); free(ho); free(lx); free(ly); free(zx); free(zy);
    free(dx); free(dy); free(wx); free(wy); free(t1); free(s); free(y); free(gs); free(r); free(p);
    return k;
}

/* Eq. 12: x_h = eta_1H u1 + eta_2H u2, x_l = eta_1L u1 + eta_2L u2, inverted
 * in closed form per pixel. */
void or_dinv(size_t n, double e1h, double e2h, double e1l, double e2l, const double *xh,
             const double *xl, double *u1, double *u2)
{
    double det = e1h * e2l - e2h * e1l;
    for (size_t i = 0; i < n; ++i) {
        u1[i] = (e2l * xh[i] - e2h * xl[i]) / det;
        u2[i] = (e1h * xl[i] - e1l * xh[i]) / det;
    }
}

/*
 * Edge map and pair weights of the penalty (the edge-weighted R after Eq. 14),
 * in FP64.  The Prewitt operator with replicated borders: gx = (sum of the
 * column to the right over rows r-1..r+1) - (sum of the column to the left),
 * gy = (sum of the row below over columns c-1..c+1) - (sum of the row above);
 * m2 = gx^2 + gy^2; a pixel is an edge where m2 > tau^2 max(m2), i.e.
 * |grad| > tau max |grad|.  e_right[r][c] couples (r,c)-(r,c+1), e_down[r][c]
 * couples (r,c)-(r+1,c): eps if either pixel is an edge, else 1; pairs that
 * leave the image get 0.  m2_out (optional) receives m2, *thr_out (optional)
 * the threshold tau^2 max(m2).
 */
void or_edges(int nx, int ny, const double *x, double tau, double eps, double *e_right,
              double *e_down, uint8_t *edge, double *m2_out, double *thr_out)
{
    size_t N = (size_t)nx * ny;
    double *m2 = malloc(N * sizeof(double));
    double mx = 0.0;
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c < nx; ++c) {
            int ru = r > 0 ? r - 1 : 0, rd = r < ny - 1 ? r + 1 : ny - 1;
            int cl = c > 0 ? c - 1 : 0, cr = c < nx - 1 ? c + 1 : nx - 1;
#define X(rr, cc) x[(size_t)(rr) * nx + (cc)]
            double gx = (X(ru, cr) + X(r, cr) + X(rd, cr)) - (X(ru, cl) + X(r, cl) + X(rd, cl));
            double gy = (X(rd, cl) + X(rd, c) + X(rd, cr)) - (X(ru, cl) + X(ru, c) + X(ru, cr));
#undef X
            double v = gx * gx + gy * gy;
            m2[(size_t)r * nx + c] = v;
            if (v > mx) mx = v;
        }
    double thr = tau * tau * mx;
    for (size_t i = 0; i < N; ++i) edge[i] = m2[i] > thr;
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c < nx; ++c) {
            size_t i = (size_t)r * nx + c;
            e_right[i] = c + 1 < nx ? ((edge[i] || edge[i + 1]) ? eps : 1.0) : 0.0;
            e_down[i] = r + 1 < ny ? ((edge[i] || edge[i + nx]) ? eps : 1.0) : 0.0;
        }
    if (m2_out) memcpy(m2_out, m2, N * sizeof(double));
    if (thr_out) *thr_out = thr;
    free(m2);
}

/* (L u)_i = sum over the 4-neighbours k of e_ik (u_i - u_k) (Eq. 14). */
void or_laplacian(int nx, int ny, const double *er, const double *ed, const double *u, double *out)
{
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c < nx; ++c) {
            size_t i = (size_t)r * nx + c;
            double s = 0.0;
            if (c + 1 < nx) s += er[i] * (u[i] - u[i + 1]);
            if (c >= 1) s += er[i - 1] * (u[i] - u[i - 1]);
            if (r + 1 < ny) s += ed[i] * (u[i] - u[i + nx]);
            if (r >= 1) s += ed[i - nx] * (u[i] - u[i - nx]);
            out[i] = s;
        }
}

/*
 * Jacobi-preconditioned CG for (I + gamma L) u = b, starting from u = b.
 * Stops when |b - (I + gamma L) u| <= tol |b| or after max_iter iterations.
 * Returns the iteration count; *relres receives the final relative residual.
 */
int or_pcg(int nx, int ny, const double *er, const double *ed, double gamma, const double *b,
           double *u, int max_iter, double tol, double *relres)
{
    size_t N = (size_t)nx * ny;
    double *res = malloc(N * sizeof(double)), *z = malloc(N * sizeof(double));
    double *p = malloc(N * sizeof(double)), *q = malloc(N * sizeof(double));
    double *dinv = malloc(N * sizeof(double));
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c < nx; ++c) {
            size_t i = (size_t)r * nx + c;
            double d = 0.0;
            if (c + 1 < nx) d += er[i];
            if (c >= 1) d += er[i - 1];
            if (r + 1 < ny) d += ed[i];
            if (r >= 1) d += ed[i - nx];
            dinv[i] = 1.0 / (1.0 + gamma * d);
        }
    memcpy(u, b, N * sizeof(double));
    or_laplacian(nx, ny, er, ed, u, q);
    for (size_t i = 0; i < N; ++i) res[i] = b[i] - (u[i] + gamma * q[i]);
    double bn = sqrt(dot(N, b, b));
    double rn = sqrt(dot(N, res, res));
    int it = 0;
    if (bn == 0.0) {
        memset(u, 0, N * sizeof(double));
        rn = 0.0;
        bn = 1.0;
    }
    for (size_t i = 0; i < N; ++i) z[i] = dinv[i] * res[i];
    memcpy(p, z, N * sizeof(double));
    double rz = dot(N, res, z);
    while (it < max_iter && rn > tol * bn) {
        or_laplacian(nx, ny, er, ed, p, q);
        for (size_t i = 0; i < N; ++i) q[i] = p[i] + gamma * q[i];
        double pq = dot(N, p, q);
        if (pq <= 0.0) break;
        double a = rz / pq;
        for (size_t i = 0; i < N; ++i) {
            u[i] += a * p[i];
            res[i] -= a * q[i];
        }
        ++it;
        rn = sqrt(dot(N, res, res));
        for (size_t i = 0; i < N; ++i) z[i] = dinv[i] * res[i];
        double rz2 = dot(N, res, z);
        double beta = rz2 / rz;
        rz = rz2;
        for (size_t i = 0; i < N; ++i) p[i] = z[i] + beta * p[i];
    }
    if (relres) *relres = rn / bn;
    free(res); free(z); free(p); free(q); free(dinv);
    return it;
}

/*
 * Attenuation-space PLS: u = (u1, u2) minimising |x - D u|^2 + gamma R(u)
 * (D applied per pixel, Eq. 12; R of Eq. 14 per material, Hessian 2L), i.e.
 * the linear system (D^T D (x) I + gamma I (x) L) u = D^T x, solved by
 * conjugate gradients preconditioned with the 2 x 2 per-pixel diagonal block
 * D^T D + gamma diag(L), from u = D^{-1} x, until |res| <= tol |D^T x| (joint
 * norms over both materials) or max_iter iterations.  Returns the iterations.
 * The core takes the grid's L (lapf on one material image) and diag(L) (dg),
 * so that the image and the volume solvers share it.
 */
typedef void (*or_lap_fn)(const void *ctx, const double *u, double *out);

static int pcg_att_core(size_t N, or_lap_fn lapf, const void *ctx, const double *dg, double e1h,
                        double e2h, double e1l, double e2l, double gamma, const double *xh,
                        const double *xl, double *u1, double *u2, int max_iter, double tol,
                        double *relres)
{
    /* D^T D = [[g11, g12], [g12, g22]] */
    const double g11 = e1h * e1h + e1l * e1l, g12 = e1h * e2h + e1l * e2l;
    const double g22 = e2h * e2h + e2l * e2l;
    double *c = malloc(2 * N * sizeof(double)), *u = malloc(2 * N * sizeof(double));
    double *res = malloc(2 * N * sizeof(double)), *z = malloc(2 * N * sizeof(double));
    double *p = malloc(2 * N * sizeof(double)), *q = malloc(2 * N * sizeof(double));
    double *lap = malloc(N * sizeof(double));
    double det = e1h * e2l - e2h * e1l;
    for (size_t i = 0; i < N; ++i) {
        c[i] = e1h * xh[i] + e1l * xl[i];
        c[N + i] = e2h * xh[i] + e2l * xl[i];
        u[i] = (e2l * xh[i] - e2h * xl[i]) / det;
        u[N + i] = (e1h * xl[i] - e1l * xh[i]) / det;
    }
    /* q = A v for the two-material vector v */
    #define APPLY(v, out)                                                         \
        for (int m = 0; m < 2; ++m) {                                             \
            lapf(ctx, (v) + m * N, lap);                                          \
            for (size_t i = 0; i < N; ++i) {                                      \
                double dd = m == 0 ? g11 * (v)[i] + g12 * (v)[N + i]              \
                                   : g12 * (v)[i] + g22 * (v)[N + i];             \
                (out)[m * N + i] = dd + gamma * lap[i];                           \
            }                                                                     \
        }
    /* z = P^{-1} res with the per-pixel block P = D^T D + gamma diag(L) I */
    #define PRECOND()                                                             \
        for (size_t i = 0; i < N; ++i) {                                          \
            double a11 = g11 + gamma * dg[i], a22 = g22 + gamma * dg[i];          \
            double dt = a11 * a22 - g12 * g12;                                    \
            z[i] = (a22 * res[i] - g12 * res[N + i]) / dt;                        \
            z[N + i] = (a11 * res[N + i] - g12 * res[i]) / dt;                    \
        }
    APPLY(u, q);
    for (size_t i = 0; i < 2 * N; ++i) res[i] = c[i] - q[i];
    double cn = sqrt(dot(2 * N, c, c)), rn = sqrt(dot(2 * N, res, res));
    if (cn == 0.0) cn = 1.0;
    PRECOND();
    memcpy(p, z, 2 * N * sizeof(double));
    double rz = dot(2 * N, res, z);
    int it = 0;
    while (it < max_iter && rn > tol * cn) {
        APPLY(p, q);
        double pq = dot(2 * N, p, q);
        if (pq <= 0.0) break;
        double a = rz / pq;
        for (size_t i = 0; i < 2 * N; ++i) {
            u[i] += a * p[i];
            res[i] -= a * q[i];
        }
        ++it;
        rn = sqrt(dot(2 * N, res, res));
        PRECOND();
        double rz2 = dot(2 * N, res, z);
        double beta = rz2 / rz;
        rz = rz2;
        for (size_t i = 0; i < 2 * N; ++i) p[i] = z[i] + beta * p[i];
    }
    #undef APPLY
    #undef PRECOND
    memcpy(u1, u, N * sizeof(double));
    memcpy(u2, u + N, N * sizeof(double));
    if (relres) *relres = rn / cn;
    free(c); free(u); free(res); free(z); free(p); free(q); free(lap);
    return it;
}

typedef struct {
    int nx, ny;
    const double *er, *ed;
} or_lap2_ctx;

static void lap2_of(const void *ctx, const double *u, double *out)
{
    const or_lap2_ctx *k = (const or_lap2_ctx *)ctx;
    or_laplacian(k->nx, k->ny, k->er, k->ed, u, out);
}

int or_pcg_att(int nx, int ny, const double *er, const double *ed, double e1h, double e2h,
               double e1l, double e2l, double gamma, const double *xh, const double *xl,
               double *u1, double *u2, int max_iter, double tol, double *relres)
{
    const size_t N = (size_t)nx * ny;
    double *dg = malloc(N * sizeof(double));
    for (int r = 0; r < ny; ++r)
        for (int cc = 0; cc < nx; ++cc) {
            size_t i = (size_t)r * nx + cc;
            double d = 0.0;
            if (cc + 1 < nx) d += er[i];
            if (cc >= 1) d += er[i - 1];
            if (r + 1 < ny) d += ed[i];
            if (r >= 1) d += ed[i - nx];
            dg[i] = d;
        }
    const or_lap2_ctx ctx = {nx, ny, er, ed};
    int it = pcg_att_core(N, lap2_of, &ctx, dg, e1h, e2h, e1l, e2l, gamma, xh, xl, u1, u2,
                          max_iter, tol, relres);
    free(dg);
    return it;
}

/*
 * ADM-TV of both energies with the TV coupled across them: the norm of
 * Eq. 2 taken over the 4-vector (grad f_high, grad f_low) at every pixel,
 * so the z-step (Eq. 8) shrinks the two energies' 2-vectors together:
 * z_e = max(|v| - 1/rho, 0) v_e / |v| with |v|^2 = |v_high|^2 + |v_low|^2.
 * Given z and lambda the f-subproblem still separates by energy, so each
 * energy keeps its own gradient step (Eq. 9), BB step and multiplier
 * (Eq. 7), exactly as in or_adm.  Fixed iteration count.
 * In:  m [2][V][B], beta[2], x0 [2][ny][nx] or NULL.
 * Out: x_out [2][ny][nx]; log [2][(K+1)][2] rows (J part, alpha^k) per
 *      energy: energy 0 carries the joint TV, energy 1 none, each its own
 *      mu/2 |r_e|^2, so that the two columns sum to the objective.
 */
void or_adm_coupled(const or_geom *g, const double *m, const double *beta, double mu, double rho,
                    double xi, int K, const double *x0, double *x_out, double *log, int nonneg)
{
    const int nx = g->nx, ny = g->ny;
    const size_t N = (size_t)nx * ny, M = (size_t)g->n_views * g->n_bins;
    double *f[2], *fo[2], *G[2], *h[2], *ho[2], *lx[2], *ly[2], *zx[2], *zy[2], *dx[2], *dy[2];
    double *wx = calloc(N, sizeof(double)), *wy = calloc(N, sizeof(double));
    double *t1 = calloc(N, sizeof(double)), *s = calloc(N, sizeof(double));
    double *y = calloc(N, sizeof(double)), *p = calloc(M, sizeof(double));
    double *gs[2], *r[2], alpha[2] = {0.0, 0.0};
    for (int e = 0; e < 2; ++e) {
        f[e] = calloc(N, sizeof(double)); fo[e] = calloc(N, sizeof(double));
        G[e] = calloc(N, sizeof(double)); h[e] = calloc(N, sizeof(double));
        ho[e] = calloc(N, sizeof(double)); lx[e] = calloc(N, sizeof(double));
        ly[e] = calloc(N, sizeof(double)); zx[e] = calloc(N, sizeof(double));
        zy[e] = calloc(N, sizeof(double)); dx[e] = calloc(N, sizeof(double));
        dy[e] = calloc(N, sizeof(double)); gs[e] = calloc(M, sizeof(double));
        r[e] = calloc(M, sizeof(double));
        for (size_t j = 0; j < M; ++j) gs[e][j] = beta[e] * m[e * M + j];
        if (x0)
            for (size_t i = 0; i < N; ++i) f[e][i] = beta[e] * x0[e * N + i];
        or_project(g, f[e], r[e]);
        for (size_t j = 0; j < M; ++j) r[e][j] -= gs[e][j];
        or_backproject(g, r[e], h[e]);
        for (size_t i = 0; i < N; ++i) h[e][i] *= mu;
    }
    int k;
    for (k = 0; k <= K; ++k) {
        for (int e = 0; e < 2; ++e) or_grad(nx, ny, f[e], dx[e], dy[e]);
        double tvj = 0.0;
        for (size_t i = 0; i < N; ++i)
            tvj += sqrt(dx[0][i] * dx[0][i] + dy[0][i] * dy[0][i] + dx[1][i] * dx[1][i] +
                        dy[1][i] * dy[1][i]);
        for (int e = 0; e < 2; ++e) {
            double *row = log + ((size_t)e * (K + 1) + k) * 2;
            row[0] = (e == 0 ? tvj : 0.0) + 0.5 * mu * dot(M, r[e], r[e]);
            row[1] = alpha[e];
        }
        if (k == K) break;
        /* joint z-step */
        for (size_t i = 0; i < N; ++i) {
            double v[4] = {dx[0][i] - lx[0][i] / rho, dy[0][i] - ly[0][i] / rho,
                           dx[1][i] - lx[1][i] / rho, dy[1][i] - ly[1][i] / rho};
            double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3]);
            double sh = n > 1.0 / rho ? (n - 1.0 / rho) / n : 0.0;
            zx[0][i] = sh * v[0];
            zy[0][i] = sh * v[1];
            zx[1][i] = sh * v[2];
            zy[1][i] = sh * v[3];
        }
        for (int e = 0; e < 2; ++e) {
            /* G (Eq. 9) */
            for (size_t i = 0; i < N; ++i) {
                wx[i] = rho * (dx[e][i] - zx[e][i]) - lx[e][i];
                wy[i] = rho * (dy[e][i] - zy[e][i]) - ly[e][i];
            }
            or_gradT(nx, ny, wx, wy, G[e]);
            for (size_t i = 0; i < N; ++i) G[e][i] += h[e][i];
            if (k == 0) {
                or_project(g, G[e], p);
                or_grad(nx, ny, G[e], wx, wy);
                double gg = dot(N, G[e], G[e]);
                double den = mu * dot(M, p, p) + rho * (dot(N, wx, wx) + dot(N, wy, wy));
                alpha[e] = den > 0.0 ? gg / den : 0.0;
                log[((size_t)e * (K + 1) + k) * 2 + 1] = alpha[e];
            }
            memcpy(fo[e], f[e], N * sizeof(double));
            memcpy(ho[e], h[e], N * sizeof(double));
            for (size_t i = 0; i < N; ++i) f[e][i] -= alpha[e] * G[e][i];
            if (nonneg)
                for (size_t i = 0; i < N; ++i) f[e][i] = f[e][i] > 0.0 ? f[e][i] : 0.0;
            or_project(g, f[e], r[e]);
            for (size_t j = 0; j < M; ++j) r[e][j] -= gs[e][j];
            or_backproject(g, r[e], h[e]);
            for (size_t i = 0; i < N; ++i) h[e][i] *= mu;
            for (size_t i = 0; i < N; ++i) s[i] = f[e][i] - fo[e][i];
            or_grad(nx, ny, s, wx, wy);
            or_gradT(nx, ny, wx, wy, t1);
            for (size_t i = 0; i < N; ++i) y[i] = (h[e][i] - ho[e][i]) + rho * t1[i];
            double ss = dot(N, s, s), sy = dot(N, s, y);
            if (sy > 0.0) alpha[e] = ss / sy;
            /* multiplier step (Eq. 7) */
            or_grad(nx, ny, f[e], wx, wy);
            for (size_t i = 0; i < N; ++i) {
                lx[e][i] -= xi * (wx[i] - zx[e][i]);
                ly[e][i] -= xi * (wy[i] - zy[e][i]);
            }
        }
    }
    for (int e = 0; e < 2; ++e)
        for (size_t i = 0; i < N; ++i) x_out[e * N + i] = f[e][i] / beta[e];
    for (int e = 0; e < 2; ++e) {
        free(f[e]); free(fo[e]); free(G[e]); free(h[e]); free(ho[e]); free(lx[e]); free(ly[e]);
        free(zx[e]); free(zy[e]); free(dx[e]); free(dy[e]); free(gs[e]); free(r[e]);
    }
    free(wx); free(wy); free(t1); free(s); free(y); free(p);
}

/* ----------------------------------------------------------- cone beam ---
 * 3-D circular cone beam (the scanner geometry of Sec. 3; the slice model
 * above is its central plane).  Source s = R (cos t, sin t, 0); flat detector
 * centred at -(D - R)(cos t, sin t, 0) with axes e_u = (-sin t, cos t, 0) and
 * e_v = (0, 0, 1); bin b of row j at u_b = (b - (B-1)/2) du + offset,
 * v_j = (j - (J-1)/2) dv.  Volume nx x ny x nz cubic voxels of side `voxel`,
 * centred on the isocentre, stored [z][y][x].  Joseph's model in 3-D: the ray
 * steps along the in-plane axis it is more aligned with and, on each plane of
 * that axis, interpolates bilinearly between the four nearest voxel centres
 * (the other in-plane axis and z); samples are scaled by the path length per
 * plane, voxel / |cos| of the angle to the driving axis; voxels outside the
 * volume are zero.  Projections are [V][J][B].
 */
typedef struct {
    int32_t nx, ny, nz;
    double voxel;
    int32_t n_views;
    const double *angles;
    int32_t n_bins, n_rows;
    double bin, row, det_offset, sod, sdd;
} or_geom3;

static double cone_walk(const or_geom3 *g, int v, int j, int b, double *X, double y, int mode)
{
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const double dl = g->voxel;
    const double th = g->angles ? g->angles[v] : 2.0 * M_PI * v / g->n_views;
    const double ct = cos(th), st = sin(th);
    const double u = (b - (g->n_bins - 1) / 2.0) * g->bin + g->det_offset;
    const double w = (j - (g->n_rows - 1) / 2.0) * g->row;
    const double sx = g->sod * ct, sy = g->sod * st, sz = 0.0;
    const double px = -(g->sdd - g->sod) * ct - u * st, py = -(g->sdd - g->sod) * st + u * ct;
    const double pz = w;
    const double dx = px - sx, dy = py - sy, dz = pz - sz;
    const double len = sqrt(dx * dx + dy * dy + dz * dz);
    const size_t plane = (size_t)nx * ny;
    double acc = 0.0;
    const int xmaj = fabs(dx) >= fabs(dy);
    const int nl = xmaj ? nx : ny, nq = xmaj ? ny : nx;
    const double L = dl * len / (xmaj ? fabs(dx) : fabs(dy));
    for (int i = 0; i < nl; ++i) {
        double t;  /* ray parameter at the plane's centre */
        if (xmaj) t = ((i - (nx - 1) / 2.0) * dl - sx) / dx;
        else t = ((i - (ny - 1) / 2.0) * dl - sy) / dy;
        const double qa = (xmaj ? sy + t * dy : sx + t * dx) / dl + (nq - 1) / 2.0;
        const double qz = (sz + t * dz) / dl + (nz - 1) / 2.0;
        const double fa = floor(qa), fz = floor(qz);
        const int a0 = (int)fa, z0 = (int)fz;
        const double wa = qa - fa, wz = qz - fz;
        for (int da = 0; da <= 1; ++da)
            for (int dz2 = 0; dz2 <= 1; ++dz2) {
                const int a = a0 + da, zz = z0 + dz2;
                if (fa < -1.0 || fa > nq - 1.0 || fz < -1.0 || fz > nz - 1.0) continue;
                if (a < 0 || a >= nq || zz < 0 || zz >= nz) continue;
                const double wt = (da ? wa : 1.0 - wa) * (dz2 ? wz : 1.0 - wz);
                const size_t idx = (size_t)zz * plane + (xmaj ? (size_t)a * nx + i : (size_t)i * nx + a);
                if (mode == 0) acc += L * wt * X[idx];
                else X[idx] += L * wt * y;
            }
    }
    return acc;
}

/* proj[v][j][b] = (A vol) */
void or_project3(const or_geom3 *g, const double *vol, double *proj)
{
    const int V = g->n_views, J = g->n_rows, B = g->n_bins;
#pragma omp parallel for schedule(static)
    for (int v = 0; v < V; ++v)
        for (int j = 0; j < J; ++j)
            for (int b = 0; b < B; ++b)
                proj[((size_t)v * J + j) * B + b] = cone_walk(g, v, j, b, (double *)vol, 0.0, 0);
}

/* vol = A^T proj, views in fixed chunks with private volumes summed in order. */
void or_backproject3(const or_geom3 *g, const double *proj, double *vol)
{
    const int V = g->n_views, J = g->n_rows, B = g->n_bins;
    const size_t N = (size_t)g->nx * g->ny * g->nz;
    int T = or_num_threads();
    if (T > V) T = V;
    if (T < 1) T = 1;
    double *buf = (double *)calloc((size_t)T * N, sizeof(double));
#pragma omp parallel for schedule(static, 1) num_threads(T)
    for (int t = 0; t < T; ++t) {
        int v0 = (int)((int64_t)V * t / T), v1 = (int)((int64_t)V * (t + 1) / T);
        double *mine = buf + (size_t)t * N;
        for (int v = v0; v < v1; ++v)
            for (int j = 0; j < J; ++j)
                for (int b = 0; b < B; ++b)
                    cone_walk(g, v, j, b, mine, proj[((size_t)v * J + j) * B + b], 1);
    }
    for (size_t i = 0; i < N; ++i) {
        double s = 0.0;
        for (int t = 0; t < T; ++t) s += buf[(size_t)t * N + i];
        vol[i] = s;
    }
    free(buf);
}

/* ------------------------------------------------------- 3-D ADM-TV ---
 * The reconstruction of Eq. 10 on a volume: Eq. 2's TV with backward
 * differences along x, y and z (zero on the first column, row and slice),
 * the isotropic shrinkage of Eq. 8 on the 3-vector, and the cone-beam
 * projector pair above in place of W.  Same steps, order, BB1 step and log
 * as or_adm (no projection, fixed iteration count).
 */
static void grad3(int nx, int ny, int nz, const double *x, double *gx, double *gy, double *gz)
{
    const size_t P = (size_t)nx * ny;
    for (int zz = 0; zz < nz; ++zz)
        for (int r = 0; r < ny; ++r)
            for (int c = 0; c < nx; ++c) {
                size_t i = (size_t)zz * P + (size_t)r * nx + c;
                gx[i] = c >= 1 ? x[i] - x[i - 1] : 0.0;
                gy[i] = r >= 1 ? x[i] - x[i - nx] : 0.0;
                gz[i] = zz >= 1 ? x[i] - x[i - P] : 0.0;
            }
}

/* Exact adjoint of grad3. */
static void gradT3(int nx, int ny, int nz, const double *px, const double *py, const double *pz,
                   double *out)
{
    const size_t P = (size_t)nx * ny;
    for (int zz = 0; zz < nz; ++zz)
        for (int r = 0; r < ny; ++r)
            for (int c = 0; c < nx; ++c) {
                size_t i = (size_t)zz * P + (size_t)r * nx + c;
                double s = 0.0;
                if (c >= 1) s += px[i];
                if (c + 1 <= nx - 1) s -= px[i + 1];
                if (r >= 1) s += py[i];
                if (r + 1 <= ny - 1) s -= py[i + nx];
                if (zz >= 1) s += pz[i];
                if (zz + 1 <= nz - 1) s -= pz[i + P];
                out[i] = s;
            }
}

void or_grad3(int nx, int ny, int nz, const double *x, double *g3)
{
    const size_t N = (size_t)nx * ny * nz;
    grad3(nx, ny, nz, x, g3, g3 + N, g3 + 2 * N);
}

void or_gradT3(int nx, int ny, int nz, const double *g3, double *out)
{
    const size_t N = (size_t)nx * ny * nz;
    gradT3(nx, ny, nz, g3, g3 + N, g3 + 2 * N, out);
}

/* m [V][J][B] projections of one energy; x_out [nz][ny][nx] = f / beta;
 * log [(K+1)][5] as in or_adm; nonneg and step_rule as in or_adm. */
int or_adm3(const or_geom3 *g, const double *m, double beta, double mu, double rho, double xi,
            int K, double tol, const double *x0, double *x_out, double *log, int nonneg,
            int step_rule)
{
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const size_t N = (size_t)nx * ny * nz;
    const size_t M = (size_t)g->n_views * g->n_rows * g->n_bins;
    double *f = calloc(N, 8), *fo = calloc(N, 8), *G = calloc(N, 8), *h = calloc(N, 8),
           *ho = calloc(N, 8), *t1 = calloc(N, 8), *sv = calloc(N, 8), *y = calloc(N, 8);
    double *l[3], *z[3], *d[3], *w[3];
    for (int a = 0; a < 3; ++a) {
        l[a] = calloc(N, 8); z[a] = calloc(N, 8); d[a] = calloc(N, 8); w[a] = calloc(N, 8);
    }
    double *gs = calloc(M, 8), *r = calloc(M, 8), *p = calloc(M, 8);
    for (size_t j = 0; j < M; ++j) gs[j] = beta * m[j];
    if (x0)  /* warm start f = beta x0; lambda = 0 either way */
        for (size_t i = 0; i < N; ++i) f[i] = beta * x0[i];
    or_project3(g, f, r);
    for (size_t j = 0; j < M; ++j) r[j] -= gs[j];
    or_backproject3(g, r, h);
    for (size_t i = 0; i < N; ++i) h[i] *= mu;
    double alpha = 0.0, relchg = 0.0;
    int k;
    for (k = 0; k < K; ++k) {
        /* z-step (Eq. 8) */
        grad3(nx, ny, nz, f, d[0], d[1], d[2]);
        double tvf = 0.0, pres = 0.0;
        for (size_t i = 0; i < N; ++i) {
            tvf += sqrt(d[0][i] * d[0][i] + d[1][i] * d[1][i] + d[2][i] * d[2][i]);
            double v0 = d[0][i] - l[0][i] / rho, v1 = d[1][i] - l[1][i] / rho,
                   v2 = d[2][i] - l[2][i] / rho;
            double mag = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
            double sh = mag > 1.0 / rho ? (mag - 1.0 / rho) / mag : 0.0;
            z[0][i] = sh * v0; z[1][i] = sh * v1; z[2][i] = sh * v2;
        }
        /* G (Eq. 9) */
        for (int a = 0; a < 3; ++a)
            for (size_t i = 0; i < N; ++i) {
                w[a][i] = rho * (d[a][i] - z[a][i]) - l[a][i];
                pres += (d[a][i] - z[a][i]) * (d[a][i] - z[a][i]);
            }
        gradT3(nx, ny, nz, w[0], w[1], w[2], G);
        for (size_t i = 0; i < N; ++i) G[i] += h[i];
        if (k == 0) {  /* exact minimiser of the f-subproblem along -G */
            or_project3(g, G, p);
            grad3(nx, ny, nz, G, w[0], w[1], w[2]);
            double den = mu * dot(M, p, p) + rho * (dot(N, w[0], w[0]) + dot(N, w[1], w[1]) +
                                                   dot(N, w[2], w[2]));
            double gg = dot(N, G, G);
            alpha = den > 0.0 ? gg / den : 0.0;
        }
        if (log) {
            double *row = log + (size_t)k * 5;
            row[0] = tvf + 0.5 * mu * dot(M, r, r);
            row[1] = alpha;
            row[2] = sqrt(pres);
            row[3] = relchg;
            row[4] = sqrt(dot(N, G, G));
        }
        memcpy(fo, f, N * 8);
        memcpy(ho, h, N * 8);
        for (size_t i = 0; i < N; ++i) f[i] -= alpha * G[i];
        if (nonneg)  /* projection onto the non-negative volumes */
            for (size_t i = 0; i < N; ++i) f[i] = f[i] > 0.0 ? f[i] : 0.0;
        or_project3(g, f, r);
        for (size_t j = 0; j < M; ++j) r[j] -= gs[j];
        or_backproject3(g, r, h);
        for (size_t i = 0; i < N; ++i) h[i] *= mu;
        /* BB1 step from s = f^{k+1} - f^k and the change of the f-gradient */
        for (size_t i = 0; i < N; ++i) sv[i] = f[i] - fo[i];
        grad3(nx, ny, nz, sv, w[0], w[1], w[2]);
        gradT3(nx, ny, nz, w[0], w[1], w[2], t1);
        for (size_t i = 0; i < N; ++i) y[i] = (h[i] - ho[i]) + rho * t1[i];
        double ss = dot(N, sv, sv), sy = dot(N, sv, y), yy = dot(N, y, y);
        if (sy > 0.0) {
            const double bb1 = ss / sy, bb2 = yy > 0.0 ? sy / yy : bb1;
            if (step_rule == 1) alpha = bb2;
            else if (step_rule == 2) alpha = bb2 / bb1 < 0.5 ? bb2 : bb1;  /* adaptive */
            else alpha = bb1;
        }
        double fn = sqrt(dot(N, fo, fo));
        relchg = fn > 0.0 ? sqrt(ss) / fn : (ss > 0.0 ? INFINITY : 0.0);
        /* multiplier step (Eq. 7) */
        grad3(nx, ny, nz, f, d[0], d[1], d[2]);
        for (int a = 0; a < 3; ++a)
            for (size_t i = 0; i < N; ++i) l[a][i] -= xi * (d[a][i] - z[a][i]);
        if (tol > 0.0 && relchg < tol) {  /* the stop rule of Sec. 3 */
            ++k;
            break;
        }
    }
    if (log) {
        grad3(nx, ny, nz, f, d[0], d[1], d[2]);
        double tvf = 0.0;
        for (size_t i = 0; i < N; ++i)
            tvf += sqrt(d[0][i] * d[0][i] + d[1][i] * d[1][i] + d[2][i] * d[2][i]);
        double *row = log + (size_t)k * 5;
        row[0] = tvf + 0.5 * mu * dot(M, r, r);
        row[1] = alpha;
        row[2] = 0.0;
        row[3] = relchg;
        row[4] = 0.0;
    }
    for (size_t i = 0; i < N; ++i) x_out[i] = f[i] / beta;
    for (int a = 0; a < 3; ++a) { free(l[a]); free(z[a]); free(d[a]); free(w[a]); }
    free(f); free(fo); free(G); free(h); free(ho); free(t1); free(sv); free(y);
    free(gs); free(r); free(p);
    return k;
}

/*
 * ADM-TV of both energies on a volume with the TV coupled across them (as
 * or_adm_coupled, with the 3-D differences): the z-step shrinks the 6-vector
 * (grad f_high, grad f_low) at every voxel, |v|^2 summed as energy 0's three
 * components and then energy 1's; each energy keeps its own f-step, BB1 step
 * and multiplier.  Fixed iteration count.
 * In:  m [2][V][J][B], beta[2], x0 [2][nz][ny][nx] or NULL.
 * Out: x_out [2][nz][ny][nx]; log [2][(K+1)][2] rows (J part, alpha^k) per
 *      energy: energy 0 carries the joint TV, energy 1 none.
 */
void or_adm3_coupled(const or_geom3 *g, const double *m, const double *beta, double mu,
                     double rho, double xi, int K, const double *x0, double *x_out, double *log,
                     int nonneg)
{
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const size_t N = (size_t)nx * ny * nz;
    const size_t M = (size_t)g->n_views * g->n_rows * g->n_bins;
    double *f[2], *fo[2], *G[2], *h[2], *ho[2], *l[2][3], *z[2][3], *d[2][3], *gs[2], *r[2];
    double *w[3], alpha[2] = {0.0, 0.0};
    for (int a = 0; a < 3; ++a) w[a] = calloc(N, 8);
    double *t1 = calloc(N, 8), *sv = calloc(N, 8), *y = calloc(N, 8), *p = calloc(M, 8);
    for (int e = 0; e < 2; ++e) {
        f[e] = calloc(N, 8); fo[e] = calloc(N, 8); G[e] = calloc(N, 8);
        h[e] = calloc(N, 8); ho[e] = calloc(N, 8);
        for (int a = 0; a < 3; ++a) {
            l[e][a] = calloc(N, 8); z[e][a] = calloc(N, 8); d[e][a] = calloc(N, 8);
        }
        gs[e] = calloc(M, 8); r[e] = calloc(M, 8);
        for (size_t j = 0; j < M; ++j) gs[e][j] = beta[e] * m[e * M + j];
        if (x0)
            for (size_t i = 0; i < N; ++i) f[e][i] = beta[e] * x0[e * N + i];
        or_project3(g, f[e], r[e]);
        for (size_t j = 0; j < M; ++j) r[e][j] -= gs[e][j];
        or_backproject3(g, r[e], h[e]);
        for (size_t i = 0; i < N; ++i) h[e][i] *= mu;
    }
    for (int k = 0; k <= K; ++k) {
        for (int e = 0; e < 2; ++e) grad3(nx, ny, nz, f[e], d[e][0], d[e][1], d[e][2]);
        double tvj = 0.0;
        for (size_t i = 0; i < N; ++i) {
            double q = 0.0;
            for (int e = 0; e < 2; ++e)
                for (int a = 0; a < 3; ++a) q += d[e][a][i] * d[e][a][i];
            tvj += sqrt(q);
        }
        for (int e = 0; e < 2; ++e) {
            double *row = log + ((size_t)e * (K + 1) + k) * 2;
            row[0] = (e == 0 ? tvj : 0.0) + 0.5 * mu * dot(M, r[e], r[e]);
            row[1] = alpha[e];
        }
        if (k == K) break;
        /* joint z-step */
        for (size_t i = 0; i < N; ++i) {
            double v[2][3], q = 0.0;
            for (int e = 0; e < 2; ++e)
                for (int a = 0; a < 3; ++a) {
                    v[e][a] = d[e][a][i] - l[e][a][i] / rho;
                    q += v[e][a] * v[e][a];
                }
            const double n = sqrt(q);
            const double sh = n > 1.0 / rho ? (n - 1.0 / rho) / n : 0.0;
            for (int e = 0; e < 2; ++e)
                for (int a = 0; a < 3; ++a) z[e][a][i] = sh * v[e][a];
        }
        for (int e = 0; e < 2; ++e) {
            /* G (Eq. 9) */
            for (int a = 0; a < 3; ++a)
                for (size_t i = 0; i < N; ++i)
                    w[a][i] = rho * (d[e][a][i] - z[e][a][i]) - l[e][a][i];
            gradT3(nx, ny, nz, w[0], w[1], w[2], G[e]);
            for (size_t i = 0; i < N; ++i) G[e][i] += h[e][i];
            if (k == 0) {  /* exact minimiser of the f-subproblem along -G */
                or_project3(g, G[e], p);
                grad3(nx, ny, nz, G[e], w[0], w[1], w[2]);
                double den = mu * dot(M, p, p) + rho * (dot(N, w[0], w[0]) + dot(N, w[1], w[1]) +
                                                       dot(N, w[2], w[2]));
                double gg = dot(N, G[e], G[e]);
                alpha[e] = den > 0.0 ? gg / den : 0.0;
                log[((size_t)e * (K + 1) + k) * 2 + 1] = alpha[e];
            }
            memcpy(fo[e], f[e], N * 8);
            memcpy(ho[e], h[e], N * 8);
            for (size_t i = 0; i < N; ++i) f[e][i] -= alpha[e] * G[e][i];
            if (nonneg)
                for (size_t i = 0; i < N; ++i) f[e][i] = f[e][i] > 0.0 ? f[e][i] : 0.0;
            or_project3(g, f[e], r[e]);
            for (size_t j = 0; j < M; ++j) r[e][j] -= gs[e][j];
            or_backproject3(g, r[e], h[e]);
            for (size_t i = 0; i < N; ++i) h[e][i] *= mu;
            for (size_t i = 0; i < N; ++i) sv[i] = f[e][i] - fo[e][i];
            grad3(nx, ny, nz, sv, w[0], w[1], w[2]);
            gradT3(nx, ny, nz, w[0], w[1], w[2], t1);
            for (size_t i = 0; i < N; ++i) y[i] = (h[e][i] - ho[e][i]) + rho * t1[i];
            double ss = dot(N, sv, sv), sy = dot(N, sv, y);
            if (sy > 0.0) alpha[e] = ss / sy;
            /* multiplier step (Eq. 7) */
            grad3(nx, ny, nz, f[e], w[0], w[1], w[2]);
            for (int a = 0; a < 3; ++a)
                for (size_t i = 0; i < N; ++i) l[e][a][i] -= xi * (w[a][i] - z[e][a][i]);
        }
    }
    for (int e = 0; e < 2; ++e)
        for (size_t i = 0; i < N; ++i) x_out[e * N + i] = f[e][i] / beta[e];
    for (int e = 0; e < 2; ++e) {
        free(f[e]); free(fo[e]); free(G[e]); free(h[e]); free(ho[e]); free(gs[e]); free(r[e]);
        for (int a = 0; a < 3; ++a) { free(l[e][a]); free(z[e][a]); free(d[e][a]); }
    }
    for (int a = 0; a < 3; ++a) free(w[a]);
    free(t1); free(sv); free(y); free(p);
}

/* ------------------------------------------------------------ 3-D PLS ---
 * Eqs. 13-15 on a volume: R of Eq. 14 over the six face neighbours, edges
 * from the 3-D Prewitt operator in FP64: per axis, the sum over the 3 x 3
 * face at +1 minus the sum over the face at -1, borders replicated;
 * m2 = gx^2 + gy^2 + gz^2; an edge where m2 > tau^2 max(m2).  Pair weights
 * e_x[i] couple i and i + 1, e_y[i] i and i + nx, e_z[i] i and i + nx ny: eps
 * if either voxel is an edge, else 1; pairs that leave the volume get 0.
 * m2_out / thr_out (optional) as in or_edges.
 */
void or_edges3(int nx, int ny, int nz, const double *x, double tau, double eps, double *ex,
               double *ey, double *ez, uint8_t *edge, double *m2_out, double *thr_out)
{
    const size_t P = (size_t)nx * ny, N = P * nz;
    double *m2 = malloc(N * sizeof(double));
    double mx = 0.0;
#define CL(v, n) ((v) < 0 ? 0 : ((v) > (n) - 1 ? (n) - 1 : (v)))
#define V3(zz, rr, cc) x[(size_t)CL(zz, nz) * P + (size_t)CL(rr, ny) * nx + CL(cc, nx)]
    for (int z = 0; z < nz; ++z)
        for (int r = 0; r < ny; ++r)
            for (int c = 0; c < nx; ++c) {
                double gx = 0.0, gy = 0.0, gz = 0.0;
                for (int a = -1; a <= 1; ++a)
                    for (int b = -1; b <= 1; ++b) {
                        gx += V3(z + a, r + b, c + 1) - V3(z + a, r + b, c - 1);
                        gy += V3(z + a, r + 1, c + b) - V3(z + a, r - 1, c + b);
                        gz += V3(z + 1, r + a, c + b) - V3(z - 1, r + a, c + b);
                    }
                double v = gx * gx + gy * gy + gz * gz;
                m2[(size_t)z * P + (size_t)r * nx + c] = v;
                if (v > mx) mx = v;
            }
#undef V3
#undef CL
    double thr = tau * tau * mx;
    for (size_t i = 0; i < N; ++i) edge[i] = m2[i] > thr;
    for (int z = 0; z < nz; ++z)
        for (int r = 0; r < ny; ++r)
            for (int c = 0; c < nx; ++c) {
                size_t i = (size_t)z * P + (size_t)r * nx + c;
                ex[i] = c + 1 < nx ? ((edge[i] || edge[i + 1]) ? eps : 1.0) : 0.0;
                ey[i] = r + 1 < ny ? ((edge[i] || edge[i + nx]) ? eps : 1.0) : 0.0;
                ez[i] = z + 1 < nz ? ((edge[i] || edge[i + P]) ? eps : 1.0) : 0.0;
            }
    if (m2_out) memcpy(m2_out, m2, N * sizeof(double));
    if (thr_out) *thr_out = thr;
    free(m2);
}

/* (L u)_i = sum over the six face neighbours k of e_ik (u_i - u_k) (Eq. 14). */
void or_laplacian3(int nx, int ny, int nz, const double *ex, const double *ey, const double *ez,
                   const double *u, double *out)
{
    const size_t P = (size_t)nx * ny;
    for (int z = 0; z < nz; ++z)
        for (int r = 0; r < ny; ++r)
            for (int c = 0; c < nx; ++c) {
                size_t i = (size_t)z * P + (size_t)r * nx + c;
                double s = 0.0;
                if (c + 1 < nx) s += ex[i] * (u[i] - u[i + 1]);
                if (c >= 1) s += ex[i - 1] * (u[i] - u[i - 1]);
                if (r + 1 < ny) s += ey[i] * (u[i] - u[i + nx]);
                if (r >= 1) s += ey[i - nx] * (u[i] - u[i - nx]);
                if (z + 1 < nz) s += ez[i] * (u[i] - u[i + P]);
                if (z >= 1) s += ez[i - P] * (u[i] - u[i - P]);
                out[i] = s;
            }
}

/* Jacobi-PCG for (I + gamma L) u = b on a volume, from u = b; as or_pcg. */
int or_pcg3(int nx, int ny, int nz, const double *ex, const double *ey, const double *ez,
            double gamma, const double *b, double *u, int max_iter, double tol, double *relres)
{
    const size_t P = (size_t)nx * ny, N = P * nz;
    double *res = malloc(N * 8), *zv = malloc(N * 8), *p = malloc(N * 8), *q = malloc(N * 8),
           *dinv = malloc(N * 8);
    for (int z = 0; z < nz; ++z)
        for (int r = 0; r < ny; ++r)
            for (int c = 0; c < nx; ++c) {
                size_t i = (size_t)z * P + (size_t)r * nx + c;
                double d = 0.0;
                if (c + 1 < nx) d += ex[i];
                if (c >= 1) d += ex[i - 1];
                if (r + 1 < ny) d += ey[i];
                if (r >= 1) d += ey[i - nx];
                if (z + 1 < nz) d += ez[i];
                if (z >= 1) d += ez[i - P];
                dinv[i] = 1.0 / (1.0 + gamma * d);
            }
    memcpy(u, b, N * 8);
    or_laplacian3(nx, ny, nz, ex, ey, ez, u, q);
    for (size_t i = 0; i < N; ++i) res[i] = b[i] - (u[i] + gamma * q[i]);
    double bn = sqrt(dot(N, b, b)), rn = sqrt(dot(N, res, res));
    int it = 0;
    if (bn == 0.0) {
        memset(u, 0, N * 8);
        rn = 0.0;
        bn = 1.0;
    }
    for (size_t i = 0; i < N; ++i) zv[i] = dinv[i] * res[i];
    memcpy(p, zv, N * 8);
    double rz = dot(N, res, zv);
    while (it < max_iter && rn > tol * bn) {
        or_laplacian3(nx, ny, nz, ex, ey, ez, p, q);
        for (size_t i = 0; i < N; ++i) q[i] = p[i] + gamma * q[i];
        double pq = dot(N, p, q);
        if (pq <= 0.0) break;
        double a = rz / pq;
        for (size_t i = 0; i < N; ++i) {
            u[i] += a * p[i];
            res[i] -= a * q[i];
        }
        ++it;
        rn = sqrt(dot(N, res, res));
        for (size_t i = 0; i < N; ++i) zv[i] = dinv[i] * res[i];
        double rz2 = dot(N, res, zv), beta = rz2 / rz;
        rz = rz2;
        for (size_t i = 0; i < N; ++i) p[i] = zv[i] + beta * p[i];
    }
    if (relres) *relres = rn / bn;
    free(res); free(zv); free(p); free(q); free(dinv);
    return it;
}

typedef struct {
    int nx, ny, nz;
    const double *ex, *ey, *ez;
} or_lap3_ctx;

static void lap3_of(const void *ctx, const double *u, double *out)
{
    const or_lap3_ctx *k = (const or_lap3_ctx *)ctx;
    or_laplacian3(k->nx, k->ny, k->nz, k->ex, k->ey, k->ez, u, out);
}

/* Attenuation-space PLS on a volume (as or_pcg_att, with R of Eq. 14 over
 * the six face neighbours). */
int or_pcg_att3(int nx, int ny, int nz, const double *ex, const double *ey, const double *ez,
                double e1h, double e2h, double e1l, double e2l, double gamma, const double *xh,
                const double *xl, double *u1, double *u2, int max_iter, double tol,
                double *relres)
{
    const size_t P = (size_t)nx * ny, N = P * nz;
    double *dg = malloc(N * sizeof(double));
    for (int z = 0; z < nz; ++z)
        for (int r = 0; r < ny; ++r)
            for (int c = 0; c < nx; ++c) {
                size_t i = (size_t)z * P + (size_t)r * nx + c;
                double d = 0.0;
                if (c + 1 < nx) d += ex[i];
                if (c >= 1) d += ex[i - 1];
                if (r + 1 < ny) d += ey[i];
                if (r >= 1) d += ey[i - nx];
                if (z + 1 < nz) d += ez[i];
                if (z >= 1) d += ez[i - P];
                dg[i] = d;
            }
    const or_lap3_ctx ctx = {nx, ny, nz, ex, ey, ez};
    int it = pcg_att_core(N, lap3_of, &ctx, dg, e1h, e2h, e1l, e2l, gamma, xh, xl, u1, u2,
                          max_iter, tol, relres);
    free(dg);
    return it;
}
