/*
 * mcrt_oracle.c -- plain FP64 CPU oracle for the Monte Carlo dust
 * radiative-transfer photon-package life cycle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * statement of what the GPU path computes.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it.  It shares no
 * code, header, table or helper with the HIP library, and the HIP library
 * never calls it.
 *
 * Paper: Camps & Baes, "SKIRT: an advanced dust radiative transfer code with
 * a user-friendly architecture" (arXiv:1410.1629).  The paper does not write
 * down the Monte Carlo equations (Sect. 1 says so explicitly); it names the
 * techniques.  Each function below cites the section that names the step and
 * the published method the step is taken from.  Readings of points the paper
 * leaves open are stated where they are used.
 *
 *   Sect. 1   photon packages, Poisson noise; peel-off at emission and
 *             scattering (Yusef-Zadeh, Morris & White 1984); continuous
 *             absorption (Lucy 1999; Niccolini et al. 2003); forced
 *             scattering (Cashwell & Everett 1959).
 *   Sect. 2.1 absorption and multiple anisotropic scattering.
 *   Sect. 2.2 packages propagate through grid cells in which density and
 *             optical properties are constant; frame instruments use
 *             parallel projection for a distant observer; direct and
 *             scattered radiation may be recorded separately; Table 1(d)
 *             lists the regular Cartesian grid.
 *   Sect. 2.3 kappa_sca, kappa_abs and the asymmetry parameter g that sets
 *             the phase function.
 *   Fig. 5    (pretty-printed parameter file) random seed, default 4357.
 *
 * Every function that has an independent check says which one in its
 * comment; the checks live in tests/test_oracle_*.py.
 *
 * Build: gcc -O2 -fno-fast-math -fopenmp -fPIC -shared (see build_oracle.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11).  The paper only
 * fixes that the generator is seeded (Fig. 5); a counter-based generator
 * makes every package reproducible from its index alone.
 * Check: tests compare against PyTorch's independent Philox engine and
 * against published known-answer vectors. */

static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void oracle_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof c);
}

/* Uniform deviate strictly inside (0,1): u = (w + 1/2) / 2^32. */
double oracle_uniform(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/* Draw number c of package p at wavelength index l: counter (p_lo, p_hi, l, c),
 * key (seed_lo, seed_hi).  Draw 0: emission position; draw 1: emission
 * direction and source choice; draw 2+n: scattering event n. */
static void draw(uint64_t seed, uint64_t p, uint32_t l, uint32_t c, double u[4])
{
    uint32_t ctr[4] = {(uint32_t)p, (uint32_t)(p >> 32), l, c};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    oracle_philox(ctr, key, w);
    for (int i = 0; i < 4; i++) u[i] = oracle_uniform(w[i]);
}

/* ------------------------------------------------------------------------ */
/* Regular Cartesian grid (Table 1(d), "LinCubDustGrid"): cells are equal
 * cuboids; cell m = i + nx*(j + ny*k), x fastest (reading).  Density is
 * constant inside each cell (Sect. 2.2). */

typedef struct {
    double lo[3], hi[3], d[3];
    int n[3];
    int64_t ncell;
    const double *pl[3]; /* rectilinear grid: the n[a] + 1 planes of axis a; NULL: regular */
    int tree;            /* tree grid: the cells are leaves with boxes leaf_lo/hi[cell] */
    double *leaf_lo, *leaf_hi;
} grid_t;

/* planes: NULL for regularly spaced cells (LinCub), else the cell-boundary
 * coordinates of x, then y, then z (n + 1 each, increasing from the box's
 * minimum to its maximum): cells spaced by any rule, such as PowCub's
 * power law (Table 1(d)). */
static void grid_free(grid_t *G);

/* tree: NULL, or a tree grid (Table 1(d): k-d tree; an octree is three
 * binary levels per level) as doubles: the node count, then per node
 * (axis, split, child) -- axis -1 marks a leaf whose cell is `child`, else
 * the node splits along `axis` at `split` into nodes child (lower side) and
 * child + 1 (upper side).  Returns 0, or -1 for a malformed tree. */
static int grid_init(grid_t *G, const double box[6], const int n[3], const double *planes, const double *tree)
{
    size_t off = 0;
    for (int a = 0; a < 3; a++) {
        G->lo[a] = box[2 * a];
        G->hi[a] = box[2 * a + 1];
        G->n[a] = n[a];
        G->d[a] = (G->hi[a] - G->lo[a]) / n[a];
        G->pl[a] = planes ? planes + off : NULL;
        off += (size_t)n[a] + 1;
    }
    G->ncell = (int64_t)n[0] * n[1] * n[2];
    G->tree = tree != NULL;
    G->leaf_lo = G->leaf_hi = NULL;
    if (!tree) return 0;
    /* leaf boxes: each node's box from its parent's, children numbered above it */
    int64_t nn = (int64_t)tree[0];
    const double *nd = tree + 1;
    double *lo = (double *)malloc(sizeof(double) * 3 * nn), *hi = (double *)malloc(sizeof(double) * 3 * nn);
    G->leaf_lo = (double *)calloc(3 * G->ncell, sizeof(double));
    G->leaf_hi = (double *)calloc(3 * G->ncell, sizeof(double));
    int ok = nn >= 1;
    for (int a = 0; a < 3 && ok; a++) {
        lo[a] = G->lo[a];
        hi[a] = G->hi[a];
    }
    for (int64_t q = 0; q < nn && ok; q++) {
        int axis = (int)nd[3 * q];
        int64_t child = (int64_t)nd[3 * q + 2];
        if (axis < 0) {
            if (child < 0 || child >= G->ncell) { ok = 0; break; }
            for (int a = 0; a < 3; a++) {
                G->leaf_lo[3 * child + a] = lo[3 * q + a];
                G->leaf_hi[3 * child + a] = hi[3 * q + a];
            }
            continue;
        }
        if (child <= q || child + 1 >= nn || axis > 2) { ok = 0; break; }
        for (int side = 0; side < 2; side++) {
            for (int a = 0; a < 3; a++) {
                lo[3 * (child + side) + a] = lo[3 * q + a];
                hi[3 * (child + side) + a] = hi[3 * q + a];
            }
        }
        hi[3 * child + axis] = nd[3 * q + 1];
        lo[3 * (child + 1) + axis] = nd[3 * q + 1];
    }
    free(lo);
    free(hi);
    if (!ok) grid_free(G);
    return ok ? 0 : -1;
}

static void grid_free(grid_t *G)
{
    free(G->leaf_lo);
    free(G->leaf_hi);
    G->leaf_lo = G->leaf_hi = NULL;
}

/* Leaf of a tree grid holding point p for a ray of direction k, by testing
 * every leaf: along each axis the leaf holds lo <= p < hi when the ray moves
 * up or parallel, lo < p <= hi when it moves down (a point on a face belongs
 * to the leaf the ray moves into).  -1 if none. */
static int64_t tree_locate(const grid_t *G, const double p[3], const double k[3])
{
    for (int64_t c = 0; c < G->ncell; c++) {
        int in = 1;
        for (int a = 0; a < 3 && in; a++) {
            double lo = G->leaf_lo[3 * c + a], hi = G->leaf_hi[3 * c + a];
            in = k[a] < 0.0 ? (lo < p[a] && p[a] <= hi) : (lo <= p[a] && p[a] < hi);
        }
        if (in) return c;
    }
    return -1;
}

/* Coordinate of plane p (0..n) along axis a. */
static double plane_at(const grid_t *G, int a, int p)
{
    return G->pl[a] ? G->pl[a][p] : G->lo[a] + p * G->d[a];
}

/* Cell along axis a holding coordinate x, before clamping: -1 below the
 * grid, n above; *on_plane tells whether x is exactly a plane's coordinate.
 * Regular grids by floor((x - lo)/d); rectilinear grids by scanning the
 * planes for the last one at or below x. */
static int axis_cell(const grid_t *G, int a, double x, int *on_plane)
{
    if (!G->pl[a]) {
        double u = (x - G->lo[a]) / G->d[a];
        double fu = floor(u);
        *on_plane = (u == fu);
        return (int)fu;
    }
    int i = -1;
    for (int p = 0; p <= G->n[a]; p++)
        if (G->pl[a][p] <= x) i = p;
    *on_plane = (i >= 0 && G->pl[a][i] == x);
    return i;
}

typedef struct {
    int64_t cell;
    double t0, t1;
} seg_t;

typedef struct {
    seg_t *v;
    size_t n, cap;
} segbuf;

static void sb_clear(segbuf *b) { b->n = 0; }

static void sb_push(segbuf *b, int64_t cell, double t0, double t1)
{
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 256;
        b->v = (seg_t *)realloc(b->v, b->cap * sizeof(seg_t));
    }
    b->v[b->n].cell = cell;
    b->v[b->n].t0 = t0;
    b->v[b->n].t1 = t1;
    b->n++;
}

/* Keeps the part of a segment list with t < len (the walk to a camera
 * inside the model stops at the camera). */
static void sb_clip(segbuf *b, double len)
{
    size_t n = 0;
    while (n < b->n && b->v[n].t0 < len) {
        if (b->v[n].t1 > len) b->v[n].t1 = len;
        n++;
    }
    b->n = n;
}

static void sb_free(segbuf *b)
{
    free(b->v);
    b->v = NULL;
    b->n = b->cap = 0;
}

/* Straight-line traversal (Sect. 2.2: packages move through the cells; the
 * walk is the voxel traversal of Amanatides & Woo, Eurographics 1987).
 * Appends, in order along the ray o + t k (t >= 0), every cell crossed with a
 * positive path length, as (cell, t_enter, t_exit), up to the grid boundary.
 * Readings: a ray starting outside enters through the slab intersection and a
 * ray that misses yields nothing; a coordinate lying exactly on a wall while
 * moving towards lower indices belongs to the lower cell; a ray parallel to
 * an axis uses floor() for that axis (half-open cells); the crossing time of
 * every plane is computed directly as (plane - o)/k; axes whose planes are
 * reached at the same t advance together; segments of zero length are
 * dropped.  Checks: analytic optical depths through uniform and
 * one-dimensional media, chord lengths, axis-parallel rays. */
static void traverse(const grid_t *G, const double o[3], const double k[3], segbuf *out)
{
    double tin = 0.0, tout = INFINITY;
    int entry = -1;
    for (int a = 0; a < 3; a++) {
        if (k[a] == 0.0) {
            if (o[a] < G->lo[a] || o[a] >= G->hi[a]) return;
            continue;
        }
        double ta = (G->lo[a] - o[a]) / k[a];
        double tb = (G->hi[a] - o[a]) / k[a];
        double tn = ta < tb ? ta : tb;
        double tf = ta < tb ? tb : ta;
        if (tn > tin) {
            tin = tn;
            entry = a;
        }
        if (tf < tout) tout = tf;
    }
    if (!(tin < tout)) return;

    if (G->tree) {
        /* tree grid: from the entry point, the leaf holding the point, left
         * through its nearest face; the exit faces' coordinates are set to
         * the faces exactly, the others advance along k */
        double p[3];
        for (int a = 0; a < 3; a++)
            p[a] = a == entry ? (k[a] > 0.0 ? G->lo[a] : G->hi[a]) : o[a] + tin * k[a];
        double t = tin;
        for (int64_t guard = 0; guard < 4 * G->ncell + 8; guard++) {
            int64_t c = tree_locate(G, p, k);
            if (c < 0) break;
            double tx[3], tm = INFINITY;
            for (int a = 0; a < 3; a++) {
                if (k[a] > 0.0)
                    tx[a] = (G->leaf_hi[3 * c + a] - p[a]) / k[a];
                else if (k[a] < 0.0)
                    tx[a] = (G->leaf_lo[3 * c + a] - p[a]) / k[a];
                else
                    tx[a] = INFINITY;
                if (tx[a] < tm) tm = tx[a];
            }
            if (!(tm < INFINITY)) break;
            if (tm > 0.0) sb_push(out, c, t, t + tm);
            int leaves_box = 0;
            for (int a = 0; a < 3; a++) {
                if (tx[a] == tm) {
                    double f = k[a] > 0.0 ? G->leaf_hi[3 * c + a] : G->leaf_lo[3 * c + a];
                    if (f == (k[a] > 0.0 ? G->hi[a] : G->lo[a])) leaves_box = 1;
                    p[a] = f;
                } else {
                    p[a] += tm * k[a];
                }
            }
            t += tm;
            if (leaves_box) break;
        }
        return;
    }

    int idx[3];
    for (int a = 0; a < 3; a++) {
        if (a == entry) {
            idx[a] = k[a] > 0.0 ? 0 : G->n[a] - 1;
            continue;
        }
        double p = o[a] + tin * k[a];
        int on_plane;
        int i = axis_cell(G, a, p, &on_plane);
        if (k[a] < 0.0 && on_plane) i -= 1;
        if (i < 0) i = 0;
        if (i > G->n[a] - 1) i = G->n[a] - 1;
        idx[a] = i;
    }

    double t = tin;
    int guard = G->n[0] + G->n[1] + G->n[2] + 8;
    while (guard-- > 0) {
        double tn[3];
        for (int a = 0; a < 3; a++) {
            if (k[a] > 0.0)
                tn[a] = (plane_at(G, a, idx[a] + 1) - o[a]) / k[a];
            else if (k[a] < 0.0)
                tn[a] = (plane_at(G, a, idx[a]) - o[a]) / k[a];
            else
                tn[a] = INFINITY;
        }
        double t1 = tn[0];
        if (tn[1] < t1) t1 = tn[1];
        if (tn[2] < t1) t1 = tn[2];
        if (t1 > t) {
            int64_t m = idx[0] + (int64_t)G->n[0] * (idx[1] + (int64_t)G->n[1] * idx[2]);
            sb_push(out, m, t, t1);
            t = t1;
        }
        int out_of_grid = 0;
        for (int a = 0; a < 3; a++) {
            if (tn[a] == t1) {
                idx[a] += k[a] > 0.0 ? 1 : -1;
                if (idx[a] < 0 || idx[a] >= G->n[a]) out_of_grid = 1;
            }
        }
        if (out_of_grid) break;
    }
}

/* Optical depth of a segment list: sum of kappa * rho_m * length. */
static double seg_tau(const segbuf *s, const double *rho, double kappa)
{
    double tau = 0.0;
    for (size_t j = 0; j < s->n; j++) tau += kappa * rho[s->v[j].cell] * (s->v[j].t1 - s->v[j].t0);
    return tau;
}

/* ------------------------------------------------------------------------ */
/* Frame instrument (Sect. 2.2, Fig. 4/5 parameters: distance, inclination
 * theta, azimuth phi, position angle omega, pixel counts, maximal extents).
 * Readings: the direction towards the observer is
 *   k_d = (sin t cos p, sin t sin p, cos t);
 * the image axes are e_x = (-sin p, cos p, 0) and
 *   e_y = (-cos t cos p, -cos t sin p, sin t), so (e_x, e_y, k_d) is
 * right-handed and theta = 90, phi = -90 gives image axes (x, z), matching the
 * instrument named "xz" in Fig. 4; omega rotates (e_x, e_y) in the image
 * plane; the extents are half-widths of the frame around the origin;
 * parallel projection, so the distance enters only as 1/D^2; a pixel holds
 * flux (luminosity / D^2).
 *
 * SED instrument (Sect. 2.2: the spectral energy distribution of the
 * received flux): the same distant observer with a single pixel that every
 * point falls in.
 *
 * Perspective instrument (Sect. 2.2: placed anywhere, even inside the
 * model).  Reading: a pinhole camera at `eye` looking at `target`; the image
 * plane passes through the target perpendicular to the view axis, with
 * e_y along `up` made perpendicular to the view axis and e_x = view x e_y;
 * a point is imaged where the line from the eye through it meets that plane
 * (points behind the eye are not seen); the peel-off ray runs from the
 * event to the eye -- optical depth along that segment only -- and counts
 * 1 / (distance to the eye)^2.  Check: the flux of a point source seen from
 * inside a uniform medium, and the image positions of points at known
 * angles. */

enum { DET_FRAME = 0, DET_SED = 1, DET_PERSPECTIVE = 2 };

typedef struct {
    int kind;
    double kd[3], ex[3], ey[3];
    double inv_d2, half_x, half_y, dpx, dpy;
    double eye[3], view[3], focal; /* perspective: eye, unit view axis, distance eye-target */
    int nx, ny;
    size_t off; /* offset of this frame inside one wavelength's image block */
} det_t;

/* par[16]: distance, inclination, azimuth, position angle, half_x, half_y,
 * kind, eye[3], target[3], up[3]. */
static void det_init(det_t *D, const double par[16], const int pix[2])
{
    double th = par[1] * (OR_PI / 180.0), ph = par[2] * (OR_PI / 180.0), om = par[3] * (OR_PI / 180.0);
    double st = sin(th), ct = cos(th), sp = sin(ph), cp = cos(ph);
    double so = sin(om), co = cos(om);
    double kd[3] = {st * cp, st * sp, ct};
    double ex[3] = {-sp, cp, 0.0};
    double ey[3] = {-ct * cp, -ct * sp, st};
    for (int a = 0; a < 3; a++) {
        D->kd[a] = kd[a];
        D->ex[a] = co * ex[a] + so * ey[a];
        D->ey[a] = -so * ex[a] + co * ey[a];
    }
    D->inv_d2 = 1.0 / (par[0] * par[0]);
    D->half_x = par[4];
    D->half_y = par[5];
    D->nx = pix[0];
    D->ny = pix[1];
    D->dpx = 2.0 * par[4] / pix[0];
    D->dpy = 2.0 * par[5] / pix[1];
    D->kind = (int)par[6];
    if (D->kind == DET_PERSPECTIVE) {
        const double *eye = par + 7, *target = par + 10, *up = par + 13;
        double v[3], n = 0.0, uv = 0.0, m = 0.0;
        for (int a = 0; a < 3; a++) {
            D->eye[a] = eye[a];
            v[a] = target[a] - eye[a];
            n += v[a] * v[a];
        }
        D->focal = sqrt(n);
        for (int a = 0; a < 3; a++) {
            D->view[a] = v[a] / D->focal;
            uv += up[a] * D->view[a];
        }
        for (int a = 0; a < 3; a++) {
            D->ey[a] = up[a] - uv * D->view[a];
            m += D->ey[a] * D->ey[a];
        }
        for (int a = 0; a < 3; a++) D->ey[a] /= sqrt(m);
        D->ex[0] = D->view[1] * D->ey[2] - D->view[2] * D->ey[1];
        D->ex[1] = D->view[2] * D->ey[0] - D->view[0] * D->ey[2];
        D->ex[2] = D->view[0] * D->ey[1] - D->view[1] * D->ey[0];
    }
}

/* Direction, 1/distance^2 and length of the peel-off ray from r to
 * instrument D (distant instruments: to the grid's boundary). */
static void det_peel_ray(const det_t *D, const double r[3], double kd[3], double *inv_d2, double *len)
{
    if (D->kind == DET_PERSPECTIVE) {
        double v[3], n = 0.0;
        for (int a = 0; a < 3; a++) {
            v[a] = D->eye[a] - r[a];
            n += v[a] * v[a];
        }
        *len = sqrt(n);
        for (int a = 0; a < 3; a++) kd[a] = v[a] / *len;
        *inv_d2 = 1.0 / n;
        return;
    }
    for (int a = 0; a < 3; a++) kd[a] = D->kd[a];
    *inv_d2 = D->inv_d2;
    *len = INFINITY;
}

/* Pixel hit by the projection of r (parallel, or through the eye), or -1
 * if outside the frame. */
static int64_t det_pixel(const det_t *D, const double r[3])
{
    if (D->kind == DET_SED) return 0;
    double xp, yp;
    if (D->kind == DET_PERSPECTIVE) {
        double d[3] = {r[0] - D->eye[0], r[1] - D->eye[1], r[2] - D->eye[2]};
        double z = d[0] * D->view[0] + d[1] * D->view[1] + d[2] * D->view[2];
        if (!(z > 0.0)) return -1;
        xp = D->focal * (d[0] * D->ex[0] + d[1] * D->ex[1] + d[2] * D->ex[2]) / z;
        yp = D->focal * (d[0] * D->ey[0] + d[1] * D->ey[1] + d[2] * D->ey[2]) / z;
    } else {
        xp = r[0] * D->ex[0] + r[1] * D->ex[1] + r[2] * D->ex[2];
        yp = r[0] * D->ey[0] + r[1] * D->ey[1] + r[2] * D->ey[2];
    }
    double fx = floor((xp + D->half_x) / D->dpx);
    double fy = floor((yp + D->half_y) / D->dpy);
    if (!(fx >= 0.0 && fx < D->nx && fy >= 0.0 && fy < D->ny)) return -1;
    return (int64_t)fy * D->nx + (int64_t)fx;
}

/* ------------------------------------------------------------------------ */
/* Henyey-Greenstein phase function (Sect. 2.3: g sets the phase function;
 * the HG form is the reading).  Normalised so that its integral over the
 * sphere is 1.  Check: the sampled cosine has mean g. */
static double hg_phase(double g, double mu)
{
    double x = 1.0 + g * g - 2.0 * g * mu;
    return (1.0 - g * g) / (4.0 * OR_PI * x * sqrt(x));
}

/* Inverse-CDF sample of the HG scattering cosine; isotropic below |g| 1e-6. */
/* d ln Phi / dg of the HG phase function at cosine mu:
 * -2g / (1 - g^2) - 3 (g - mu) / (1 + g^2 - 2 g mu). */
static double hg_dlng(double g, double mu) { return -2.0 * g / (1.0 - g * g) - 3.0 * (g - mu) / (1.0 + g * g - 2.0 * g * mu); }

double oracle_hg_mu(double g, double u)
{
    if (fabs(g) < 1e-6) return 2.0 * u - 1.0;
    double f = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
    double mu = (1.0 + g * g - f * f) / (2.0 * g);
    if (mu < -1.0) mu = -1.0;
    if (mu > 1.0) mu = 1.0;
    return mu;
}

/* New direction at polar cosine mu and azimuth psi around k, using the
 * orthonormal basis of Duff, Burgess, Christensen, Hery, Kensler, Liani &
 * Villemin (JCGT 2017); renormalised afterwards.  Check: unit norm and mean
 * k.k' = g over many samples. */
void oracle_rotate(const double k[3], double mu, double psi, double out[3])
{
    double s = k[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (s + k[2]);
    double b = k[0] * k[1] * a;
    double b1[3] = {1.0 + s * k[0] * k[0] * a, s * b, -s * k[0]};
    double b2[3] = {b, s + k[1] * k[1] * a, -k[1]};
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double cp = cos(psi), sp = sin(psi);
    double n2 = 0.0;
    for (int i = 0; i < 3; i++) {
        out[i] = st * (cp * b1[i] + sp * b2[i]) + mu * k[i];
        n2 += out[i] * out[i];
    }
    double inv = 1.0 / sqrt(n2);
    for (int i = 0; i < 3; i++) out[i] *= inv;
}

/* ------------------------------------------------------------------------ */
/* Sources (Sect. 2.2, Table 1(a): point geometry and exponential disk; the
 * geometry draws random positions).  Exponential disk density
 * rho ~ exp(-R/h_R - |z|/h_z), untruncated: R follows Gamma(2, h_R) because
 * of the area element 2 pi R dR, so R = -h_R ln(u0 u1); phi = 2 pi u2; z
 * follows a Laplace law with scale h_z.  Check: moments E[R] = 2 h_R,
 * E[|z|] = h_z, and the dust-free face-on image of the disk. */

enum { SRC_POINT = 0, SRC_EXPDISK = 1, SRC_CELLS = 2 };

typedef struct {
    int kind;
    double c[3], hr, hz;
} src_t;

void oracle_emit_position(int kind, const double par[5], const double u[4], double r[3])
{
    r[0] = par[0];
    r[1] = par[1];
    r[2] = par[2];
    if (kind == SRC_EXPDISK) {
        double R = -par[3] * log(u[0] * u[1]);
        double phi = 2.0 * OR_PI * u[2];
        double z = u[3] < 0.5 ? par[4] * log(2.0 * u[3]) : -par[4] * log(2.0 * (1.0 - u[3]));
        r[0] += R * cos(phi);
        r[1] += R * sin(phi);
        r[2] += z;
    }
}

/* Isotropic emission direction: mu = 2 u0 - 1, psi = 2 pi u1. */
void oracle_emit_direction(const double u[4], double k[3])
{
    double mu = 2.0 * u[0] - 1.0;
    double psi = 2.0 * OR_PI * u[1];
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    k[0] = st * cos(psi);
    k[1] = st * sin(psi);
    k[2] = mu;
}

/* Box of cell c: along each axis between consecutive planes (regular and
 * rectilinear grids, c = i + nx (j + ny k)), or the leaf's box (tree grids). */
static void cell_bounds(const grid_t *G, int64_t c, double lo[3], double hi[3])
{
    if (G->tree) {
        for (int a = 0; a < 3; a++) {
            lo[a] = G->leaf_lo[3 * c + a];
            hi[a] = G->leaf_hi[3 * c + a];
        }
        return;
    }
    int64_t i[3] = {c % G->n[0], (c / G->n[0]) % G->n[1], c / ((int64_t)G->n[0] * G->n[1])};
    for (int a = 0; a < 3; a++) {
        lo[a] = plane_at(G, a, (int)i[a]);
        hi[a] = plane_at(G, a, (int)i[a] + 1);
    }
}

/* Emission point of a cell source (the grid's cells emit: dust emission,
 * Sect. 1 and 2.1).  cum[0..ncell] are the exclusive prefix sums of the
 * cells' luminosities at this wavelength; the cell is the last c with
 * cum[c] <= u0 cum[ncell], so it is drawn with probability proportional to
 * its luminosity (and never with zero luminosity); the point is
 * lo + u (hi - lo) in its box from u1, u2, u3.  Check: the cell counts and
 * the positions inside a cell against their laws, with no dust on the way. */
static void cell_emit_position(const grid_t *G, const double *cum, const double u[4], double r[3])
{
    double target = u[0] * cum[G->ncell];
    int64_t lo = 0, hi = G->ncell - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) / 2;
        if (cum[mid] <= target)
            lo = mid;
        else
            hi = mid - 1;
    }
    double bl[3], bh[3];
    cell_bounds(G, lo, bl, bh);
    for (int a = 0; a < 3; a++) r[a] = bl[a] + u[1 + a] * (bh[a] - bl[a]);
}

/* Forced scattering (Sect. 1, Cashwell & Everett 1959): the optical depth of
 * the interaction point is drawn from exp(-tau) truncated to [0, T]:
 * tau_s = -ln(1 - u (1 - e^-T)).  Check: the histogram against the
 * truncated-exponential law. */
double oracle_forced_tau(double T, double u) { return -log1p(u * expm1(-T)); }

/* ------------------------------------------------------------------------ */
/* The simulation. */

enum { FLAG_PEEL_EMIT = 1, FLAG_PEEL_SCAT = 2, FLAG_ABSORB = 4, FLAG_SPLIT = 8 };
enum { MODE_FORWARD = 0, MODE_GRAD = 1, MODE_REWEIGHT = 2, MODE_ATTACHED = 3 };
enum { ST_EMITTED, ST_ABSORBED, ST_ESCAPED, ST_TRUNCATED, ST_XPATH, ST_XLOCATE, ST_XPEEL, ST_EVENTS, ST_PACKAGES, ST_N };

#define MAX_DET 16
#define MAX_SRC 16

typedef struct {
    grid_t G;
    const double *rho;      /* density used to sample paths */
    const double *rho_eval; /* REWEIGHT: density at which weights are evaluated */
    int n_lambda;
    const double *kappa, *albedo, *g;
    int n_src;
    src_t src[MAX_SRC];
    const double *lum; /* [n_src][n_lambda]; a cell source's row holds its per-wavelength totals */
    double *lum_own;   /* the copy of the source luminosities that lum points to */
    int cell_src;      /* index of the cell source, -1 if none */
    double *cell_cum;  /* cell source: [n_lambda][ncell + 1] exclusive prefix sums of its luminosities */
    int n_det;
    det_t det[MAX_DET];
    size_t pix_lambda; /* pixels of all frames for one wavelength */
    uint64_t n_pkg, first, seed;
    double w_min;
    int max_scatter;
    unsigned flags;
    int mode;
    const double *adj; /* GRAD: dL/dI, same layout as the images */
    const double *adj_abs; /* GRAD: dL/dA of the absorbed tally [n_lambda][ncell], or NULL */
    /* REWEIGHT: albedo [n_lambda], g [n_lambda] and source luminosities
     * [n_src][n_lambda] at which weights are evaluated (NULL: the sampling
     * values) */
    const double *alb_eval, *g_eval, *lum_eval;
} problem_t;

/* One recorded peel-off contribution (GRAD mode). */
typedef struct {
    int event;    /* 0 = emission, i >= 1 = scattering i */
    double a_c;   /* dL/dI at the pixel times the contribution */
    double dlng;  /* d ln(contribution) / dg: scores of the sampled directions and the peel phase */
    int absorbed; /* 1: the absorbed-tally term of the path after the event (images' optics gradients skip it) */
    int det;      /* the instrument it goes to */
    size_t beg, end; /* peel segments inside the peel buffer */
} contrib_t;

/* One event of a package as the attached derivative needs it (ATTACHED
 * mode): the position and the weight after the event and, when a path leg
 * follows it, the leg's direction k, optical depth T to the boundary,
 * forced-scattering depth tau_s, length s to the next event, the density of
 * the cell where that event lies and the leg's full path (segments up to
 * the boundary, in the legs buffer). */
typedef struct {
    double r[3], w;
    int leg;
    double k[3], T, tau_s, s, rho_s;
    size_t beg, end;
} att_ev_t;

typedef struct {
    double *images;   /* full image array */
    double *absorbed; /* [ncell] slice of the current wavelength, or NULL */
    double *grad;     /* [ncell] or NULL */
    double stats[ST_N];
    double gopt[2 + MAX_SRC]; /* GRAD: dL/d albedo, dL/d g, dL/d L_s of the current wavelength */
    segbuf path, peel, legs, gpeel;
    /* GRAD bookkeeping of the current package */
    size_t *leg_beg, *leg_end;
    int64_t *leg_cell;
    int nleg_cap;
    contrib_t *con;
    int ncon, ncon_cap;
    att_ev_t *aev; /* ATTACHED: the package's events */
    int naev, naev_cap;
} accum_t;

static size_t image_index(const problem_t *P, int comp, int l, int d, int64_t pix)
{
    return ((size_t)comp * P->n_lambda + l) * P->pix_lambda + P->det[d].off + (size_t)pix;
}

static void grad_reserve_legs(accum_t *A, int n)
{
    if (n <= A->nleg_cap) return;
    int cap = A->nleg_cap ? A->nleg_cap : 64;
    while (cap < n) cap *= 2;
    A->leg_beg = (size_t *)realloc(A->leg_beg, cap * sizeof(size_t));
    A->leg_end = (size_t *)realloc(A->leg_end, cap * sizeof(size_t));
    A->leg_cell = (int64_t *)realloc(A->leg_cell, cap * sizeof(int64_t));
    A->nleg_cap = cap;
}

static contrib_t *grad_new_contrib(accum_t *A)
{
    if (A->ncon == A->ncon_cap) {
        A->ncon_cap = A->ncon_cap ? 2 * A->ncon_cap : 64;
        A->con = (contrib_t *)realloc(A->con, A->ncon_cap * sizeof(contrib_t));
    }
    return &A->con[A->ncon++];
}

/* Peel-off (Sect. 1, Yusef-Zadeh et al. 1984): the deterministic part of an
 * emission or scattering event that leaves towards each frame, attenuated by
 * the optical depth from r to the grid boundary along k_d.  The phase value
 * is 1/(4 pi) at emission and HG(k_in . k_d) at scattering.  The weight
 * passed in is the package weight after the event (reading: at scattering,
 * after the forced-scattering weight update).
 * w_eval / rho_eval: REWEIGHT mode evaluates the contribution at another
 * density along the same geometry. */
static void peel_event(const problem_t *P, accum_t *A, int l, int event, const double r[3],
                       const double *k_in, double w, double w_eval, double score)
{
    int comp = (P->flags & FLAG_SPLIT) && event > 0 ? 1 : 0;
    double kappa = P->kappa[l], g = P->g[l];
    for (int d = 0; d < P->n_det; d++) {
        const det_t *D = &P->det[d];
        int64_t pix = det_pixel(D, r);
        if (pix < 0) continue;
        double kd[3], inv_d2, len;
        det_peel_ray(D, r, kd, &inv_d2, &len);
        double phase = k_in ? hg_phase(g, k_in[0] * kd[0] + k_in[1] * kd[1] + k_in[2] * kd[2])
                            : 1.0 / (4.0 * OR_PI);
        sb_clear(&A->peel);
        traverse(&P->G, r, kd, &A->peel);
        sb_clip(&A->peel, len);
        A->stats[ST_XPEEL] += (double)A->peel.n;
        size_t ii = image_index(P, comp, l, d, pix);
        if (P->mode == MODE_REWEIGHT) {
            double tau = seg_tau(&A->peel, P->rho_eval, kappa);
            double phase_eval = phase;
            if (k_in && P->g_eval) phase_eval = hg_phase(P->g_eval[l], k_in[0] * kd[0] + k_in[1] * kd[1] + k_in[2] * kd[2]);
            A->images[ii] += w_eval * phase_eval * exp(-tau) * inv_d2;
        } else {
            double tau = seg_tau(&A->peel, P->rho, kappa);
            double c = w * phase * exp(-tau) * inv_d2;
            A->images[ii] += c;
            if (P->mode == MODE_GRAD || P->mode == MODE_ATTACHED) {
                contrib_t *C = grad_new_contrib(A);
                C->event = event;
                C->a_c = P->adj[ii] * c;
                C->dlng = k_in ? score + hg_dlng(g, k_in[0] * kd[0] + k_in[1] * kd[1] + k_in[2] * kd[2]) : 0.0;
                C->absorbed = 0;
                C->det = d;
                C->beg = A->gpeel.n;
                for (size_t j = 0; j < A->peel.n; j++)
                    sb_push(&A->gpeel, A->peel.v[j].cell, A->peel.v[j].t0, A->peel.v[j].t1);
                C->end = A->gpeel.n;
            }
        }
    }
}

/* Gradient of the image loss for one package, from its recorded legs and
 * contributions (detached "perturbation Monte Carlo" derivative, Hayakawa et
 * al., Opt. Lett. 2001).  With paths held fixed, a contribution C of event e
 * scales with density as
 *   prod_{i<=e} rho(c_i) exp(-tau(leg_i)) * exp(-tau(peel)),
 * the forced-scattering normalisation 1 - e^-T cancelling against the
 * sampling density.  Hence
 *   dC/drho_m = C [ sum_{i<=e} (delta(m,c_i)/rho_m - kappa l_m(leg_i))
 *                   - kappa l_m(peel) ],
 * and dL/drho_m = sum over contributions of (dL/dI_pixel) dC/drho_m.  Written
 * out plainly, without the suffix-sum reorganisation the GPU uses.
 * Check: finite differences of the reweighted estimator, and the closed form
 * for a non-scattering medium. */
static void grad_flush_package(const problem_t *P, accum_t *A, int l, int src)
{
    double kappa = P->kappa[l], alb = P->albedo[l], lum = P->lum[(size_t)src * P->n_lambda + l];
    for (int q = 0; q < A->ncon; q++) {
        const contrib_t *C = &A->con[q];
        if (C->a_c == 0.0) continue;
        if (C->absorbed) goto legs; /* the optics gradients are those of the image loss */
        /* optics and luminosity: a contribution after n scatterings scales as
         * albedo^n, with the scores of its sampled directions and its peel
         * phase in g, and as the luminosity of its package's source */
        if (alb > 0.0) A->gopt[0] += C->a_c * C->event / alb;
        A->gopt[1] += C->a_c * C->dlng;
        if (lum > 0.0) A->gopt[2 + src] += C->a_c / lum;
    legs:
        for (int i = 1; i <= C->event; i++) {
            int64_t c = A->leg_cell[i];
            A->grad[c] += C->a_c / P->rho[c];
            for (size_t j = A->leg_beg[i]; j < A->leg_end[i]; j++) {
                const seg_t *s = &A->legs.v[j];
                A->grad[s->cell] -= C->a_c * kappa * (s->t1 - s->t0);
            }
        }
        for (size_t j = C->beg; j < C->end; j++) {
            const seg_t *s = &A->gpeel.v[j];
            A->grad[s->cell] -= C->a_c * kappa * (s->t1 - s->t0);
        }
    }
}

/* Appends an event at r with weight w to the package's record (ATTACHED). */
static void att_push(accum_t *A, const double r[3], double w)
{
    if (A->naev == A->naev_cap) {
        A->naev_cap = A->naev_cap ? 2 * A->naev_cap : 64;
        A->aev = (att_ev_t *)realloc(A->aev, A->naev_cap * sizeof(att_ev_t));
    }
    att_ev_t *E = &A->aev[A->naev++];
    memset(E, 0, sizeof *E);
    for (int a = 0; a < 3; a++) E->r[a] = r[a];
    E->w = w;
}

/* Derivative of a ray's optical depth with respect to its origin o, for the
 * segment list b[beg, end) of the ray o + t k (contiguous, up to the grid's
 * boundary).  Moving the origin by dr moves the crossing of a plane normal
 * to axis a by dt = -dr_a / k_a, and the optical depth changes there by
 * kappa (rho_before - rho_after) dt (after the last segment: rho_after = 0,
 * outside the grid).  The plane of each crossing is the face through which
 * the ray leaves the cell before it: the axis with the earliest exit time
 * from that cell's box (on an edge or corner, where the derivative does not
 * exist, the lowest such axis).  Each crossing's term is weighted by
 * w_before when it lies before t_cut, else by w_after, and added to out.
 * Check: finite differences of whole runs with the random numbers held
 * fixed (the attached derivative it is part of). */
static void tau_grad_origin(const grid_t *G, const segbuf *b, size_t beg, size_t end, const double o[3],
                            const double k[3], const double *rho, double kappa, double t_cut, double w_before,
                            double w_after, double out[3])
{
    for (size_t j = beg; j < end; j++) {
        const seg_t *s = &b->v[j];
        double after = j + 1 < end ? rho[b->v[j + 1].cell] : 0.0;
        double jump = kappa * (rho[s->cell] - after);
        if (jump == 0.0) continue;
        double lo[3], hi[3];
        cell_bounds(G, s->cell, lo, hi);
        int ax = -1;
        double tm = INFINITY;
        for (int a = 0; a < 3; a++) {
            if (k[a] == 0.0) continue;
            double te = ((k[a] > 0.0 ? hi[a] : lo[a]) - o[a]) / k[a];
            if (te < tm) {
                tm = te;
                ax = a;
            }
        }
        if (ax < 0) continue;
        out[ax] -= (s->t1 < t_cut ? w_before : w_after) * jump / k[ax];
    }
}

/* Gradient of the image loss for one package by the attached (pathwise)
 * derivative: the random numbers are held fixed and the package's events
 * move with the densities.  The directions do not depend on the densities
 * (each is the previous one turned by angles drawn from the random
 * numbers); the positions do, through the forced-scattering step.  With
 * event n at r_n, weight w_n and the leg after it along k_n of optical
 * depth T_n to the boundary:
 *   tau_s,n = -ln(1 - u (1 - e^-T_n))   (fixed u),
 *   s_n solves tau(r_n, k_n, s_n) = tau_s,n,   r_{n+1} = r_n + s_n k_n,
 *   w_{n+1} = w_n albedo (1 - e^-T_n),
 * and a peel-off contribution of event n is C = w_n Phi e^-tau_peel(r_n) / D^2
 * (frames and SED instruments: the direction and distance of the observer
 * do not depend on r_n).  The loss is the sum of a C over the package's
 * contributions (a = dL/dI of the pixel the event projects into; pixel
 * choices, the escape test T = 0 and the termination test are held fixed:
 * the derivative is that of the per-package estimator where it is smooth).
 * Reverse accumulation over the events, from the last one back, with the
 * adjoints lbar of ln w_n and rbar of r_n:
 *   each contribution q = a C of event n: lbar += q, d/drho -= q kappa l
 *     along its peel ray, rbar -= q dtau_peel/dr_n;
 *   the leg from event n-1 to event n: sbar = rbar . k,
 *     taubar = sbar / (kappa rho_s)          (ds/dtau_s = 1/(kappa rho_s)),
 *     Tbar = taubar dtau_s/dT + lbar dln(1 - e^-T)/dT
 *          = taubar e^(tau_s - T) (1 - e^-tau_s)/(1 - e^-T) + lbar e^-T/(1 - e^-T),
 *     d/drho_m += Tbar kappa l_m(leg to the boundary) - (sbar / rho_s) l_m(leg up to s),
 *     rbar of r_{n-1} = rbar + Tbar dT/dr - taubar dtau(r, k, s)/dr (s fixed);
 *   lbar carries over unchanged (ln w_n = ln w_{n-1} + ln albedo + ln(1 - e^-T)),
 *   and the emission point does not move.
 * Check: finite differences of whole runs at rho (1 +- h v) with the same
 * random numbers, for instruments without pixel edges (SED) and
 * termination by count; the detached gradient in expectation; the
 * detached gradient exactly for a medium that does not scatter. */
static void attached_flush_package(const problem_t *P, accum_t *A, int l)
{
    const grid_t *G = &P->G;
    const double kappa = P->kappa[l];
    double lbar = 0.0, rbar[3] = {0.0, 0.0, 0.0};
    for (int n = A->naev - 1; n >= 0; n--) {
        const att_ev_t *E = &A->aev[n];
        for (int q = 0; q < A->ncon; q++) {
            const contrib_t *C = &A->con[q];
            if (C->event != n || C->a_c == 0.0) continue;
            lbar += C->a_c;
            for (size_t j = C->beg; j < C->end; j++) {
                const seg_t *s = &A->gpeel.v[j];
                A->grad[s->cell] -= C->a_c * kappa * (s->t1 - s->t0);
            }
            if (n > 0) {
                double d[3] = {0.0, 0.0, 0.0};
                tau_grad_origin(G, &A->gpeel, C->beg, C->end, E->r, P->det[C->det].kd, P->rho, kappa, INFINITY, 1.0,
                                1.0, d);
                for (int a = 0; a < 3; a++) rbar[a] -= C->a_c * d[a];
            }
        }
        if (n == 0) break;
        const att_ev_t *L = &A->aev[n - 1];
        double sbar = rbar[0] * L->k[0] + rbar[1] * L->k[1] + rbar[2] * L->k[2];
        double taubar = sbar / (kappa * L->rho_s);
        double Tbar = (taubar * exp(L->tau_s - L->T) * -expm1(-L->tau_s) + lbar * exp(-L->T)) / -expm1(-L->T);
        for (size_t j = L->beg; j < L->end; j++) {
            const seg_t *s = &A->legs.v[j];
            double part = s->t0 < L->s ? fmin(s->t1, L->s) - s->t0 : 0.0;
            A->grad[s->cell] += Tbar * kappa * (s->t1 - s->t0) - sbar / L->rho_s * part;
        }
        if (n - 1 > 0) {
            double d[3] = {0.0, 0.0, 0.0};
            tau_grad_origin(G, &A->legs, L->beg, L->end, L->r, L->k, P->rho, kappa, L->s, Tbar - taubar, Tbar, d);
            for (int a = 0; a < 3; a++) rbar[a] += d[a];
        }
    }
}

/* Life cycle of package p at wavelength l (Sect. 1: emission, a number of
 * scattering events, then absorption or escape; with the three techniques
 * named there):
 *   1. emit: source chosen by cumulative luminosity, position from its
 *      geometry, isotropic direction, weight W0 = L_total / N;
 *   2. peel-off at emission;
 *   3. repeat: traverse to the boundary (segments, optical depths, total T);
 *      T = 0 means the package leaves unhindered; continuous absorption
 *      deposits W (1 - albedo) e^-tau_{j-1} (1 - e^-dtau_j) in each cell
 *      crossed and W e^-T escapes; forced scattering draws tau_s in [0, T]
 *      and locates the interaction point; W <- W albedo (1 - e^-T); peel-off
 *      at scattering with the incoming direction; stop below w_min * W0 or
 *      after max_scatter scatterings (the remaining weight is tallied as
 *      truncated); draw the new direction from HG.
 * Energy: emitted = absorbed + escaped + truncated per package up to
 * rounding (each event splits W into these parts and the scattered part). */
static void run_package(const problem_t *P, accum_t *A, uint64_t p, int l)
{
    const grid_t *G = &P->G;
    const double kappa = P->kappa[l], alb = P->albedo[l], g = P->g[l];
    double u[4];

    double ltot = 0.0;
    for (int s = 0; s < P->n_src; s++) ltot += P->lum[(size_t)s * P->n_lambda + l];
    const double w0 = ltot / (double)P->n_pkg;
    if (ltot == 0.0) { /* nothing is emitted at this wavelength: no package is launched */
        A->stats[ST_PACKAGES] += 1.0;
        return;
    }

    /* 1. emission */
    double r[3], k[3];
    draw(P->seed, p, (uint32_t)l, 1, u);
    int sidx = P->n_src - 1;
    {
        double target = u[2] * ltot, cum = 0.0;
        for (int s = 0; s < P->n_src; s++) {
            cum += P->lum[(size_t)s * P->n_lambda + l];
            if (target < cum) {
                sidx = s;
                break;
            }
        }
    }
    oracle_emit_direction(u, k);
    draw(P->seed, p, (uint32_t)l, 0, u);
    {
        const src_t *S = &P->src[sidx];
        double par[5] = {S->c[0], S->c[1], S->c[2], S->hr, S->hz};
        if (S->kind == SRC_CELLS)
            cell_emit_position(G, P->cell_cum + (size_t)l * (G->ncell + 1), u, r);
        else
            oracle_emit_position(S->kind, par, u, r);
    }
    double w = w0, w_eval = w0, score = 0.0;
    if (P->mode == MODE_REWEIGHT && P->lum_eval)
        w_eval = w0 * P->lum_eval[(size_t)sidx * P->n_lambda + l] / P->lum[(size_t)sidx * P->n_lambda + l];
    A->stats[ST_EMITTED] += w0;
    A->stats[ST_PACKAGES] += 1.0;

    if (P->mode == MODE_GRAD || P->mode == MODE_ATTACHED) {
        A->ncon = 0;
        sb_clear(&A->legs);
        sb_clear(&A->gpeel);
        grad_reserve_legs(A, 2);
    }
    if (P->mode == MODE_ATTACHED) {
        A->naev = 0;
        att_push(A, r, w);
    }

    /* 2. peel-off at emission */
    if (P->flags & FLAG_PEEL_EMIT) peel_event(P, A, l, 0, r, NULL, w, w_eval, 0.0);

    /* 3. scattering loop */
    for (int n = 0;; n++) {
        sb_clear(&A->path);
        traverse(G, r, k, &A->path);
        A->stats[ST_XPATH] += (double)A->path.n;
        double T = seg_tau(&A->path, P->rho, kappa);
        if (T == 0.0) {
            A->stats[ST_ESCAPED] += w;
            break;
        }
        /* continuous absorption along the whole path */
        {
            double tau = 0.0, tau_eval = 0.0;
            for (size_t j = 0; j < A->path.n; j++) {
                const seg_t *s = &A->path.v[j];
                double dtau = kappa * P->rho[s->cell] * (s->t1 - s->t0);
                double dep = w * (1.0 - alb) * exp(-tau) * (-expm1(-dtau));
                A->stats[ST_ABSORBED] += dep;
                if (A->absorbed && P->mode != MODE_REWEIGHT) A->absorbed[s->cell] += dep;
                if (A->absorbed && P->mode == MODE_REWEIGHT) { /* the same deposits at rho_eval, weight w_eval */
                    double dte = kappa * P->rho_eval[s->cell] * (s->t1 - s->t0);
                    A->absorbed[s->cell] += w_eval * (1.0 - (P->alb_eval ? P->alb_eval[l] : alb)) * exp(-tau_eval) *
                                            (-expm1(-dte));
                    tau_eval += dte;
                }
                tau += dtau;
            }
            A->stats[ST_ESCAPED] += w * exp(-T);
        }
        /* the absorbed tally's adjoint (GRAD with adj_abs): the path's deposits
         * dep_j = w (1 - albedo) e^-tau_{j-1} (1 - e^-dtau_j) weighted by
         * b = dL/dA of their cells sum to B; with paths held fixed, B carries
         * the density dependence of the weight w (the legs up to this event,
         * as a contribution of this event does), and each deposit that of its
         * own factor: -kappa l_k for every cell k crossed before it and
         * kappa l_j e^-dtau_j / (1 - e^-dtau_j) for its own cell.  Summed over
         * the path: cell k of segment j_k gets -kappa l_k (B - P_k), P_k the
         * sum of b dep up to and including segment j_k, plus
         * b_k w (1 - albedo) e^-tau_{j_k - 1} e^-dtau_k kappa l_k. */
        if (P->mode == MODE_GRAD && P->adj_abs) {
            const double *b = P->adj_abs + (size_t)l * G->ncell;
            double B = 0.0, tau = 0.0;
            for (size_t j = 0; j < A->path.n; j++) {
                const seg_t *s = &A->path.v[j];
                double dtau = kappa * P->rho[s->cell] * (s->t1 - s->t0);
                B += b[s->cell] * w * (1.0 - alb) * exp(-tau) * (-expm1(-dtau));
                tau += dtau;
            }
            double Pk = 0.0;
            tau = 0.0;
            for (size_t j = 0; j < A->path.n; j++) {
                const seg_t *s = &A->path.v[j];
                double len = s->t1 - s->t0, dtau = kappa * P->rho[s->cell] * len;
                Pk += b[s->cell] * w * (1.0 - alb) * exp(-tau) * (-expm1(-dtau));
                A->grad[s->cell] += -kappa * len * (B - Pk) +
                                    b[s->cell] * w * (1.0 - alb) * exp(-tau) * exp(-dtau) * kappa * len;
                tau += dtau;
            }
            if (B != 0.0) {
                contrib_t *C = grad_new_contrib(A);
                C->event = n;
                C->a_c = B;
                C->dlng = 0.0;
                C->absorbed = 1;
                C->det = -1;
                C->beg = C->end = A->gpeel.n;
            }
        }
        /* forced scattering: interaction point */
        draw(P->seed, p, (uint32_t)l, 2u + (uint32_t)n, u);
        double tau_s = oracle_forced_tau(T, u[0]);
        double tau = 0.0, s_hit = -1.0;
        int64_t c_hit = -1;
        size_t j_hit = 0, j_last = 0;
        for (size_t j = 0; j < A->path.n; j++) {
            const seg_t *s = &A->path.v[j];
            double ext = kappa * P->rho[s->cell];
            double dtau = ext * (s->t1 - s->t0);
            if (dtau > 0.0) j_last = j;
            if (tau <= tau_s && tau_s < tau + dtau) {
                s_hit = s->t0 + (tau_s - tau) / ext;
                c_hit = s->cell;
                j_hit = j;
                break;
            }
            tau += dtau;
        }
        if (c_hit < 0) { /* tau_s >= T through rounding: end of the last absorbing segment */
            s_hit = A->path.v[j_last].t1;
            c_hit = A->path.v[j_last].cell;
            j_hit = j_last;
        }
        A->stats[ST_XLOCATE] += (double)(j_hit + 1);
        A->stats[ST_EVENTS] += 1.0;

        if (P->mode == MODE_GRAD) { /* leg r_{n} -> s: full segments then the partial one */
            int i = n + 1;
            grad_reserve_legs(A, i + 1);
            A->leg_beg[i] = A->legs.n;
            for (size_t j = 0; j < j_hit; j++) sb_push(&A->legs, A->path.v[j].cell, A->path.v[j].t0, A->path.v[j].t1);
            sb_push(&A->legs, c_hit, A->path.v[j_hit].t0, s_hit);
            A->leg_end[i] = A->legs.n;
            A->leg_cell[i] = c_hit;
        }
        if (P->mode == MODE_REWEIGHT) {
            double dtau_leg = 0.0;
            for (size_t j = 0; j < j_hit; j++) {
                const seg_t *s = &A->path.v[j];
                dtau_leg += kappa * (P->rho_eval[s->cell] - P->rho[s->cell]) * (s->t1 - s->t0);
            }
            dtau_leg += kappa * (P->rho_eval[c_hit] - P->rho[c_hit]) * (s_hit - A->path.v[j_hit].t0);
            w_eval *= (P->alb_eval ? P->alb_eval[l] : alb) * (-expm1(-T)) * (P->rho_eval[c_hit] / P->rho[c_hit]) *
                      exp(-dtau_leg);
        }

        if (P->mode == MODE_ATTACHED) { /* the leg after the current event: its whole path to the boundary */
            att_ev_t *E = &A->aev[A->naev - 1];
            E->leg = 1;
            for (int a = 0; a < 3; a++) E->k[a] = k[a];
            E->T = T;
            E->tau_s = tau_s;
            E->s = s_hit;
            E->rho_s = P->rho[c_hit];
            E->beg = A->legs.n;
            for (size_t j = 0; j < A->path.n; j++)
                sb_push(&A->legs, A->path.v[j].cell, A->path.v[j].t0, A->path.v[j].t1);
            E->end = A->legs.n;
        }

        for (int a = 0; a < 3; a++) r[a] += s_hit * k[a];
        w *= alb * (-expm1(-T));
        if (P->mode == MODE_ATTACHED) att_push(A, r, w);

        if (P->flags & FLAG_PEEL_SCAT) peel_event(P, A, l, n + 1, r, k, w, w_eval, score);

        if (w < P->w_min * w0 || n + 1 >= P->max_scatter) {
            A->stats[ST_TRUNCATED] += w;
            break;
        }
        /* new direction: HG polar cosine and uniform azimuth */
        double mu = oracle_hg_mu(g, u[1]);
        score += hg_dlng(g, mu);
        if (P->mode == MODE_REWEIGHT && P->g_eval) w_eval *= hg_phase(P->g_eval[l], mu) / hg_phase(g, mu);
        double psi = 2.0 * OR_PI * u[2];
        double kn[3];
        oracle_rotate(k, mu, psi, kn);
        k[0] = kn[0];
        k[1] = kn[1];
        k[2] = kn[2];
    }

    if (P->mode == MODE_GRAD) grad_flush_package(P, A, l, sidx);
    if (P->mode == MODE_ATTACHED) attached_flush_package(P, A, l);
}

static void accum_free(accum_t *A)
{
    sb_free(&A->path);
    sb_free(&A->peel);
    sb_free(&A->legs);
    sb_free(&A->gpeel);
    free(A->leg_beg);
    free(A->leg_end);
    free(A->leg_cell);
    free(A->con);
    free(A->aev);
}

static int setup_problem(problem_t *P, const double box[6], const int n[3], const double *rho, int n_lambda,
                         const double *kappa, const double *albedo, const double *g, int n_src, const int *src_kind,
                         const double *src_par, const double *src_lum, int n_det, const double *det_par,
                         const int *det_pix, uint64_t n_pkg, uint64_t first, uint64_t seed, double w_min,
                         int max_scatter, unsigned flags, const double *planes, const double *tree,
                         const double *cell_lum)
{
    if (n_src < 1 || n_src > MAX_SRC || n_det < 0 || n_det > MAX_DET || n_lambda < 1 || n_pkg < 1) return -1;
    for (int a = 0; a < 3; a++)
        if (n[a] < 1 || !(box[2 * a + 1] > box[2 * a])) return -1;
    memset(P, 0, sizeof *P);
    if (grid_init(&P->G, box, n, planes, tree)) return -1;
    P->rho = rho;
    P->n_lambda = n_lambda;
    P->kappa = kappa;
    P->albedo = albedo;
    P->g = g;
    P->n_src = n_src;
    P->cell_src = -1;
    for (int s = 0; s < n_src; s++) {
        P->src[s].kind = src_kind[s];
        for (int a = 0; a < 3; a++) P->src[s].c[a] = src_par[5 * s + a];
        P->src[s].hr = src_par[5 * s + 3];
        P->src[s].hz = src_par[5 * s + 4];
        if (src_kind[s] == SRC_CELLS) {
            if (P->cell_src >= 0 || !cell_lum) {
                grid_free(&P->G);
                return -1;
            }
            P->cell_src = s;
        }
    }
    /* a cell source's luminosity at each wavelength is the sum over its cells */
    P->lum_own = (double *)malloc(sizeof(double) * (size_t)n_src * n_lambda);
    memcpy(P->lum_own, src_lum, sizeof(double) * (size_t)n_src * n_lambda);
    if (P->cell_src >= 0) {
        int64_t nc = P->G.ncell;
        P->cell_cum = (double *)malloc(sizeof(double) * (size_t)n_lambda * (nc + 1));
        for (int l = 0; l < n_lambda; l++) {
            double *cum = P->cell_cum + (size_t)l * (nc + 1), acc = 0.0;
            for (int64_t m = 0; m < nc; m++) {
                cum[m] = acc;
                acc += cell_lum[(size_t)l * nc + m];
            }
            cum[nc] = acc;
            P->lum_own[(size_t)P->cell_src * n_lambda + l] = acc;
        }
    }
    P->lum = P->lum_own;
    P->n_det = n_det;
    size_t off = 0;
    for (int d = 0; d < n_det; d++) {
        det_init(&P->det[d], det_par + 16 * d, det_pix + 2 * d);
        P->det[d].off = off;
        off += (size_t)det_pix[2 * d] * det_pix[2 * d + 1];
    }
    P->pix_lambda = off;
    P->n_pkg = n_pkg;
    P->first = first;
    P->seed = seed;
    P->w_min = w_min;
    P->max_scatter = max_scatter;
    P->flags = flags;
    return 0;
}

static void problem_free(problem_t *P)
{
    free(P->lum_own);
    free(P->cell_cum);
    P->lum_own = P->cell_cum = NULL;
    grid_free(&P->G);
}

/* Runs packages [first, first + n_pkg) for every wavelength.  Each thread
 * works on its own accumulators; the wavelength slices are summed in thread
 * order afterwards, so a single thread gives the plain serial sums. */
static int simulate(problem_t *P, double *images, double *absorbed, double *grad, double *grad_opt, double stats[ST_N],
                    int n_threads)
{
    int comps = (P->flags & FLAG_SPLIT) ? 2 : 1;
    size_t nimg = (size_t)comps * P->n_lambda * P->pix_lambda;
    int64_t ncell = P->G.ncell;
    memset(images, 0, nimg * sizeof(double));
    if (absorbed) memset(absorbed, 0, (size_t)P->n_lambda * ncell * sizeof(double));
    if (grad) memset(grad, 0, (size_t)ncell * sizeof(double));
    if (grad_opt) memset(grad_opt, 0, (size_t)(2 + P->n_src) * P->n_lambda * sizeof(double));
    for (int i = 0; i < ST_N; i++) stats[i] = 0.0;
    if (n_threads < 1) n_threads = 1;

    for (int l = 0; l < P->n_lambda; l++) {
        accum_t *acc = (accum_t *)calloc((size_t)n_threads, sizeof(accum_t));
        for (int t = 0; t < n_threads; t++) {
            acc[t].images = (double *)calloc(nimg, sizeof(double));
            if (absorbed) acc[t].absorbed = (double *)calloc((size_t)ncell, sizeof(double));
            if (grad) acc[t].grad = (double *)calloc((size_t)ncell, sizeof(double));
        }
        int64_t npk = (int64_t)P->n_pkg;
#pragma omp parallel for num_threads(n_threads) schedule(dynamic, 64)
        for (int64_t q = 0; q < npk; q++) {
            int t = 0;
#ifdef _OPENMP
            t = omp_get_thread_num();
#endif
            run_package(P, &acc[t], P->first + (uint64_t)q, l);
        }
        for (int t = 0; t < n_threads; t++) {
            for (size_t i = 0; i < nimg; i++) images[i] += acc[t].images[i];
            if (absorbed)
                for (int64_t m = 0; m < ncell; m++) absorbed[(size_t)l * ncell + m] += acc[t].absorbed[m];
            if (grad)
                for (int64_t m = 0; m < ncell; m++) grad[m] += acc[t].grad[m];
            for (int i = 0; i < ST_N; i++) stats[i] += acc[t].stats[i];
            if (grad_opt)
                for (int i = 0; i < 2 + P->n_src; i++) grad_opt[(size_t)i * P->n_lambda + l] += acc[t].gopt[i];
            free(acc[t].images);
            free(acc[t].absorbed);
            free(acc[t].grad);
            accum_free(&acc[t]);
        }
        free(acc);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Public entry points (ctypes).  Arrays:
 *   box[6]      xmin,xmax,ymin,ymax,zmin,zmax;  n[3] cells per axis
 *   rho[ncell]  density, cell m = i + nx (j + ny k)
 *   kappa, albedo, g [n_lambda]
 *   src_kind[n_src] (0 point, 1 exponential disk, 2 cells); src_par[n_src][5]
 *     = x, y, z, h_R, h_z;  src_lum[n_src][n_lambda]; cell_lum [n_lambda][ncell]
 *     of the cell source or NULL
 *   det_par[n_det][16] = distance, inclination, azimuth, position angle (deg),
 *     half-extent x, half-extent y, kind (0 frame, 1 SED, 2 perspective),
 *     eye[3], target[3], up[3];  det_pix[n_det][2] = nx, ny
 *   images [comps][n_lambda][sum over frames of ny*nx], comps = 2 with the
 *     split flag (0 direct, 1 scattered), else 1
 *   absorbed [n_lambda][ncell] or NULL
 *   stats[9] emitted, absorbed, escaped, truncated, path crossings, locate
 *     crossings, peel crossings, scattering events, packages
 * Returns 0, or -1 on invalid arguments. */

int oracle_run(const double box[6], const int n[3], const double *rho, int n_lambda, const double *kappa,
               const double *albedo, const double *g, int n_src, const int *src_kind, const double *src_par,
               const double *src_lum, int n_det, const double *det_par, const int *det_pix, uint64_t n_pkg,
               uint64_t first, uint64_t seed, double w_min, int max_scatter, unsigned flags, double *images,
               double *absorbed, double *stats, int n_threads, const double *planes, const double *tree,
               const double *cell_lum)
{
    problem_t P;
    if (setup_problem(&P, box, n, rho, n_lambda, kappa, albedo, g, n_src, src_kind, src_par, src_lum, n_det,
                      det_par, det_pix, n_pkg, first, seed, w_min, max_scatter, flags, planes, tree, cell_lum))
        return -1;
    P.mode = MODE_FORWARD;
    int rc = simulate(&P, images, (flags & FLAG_ABSORB) ? absorbed : NULL, NULL, NULL, stats, n_threads);
    problem_free(&P);
    return rc;
}

/* Gradient of L with respect to every cell density, given adj = dL/dI in
 * the image layout of oracle_run with the same flags.  Also returns the
 * images of the same run, and (grad_opt non-NULL, [2 + n_src][n_lambda])
 * the gradients with respect to the albedo, g and each source's luminosity
 * per wavelength.  Reading: the same detached derivative with paths held
 * fixed.  A contribution after n scatterings scales as albedo^n
 * (d/dalbedo = n C / albedo; reported 0 at albedo = 0); in g it carries
 * the log-derivative of the HG density of each direction sampled before it
 * and of its peel phase (the scores of a fixed path); and it scales as the
 * luminosity of its package's source (weight L_total / N times choice
 * probability L_s / L_total; d/dL_s = C / L_s, reported 0 for a dark
 * source).  Check: finite differences of the reweighted estimator in each
 * parameter, and the linear cases (one scattering at most; one source).
 * adj_abs non-NULL ([n_lambda][ncell], dL/dA): the loss also has a term in
 * the absorbed tally, and the density gradient includes it (the optics
 * gradients stay those of the images). */
int oracle_grad(const double box[6], const int n[3], const double *rho, int n_lambda, const double *kappa,
                const double *albedo, const double *g, int n_src, const int *src_kind, const double *src_par,
                const double *src_lum, int n_det, const double *det_par, const int *det_pix, uint64_t n_pkg,
                uint64_t first, uint64_t seed, double w_min, int max_scatter, unsigned flags, const double *adj,
                double *images, double *grad, double *stats, int n_threads, const double *planes,
                const double *tree, const double *cell_lum, double *grad_opt, const double *adj_abs)
{
    problem_t P;
    if (setup_problem(&P, box, n, rho, n_lambda, kappa, albedo, g, n_src, src_kind, src_par, src_lum, n_det,
                      det_par, det_pix, n_pkg, first, seed, w_min, max_scatter, flags, planes, tree, cell_lum))
        return -1;
    P.mode = MODE_GRAD;
    P.adj = adj;
    P.adj_abs = adj_abs;
    int rc = simulate(&P, images, NULL, grad, grad_opt, stats, n_threads);
    problem_free(&P);
    return rc;
}

/* Gradient of the same image loss with respect to every cell density by the
 * attached (pathwise) derivative (attached_flush_package): the random
 * numbers are held fixed and the scattering points move with the
 * densities.  Frames and SED instruments only (-1 with a perspective
 * instrument).  Also returns the images of the same run. */
int oracle_grad_attached(const double box[6], const int n[3], const double *rho, int n_lambda, const double *kappa,
                         const double *albedo, const double *g, int n_src, const int *src_kind,
                         const double *src_par, const double *src_lum, int n_det, const double *det_par,
                         const int *det_pix, uint64_t n_pkg, uint64_t first, uint64_t seed, double w_min,
                         int max_scatter, unsigned flags, const double *adj, double *images, double *grad,
                         double *stats, int n_threads, const double *planes, const double *tree,
                         const double *cell_lum)
{
    for (int d = 0; d < n_det; d++)
        if ((int)det_par[16 * d + 6] == DET_PERSPECTIVE) return -1;
    problem_t P;
    if (setup_problem(&P, box, n, rho, n_lambda, kappa, albedo, g, n_src, src_kind, src_par, src_lum, n_det,
                      det_par, det_pix, n_pkg, first, seed, w_min, max_scatter, flags, planes, tree, cell_lum))
        return -1;
    P.mode = MODE_ATTACHED;
    P.adj = adj;
    int rc = simulate(&P, images, NULL, grad, NULL, stats, n_threads);
    problem_free(&P);
    return rc;
}

/* Images of the estimator whose paths are sampled at rho0 and whose weights
 * are evaluated at rho (reweighting; a smooth function of rho whose
 * derivative at rho = rho0 is oracle_grad); likewise at the albedos, g and
 * source luminosities alb_eval, g_eval, lum_eval when given (NULL: the
 * sampling values): weights carry (albedo_eval)^n, the ratios of the HG
 * densities of the sampled directions and the peel phase at g_eval, and
 * the ratio of the package source's luminosities.  absorbed non-NULL
 * ([n_lambda][ncell]): the absorbed tally of the same estimator. */
int oracle_reweight(const double box[6], const int n[3], const double *rho0, const double *rho, int n_lambda,
                    const double *kappa, const double *albedo, const double *g, int n_src, const int *src_kind,
                    const double *src_par, const double *src_lum, int n_det, const double *det_par,
                    const int *det_pix, uint64_t n_pkg, uint64_t first, uint64_t seed, double w_min,
                    int max_scatter, unsigned flags, double *images, double *stats, int n_threads,
                    const double *planes, const double *tree, const double *cell_lum, const double *alb_eval,
                    const double *g_eval, const double *lum_eval, double *absorbed)
{
    problem_t P;
    if (setup_problem(&P, box, n, rho0, n_lambda, kappa, albedo, g, n_src, src_kind, src_par, src_lum, n_det,
                      det_par, det_pix, n_pkg, first, seed, w_min, max_scatter, flags, planes, tree, cell_lum))
        return -1;
    P.mode = MODE_REWEIGHT;
    P.rho_eval = rho;
    P.alb_eval = alb_eval;
    P.g_eval = g_eval;
    P.lum_eval = lum_eval;
    int rc = simulate(&P, images, absorbed, NULL, NULL, stats, n_threads);
    problem_free(&P);
    return rc;
}

/* Per-ray optical depth to the grid boundary, and optionally the segment
 * list (cell, length) of the first max_seg segments; n_seg gets the true
 * count.  Returns the total number of segments. */
int64_t oracle_trace(const double box[6], const int n[3], const double *rho, double kappa, int64_t n_rays,
                     const double *origin, const double *dir, double *tau, int max_seg, int64_t *seg_cell,
                     double *seg_len, int *n_seg, const double *planes, const double *tree)
{
    grid_t G;
    if (grid_init(&G, box, n, planes, tree)) return -1;
    segbuf sb = {0};
    int64_t total = 0;
    for (int64_t q = 0; q < n_rays; q++) {
        sb_clear(&sb);
        traverse(&G, origin + 3 * q, dir + 3 * q, &sb);
        tau[q] = seg_tau(&sb, rho, kappa);
        total += (int64_t)sb.n;
        if (n_seg) n_seg[q] = (int)sb.n;
        if (seg_cell && seg_len) {
            for (size_t j = 0; j < sb.n && (int)j < max_seg; j++) {
                seg_cell[q * max_seg + j] = sb.v[j].cell;
                seg_len[q * max_seg + j] = sb.v[j].t1 - sb.v[j].t0;
            }
        }
    }
    sb_free(&sb);
    grid_free(&G);
    return total;
}

/* Peel-off of a list of events into the frames of one wavelength:
 * images[frames] += w * phase * exp(-tau(r, k_d)) / D^2.  dir_in == NULL
 * means isotropic emission (phase 1/4pi), else HG with parameter g. */
int oracle_peel(const double box[6], const int n[3], const double *rho, double kappa, double g, int64_t n_events,
                const double *pos, const double *dir_in, const double *w, int n_det, const double *det_par,
                const int *det_pix, double *images, const double *planes, const double *tree)
{
    if (n_det < 1 || n_det > MAX_DET) return -1;
    grid_t G;
    if (grid_init(&G, box, n, planes, tree)) return -1;
    det_t det[MAX_DET];
    size_t off = 0;
    for (int d = 0; d < n_det; d++) {
        det_init(&det[d], det_par + 16 * d, det_pix + 2 * d);
        det[d].off = off;
        off += (size_t)det_pix[2 * d] * det_pix[2 * d + 1];
    }
    segbuf sb = {0};
    for (int64_t e = 0; e < n_events; e++) {
        const double *r = pos + 3 * e;
        for (int d = 0; d < n_det; d++) {
            int64_t pix = det_pixel(&det[d], r);
            if (pix < 0) continue;
            const double *kin = dir_in ? dir_in + 3 * e : NULL;
            double kd[3], inv_d2, len;
            det_peel_ray(&det[d], r, kd, &inv_d2, &len);
            double phase = kin ? hg_phase(g, kin[0] * kd[0] + kin[1] * kd[1] + kin[2] * kd[2]) : 1.0 / (4.0 * OR_PI);
            sb_clear(&sb);
            traverse(&G, r, kd, &sb);
            sb_clip(&sb, len);
            double tau = seg_tau(&sb, rho, kappa);
            images[det[d].off + (size_t)pix] += w[e] * phase * exp(-tau) * inv_d2;
        }
    }
    sb_free(&sb);
    grid_free(&G);
    return 0;
}

/* Detector geometry, exposed for the geometry checks: kd, ex, ey [9]
 * (perspective: the view axis, ex, ey). */
void oracle_detector_basis(const double par[16], double out[9])
{
    det_t D;
    int pix[2] = {1, 1};
    det_init(&D, par, pix);
    for (int a = 0; a < 3; a++) {
        out[a] = D.kind == DET_PERSPECTIVE ? D.view[a] : D.kd[a];
        out[3 + a] = D.ex[a];
        out[6 + a] = D.ey[a];
    }
}

/* HG phase value, exposed for the normalisation check. */
double oracle_hg_phase(double g, double mu) { return hg_phase(g, mu); }

/* Raw Philox words of draw c for packages p0 .. p0+n-1 at wavelength l:
 * out[4n].  Used by the statistical checks of the uniform deviates. */
void oracle_draw_words(uint64_t seed, uint64_t p0, int64_t n, uint32_t l, uint32_t c, uint32_t *out)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t q = 0; q < n; q++) {
        uint64_t p = p0 + (uint64_t)q;
        uint32_t ctr[4] = {(uint32_t)p, (uint32_t)(p >> 32), l, c};
        oracle_philox(ctr, key, out + 4 * q);
    }
}

/* ------------------------------------------------------------------------ */
/* Dust emission (Sect. 1: the dust absorbs and re-emits; Sect. 2.1:
 * panchromatic simulations).  Reading: the grains are modified black bodies
 * in radiative equilibrium.  A cell of dust mass M = rho V at temperature T
 * emits emissivity * M * sum_i kappa_abs_i B(lambda_i, T) dlambda_i with
 * B(lambda, T) = lambda^-5 / (exp(c2 / (lambda T)) - 1), c2 = hc/k =
 * 14387.77 um K (lambda in um), and its temperature is the one at which it
 * emits what it absorbed.  Checks: the closed form for one wavelength, the
 * Stefan-Boltzmann-type integrals of grey and lambda^-2 dust, Wien's
 * displacement law, and energy conservation per cell. */

#define OR_C2 14387.77

double oracle_mbb_sum(int nl, const double *lambda, const double *dlambda, const double *kabs, double T)
{
    double s = 0.0;
    for (int i = 0; i < nl; i++) {
        double l = lambda[i];
        s += kabs[i] * dlambda[i] / (l * l * l * l * l * expm1(OR_C2 / (l * T)));
    }
    return s;
}

/* Per cell: L = the cell's absorbed luminosity (sum of the n_abs rows),
 * M = rho V.  L <= 0 or M <= 0: T = 0 and no emission.  Else T solves
 * mbb_sum(T) = L / (emissivity M), by bisection in ln T over [ln 1, ln 1e5]
 * until no double lies strictly between the ends (a root outside the range
 * ends at its nearer end), and the cell emits L kappa_abs_i B(lambda_i, T)
 * dlambda_i / mbb_sum(T) at wavelength i (nothing if that sum is 0). */
int oracle_dust_emission(const double box[6], const int n[3], const double *planes, const double *tree,
                         const double *rho, int n_abs, const double *absorbed, int nl, const double *lambda,
                         const double *dlambda, const double *kabs, double emissivity, double *T_out,
                         double *emission)
{
    grid_t G;
    if (n_abs < 1 || nl < 1 || !(emissivity > 0.0)) return -1;
    if (grid_init(&G, box, n, planes, tree)) return -1;
    for (int64_t m = 0; m < G.ncell; m++) {
        double L = 0.0;
        for (int r = 0; r < n_abs; r++) L += absorbed[(size_t)r * G.ncell + m];
        double lo[3], hi[3];
        cell_bounds(&G, m, lo, hi);
        double M = rho[m] * (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
        double T = 0.0, S = 0.0;
        if (L > 0.0 && M > 0.0) {
            double y = L / (emissivity * M), a = 0.0, b = log(1e5);
            for (;;) {
                double mid = 0.5 * (a + b);
                if (!(mid > a && mid < b)) break;
                if (oracle_mbb_sum(nl, lambda, dlambda, kabs, exp(mid)) < y)
                    a = mid;
                else
                    b = mid;
            }
            T = exp(a);
            S = oracle_mbb_sum(nl, lambda, dlambda, kabs, T);
        }
        T_out[m] = T;
        for (int i = 0; i < nl; i++) {
            double l = lambda[i];
            emission[(size_t)i * G.ncell + m] =
                S > 0.0 ? L * (kabs[i] * dlambda[i] / (l * l * l * l * l * expm1(OR_C2 / (l * T)))) / S : 0.0;
        }
    }
    grid_free(&G);
    return 0;
}
