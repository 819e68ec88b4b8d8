/*
 * merf_oracle.c -- FP64 CPU oracle for MERF deferred volume rendering.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU renderer is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it; the renderer itself never
 * links, imports or calls it, and it shares no code, header or table with the
 * GPU library.
 *
 * Everything is computed in double precision, one ray at a time, in the order
 * the paper describes (MERF, arXiv 2302.12249):
 *   ray  ->  piecewise-projective contraction (Sec. 4.2, Eq. 7), split into
 *   straight contracted segments  ->  uniform lattice of samples in contracted
 *   space  ->  occupancy test on every level (Sec. 6)  ->  feature lookup
 *   t = V + P_x + P_y + P_z (Sec. 4.1, Eq. 5) from byte values dequantised by
 *   Eq. 8  ->  nonlinearities (Eq. 6)  ->  emission-absorption compositing of
 *   density, diffuse colour and features (Sec. 3, Eq. 1-2) with early
 *   termination (Sec. 6)  ->  deferred MLP once per ray (Eq. 3, App. B).
 *
 * There is no empty-space *skipping* here: every lattice sample is tested
 * against the occupancy levels one by one.  Skipping to a cell exit (Sec. 6)
 * only avoids testing samples that lie in an empty cell, so the set of
 * evaluated samples -- and hence the image -- is the same; the GPU path that
 * does skip is checked against this definition.
 *
 * Readings taken where the paper is silent (each is listed with its reason in
 * the design notes that accompany the repository):
 *   - Eq. 7 ties: the region axis is the first index j with |x_j| = ||x||_inf.
 *   - Rays start at the camera centre (t = 0) and go to t = infinity, whose
 *     contracted image is a finite limit point.
 *   - Samples: each straight contracted segment is cut, from its start, into
 *     intervals of contracted length `step` (the last one shorter); one sample
 *     at each interval midpoint; delta = the interval's contracted length
 *     (delta_mode 0) or the world length of its preimage (delta_mode 1).
 *   - Texels are cell-centred at -2 + (k + 1/2) * 4/N with clamp-to-edge;
 *     an absent block reads byte 0 on every channel.
 *   - Plane P_x is indexed (u, v) = (y, z), P_y (x, z), P_z (x, y).
 *   - Occupancy cell of level r: clamp(floor((p + 2) r / 4), 0, r - 1).
 *   - Deferred MLP input: [C_d(3), F(4), d(3), sin(2^k d), cos(2^k d) for
 *     k = 0..3] = 34 values, ReLU hidden layers, linear output, RGB = C_d + h.
 *   - Output alpha = 1 - T_final; no background term.
 *
 * The functions exported below are also called one by one by the tests that
 * pin this oracle to closed forms and invariants.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_LEVELS 4
#define OR_MAX_SEG 8
#define OR_MAX_CAND 12

typedef struct {
    int32_t L, B, R, C;
    int32_t num_blocks;
    int32_t occ_levels;
    const int32_t *block_index;   /* [(L/B)^3] z-major, -1 = absent            */
    const uint8_t *blocks;        /* [num_blocks][B][B][B][C]  (z, y, x, c)     */
    const uint8_t *planes;        /* [3][R][R][C]: P_x[z][y], P_y[z][x], P_z[y][x] */
    int32_t occ_res[OR_MAX_LEVELS];
    const uint8_t *occ[OR_MAX_LEVELS]; /* coarse -> fine, [r][r][r] z-major    */
    double m_density, m_feature;  /* Eq. 8 ranges: 14 and 7                     */
    int32_t mlp_in, mlp_hidden;
    const float *mlp;             /* W0[in][h] b0[h] W1[h][h] b1[h] W2[h][3] b2[3] */
} or_scene;

typedef struct {
    double c2w[12];               /* row-major 3x4 camera-to-world (OpenCV axes) */
    double fx, fy, cx, cy;
    int32_t width, height;
} or_camera;

typedef struct {
    double step;                  /* contracted step between samples            */
    double t_min;                 /* transmittance threshold, 2e-4 (Sec. 6)     */
    int32_t delta_mode;           /* 0 = contracted interval, 1 = world interval */
    int32_t want_fragile;         /* also compute the fragility flag            */
    double eps_occ;               /* fragility margin to occupancy faces        */
    double eps_int;               /* fragility margin on interval counts        */
} or_params;

/* ------------------------------------------------------------------------ */
/* Eq. 7: piecewise-projective contraction                                   */
/* ------------------------------------------------------------------------ */

/* Region of a point: 0 = unit cube; otherwise 1 + 2j + (x_j < 0) for the
 * first axis j reaching the infinity norm. */
int or_region(const double x[3])
{
    double r = fabs(x[0]);
    int j = 0;
    for (int k = 1; k < 3; ++k)
        if (fabs(x[k]) > r) { r = fabs(x[k]); j = k; }
    if (r <= 1.0) return 0;
    return 1 + 2 * j + (x[j] < 0.0 ? 1 : 0);
}

/* The projective map that Eq. 7 uses inside region `reg`, applied to x.
 * Region (j, s): y_j = (2 - 1/|x_j|) s and y_k = x_k / |x_j|. */
void or_map_region(int reg, const double x[3], double y[3])
{
    if (reg == 0) { y[0] = x[0]; y[1] = x[1]; y[2] = x[2]; return; }
    int j = (reg - 1) / 2;
    double s = ((reg - 1) & 1) ? -1.0 : 1.0;
    double a = fabs(x[j]);
    for (int k = 0; k < 3; ++k) y[k] = x[k] / a;
    y[j] = (2.0 - 1.0 / a) * s;
}

void or_contract(const double x[3], double y[3])
{
    or_map_region(or_region(x), x, y);
}

/* Inverse of the region map (used for world-space deltas and by tests). */
void or_unmap_region(int reg, const double y[3], double x[3])
{
    if (reg == 0) { x[0] = y[0]; x[1] = y[1]; x[2] = y[2]; return; }
    int j = (reg - 1) / 2;
    double s = ((reg - 1) & 1) ? -1.0 : 1.0;
    double a = 1.0 / (2.0 - s * y[j]);   /* |x_j| */
    for (int k = 0; k < 3; ++k) x[k] = y[k] * a;
    x[j] = s * a;
}

/* Contracted image of the point at infinity of a ray with direction d that
 * ends in region `reg`: y_j = 2 s, y_k = d_k / |d_j|. */
static void or_limit_point(int reg, const double d[3], double y[3])
{
    int j = (reg - 1) / 2;
    double s = ((reg - 1) & 1) ? -1.0 : 1.0;
    double a = fabs(d[j]);
    for (int k = 0; k < 3; ++k) y[k] = d[k] / a;
    y[j] = 2.0 * s;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Candidate parameters t > 0 where the region of o + t d can change: the
 * cube faces x_j = +-1 and the seams x_j = +-x_k.  Returns the count. */
int or_candidates(const double o[3], const double d[3], double cand[OR_MAX_CAND])
{
    int n = 0;
    for (int j = 0; j < 3; ++j) {
        if (d[j] != 0.0) {
            double t1 = (1.0 - o[j]) / d[j], t2 = (-1.0 - o[j]) / d[j];
            if (t1 > 0.0 && isfinite(t1)) cand[n++] = t1;
            if (t2 > 0.0 && isfinite(t2)) cand[n++] = t2;
        }
    }
    for (int j = 0; j < 3; ++j)
        for (int k = j + 1; k < 3; ++k) {
            double den1 = d[j] - d[k], den2 = d[j] + d[k];
            if (den1 != 0.0) {
                double t = (o[k] - o[j]) / den1;
                if (t > 0.0 && isfinite(t)) cand[n++] = t;
            }
            if (den2 != 0.0) {
                double t = (-o[k] - o[j]) / den2;
                if (t > 0.0 && isfinite(t)) cand[n++] = t;
            }
        }
    qsort(cand, (size_t)n, sizeof(double), cmp_double);
    return n;
}

/* Split the ray o + t d, t in [0, inf), into maximal intervals of constant
 * region.  Outputs per segment: world end parameters ta[i] < tb[i]
 * (tb = INFINITY for the last), region reg[i], and contracted end points
 * ya[i], yb[i].  Returns the number of segments (at most 7). */
int or_segments(const double o[3], const double d[3], double ta[OR_MAX_SEG], double tb[OR_MAX_SEG],
                int reg[OR_MAX_SEG], double ya[OR_MAX_SEG][3], double yb[OR_MAX_SEG][3])
{
    double cand[OR_MAX_CAND];
    int nc = or_candidates(o, d, cand);
    double bnd[OR_MAX_CAND + 2];
    int nb = 0;
    bnd[nb++] = 0.0;
    for (int i = 0; i < nc; ++i) bnd[nb++] = cand[i];
    bnd[nb++] = INFINITY;
    int ns = 0;
    for (int i = 0; i + 1 < nb; ++i) {
        double a = bnd[i], b = bnd[i + 1];
        if (!(b > a)) continue;
        double tm = isinf(b) ? 2.0 * a + 1.0 : 0.5 * (a + b);
        double xm[3] = {o[0] + tm * d[0], o[1] + tm * d[1], o[2] + tm * d[2]};
        int r = or_region(xm);
        if (ns > 0 && reg[ns - 1] == r) { tb[ns - 1] = b; continue; }
        ta[ns] = a; tb[ns] = b; reg[ns] = r; ++ns;
    }
    for (int i = 0; i < ns; ++i) {
        double xa[3] = {o[0] + ta[i] * d[0], o[1] + ta[i] * d[1], o[2] + ta[i] * d[2]};
        or_map_region(reg[i], xa, ya[i]);
        if (isinf(tb[i])) {
            or_limit_point(reg[i], d, yb[i]);
        } else {
            double xb[3] = {o[0] + tb[i] * d[0], o[1] + tb[i] * d[1], o[2] + tb[i] * d[2]};
            or_map_region(reg[i], xb, yb[i]);
        }
    }
    return ns;
}

/* ------------------------------------------------------------------------ */
/* Eq. 8: dequantisation; Sec. 4.1 (Eq. 5): feature lookup                    */
/* ------------------------------------------------------------------------ */

double or_dequant(int b, double m)
{
    return 2.0 * m * (double)b / 255.0 - m;
}

static double channel_m(const or_scene *s, int c)
{
    return c == 0 ? s->m_density : s->m_feature;
}

/* Cell-centred texel coordinate with clamp-to-edge: lower index and weight. */
static void texel_coord(double p, int n, int *i0, int *i1, double *f)
{
    double g = (p + 2.0) * (double)n / 4.0 - 0.5;
    double fl = floor(g);
    int a = (int)fl;
    *f = g - fl;
    int b = a + 1;
    *i0 = a < 0 ? 0 : (a > n - 1 ? n - 1 : a);
    *i1 = b < 0 ? 0 : (b > n - 1 ? n - 1 : b);
}

/* Byte of the sparse 3D grid V at voxel (x, y, z); 0 in an absent block. */
static int grid_byte(const or_scene *s, int x, int y, int z, int c)
{
    int B = s->B, nb = s->L / B;
    int bi = s->block_index[((size_t)(z / B) * nb + (size_t)(y / B)) * nb + (size_t)(x / B)];
    if (bi < 0) return 0;
    size_t off = ((((size_t)bi * B + (size_t)(z % B)) * B + (size_t)(y % B)) * B + (size_t)(x % B)) * s->C + c;
    return s->blocks[off];
}

static int plane_byte(const or_scene *s, int plane, int u, int v, int c)
{
    size_t R = (size_t)s->R;
    return s->planes[(((size_t)plane * R + (size_t)v) * R + (size_t)u) * s->C + c];
}

/* Eq. 5: t(p) = V(p) + P_x(p_y, p_z) + P_y(p_x, p_z) + P_z(p_x, p_y), with
 * each stored byte dequantised (Eq. 8) before interpolation.  A scene without
 * the 3D grid (L = 0, the representation the paper ablates in Sec. 7) sums the
 * planes only; a scene without planes (R = 0) is the sparse grid alone. */
void or_features(const or_scene *s, const double p[3], double t[8])
{
    const int has_grid = s->L > 0, has_planes = s->R > 0;
    int gi[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    double gf[3] = {0, 0, 0};
    if (has_grid)
        for (int a = 0; a < 3; ++a) texel_coord(p[a], s->L, &gi[a][0], &gi[a][1], &gf[a]);
    int pi[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    double pf[3] = {0, 0, 0};
    if (has_planes)
        for (int a = 0; a < 3; ++a) texel_coord(p[a], s->R, &pi[a][0], &pi[a][1], &pf[a]);
    /* (u axis, v axis) of planes P_x, P_y, P_z */
    static const int uax[3] = {1, 0, 0}, vax[3] = {2, 2, 1};
    for (int c = 0; c < s->C; ++c) {
        double m = channel_m(s, c);
        double v = 0.0;
        for (int dz = 0; dz < 2 && has_grid; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    double w = (dx ? gf[0] : 1.0 - gf[0]) * (dy ? gf[1] : 1.0 - gf[1]) *
                               (dz ? gf[2] : 1.0 - gf[2]);
                    v += w * or_dequant(grid_byte(s, gi[0][dx], gi[1][dy], gi[2][dz], c), m);
                }
        for (int pl = 0; pl < 3 && has_planes; ++pl) {
            int ua = uax[pl], va = vax[pl];
            for (int dv = 0; dv < 2; ++dv)
                for (int du = 0; du < 2; ++du) {
                    double w = (du ? pf[ua] : 1.0 - pf[ua]) * (dv ? pf[va] : 1.0 - pf[va]);
                    v += w * or_dequant(plane_byte(s, pl, pi[ua][du], pi[va][dv], c), m);
                }
        }
        t[c] = v;
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. 6: occupancy                                                          */
/* ------------------------------------------------------------------------ */

static int occ_cell(double p, int r)
{
    double g = floor((p + 2.0) * (double)r / 4.0);
    if (g < 0.0) return 0;
    if (g > (double)(r - 1)) return r - 1;
    return (int)g;
}

/* 1 iff every occupancy level marks the cell containing p as occupied. */
int or_occupied(const or_scene *s, const double p[3])
{
    for (int l = 0; l < s->occ_levels; ++l) {
        int r = s->occ_res[l];
        size_t idx = ((size_t)occ_cell(p[2], r) * r + (size_t)occ_cell(p[1], r)) * r + (size_t)occ_cell(p[0], r);
        if (!s->occ[l][idx]) return 0;
    }
    return 1;
}

/* A sample is fragile when it lies within eps of a face of some occupancy
 * cell and moving it across that face changes the all-levels decision: an
 * FP32 renderer may legitimately decide it the other way. */
static int occ_fragile(const or_scene *s, const double p[3], double eps)
{
    int here = or_occupied(s, p);
    for (int a = 0; a < 3; ++a) {
        int near = 0;
        for (int l = 0; l < s->occ_levels && !near; ++l) {
            double g = (p[a] + 2.0) * (double)s->occ_res[l] / 4.0;
            double h = 4.0 / (double)s->occ_res[l];
            double fr = g - floor(g);
            if (fr * h < eps || (1.0 - fr) * h < eps) near = 1;
        }
        if (!near) continue;
        double q[3] = {p[0], p[1], p[2]};
        q[a] = p[a] + 2.0 * eps;
        if (or_occupied(s, q) != here) return 1;
        q[a] = p[a] - 2.0 * eps;
        if (or_occupied(s, q) != here) return 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Eq. 3 / App. B: deferred MLP                                               */
/* ------------------------------------------------------------------------ */

/* MLP input: diffuse colour, features, view direction and its sin/cos
 * encoding with 4 frequencies 2^0..2^3. */
void or_encode(const double cd[3], const double f[4], const double d[3], double x[34])
{
    int n = 0;
    for (int i = 0; i < 3; ++i) x[n++] = cd[i];
    for (int i = 0; i < 4; ++i) x[n++] = f[i];
    for (int i = 0; i < 3; ++i) x[n++] = d[i];
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 3; ++i) x[n++] = sin(ldexp(d[i], k));
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 3; ++i) x[n++] = cos(ldexp(d[i], k));
}

/* h(x): in -> hidden (ReLU) -> hidden (ReLU) -> 3 (linear). */
void or_mlp(const or_scene *s, const double *x, double y[3])
{
    int in = s->mlp_in, h = s->mlp_hidden;
    const float *W0 = s->mlp, *b0 = W0 + in * h, *W1 = b0 + h, *b1 = W1 + h * h, *W2 = b1 + h,
                *b2 = W2 + h * 3;
    double h1[64], h2[64];
    for (int o = 0; o < h; ++o) {
        double a = b0[o];
        for (int i = 0; i < in; ++i) a += x[i] * (double)W0[i * h + o];
        h1[o] = a > 0.0 ? a : 0.0;
    }
    for (int o = 0; o < h; ++o) {
        double a = b1[o];
        for (int i = 0; i < h; ++i) a += h1[i] * (double)W1[i * h + o];
        h2[o] = a > 0.0 ? a : 0.0;
    }
    for (int o = 0; o < 3; ++o) {
        double a = b2[o];
        for (int i = 0; i < h; ++i) a += h2[i] * (double)W2[i * 3 + o];
        y[o] = a;
    }
}

/* ------------------------------------------------------------------------ */
/* One ray                                                                   */
/* ------------------------------------------------------------------------ */

static double sigmoid(double v) { return 1.0 / (1.0 + exp(-v)); }

/* Optional per-sample log for tests: position, delta, evaluated flag, alpha,
 * transmittance before the sample, segment index. */
typedef struct {
    double p[3], delta, alpha, T;
    int32_t evaluated, segment;
} or_sample;

/* Per-ray statistics (all optional). */
typedef struct {
    double visited, evaluated, contributing, sum_w, T, segments, fragile;
    double cd[3], feat[4];
} or_ray_stats;

/* World length of the preimage of the contracted interval [y0, y1] in region reg. */
static double world_delta(int reg, const double y0[3], const double y1[3])
{
    if (reg != 0) {
        int j = (reg - 1) / 2;
        double s = ((reg - 1) & 1) ? -1.0 : 1.0;
        if (s * y1[j] >= 2.0 || s * y0[j] >= 2.0) return INFINITY;
    }
    double x0[3], x1[3];
    or_unmap_region(reg, y0, x0);
    or_unmap_region(reg, y1, x1);
    double dx = x1[0] - x0[0], dy = x1[1] - x0[1], dz = x1[2] - x0[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* Render one ray.  out = (R, G, B, 1 - T).  Returns the number of samples
 * written to `log` (if log != NULL, at most log_cap are written). */
int or_render_ray(const or_scene *s, const or_params *P, const double o[3], const double d[3],
                  double out[4], or_ray_stats *st, or_sample *log, int log_cap)
{
    double ta[OR_MAX_SEG], tb[OR_MAX_SEG], ya[OR_MAX_SEG][3], yb[OR_MAX_SEG][3];
    int reg[OR_MAX_SEG];
    int ns = or_segments(o, d, ta, tb, reg, ya, yb);

    double T = 1.0, cd[3] = {0, 0, 0}, F[4] = {0, 0, 0, 0}, sum_w = 0.0;
    double visited = 0, evaluated = 0, contributing = 0;
    int fragile = 0, nlog = 0, done = 0;
    const double step = P->step;

    if (P->want_fragile) {
        /* Grazing: two region-candidate parameters almost equal, at a point on
         * or outside the unit cube (inside it the seams do not change the
         * region) that is occupied, may give an extra or a missing tiny
         * segment in FP32. */
        double cand[OR_MAX_CAND];
        int nc = or_candidates(o, d, cand);
        for (int i = 0; i + 1 < nc; ++i) {
            if (cand[i + 1] - cand[i] <= 1e-6 * fmax(1.0, cand[i])) {
                double x[3] = {o[0] + cand[i] * d[0], o[1] + cand[i] * d[1], o[2] + cand[i] * d[2]};
                double r = fmax(fabs(x[0]), fmax(fabs(x[1]), fabs(x[2])));
                if (r < 1.0 - 1e-6) continue;
                double y[3];
                or_contract(x, y);
                if (or_occupied(s, y)) fragile = 1;
            }
        }
    }

    for (int sg = 0; sg < ns && !done; ++sg) {
        double dir[3] = {yb[sg][0] - ya[sg][0], yb[sg][1] - ya[sg][1], yb[sg][2] - ya[sg][2]};
        double len = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
        if (!(len > 0.0)) continue;
        for (int a = 0; a < 3; ++a) dir[a] /= len;
        long n = (long)ceil(len / step);
        if (P->want_fragile) {
            /* Interval count close to an integer: an FP32 renderer may add or
             * drop a vanishing last interval, which matters when occupied. */
            double q = len / step;
            if (fabs(q - floor(q + 0.5)) < P->eps_int && or_occupied(s, yb[sg])) fragile = 1;
        }
        for (long k = 0; k < n; ++k) {
            double u0 = (double)k * step;
            double u1 = fmin((double)(k + 1) * step, len);
            double um = 0.5 * (u0 + u1);
            double p[3] = {ya[sg][0] + um * dir[0], ya[sg][1] + um * dir[1], ya[sg][2] + um * dir[2]};
            double delta = u1 - u0;
            if (P->delta_mode == 1) {
                double y0[3] = {ya[sg][0] + u0 * dir[0], ya[sg][1] + u0 * dir[1], ya[sg][2] + u0 * dir[2]};
                double y1[3] = {ya[sg][0] + u1 * dir[0], ya[sg][1] + u1 * dir[1], ya[sg][2] + u1 * dir[2]};
                if (k == n - 1) { y1[0] = yb[sg][0]; y1[1] = yb[sg][1]; y1[2] = yb[sg][2]; }
                delta = world_delta(reg[sg], y0, y1);
            }
            visited += 1;
            if (P->want_fragile && !fragile && occ_fragile(s, p, P->eps_occ)) fragile = 1;
            int ev = or_occupied(s, p);
            double alpha = 0.0, Tb = T;
            if (ev) {
                evaluated += 1;
                double t[8];
                or_features(s, p, t);
                double tau = exp(t[0]);                                  /* Eq. 6 */
                alpha = isinf(delta) ? (tau > 0.0 ? 1.0 : 0.0) : -expm1(-tau * delta); /* Eq. 1 */
                double w = T * alpha;
                if (alpha > 0.0) contributing += 1;
                for (int c = 0; c < 3; ++c) cd[c] += w * sigmoid(t[1 + c]);   /* Eq. 2 */
                for (int c = 0; c < 4; ++c) F[c] += w * sigmoid(t[4 + c]);
                sum_w += w;
                T *= (1.0 - alpha);
            }
            if (log && nlog < log_cap) {
                or_sample *e = &log[nlog];
                e->p[0] = p[0]; e->p[1] = p[1]; e->p[2] = p[2];
                e->delta = delta; e->alpha = alpha; e->T = Tb; e->evaluated = ev; e->segment = sg;
            }
            ++nlog;
            if (T < P->t_min) { done = 1; break; }                         /* Sec. 6 */
        }
    }

    double x[64], y[3];
    or_encode(cd, F, d, x);
    or_mlp(s, x, y);                                                       /* Eq. 3 */
    out[0] = cd[0] + y[0];
    out[1] = cd[1] + y[1];
    out[2] = cd[2] + y[2];
    out[3] = 1.0 - T;
    if (st) {
        st->visited = visited; st->evaluated = evaluated; st->contributing = contributing;
        st->sum_w = sum_w; st->T = T; st->segments = ns; st->fragile = fragile;
        for (int c = 0; c < 3; ++c) st->cd[c] = cd[c];
        for (int c = 0; c < 4; ++c) st->feat[c] = F[c];
    }
    return nlog;
}

/* Pinhole ray through the centre of pixel (row i, column j), unit direction. */
void or_camera_ray(const or_camera *cam, int i, int j, double o[3], double d[3])
{
    double v[3] = {((double)j + 0.5 - cam->cx) / cam->fx, ((double)i + 0.5 - cam->cy) / cam->fy, 1.0};
    double n = 0.0;
    for (int r = 0; r < 3; ++r) {
        o[r] = cam->c2w[4 * r + 3];
        d[r] = cam->c2w[4 * r + 0] * v[0] + cam->c2w[4 * r + 1] * v[1] + cam->c2w[4 * r + 2] * v[2];
        n += d[r] * d[r];
    }
    n = sqrt(n);
    for (int r = 0; r < 3; ++r) d[r] /= n;
}

/* Render a batch of cameras.  Pixels are stored camera after camera, each
 * camera row-major; out is [pixels][4].  `rows_stride` > 1 renders only
 * every rows_stride-th row of every camera (row_offset first) and packs the
 * results densely (used for bounded CPU timing samples).  stats may be NULL.
 * Returns the number of pixels rendered. */
long or_render(const or_scene *s, const or_camera *cams, int ncams, const or_params *P, double *out,
               or_ray_stats *stats, int nthreads, int rows_stride, int row_offset)
{
    if (rows_stride < 1) rows_stride = 1;
    long total = 0;
    for (int c = 0; c < ncams; ++c) {
        const or_camera *cam = &cams[c];
        int nrows = 0;
        for (int i = row_offset; i < cam->height; i += rows_stride) ++nrows;
        long base = total;
#ifdef _OPENMP
        /* a thread count for this call only (omp_set_num_threads would
         * persist into later calls) */
        const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
        for (int ri = 0; ri < nrows; ++ri) {
            int i = row_offset + ri * rows_stride;
            for (int j = 0; j < cam->width; ++j) {
                long px = base + (long)ri * cam->width + j;
                double o[3], d[3];
                or_camera_ray(cam, i, j, o, d);
                or_render_ray(s, P, o, d, out + 4 * px, stats ? stats + px : NULL, NULL, 0);
            }
        }
        total += (long)nrows * cam->width;
    }
    return total;
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
