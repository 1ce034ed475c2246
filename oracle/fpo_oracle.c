/*
 * Fourier PlenOctree oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of what the render and fine-tune
 * path computes.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load it; the product path never does.  It shares no code
 * with the HIP library: its own basis, spherical harmonics, camera model,
 * point location (a hash of leaf keys), finest-lattice DDA, compositing,
 * gradient and time bake.
 *
 * Paper: Wang et al., "Fourier PlenOctrees for Dynamic Radiance Field
 * Rendering in Real-time", CVPR 2022.
 *   - Eq. 1 (Sec. 3): colour c(d; z) = sigmoid(sum_{l<=2} sum_m z_{m,l} Y_{m,l}(d)).
 *   - Eq. 6 (Sec. 4.1): a leaf holds k^sigma (n1) and k^z (n2 x 9 x 3).
 *   - Eq. 7, 9 (Sec. 4.1): sigma(t) and z_{m,l}(t) are sums of k_i IDFT_i(t).
 *   - Eq. 8 (Sec. 4.1): IDFT_i(t) = cos(i pi t / T), i even; sin((i+1) pi t / T), i odd.
 *   - Eq. 13 (Sec. 4.3): the L2 photometric loss that fine-tuning minimises.
 * Volume rendering itself is inherited from NeRF / PlenOctree (Sec. 1, Sec. 3,
 * and the transmittance T_i of Sec. 3): along a ray the field at time t is
 * piecewise constant over leaves, so the rendered colour is exactly
 *     C = sum_i T_i (1 - exp(-sigma_i delta_i)) c_i + T_N bg,
 *     T_i = exp(-sum_{j<i} sigma_j delta_j).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - density: sigma_eff = s * max(sigma(t), 0) per unit-cube length;
 *   - scene: the unit cube [0,1]^3, leaf (d,i,j,k) covers [i,i+1) 2^-d x ...;
 *   - SH: real orthonormal basis with the Condon-Shortley phase, j = l^2+l+m;
 *   - early termination: stop after the segment that drives T below tau;
 *   - camera: pinhole through pixel centres, y up.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_N_SH 9
#define OR_MAX_COEFF 512

/* ------------------------------------------------------------------------ */
/* Eq. 8: the real Fourier basis.                                            */
/* ------------------------------------------------------------------------ */
void or_basis(double t, double period, int32_t n, double* out)
{
    for (int32_t i = 0; i < n; ++i) {
        if (i % 2 == 0)
            out[i] = cos((double)i * M_PI * t / period);
        else
            out[i] = sin((double)(i + 1) * M_PI * t / period);
    }
}

/* ------------------------------------------------------------------------ */
/* Eq. 1: real spherical harmonics up to degree 2 of a unit direction.       */
/* Orthonormal on the sphere, Condon-Shortley phase, index j = l^2 + l + m.  */
/* ------------------------------------------------------------------------ */
void or_sh9(const double dir[3], double out[9])
{
    const double x = dir[0], y = dir[1], z = dir[2];
    const double c0 = 0.5 * sqrt(1.0 / M_PI);          /* Y_00            */
    const double c1 = sqrt(3.0 / (4.0 * M_PI));         /* Y_1m            */
    const double c2 = 0.5 * sqrt(15.0 / M_PI);          /* Y_2,{-2,-1,1}   */
    const double c20 = 0.25 * sqrt(5.0 / M_PI);         /* Y_20            */
    const double c22 = 0.25 * sqrt(15.0 / M_PI);        /* Y_22            */
    out[0] = c0;
    out[1] = -c1 * y;
    out[2] = c1 * z;
    out[3] = -c1 * x;
    out[4] = c2 * x * y;
    out[5] = -c2 * y * z;
    out[6] = c20 * (3.0 * z * z - 1.0);
    out[7] = -c2 * x * z;
    out[8] = c22 * (x * x - y * y);
}

/* ------------------------------------------------------------------------ */
/* Pinhole camera through pixel centres, y up.                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    double eye[3], fwd[3], up[3];
    double fov_y_deg;
    int32_t width, height;
    double time;
} or_camera;

static void or_normalize(double v[3])
{
    double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n; v[1] /= n; v[2] /= n;
}

static void or_cross(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

void or_camera_ray(const or_camera* cam, int32_t px, int32_t py, double o[3], double d[3])
{
    double f[3] = {cam->fwd[0], cam->fwd[1], cam->fwd[2]};
    or_normalize(f);
    double r[3];
    or_cross(f, cam->up, r);
    or_normalize(r);
    double u[3];
    or_cross(r, f, u);
    const double tan_h = tan(0.5 * cam->fov_y_deg * M_PI / 180.0);
    const double aspect = (double)cam->width / (double)cam->height;
    const double sx = (2.0 * ((double)px + 0.5) / (double)cam->width - 1.0) * tan_h * aspect;
    const double sy = (1.0 - 2.0 * ((double)py + 0.5) / (double)cam->height) * tan_h;
    for (int a = 0; a < 3; ++a) {
        o[a] = cam->eye[a];
        d[a] = f[a] + sx * r[a] + sy * u[a];
    }
    or_normalize(d);
}

/* Rays for n pixels of one camera. */
void or_camera_rays(const or_camera* cam, int64_t n, const int32_t* px, const int32_t* py,
                    double* o, double* d)
{
    for (int64_t r = 0; r < n; ++r) or_camera_ray(cam, px[r], py[r], o + 3 * r, d + 3 * r);
}

/* ------------------------------------------------------------------------ */
/* Octree leaves, located through a hash of (depth, i, j, k).                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t max_depth;
    int64_t n_leaves;
    uint64_t mask;
    uint64_t* keys; /* 0 = empty slot */
    int64_t* vals;
} or_tree;

static uint64_t or_key(int32_t d, int64_t i, int64_t j, int64_t k)
{
    return 1u + (((uint64_t)d << 60) | ((uint64_t)i << 40) | ((uint64_t)j << 20) | (uint64_t)k);
}

static uint64_t or_mix(uint64_t x)
{
    /* splitmix64 finaliser */
    x ^= x >> 30; x *= 0xbf58476d1ce4e5b9ULL;
    x ^= x >> 27; x *= 0x94d049bb133111ebULL;
    x ^= x >> 31;
    return x;
}

static int64_t or_lookup(const or_tree* tr, uint64_t key)
{
    uint64_t h = or_mix(key) & tr->mask;
    for (;;) {
        if (tr->keys[h] == key) return tr->vals[h];
        if (tr->keys[h] == 0) return -1;
        h = (h + 1) & tr->mask;
    }
}

/* insert; returns 0 ok, 1 duplicate */
static int or_insert(or_tree* tr, uint64_t key, int64_t val)
{
    uint64_t h = or_mix(key) & tr->mask;
    for (;;) {
        if (tr->keys[h] == key) return 1;
        if (tr->keys[h] == 0) { tr->keys[h] = key; tr->vals[h] = val; return 0; }
        h = (h + 1) & tr->mask;
    }
}

void or_tree_free(or_tree* tr)
{
    if (!tr) return;
    free(tr->keys);
    free(tr->vals);
    free(tr);
}

/* Error codes: 0 ok, 1 bad depth, 2 coordinate out of range, 3 duplicate,
 * 4 a leaf lies inside another leaf, 5 out of memory. */
or_tree* or_tree_build(const int32_t* dijk, int64_t n, int32_t max_depth, int32_t* err)
{
    *err = 0;
    if (max_depth < 1 || max_depth > 16) { *err = 1; return NULL; }
    uint64_t cap = 16;
    while (cap < (uint64_t)(2 * n + 16)) cap <<= 1;
    or_tree* tr = (or_tree*)calloc(1, sizeof(or_tree));
    if (!tr) { *err = 5; return NULL; }
    tr->max_depth = max_depth;
    tr->n_leaves = n;
    tr->mask = cap - 1;
    tr->keys = (uint64_t*)calloc(cap, sizeof(uint64_t));
    tr->vals = (int64_t*)calloc(cap, sizeof(int64_t));
    if (!tr->keys || !tr->vals) { or_tree_free(tr); *err = 5; return NULL; }
    for (int64_t l = 0; l < n; ++l) {
        const int32_t d = dijk[4 * l], i = dijk[4 * l + 1], j = dijk[4 * l + 2], k = dijk[4 * l + 3];
        if (d < 1 || d > max_depth) { *err = 1; or_tree_free(tr); return NULL; }
        const int64_t g = (int64_t)1 << d;
        if (i < 0 || j < 0 || k < 0 || i >= g || j >= g || k >= g) { *err = 2; or_tree_free(tr); return NULL; }
        if (or_insert(tr, or_key(d, i, j, k), l)) { *err = 3; or_tree_free(tr); return NULL; }
    }
    /* no leaf may have a leaf among its ancestors */
    for (int64_t l = 0; l < n; ++l) {
        const int32_t d = dijk[4 * l], i = dijk[4 * l + 1], j = dijk[4 * l + 2], k = dijk[4 * l + 3];
        for (int32_t a = 1; a < d; ++a) {
            const int sh = d - a;
            if (or_lookup(tr, or_key(a, i >> sh, j >> sh, k >> sh)) >= 0) { *err = 4; or_tree_free(tr); return NULL; }
        }
    }
    return tr;
}

/* Leaf containing the finest-lattice cell (x, y, z), or -1 if the cell is empty. */
int64_t or_tree_locate(const or_tree* tr, int64_t x, int64_t y, int64_t z)
{
    for (int32_t d = 1; d <= tr->max_depth; ++d) {
        const int sh = tr->max_depth - d;
        const int64_t l = or_lookup(tr, or_key(d, x >> sh, y >> sh, z >> sh));
        if (l >= 0) return l;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Ray / unit-cube slab test.  Returns 0 if the ray misses; else t_in, t_out  */
/* with t_in >= 0.  d need not be normalised.                                */
/* ------------------------------------------------------------------------ */
static int or_slab(const double o[3], const double d[3], double* t_in, double* t_out)
{
    double lo = 0.0, hi = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < 0.0 || o[a] > 1.0) return 0;
            continue;
        }
        double t1 = (0.0 - o[a]) / d[a];
        double t2 = (1.0 - o[a]) / d[a];
        if (t1 > t2) { double s = t1; t1 = t2; t2 = s; }
        if (t1 > lo) lo = t1;
        if (t2 < hi) hi = t2;
    }
    if (!(lo < hi)) return 0;
    *t_in = lo;
    *t_out = hi;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Segment list of a ray: a 3D-DDA over the finest lattice (Amanatides and   */
/* Woo 1987) with axis tie-break x < y < z, consecutive cells of the same    */
/* leaf merged, segments of zero length dropped.  d must be unit length.     */
/* Returns the number of segments; writes at most cap of them.               */
/* ------------------------------------------------------------------------ */
int64_t or_trace(const or_tree* tr, const double o[3], const double d[3], int64_t cap,
                 int64_t* leaf, double* t0, double* t1)
{
    double t_in, t_out;
    if (!or_slab(o, d, &t_in, &t_out)) return 0;
    const int64_t G = (int64_t)1 << tr->max_depth;
    int64_t c[3];
    int step[3];
    for (int a = 0; a < 3; ++a) {
        double p = o[a] + t_in * d[a];
        int64_t ci = (int64_t)floor(p * (double)G);
        if (ci < 0) ci = 0;
        if (ci > G - 1) ci = G - 1;
        c[a] = ci;
        step[a] = d[a] > 0.0 ? 1 : (d[a] < 0.0 ? -1 : 0);
    }
    int64_t count = 0;
    int64_t cur_leaf = -1;
    double cur_t0 = 0.0, cur_t1 = 0.0;
    double t_cur = t_in;
    for (;;) {
        double tn[3];
        for (int a = 0; a < 3; ++a) {
            if (step[a] == 0) { tn[a] = INFINITY; continue; }
            const int64_t plane = c[a] + (step[a] > 0 ? 1 : 0);
            tn[a] = ((double)plane / (double)G - o[a]) / d[a];
        }
        int ax = 0;
        if (tn[1] < tn[ax]) ax = 1;
        if (tn[2] < tn[ax]) ax = 2;
        double t_exit = tn[ax] < t_out ? tn[ax] : t_out;
        if (t_exit < t_cur) t_exit = t_cur;
        const int64_t l = or_tree_locate(tr, c[0], c[1], c[2]);
        if (l >= 0 && l == cur_leaf && cur_t1 == t_cur) {
            cur_t1 = t_exit;              /* same leaf continues */
        } else {
            if (cur_leaf >= 0 && cur_t1 > cur_t0) {
                if (count < cap) { leaf[count] = cur_leaf; t0[count] = cur_t0; t1[count] = cur_t1; }
                ++count;
            }
            cur_leaf = l;
            cur_t0 = t_cur;
            cur_t1 = t_exit;
        }
        if (tn[ax] >= t_out) break;
        c[ax] += step[ax];
        if (c[ax] < 0 || c[ax] >= G) break;
        t_cur = t_exit;
    }
    if (cur_leaf >= 0 && cur_t1 > cur_t0) {
        if (count < cap) { leaf[count] = cur_leaf; t0[count] = cur_t0; t1[count] = cur_t1; }
        ++count;
    }
    return count;
}

/* ------------------------------------------------------------------------ */
/* Rendering.                                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_sigma;       /* n1 */
    int32_t n_sh_fourier;  /* n2 */
    double period;         /* T */
    double sigma_scale;    /* s */
    double stop_T;         /* tau; 0 disables early termination */
    double band;           /* relative band around tau inside which both outcomes are kept */
    double bg[3];
} or_params;

static int32_t or_ncoeff(const or_params* p)
{
    return p->n_sigma + 3 * OR_N_SH * p->n_sh_fourier;
}

/* Density (pre-activation) and the 3 x 9 SH coefficients of one leaf at time
 * t: Eq. 7 and Eq. 9, or the stored snapshot values when `snap` is set. */
static void or_leaf_values(const or_params* p, const double* k, const double* b,
                           const double* snap, int64_t leaf, int64_t n_leaves,
                           double* sigma_raw, double z[27])
{
    if (snap) {
        *sigma_raw = snap[leaf];
        for (int q = 0; q < 27; ++q) z[q] = snap[(int64_t)(q + 1) * n_leaves + leaf];
        return;
    }
    double s = 0.0;
    for (int32_t i = 0; i < p->n_sigma; ++i) s += k[i] * b[i];
    *sigma_raw = s;
    for (int q = 0; q < 27; ++q) {
        const double* kz = k + p->n_sigma + q * p->n_sh_fourier;
        double v = 0.0;
        for (int32_t i = 0; i < p->n_sh_fourier; ++i) v += kz[i] * b[i];
        z[q] = v;
    }
}

typedef struct {
    double rgb[2][3];   /* [0]: earliest admissible stop, [1]: latest */
    double T[2];
    int64_t n_seg[2];   /* composited segments */
    int64_t n_opaque[2];/* composited segments with sigma_eff * delta > 0 */
    int64_t n_cells;    /* all segments the ray crosses (no early stop) */
} or_ray_result;

/* Render one ray.  coeffs: [L][ncoeff] caller order; snap (optional):
 * [28][L] baked values.  Two early-termination outcomes are produced: one
 * with threshold tau (1 + band), one with tau (1 - band); they agree unless
 * the FP64 transmittance straddles tau within the band. */
static void or_render_one(const or_tree* tr, const double* coeffs, const double* snap,
                          const or_params* p, const double* b,
                          const double o[3], const double d_in[3],
                          int64_t* seg_leaf, double* seg_t0, double* seg_t1, int64_t seg_cap,
                          or_ray_result* res)
{
    double d[3] = {d_in[0], d_in[1], d_in[2]};
    or_normalize(d);
    const int64_t n = or_trace(tr, o, d, seg_cap, seg_leaf, seg_t0, seg_t1);
    double Y[9];
    or_sh9(d, Y);
    const int32_t nc = or_ncoeff(p);
    res->n_cells = n;
    for (int v = 0; v < 2; ++v) {
        const double thr = p->stop_T > 0.0 ? p->stop_T * (v == 0 ? 1.0 + p->band : 1.0 - p->band) : 0.0;
        double T = 1.0, C[3] = {0.0, 0.0, 0.0};
        int64_t used = 0, opaque = 0;
        for (int64_t s = 0; s < n && s < seg_cap; ++s) {
            const int64_t l = seg_leaf[s];
            double sraw, z[27];
            or_leaf_values(p, coeffs + l * nc, b, snap, l, tr->n_leaves, &sraw, z);
            const double sigma = p->sigma_scale * (sraw > 0.0 ? sraw : 0.0);
            const double delta = seg_t1[s] - seg_t0[s];
            const double alpha = -expm1(-sigma * delta);
            for (int c = 0; c < 3; ++c) {
                double h = 0.0;
                for (int j = 0; j < 9; ++j) h += z[c * 9 + j] * Y[j];
                const double rgb = 1.0 / (1.0 + exp(-h));
                C[c] += T * alpha * rgb;
            }
            T *= exp(-sigma * delta);
            ++used;
            if (sigma * delta > 0.0) ++opaque;
            if (thr > 0.0 && T < thr) break;
        }
        for (int c = 0; c < 3; ++c) res->rgb[v][c] = C[c] + T * p->bg[c];
        res->T[v] = T;
        res->n_seg[v] = used;
        res->n_opaque[v] = opaque;
    }
}

typedef struct {
    const or_tree* tr;
    const double* coeffs;
    const double* snap;
    const or_params* p;
    const double* basis;    /* [n_t][n_max] */
    int32_t n_bmax;
    const double* o;
    const double* d;
    const int32_t* t_idx;
    int64_t n;
    double* rgb;            /* [n][2][3] */
    double* T;              /* [n][2] */
    int64_t* n_seg;         /* [n][2] */
    int64_t* n_opaque;      /* [n][2] */
    int64_t* n_cells;       /* [n] */
    int64_t begin, end;
    int32_t status;
} or_job;

static void* or_render_worker(void* arg)
{
    or_job* job = (or_job*)arg;
    const int64_t cap = 3 * ((int64_t)1 << job->tr->max_depth) + 8;
    int64_t* sl = (int64_t*)malloc(sizeof(int64_t) * cap);
    double* s0 = (double*)malloc(sizeof(double) * cap);
    double* s1 = (double*)malloc(sizeof(double) * cap);
    if (!sl || !s0 || !s1) { job->status = 5; free(sl); free(s0); free(s1); return NULL; }
    for (int64_t r = job->begin; r < job->end; ++r) {
        or_ray_result res;
        const double* b = job->basis + (int64_t)job->t_idx[r] * job->n_bmax;
        or_render_one(job->tr, job->coeffs, job->snap, job->p, b, job->o + 3 * r, job->d + 3 * r,
                      sl, s0, s1, cap, &res);
        for (int v = 0; v < 2; ++v) {
            for (int c = 0; c < 3; ++c) job->rgb[r * 6 + v * 3 + c] = res.rgb[v][c];
            job->T[r * 2 + v] = res.T[v];
            job->n_seg[r * 2 + v] = res.n_seg[v];
            job->n_opaque[r * 2 + v] = res.n_opaque[v];
        }
        job->n_cells[r] = res.n_cells;
    }
    free(sl); free(s0); free(s1);
    return NULL;
}

/* Render n rays.  times: [n_t]; t_idx: [n] index into times.  coeffs may be
 * NULL when snap ([28][L]) is given.  Outputs: rgb [n][2][3], T [n][2],
 * n_seg [n][2], n_opaque [n][2], n_cells [n].  Returns 0 on success. */
int32_t or_render_rays(const or_tree* tr, const double* coeffs, const double* snap,
                       const or_params* p, const double* times, int32_t n_t,
                       const double* o, const double* d, const int32_t* t_idx, int64_t n,
                       int32_t n_threads, double* rgb, double* T, int64_t* n_seg, int64_t* n_opaque,
                       int64_t* n_cells)
{
    const int32_t nb = p->n_sigma > p->n_sh_fourier ? p->n_sigma : p->n_sh_fourier;
    double* basis = (double*)malloc(sizeof(double) * (size_t)(n_t > 0 ? n_t : 1) * nb);
    if (!basis) return 5;
    for (int32_t t = 0; t < n_t; ++t) or_basis(times[t], p->period, nb, basis + (int64_t)t * nb);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    if ((int64_t)n_threads > n) n_threads = (int32_t)(n > 0 ? n : 1);
    pthread_t th[256];
    or_job jobs[256];
    int32_t status = 0;
    for (int32_t w = 0; w < n_threads; ++w) {
        or_job* j = &jobs[w];
        j->tr = tr; j->coeffs = coeffs; j->snap = snap; j->p = p; j->basis = basis; j->n_bmax = nb;
        j->o = o; j->d = d; j->t_idx = t_idx; j->n = n;
        j->rgb = rgb; j->T = T; j->n_seg = n_seg; j->n_opaque = n_opaque; j->n_cells = n_cells;
        j->begin = n * w / n_threads;
        j->end = n * (w + 1) / n_threads;
        j->status = 0;
    }
    for (int32_t w = 1; w < n_threads; ++w) pthread_create(&th[w], NULL, or_render_worker, &jobs[w]);
    or_render_worker(&jobs[0]);
    for (int32_t w = 1; w < n_threads; ++w) pthread_join(th[w], NULL);
    for (int32_t w = 0; w < n_threads; ++w) if (jobs[w].status) status = jobs[w].status;
    free(basis);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Gradient of the loss w.r.t. the leaf coefficients (Eq. 13 fine-tuning).    */
/* The analytic reverse of the per-ray compositing above, FP64, with the     */
/* nominal early-termination rule (threshold tau).  grad_rgb: [n][3] = dL/dC */
/* per ray.  grad: [L][ncoeff] caller order, accumulated (+=).               */
/* Also writes the forward colour rgb [n][3].                                */
/* Threads take contiguous ranges of rays and list each composited segment's */
/* ncoeff derivatives; the lists are added into grad in ray order, so the    */
/* sums are formed in the same order for any thread count.                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    const or_tree* tr;
    const double* coeffs;
    const or_params* p;
    const double* basis;     /* [n_t][nb] */
    int32_t nb;
    const double* o;
    const double* d_in;
    const int32_t* t_idx;
    const double* grad_rgb;
    double* rgb_out;
    int64_t begin, end;
    int64_t* leaves;         /* one per listed segment */
    double* vals;            /* ncoeff per listed segment */
    int64_t n_list, cap_list;
    int32_t status;
} or_grad_job;

static int or_grad_push(or_grad_job* job, int64_t leaf, int32_t nc, double** row)
{
    if (job->n_list == job->cap_list) {
        const int64_t cap = job->cap_list ? 2 * job->cap_list : 1024;
        int64_t* l = (int64_t*)realloc(job->leaves, sizeof(int64_t) * cap);
        if (!l) return 5;
        job->leaves = l;
        double* v = (double*)realloc(job->vals, sizeof(double) * cap * nc);
        if (!v) return 5;
        job->vals = v;
        job->cap_list = cap;
    }
    job->leaves[job->n_list] = leaf;
    *row = job->vals + job->n_list * nc;
    for (int32_t q = 0; q < nc; ++q) (*row)[q] = 0.0;
    ++job->n_list;
    return 0;
}

static void* or_grad_worker(void* arg)
{
    or_grad_job* job = (or_grad_job*)arg;
    const or_tree* tr = job->tr;
    const or_params* p = job->p;
    const int32_t nc = or_ncoeff(p);
    const int64_t cap = 3 * ((int64_t)1 << tr->max_depth) + 8;
    int64_t* sl = (int64_t*)malloc(sizeof(int64_t) * cap);
    double* s0 = (double*)malloc(sizeof(double) * cap);
    double* s1 = (double*)malloc(sizeof(double) * cap);
    /* per segment: sigma_raw, sigma, delta, T_before, alpha, rgb[3] */
    double* st = (double*)malloc(sizeof(double) * cap * 8);
    if (!sl || !s0 || !s1 || !st) { job->status = 5; free(sl); free(s0); free(s1); free(st); return NULL; }
    for (int64_t r = job->begin; r < job->end; ++r) {
        const double* b = job->basis + (int64_t)job->t_idx[r] * job->nb;
        double d[3] = {job->d_in[3 * r], job->d_in[3 * r + 1], job->d_in[3 * r + 2]};
        or_normalize(d);
        const int64_t nseg = or_trace(tr, job->o + 3 * r, d, cap, sl, s0, s1);
        double Y[9];
        or_sh9(d, Y);
        double T = 1.0, C[3] = {0.0, 0.0, 0.0};
        int64_t used = 0;
        for (int64_t s = 0; s < nseg; ++s) {
            const int64_t l = sl[s];
            double sraw, z[27];
            or_leaf_values(p, job->coeffs + l * nc, b, NULL, l, tr->n_leaves, &sraw, z);
            const double sigma = p->sigma_scale * (sraw > 0.0 ? sraw : 0.0);
            const double delta = s1[s] - s0[s];
            const double alpha = -expm1(-sigma * delta);
            double* e = st + 8 * s;
            e[0] = sraw; e[1] = sigma; e[2] = delta; e[3] = T; e[4] = alpha;
            for (int c = 0; c < 3; ++c) {
                double h = 0.0;
                for (int j = 0; j < 9; ++j) h += z[c * 9 + j] * Y[j];
                e[5 + c] = 1.0 / (1.0 + exp(-h));
                C[c] += T * alpha * e[5 + c];
            }
            T *= exp(-sigma * delta);
            ++used;
            if (p->stop_T > 0.0 && T < p->stop_T) break;
        }
        double Cf[3];
        for (int c = 0; c < 3; ++c) Cf[c] = C[c] + T * p->bg[c];
        if (job->rgb_out) for (int c = 0; c < 3; ++c) job->rgb_out[3 * r + c] = Cf[c];
        const double* g = job->grad_rgb + 3 * r;
        /* R_i = C_final - sum_{j<=i} T_j alpha_j c_j */
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t s = 0; s < used; ++s) {
            const double* e = st + 8 * s;
            const double Tb = e[3], alpha = e[4], sigma_delta = e[1] * e[2];
            const double T_after = Tb * exp(-sigma_delta);
            double dsig = 0.0;
            double dh[3];
            for (int c = 0; c < 3; ++c) {
                acc[c] += Tb * alpha * e[5 + c];
                const double R = Cf[c] - acc[c];
                dsig += g[c] * e[2] * (T_after * e[5 + c] - R);
                const double dc = g[c] * Tb * alpha;
                dh[c] = dc * e[5 + c] * (1.0 - e[5 + c]);
            }
            double* gl;
            if ((job->status = or_grad_push(job, sl[s], nc, &gl)) != 0) break;
            if (e[0] > 0.0) {
                const double ds_raw = dsig * p->sigma_scale;
                for (int32_t i = 0; i < p->n_sigma; ++i) gl[i] = ds_raw * b[i];
            }
            for (int c = 0; c < 3; ++c)
                for (int j = 0; j < 9; ++j) {
                    const double dz = dh[c] * Y[j];
                    double* gz = gl + p->n_sigma + (c * 9 + j) * p->n_sh_fourier;
                    for (int32_t i = 0; i < p->n_sh_fourier; ++i) gz[i] = dz * b[i];
                }
        }
        if (job->status) break;
    }
    free(sl); free(s0); free(s1); free(st);
    return NULL;
}

int32_t or_render_grad(const or_tree* tr, const double* coeffs, const or_params* p,
                       const double* times, int32_t n_t,
                       const double* o, const double* d_in, const int32_t* t_idx, int64_t n,
                       const double* grad_rgb, int32_t n_threads, double* grad, double* rgb_out)
{
    const int32_t nc = or_ncoeff(p);
    const int32_t nb = p->n_sigma > p->n_sh_fourier ? p->n_sigma : p->n_sh_fourier;
    double* basis = (double*)malloc(sizeof(double) * (size_t)(n_t > 0 ? n_t : 1) * nb);
    if (!basis) return 5;
    for (int32_t t = 0; t < n_t; ++t) or_basis(times[t], p->period, nb, basis + (int64_t)t * nb);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    pthread_t th[256];
    or_grad_job jobs[256];
    memset(jobs, 0, sizeof(jobs));
    int32_t status = 0;
    /* rays in chunks, so that the segment lists stay small */
    const int64_t chunk = (int64_t)n_threads * 2048;
    for (int64_t c0 = 0; c0 < n && status == 0; c0 += chunk) {
        const int64_t m = n - c0 < chunk ? n - c0 : chunk;
        for (int32_t w = 0; w < n_threads; ++w) {
            or_grad_job* j = &jobs[w];
            j->tr = tr; j->coeffs = coeffs; j->p = p; j->basis = basis; j->nb = nb;
            j->o = o; j->d_in = d_in; j->t_idx = t_idx; j->grad_rgb = grad_rgb; j->rgb_out = rgb_out;
            j->begin = c0 + m * w / n_threads;
            j->end = c0 + m * (w + 1) / n_threads;
            j->n_list = 0;
            j->status = 0;
        }
        for (int32_t w = 1; w < n_threads; ++w) pthread_create(&th[w], NULL, or_grad_worker, &jobs[w]);
        or_grad_worker(&jobs[0]);
        for (int32_t w = 1; w < n_threads; ++w) pthread_join(th[w], NULL);
        for (int32_t w = 0; w < n_threads; ++w) {
            if (jobs[w].status) { status = jobs[w].status; break; }
            for (int64_t e = 0; e < jobs[w].n_list; ++e) {
                double* gl = grad + jobs[w].leaves[e] * nc;
                const double* v = jobs[w].vals + e * nc;
                for (int32_t q = 0; q < nc; ++q) gl[q] += v[q];
            }
        }
    }
    for (int32_t w = 0; w < n_threads; ++w) { free(jobs[w].leaves); free(jobs[w].vals); }
    free(basis);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Time bake: Eq. 7 and Eq. 9 evaluated at n_t times for every leaf.         */
/* out: [n_t][28][L]; row 0 = sigma(t) (before activation), row 1 + c*9 + j  */
/* = z_{c,j}(t).  coeffs: [L][ncoeff].                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    const double* coeffs;
    int64_t n_leaves;
    const or_params* p;
    const double* times;
    int32_t n_t;
    double* out;
    int64_t begin, end;      /* leaf range of this thread */
} or_bake_job;

static void* or_bake_worker(void* arg)
{
    const or_bake_job* job = (const or_bake_job*)arg;
    const or_params* p = job->p;
    const int32_t nc = or_ncoeff(p);
    const int64_t L = job->n_leaves;
    double b[OR_MAX_COEFF];
    const int32_t nb = p->n_sigma > p->n_sh_fourier ? p->n_sigma : p->n_sh_fourier;
    for (int32_t t = 0; t < job->n_t; ++t) {
        or_basis(job->times[t], p->period, nb, b);
        double* o = job->out + (int64_t)t * 28 * L;
        for (int64_t l = job->begin; l < job->end; ++l) {
            double sraw, z[27];
            or_leaf_values(p, job->coeffs + l * nc, b, NULL, l, L, &sraw, z);
            o[l] = sraw;
            for (int q = 0; q < 27; ++q) o[(int64_t)(q + 1) * L + l] = z[q];
        }
    }
    return NULL;
}

/* Leaves are independent: threads take contiguous leaf ranges. */
void or_bake(const double* coeffs, int64_t n_leaves, const or_params* p,
             const double* times, int32_t n_t, int32_t n_threads, double* out)
{
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    if ((int64_t)n_threads > n_leaves) n_threads = (int32_t)(n_leaves > 0 ? n_leaves : 1);
    pthread_t th[256];
    or_bake_job jobs[256];
    for (int32_t w = 0; w < n_threads; ++w) {
        or_bake_job* j = &jobs[w];
        j->coeffs = coeffs; j->n_leaves = n_leaves; j->p = p; j->times = times; j->n_t = n_t; j->out = out;
        j->begin = n_leaves * w / n_threads;
        j->end = n_leaves * (w + 1) / n_threads;
    }
    for (int32_t w = 1; w < n_threads; ++w) pthread_create(&th[w], NULL, or_bake_worker, &jobs[w]);
    or_bake_worker(&jobs[0]);
    for (int32_t w = 1; w < n_threads; ++w) pthread_join(th[w], NULL);
}

/* ------------------------------------------------------------------------ */
/* Proposal labels: hit = some composited segment has sigma_eff delta > 0;   */
/* s_in / s_out = where the first such segment starts / the last composited  */
/* such segment ends, as fractions of the ray's chord [t_in, t_out] through  */
/* the unit cube.  Early termination uses the nominal threshold tau.         */
/* labels: [n][3] (hit, s_in, s_out); s_in = s_out = 0 when there is no hit. */
/* ------------------------------------------------------------------------ */
int32_t or_ray_labels(const or_tree* tr, const double* coeffs, const or_params* p,
                      const double* times, int32_t n_t, const double* o, const double* d_in,
                      const int32_t* t_idx, int64_t n, double* labels)
{
    const int32_t nc = or_ncoeff(p);
    const int32_t nb = p->n_sigma > p->n_sh_fourier ? p->n_sigma : p->n_sh_fourier;
    const int64_t cap = 3 * ((int64_t)1 << tr->max_depth) + 8;
    int64_t* sl = (int64_t*)malloc(sizeof(int64_t) * cap);
    double* s0 = (double*)malloc(sizeof(double) * cap);
    double* s1 = (double*)malloc(sizeof(double) * cap);
    double* basis = (double*)malloc(sizeof(double) * (size_t)(n_t > 0 ? n_t : 1) * nb);
    if (!sl || !s0 || !s1 || !basis) { free(sl); free(s0); free(s1); free(basis); return 5; }
    for (int32_t t = 0; t < n_t; ++t) or_basis(times[t], p->period, nb, basis + (int64_t)t * nb);
    for (int64_t r = 0; r < n; ++r) {
        double d[3] = {d_in[3 * r], d_in[3 * r + 1], d_in[3 * r + 2]};
        or_normalize(d);
        double* lab = labels + 3 * r;
        lab[0] = lab[1] = lab[2] = 0.0;
        double t_in, t_out;
        if (!or_slab(o + 3 * r, d, &t_in, &t_out)) continue;
        const double* b = basis + (int64_t)t_idx[r] * nb;
        const int64_t nseg = or_trace(tr, o + 3 * r, d, cap, sl, s0, s1);
        double T = 1.0;
        int hit = 0;
        double first = 0.0, last = 0.0;
        for (int64_t s = 0; s < nseg; ++s) {
            double sraw, z[27];
            or_leaf_values(p, coeffs + sl[s] * nc, b, NULL, sl[s], tr->n_leaves, &sraw, z);
            const double sigma = p->sigma_scale * (sraw > 0.0 ? sraw : 0.0);
            const double delta = s1[s] - s0[s];
            if (sigma * delta > 0.0) {
                if (!hit) first = s0[s];
                hit = 1;
                last = s1[s];
            }
            T *= exp(-sigma * delta);
            if (p->stop_T > 0.0 && T < p->stop_T) break;
        }
        if (hit) {
            const double len = t_out - t_in;
            lab[0] = 1.0;
            lab[1] = (first - t_in) / len;
            lab[2] = (last - t_in) / len;
        }
    }
    free(sl); free(s0); free(s1); free(basis);
    return 0;
}
