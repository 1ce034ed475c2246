// Driver for the ASan/UBSan build of libfpo's host code (fpo_host.cpp) and the
// FP64 oracle (fpo_oracle.c), built with the host compilers only: no device
// code is involved.  It exercises every host entry point and every oracle
// function on random mixed-depth trees, including their error paths and the
// oracle's threaded loops, and cross-checks the two point locations.  Exit
// status 0 and no sanitizer report is a pass.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "fpo.h"

extern "C" {
typedef struct {
    double eye[3], fwd[3], up[3];
    double fov_y_deg;
    int32_t width, height;
    double time;
} or_camera;
typedef struct {
    int32_t n_sigma, n_sh_fourier;
    double period, sigma_scale, stop_T, band;
    double bg[3];
} or_params;
struct or_tree;
void or_basis(double t, double period, int32_t n, double* out);
void or_sh9(const double dir[3], double out[9]);
void or_camera_rays(const or_camera* cam, int64_t n, const int32_t* px, const int32_t* py, double* o, double* d);
or_tree* or_tree_build(const int32_t* dijk, int64_t n, int32_t max_depth, int32_t* err);
void or_tree_free(or_tree* tr);
int64_t or_tree_locate(const or_tree* tr, int64_t x, int64_t y, int64_t z);
int64_t or_trace(const or_tree* tr, const double o[3], const double d[3], int64_t cap, int64_t* leaf, double* t0,
                 double* t1);
int32_t or_render_rays(const or_tree* tr, const double* coeffs, const double* snap, const or_params* p,
                       const double* times, int32_t n_t, const double* o, const double* d, const int32_t* t_idx,
                       int64_t n, int32_t n_threads, double* rgb, double* T, int64_t* n_seg, int64_t* n_opaque,
                       int64_t* n_cells);
int32_t or_render_grad(const or_tree* tr, const double* coeffs, const or_params* p, const double* times,
                       int32_t n_t, const double* o, const double* d_in, const int32_t* t_idx, int64_t n,
                       const double* grad_rgb, int32_t n_threads, double* grad, double* rgb_out);
void or_bake(const double* coeffs, int64_t n_leaves, const or_params* p, const double* times, int32_t n_t,
             int32_t n_threads, double* out);
int32_t or_ray_labels(const or_tree* tr, const double* coeffs, const or_params* p, const double* times,
                      int32_t n_t, const double* o, const double* d_in, const int32_t* t_idx, int64_t n,
                      double* labels);
}

static uint64_t g_state = 0x2202086142022ull;
static double urand()
{
    g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}

#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            std::exit(1);                                                        \
        }                                                                        \
    } while (0)

// Random mixed-depth partition: split cells with probability p_split.
static void subdivide(int d, int i, int j, int k, int max_depth, double p_split, std::vector<int32_t>& out)
{
    if (d > 0 && (d == max_depth || urand() > p_split)) {
        if (urand() < 0.7) {
            out.push_back(d); out.push_back(i); out.push_back(j); out.push_back(k);
        }
        return;
    }
    for (int c = 0; c < 8; ++c)
        subdivide(d + 1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + ((c >> 2) & 1), max_depth, p_split, out);
}

static int64_t descend(const std::vector<int32_t>& ch, int D, int x, int y, int z)
{
    int64_t node = 0;
    for (int lvl = 0; lvl < D; ++lvl) {
        const int sh = D - 1 - lvl;
        const int oct = ((x >> sh) & 1) | (((y >> sh) & 1) << 1) | (((z >> sh) & 1) << 2);
        const int32_t c = ch[node * 8 + oct];
        if (c > 0) { node = c; continue; }
        return c < 0 ? -(int64_t)c - 1 : -1;
    }
    return -2;
}

int main()
{
    const int D = 6;
    for (int trial = 0; trial < 3; ++trial) {
        std::vector<int32_t> dijk;
        subdivide(0, 0, 0, 0, D, 0.55, dijk);
        const int64_t L = (int64_t)dijk.size() / 4;
        CHECK(L > 10);
        // tree build: size query, too small a capacity, build
        int64_t n_nodes = 0;
        CHECK(fpo_build_tree(dijk.data(), L, D, nullptr, 0, &n_nodes, nullptr) == FPO_OK && n_nodes > 0);
        std::vector<int32_t> ch((size_t)n_nodes * 8);
        std::vector<int64_t> perm((size_t)L);
        int64_t n2 = 0;
        CHECK(fpo_build_tree(dijk.data(), L, D, ch.data(), n_nodes - 1, &n2, perm.data()) == FPO_E_CAPACITY);
        CHECK(fpo_build_tree(dijk.data(), L, D, ch.data(), n_nodes, &n2, perm.data()) == FPO_OK && n2 == n_nodes);
        // point location agrees with the oracle's hash on every finest cell
        int32_t err = 0;
        or_tree* ot = or_tree_build(dijk.data(), L, D, &err);
        CHECK(ot && err == 0);
        const int G = 1 << D;
        for (int x = 0; x < G; x += 3)
            for (int y = 0; y < G; y += 2)
                for (int z = 0; z < G; ++z) {
                    const int64_t slot = descend(ch, D, x, y, z);
                    const int64_t want = or_tree_locate(ot, x, y, z);
                    CHECK((slot < 0 && want < 0) || (slot >= 0 && want >= 0 && perm[(size_t)slot] == want));
                }
        // error paths
        std::vector<int32_t> dup(dijk.begin(), dijk.begin() + 8);
        dup[4] = dup[0]; dup[5] = dup[1]; dup[6] = dup[2]; dup[7] = dup[3];
        CHECK(fpo_build_tree(dup.data(), 2, D, nullptr, 0, &n2, nullptr) == FPO_E_INVALID);
        CHECK(std::strlen(fpo_last_error()) > 0);
        int32_t bad[4] = {2, 4, 0, 0};
        CHECK(fpo_build_tree(bad, 1, D, nullptr, 0, &n2, nullptr) == FPO_E_INVALID);
        int32_t nested[8] = {1, 0, 0, 0, 2, 0, 0, 0};
        CHECK(fpo_build_tree(nested, 2, D, nullptr, 0, &n2, nullptr) == FPO_E_INVALID);
        CHECK(fpo_build_tree(dijk.data(), L, 11, nullptr, 0, &n2, nullptr) == FPO_E_INVALID);
        // union of two "frames" (this tree and a coarser copy of half of it), pruning, occupancy
        std::vector<int32_t> cells(dijk);
        for (int64_t l = 0; l < L; l += 2)
            if (dijk[4 * l] > 1) {
                cells.push_back(dijk[4 * l] - 1);
                cells.push_back(dijk[4 * l + 1] >> 1);
                cells.push_back(dijk[4 * l + 2] >> 1);
                cells.push_back(dijk[4 * l + 3] >> 1);
            }
        int64_t n_union = 0;
        CHECK(fpo_union_leaves(cells.data(), (int64_t)cells.size() / 4, D, nullptr, 0, &n_union) == FPO_OK);
        std::vector<int32_t> un((size_t)n_union * 4);
        CHECK(fpo_union_leaves(cells.data(), (int64_t)cells.size() / 4, D, un.data(), n_union, &n_union) == FPO_OK);
        std::vector<float> smax((size_t)n_union);
        for (auto& v : smax) v = (float)(urand() * 2e-3);
        std::vector<int64_t> keep((size_t)n_union);
        int64_t n_keep = 0;
        CHECK(fpo_prune_leaves(smax.data(), n_union, 1e-3f, keep.data(), &n_keep) == FPO_OK);
        CHECK(n_keep > 0 && n_keep < n_union);
        std::vector<uint32_t> bits(FPO_COARSE_WORDS);
        CHECK(fpo_coarse_occupancy(dijk.data(), L, D, bits.data()) == FPO_OK);
        // basis and cameras
        fpo_layout lay = {FPO_N_SIGMA, FPO_N_SH_FOURIER, FPO_SH_DEGREE, 60.0f, 64.0f};
        double times[3] = {0.0, 22.2, -7.5};
        std::vector<float> basis(3 * FPO_BASIS_STRIDE);
        CHECK(fpo_time_basis(times, 3, &lay, basis.data()) == FPO_OK);
        double ref[FPO_N_SIGMA];
        or_basis(22.2, 60.0, FPO_N_SIGMA, ref);
        for (int i = 0; i < FPO_N_SIGMA; ++i) CHECK(std::fabs(basis[FPO_BASIS_STRIDE + i] - ref[i]) < 1e-6);
        fpo_camera cam = {{1.5f, 0.6f, 0.4f}, {-1.0f, -0.1f, 0.1f}, {0.0f, 1.0f, 0.0f}, 40.0f, 17, 11, 3.0};
        std::vector<float> table(FPO_CAMERA_FLOATS);
        CHECK(fpo_camera_pack(&cam, 1, table.data()) == FPO_OK);
        // oracle: rays, traces, renders (threaded), gradient (threaded), bake (threaded), labels
        or_camera oc = {{1.5, 0.6, 0.4}, {-1.0, -0.1, 0.1}, {0.0, 1.0, 0.0}, 40.0, 17, 11, 3.0};
        const int64_t n = 17 * 11;
        std::vector<int32_t> px(n), py(n), t_idx(n);
        for (int64_t r = 0; r < n; ++r) { px[r] = (int32_t)(r % 17); py[r] = (int32_t)(r / 17); t_idx[r] = (int32_t)(r % 3); }
        std::vector<double> o(3 * n), d(3 * n);
        or_camera_rays(&oc, n, px.data(), py.data(), o.data(), d.data());
        const int64_t cap = 3 * ((int64_t)1 << D) + 8;
        std::vector<int64_t> lf(cap);
        std::vector<double> t0(cap), t1(cap);
        for (int64_t r = 0; r < n; ++r) {
            const int64_t m = or_trace(ot, &o[3 * r], &d[3 * r], cap, lf.data(), t0.data(), t1.data());
            CHECK(m >= 0 && m <= cap);
            for (int64_t s = 1; s < m; ++s) CHECK(t0[s] >= t1[s - 1] - 1e-12);
        }
        const int nc = 166;
        std::vector<double> k((size_t)L * nc);
        for (auto& v : k) v = urand() - 0.45;
        or_params p = {31, 5, 60.0, 16.0, 1e-2, 1e-3, {0.1, 0.2, 0.3}};
        std::vector<double> rgb(6 * n), T(2 * n), rgb1(3 * n), g(3 * n), grad((size_t)L * nc), lab(3 * n);
        std::vector<int64_t> nseg(2 * n), nopq(2 * n), ncell(n);
        CHECK(or_render_rays(ot, k.data(), nullptr, &p, times, 3, o.data(), d.data(), t_idx.data(), n, 4, rgb.data(),
                             T.data(), nseg.data(), nopq.data(), ncell.data()) == 0);
        for (int64_t r = 0; r < n; ++r) CHECK(T[2 * r] >= 0.0 && T[2 * r] <= 1.0);
        for (auto& v : g) v = urand() - 0.5;
        CHECK(or_render_grad(ot, k.data(), &p, times, 3, o.data(), d.data(), t_idx.data(), n, g.data(), 3,
                             grad.data(), rgb1.data()) == 0);
        std::vector<double> bk((size_t)3 * 28 * L);
        or_bake(k.data(), L, &p, times, 3, 2, bk.data());
        std::vector<double> snap(bk.begin() + 28 * L, bk.begin() + 56 * L);
        CHECK(or_render_rays(ot, nullptr, snap.data(), &p, times, 3, o.data(), d.data(), t_idx.data(), n, 2,
                             rgb.data(), T.data(), nseg.data(), nopq.data(), ncell.data()) == 0);
        CHECK(or_ray_labels(ot, k.data(), &p, times, 3, o.data(), d.data(), t_idx.data(), n, lab.data()) == 0);
        or_tree_free(ot);
    }
    std::printf("sanitize_host ok\n");
    return 0;
}
