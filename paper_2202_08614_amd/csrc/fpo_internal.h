// Internal helpers shared by the host-side translation units of libfpo.
#pragma once

#include <cstdint>
#include <string>

#include "fpo.h"

namespace fpo {

// Record a message for fpo_last_error() and return `st`.
fpo_status fail(fpo_status st, const std::string& msg);
fpo_status ok();

// Words per 16-byte packed word and number of planes for a coefficient dtype.
inline int coeffs_per_word(fpo_dtype dt) { return dt == FPO_F32 ? 4 : (dt == FPO_BF16 ? 8 : 16); }
inline int n_planes(fpo_dtype dt)
{
    const int w = coeffs_per_word(dt);
    return (FPO_N_COEFF + w - 1) / w;
}

// Coefficient layouts (n1, n2) with compiled kernels: the default (31, 5)
// everywhere; (11 | 21 | 31, 5 | 11) for packing, Fourier-mode F32 renders and
// the per-time IDFT pass.
inline bool layout_supported(int n1, int n2)
{
    return (n1 == 11 || n1 == 21 || n1 == 31) && (n2 == 5 || n2 == 11);
}
inline bool default_layout(const fpo_layout& L)
{
    return L.n_sigma == FPO_N_SIGMA && L.n_sh_fourier == FPO_N_SH_FOURIER;
}
// 16-byte words per leaf record (whole 128-byte lines).
inline int record_words(fpo_dtype dt, int n1, int n2)
{
    const int w = coeffs_per_word(dt);
    return ((n1 + 3 * FPO_N_SH * n2 + w - 1) / w + 7) / 8 * 8;
}

// Validate a tree view (host-visible fields only).  allow_layouts: the call
// handles every layout_supported() layout (else only the default one).
fpo_status check_tree(const fpo_tree_view* tree, bool need_coeffs, bool allow_layouts = false);
// allow_skip: the call accepts the skip flags (fpo_render only); allow_record:
// it accepts FPO_RAYS_RECORD (fpo_render_rays, fpo_render_backward);
// skip_workspace: skip modes need opts->workspace (not so for a call that
// brings its own scratch).
fpo_status check_opts(const fpo_render_opts* opts, const fpo_tree_view* tree, bool allow_skip = false,
                      bool allow_record = false, bool skip_workspace = true);

// Segment records in opts->workspace (FPO_RAYS_RECORD): per-ray counts at the
// start, records of FPO_RECORD_BYTES from the next 256-byte boundary, cap
// records per ray (at least 1).
struct RecordLayout {
    int32_t* count;
    void* records;
    int32_t cap;
};
fpo_status record_layout(const fpo_render_opts* opts, int64_t n_rays, RecordLayout& out);

// Camera frame in FP64, rounded to FP32: eye, unit forward, right * tan_x, up' * tan_y.
fpo_status camera_frame(const fpo_camera& cam, float out[12]);

// FP64 basis of Eq. 8 rounded to FP32 (FPO_BASIS_STRIDE values, zero padded).
void basis_row(double t, double period, int n, float* out);

// FPO_E_DEVICE with the HIP error string if the last launch failed, else FPO_OK.
fpo_status launch_status(const char* what);

// A roctx range around one library call (push on construction, pop on
// destruction), so that a profiler's marker trace shows each call.
struct ApiRange {
    explicit ApiRange(const char* name);
    ~ApiRange();
    ApiRange(const ApiRange&) = delete;
    ApiRange& operator=(const ApiRange&) = delete;
};

// Debug switches from the environment: FPO_FAULT=alloc (host allocations
// fail: throws std::bad_alloc) and FPO_FORCE_FALLBACK=1 (skip flags ignored).
void fault_point_alloc();
bool force_fallback();

}  // namespace fpo
