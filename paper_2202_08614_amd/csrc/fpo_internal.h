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

// Validate a tree view (host-visible fields only).
fpo_status check_tree(const fpo_tree_view* tree, bool need_coeffs);
// allow_skip: the call accepts the skip flags (fpo_render only).
fpo_status check_opts(const fpo_render_opts* opts, const fpo_tree_view* tree, bool allow_skip = false);

// Camera frame in FP64, rounded to FP32: eye, unit forward, right * tan_x, up' * tan_y.
fpo_status camera_frame(const fpo_camera& cam, float out[12]);

// FP64 basis of Eq. 8 rounded to FP32 (FPO_BASIS_STRIDE values, zero padded).
void basis_row(double t, double period, int n, float* out);

// FPO_E_DEVICE with the HIP error string if the last launch failed, else FPO_OK.
fpo_status launch_status(const char* what);

}  // namespace fpo
