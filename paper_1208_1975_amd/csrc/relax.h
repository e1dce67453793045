// Sweep-driver internals shared by the host files.
#pragma once

#include "patchset.h"

namespace bs {

int scheme_mode(int axis, bs_scheme scheme);
bs_status get_worklist(bs_patchset *ps, int kind, int axis, int popt, int tx, int colour_mode, WorkList **out,
                       int chunk = 0);
LineCfg default_line_cfg(const bs_patchset *ps, int axis, int colour_mode);
bs_status check_line_cfg(const bs_patchset *ps, int axis, const LineCfg &c);
size_t line_lds_bytes(const bs_patchset *ps, int axis, const LineCfg &c);
// rhs_mode 0: right-hand side = residual of src; 1: = src itself.
// out_mode 0: dst = src + omega du; 1: dst = du.
// f32: block solve in FP32 (residual and update stay FP64).
bs_status line_pass(bs_patchset *ps, int axis, const LineCfg &c, int colour_mode, int run, const double *src,
                    double *dst, const double *f, double omega, hipStream_t stream, int patch, int rhs_mode,
                    int out_mode, int f32 = 0);
const LineCfg &line_cfg(bs_patchset *ps, int axis, int colour_mode);
bs_status enqueue_line_sweeps(bs_patchset *ps, int axis, bs_scheme scheme, const LineCfg &c, double omega,
                              int nsweeps, double *u, const double *f, double *work, hipStream_t stream,
                              bool per_patch, int f32 = 0);
bs_status prepare_lists(bs_patchset *ps, int axis, const LineCfg &c, int colour_mode);
// Chaotic GS dispatch: tiles per even/odd chunk of the one-launch order, and
// whether the sweep is instead dispatched colour-major in two launches.
int chaotic_chunk_for(bs_patchset *ps, int axis, const LineCfg &c);
bool chaotic_colour_major(bs_patchset *ps, int axis, const LineCfg &c);
void clear_graphs(bs_patchset *ps);
bs_status check_line_ps_ext(const bs_patchset *ps, int32_t axis, const char *fn);

}  // namespace bs
