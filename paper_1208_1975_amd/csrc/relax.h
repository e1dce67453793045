// Sweep-driver internals shared by the host files.
#pragma once

#include "patchset.h"

namespace bs {

int scheme_mode(int axis, bs_scheme scheme);
bs_status get_worklist(bs_patchset *ps, int kind, int axis, int popt, int tx, int colour_mode, WorkList **out,
                       int chunk = 0);
// direct: the configuration for sweeps that may run in the direct Jacobi form
// (FP64, no solve-only or field right-hand-side modes)
LineCfg default_line_cfg(const bs_patchset *ps, int axis, int colour_mode, bool direct = true);
bs_status check_line_cfg(const bs_patchset *ps, int axis, const LineCfg &c);
size_t line_lds_bytes(const bs_patchset *ps, int axis, const LineCfg &c);
// rhs_mode 0: right-hand side = residual of src; 1: = src itself.
// out_mode 0: dst = src + omega du; 1: dst = du; 2 (y/z lines, Jacobi, FP64):
// dst = src + omega du and dst2 = du.
// f32: block solve in FP32 (residual and update stay FP64).
bs_status line_pass(bs_patchset *ps, int axis, const LineCfg &c, int colour_mode, int run, const double *src,
                    double *dst, const double *f, double omega, hipStream_t stream, int patch, int rhs_mode,
                    int out_mode, int f32 = 0, double *dst2 = nullptr);
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

// Ghost updates and extrapolated faces (ghost.cpp).
struct FaceOpsBuild {
    DevBuf ops, items;
    int nfill = 0, nitems = 0;
};
bs_status make_face_ops(const bs_patchset *ps, const std::vector<int32_t> &bc, const std::vector<int32_t> &links,
                        FaceOpsBuild &out);
void commit_face_ops(bs_patchset *ps, FaceOpsBuild &b);
bool ghost_active(const bs_patchset *ps);
bool any_bc(const bs_patchset *ps);
// fill_only: the extrapolated faces alone; else the whole update (links too)
hipError_t ghost_update(const bs_patchset *ps, double *u, bool fill_only, hipStream_t s);
bool bline_any(const bs_patchset *ps, int axis);
bs_status bline_prepare(bs_patchset *ps, int axis);
bs_status bline_pass(bs_patchset *ps, int axis, int colour, const double *src, double *dst, const double *f,
                     double omega, hipStream_t s);
void reset_bc_state(bs_patchset *ps);

// Plane pieces of the adjoint (plane.cpp, FP64): one half-step src -> dst on
// the planes of `colour` (-1 all), and out = M^{-1} P rhs with rhs = r(src)
// (f given) or src's interior (f null), into an out that is zero there.
bs_status plane_step(bs_patchset *ps, int normal, int colour, const double *src, double *dst, const double *f,
                     double omega, hipStream_t s);
bs_status plane_solve(bs_patchset *ps, int normal, int colour, const double *src, const double *f, double *out,
                      hipStream_t s);

// bs_line_relax with graph capture of the sequence allowed or not (a caller
// that captures its own sequence enqueues the sweeps directly).
bs_status line_relax_impl(bs_patchset *ps, int32_t axis, bs_scheme scheme, double omega, int32_t nsweeps,
                          bs_precision prec, double *u, const double *f, double *work, hipStream_t stream,
                          bool allow_graph);

}  // namespace bs
