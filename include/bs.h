/*
 * bs.h -- C ABI of the block-smoothing library (libblocksmooth.so): line- and
 * plane-block relaxation of the constant-coefficient 7-point stencil on
 * structured patches, for AMD MI355X (gfx950).
 *
 * Method: Birke, Philip, Wang, Berrill, "Block-Relaxation Methods for 3D
 * Constant-Coefficient Stencils on GPUs and Multicore CPUs".
 *   - operator: eq. (stencil3d7), generalised to one weight per axis:
 *       (A u)_c = sum_a eps_a (2u_c - u_{c-e_a} - u_{c+e_a}) = h^2 f_c;
 *   - iteration: eq. (blockiteration2), u <- u + omega M^{-1} r, r = h^2 f - A u,
 *     with M the block diagonal (Jacobi) or the block triangle in the visiting
 *     order (block Gauss-Seidel, eq. sm:blockm);
 *   - schemes: damped block Jacobi and chaotic block Gauss-Seidel (section 2,
 *     Algorithm 1), plus a deterministic two-colour block Gauss-Seidel;
 *   - blocks: whole x/y/z lines (tridiagonal, solved exactly) and whole planes
 *     (solved exactly by fast diagonalisation); the paper's partition admits
 *     any block split of A (section 2, discussion of eq. sm:blocka).
 *
 * Storage (section 2.1, index spaces): a patch of nx*ny*nz cells stores u WITH
 * one ghost layer -- (nz+2)(ny+2)(nx+2) doubles, x fastest, interior cell
 * (i,j,k) at ((k+1)(ny+2)+(j+1))(nx+2)+(i+1) -- and f WITHOUT ghosts --
 * nz*ny*nx doubles, cell (i,j,k) at (k*ny+j)*nx+i.  A patch set concatenates
 * its patches; element offsets come from bs_layout (the library may leave
 * alignment gaps between patches; gap contents are never read or written).
 *
 * Ghosts are inputs that the caller owns and updates between calls (section
 * 2: ghost cells are refreshed after a full smoothing step); every call leaves
 * u's ghost cells bit-unchanged, except the ghosts of extrapolated faces
 * (bs_set_bc) and of linked faces (bs_set_links), which the library updates
 * after every sweep.  Edge and corner ghosts are never read.
 *
 * Pointers named *_host are host memory; every other buffer pointer is device
 * memory on the device that was current at bs_create_patchset.  The caller
 * owns u, f, work, r and gradient buffers; the library owns the patch set and
 * everything it allocates (factor tables, sine bases, work lists, graphs).
 *
 * Asynchrony: every call taking a hipStream_t enqueues work on that stream and
 * returns without synchronising.  bs_create_patchset, bs_set_eps and
 * bs_destroy_patchset are synchronous.  Calls on one patch set must not run
 * concurrently from several host threads.
 *
 * Errors: arguments are validated before anything is enqueued; on a non-OK
 * status nothing has been launched, except BS_ERR_HIP, which reports a failed
 * HIP call (its message is in bs_last_error()).  No C++ exception crosses
 * this interface.
 */
#ifndef BS_H
#define BS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bs_patchset bs_patchset;   /* opaque, library-owned */

typedef enum {
    BS_OK = 0,
    BS_ERR_INVALID = 1,      /* bad argument: null pointer, range, size */
    BS_ERR_UNSUPPORTED = 2,  /* valid but not provided (see each call) */
    BS_ERR_OOM = 3,          /* device or host allocation failed */
    BS_ERR_HIP = 4           /* a HIP runtime call failed */
} bs_status;

typedef enum {
    BS_JACOBI = 0,       /* every block from the old u, result via a second vector */
    BS_CHAOTIC_GS = 1,   /* every block updated once, in place, no ordering between
                            blocks (Algorithm 1); blocks are dispatched colour-major
                            in one launch; results are not bit-reproducible */
    BS_COLORED_GS = 2    /* two-colour block GS: colour = (sum of a line's two free
                            indices) mod 2, or plane index mod 2; colour 0 first;
                            deterministic */
} bs_scheme;

typedef enum {
    BS_FP64 = 0,         /* everything in FP64 */
    BS_MIXED_FP32 = 1,   /* FP64 residual and update, FP32 block solve */
    BS_MIXED_BF16 = 2    /* FP64 residual and update, BF16 transforms with FP32
                            accumulation (planes only) */
} bs_precision;

/* Layout of a patch set, computed on the host with no device work.
 * dims_host: [3*npatch] = nx,ny,nz per patch (each >= 1).
 * Outputs: total doubles of u (padded) and f (unpadded); optional per-patch
 * element offsets ([npatch] each, may be NULL).  Patches start on 256-byte
 * boundaries.  BS_ERR_INVALID on npatch < 1, a null dims/numel pointer, or
 * dims < 1. */
bs_status bs_layout_plan(int32_t npatch, const int32_t *dims_host, int64_t *u_numel,
                         int64_t *f_numel, int64_t *u_off_host, int64_t *f_off_host);

/* Create a patch set: per patch dims (nx,ny,nz), axis weights eps (eps_x,
 * eps_y, eps_z > 0) and cell width h > 0.  Builds every precomputed table on
 * the current device (section 2: the block inverse is formed once before the
 * smoothing iterations): the LU factors and interface-coupling tables of the
 * exact line solves, and the sine eigenbases and eigenvalues of the exact
 * plane solves.  Synchronous.  BS_ERR_INVALID on bad sizes or non-positive
 * eps/h; BS_ERR_UNSUPPORTED for an edge above 4096 or a patch whose padded u
 * reaches 4 GiB ((nx+2)(ny+2)(nz+2) >= 2^29, about 810^3 cells: split such a
 * domain into patches); BS_ERR_OOM / BS_ERR_HIP on allocation or copy
 * failures. */
bs_status bs_create_patchset(int32_t npatch, const int32_t *dims_host, const double *eps_host,
                             const double *h_host, bs_patchset **out);

/* Free a patch set and everything it owns.  Waits for the device.  NULL ok. */
void bs_destroy_patchset(bs_patchset *ps);

/* Replace every patch's eps ([3*npatch], > 0) and rebuild the tables that
 * depend on it.  Synchronous.  The new line tables are built aside and swapped
 * in only when every allocation and copy succeeded: on BS_ERR_OOM / BS_ERR_HIP
 * from that step the patch set keeps its previous eps and stays usable.  Cube
 * block sizes prepared with bs_cube_prepare are rebuilt afterwards; if one of
 * those rebuilds fails, the call returns its status with the new eps in force,
 * and that size and every prepared size not yet rebuilt are dropped (they must
 * be prepared again). */
bs_status bs_set_eps(bs_patchset *ps, const double *eps_host);

/* Boundary condition per face: bc_host[npatch] holds a 6-bit mask per patch,
 * bit 2a = the low face of axis a (cells at index 0), bit 2a+1 = the high face.
 * A set bit marks an extrapolated Dirichlet face (section 1.1: boundary
 * conditions are extrapolated into the ghost layer; the value at the face is
 * zero): its ghost is the negated adjacent interior value, which folds into
 * the operator as +eps_a on the diagonal of the cells next to the face and
 * into every block that contains them.  A clear bit (the default) keeps the
 * ghosts of that face as caller data.  The ghost cells of an extrapolated face
 * are the library's: the sweeps overwrite them with the negated adjacent
 * interior values, and bs_residual ignores them.  Rebuilds the line tables
 * (raised end diagonals) and drops prepared cube block sizes.  Synchronous.
 * BS_ERR_INVALID for a mask outside 0..63 or one that marks a linked face
 * (bs_set_links); on BS_ERR_OOM / BS_ERR_HIP the set keeps its previous
 * conditions.  Lines, planes (FP64) and cube blocks take any mask (a cube
 * block touching an extrapolated face gets its own inverse); mixed-precision
 * planes return BS_ERR_UNSUPPORTED on a patch set with any extrapolated
 * face. */
bs_status bs_set_bc(bs_patchset *ps, const int32_t *bc_host);

/* Face adjacency (section 2: ghosts are updated Jacobi-fashion after every
 * smoothing step; section 1.1: the ghosts of faces between patches keep the
 * patches consistent).  links_host[3*nlinks] holds (a, axis, b): patch b lies
 * on patch a's high side along `axis`, with equal extents along the other two
 * axes.  Afterwards every sweep of bs_line_relax, bs_plane_relax and
 * bs_cube_relax is followed by a ghost update on the new iterate: a's high
 * ghost layer along `axis` takes b's first interior layer and b's low ghost
 * layer a's last one (and extrapolated faces take their negated interior
 * values).  nlinks = 0 removes the links.  Synchronous.  BS_ERR_INVALID for
 * an index out of range, a == b, unequal extents, a face used by two links,
 * or a face that is extrapolated; nothing changes on any error. */
bs_status bs_set_links(bs_patchset *ps, int32_t nlinks, const int32_t *links_host);

/* One ghost update of u (device, u layout) as the sweeps apply it after every
 * step: the linked faces' ghosts from their neighbours, the extrapolated
 * faces' ghosts from their own interior.  Edge and corner ghosts are never
 * touched.  Asynchronous on `stream`. */
bs_status bs_exchange_ghosts(const bs_patchset *ps, double *u, hipStream_t stream);

/* Layout of an existing patch set (same meaning as bs_layout_plan). */
bs_status bs_layout(const bs_patchset *ps, int64_t *u_numel, int64_t *f_numel,
                    int64_t *u_off_host, int64_t *f_off_host);

/* Residual r = h^2 f - A u over interior cells (eq. stencil3d7 with axis
 * weights; section 3 monitors its 2-norm).  r: f-layout output, or NULL for
 * norms only.  rnorm2: [npatch] device doubles receiving sum(r^2) per patch,
 * or NULL.  The sums are reduced in a fixed order, so they are bit-identical
 * from run to run.  At least one of r, rnorm2 must be non-NULL. */
bs_status bs_residual(const bs_patchset *ps, const double *u, const double *f, double *r,
                      double *rnorm2, hipStream_t stream);

/* nsweeps sweeps of line-block relaxation along `axis` (0=x, 1=y, 2=z) on every
 * patch of the set: each line's residual is formed from the current u
 * (off-line neighbours and ghosts included), the line's tridiagonal block
 * tridiag(-eps_a, 2(eps_x+eps_y+eps_z), -eps_a) is solved exactly, and the
 * line is updated by omega times the correction (Algorithm 1; Algorithm 2's
 * residual / block solve / update structure).
 *   u     in/out, u-layout; on return it holds the result (also for Jacobi
 *         with an odd sweep count).
 *   f     f-layout.
 *   work  u-layout scratch for BS_JACOBI (the paper's second vector v); may
 *         be NULL for the Gauss-Seidel schemes.  Its ghosts are overwritten.
 *   omega in (0, 2).  nsweeps >= 0 (0 enqueues nothing).
 *   prec  BS_FP64, or BS_MIXED_FP32: the line solve (chunk factors and
 *         interface coupling) in FP32 while the residual and the update
 *         u += omega du stay in FP64; every sweep recomputes the FP64
 *         residual, so the sweeps themselves act as the defect correction and
 *         the exact discrete solution stays a fixed point.
 * Every patch of the set is relaxed by the same launches (one per sweep, or
 * per colour for BS_COLORED_GS), larger patches first.  BS_CHAOTIC_GS on y/z
 * lines updates each tile's colour-0 lines, then its colour-1 lines from the
 * new in-tile values, in place, tiles of even tile rows dispatched first.  A
 * sequence of two or more sweeps is captured into a HIP graph on its first
 * call and replayed by later calls with the same arguments and buffers.
 * When a patch set has fewer tiles of lines than one even/odd dispatch chunk per
 * XCD (so that every tile would run at once and tiles could not see their
 * neighbours' new values), BS_CHAOTIC_GS is dispatched colour-major instead:
 * all colour-0 lines in one launch, then all colour-1 lines, which is the
 * two-colour sweep (one of the orders a chaotic sweep may take).
 * Line lengths: every line is solved whole; the supported lengths are x-lines
 * of up to 256 cells and y- or z-lines of up to 1024 cells (the kernels hold a
 * line in the registers of at most 16 wavefronts, and 64 x-lines of a tile in
 * LDS).  A longer line along `axis` in any patch of the set returns
 * BS_ERR_UNSUPPORTED before anything is enqueued (split such patches, or use
 * plane blocks, which accept in-plane edges up to 1024).
 * BS_ERR_UNSUPPORTED for BS_MIXED_BF16 (BF16 is offered for planes only). */
bs_status bs_line_relax(bs_patchset *ps, int32_t axis, bs_scheme scheme, double omega,
                        int32_t nsweeps, bs_precision prec, double *u, const double *f,
                        double *work, hipStream_t stream);

/* nsweeps sweeps of plane-block relaxation with planes normal to normal_axis.
 * Each plane block M_P = d I - eps_a(S_a + S_a^T) - eps_b(S_b + S_b^T) is
 * solved exactly by fast diagonalisation with the orthonormal DST-I bases of
 * the two in-plane axes.  refine >= 0 inner defect-correction steps are
 * applied to the block solve for the mixed precisions (ignored for FP64).
 * Other arguments as bs_line_relax.  BS_ERR_UNSUPPORTED if an in-plane edge
 * exceeds 1024. */
bs_status bs_plane_relax(bs_patchset *ps, int32_t normal_axis, bs_scheme scheme, double omega,
                         int32_t nsweeps, bs_precision prec, int32_t refine, double *u,
                         const double *f, double *work, hipStream_t stream);

/* Geometric cube blocks (section 2's lexicographically ordered geometric
 * blocks; the block Jacobi algorithm on GPUs; the block-inversion section).
 * Blocks of bx x by x bz cells tile every patch from its origin; an edge
 * longer than the patch is clipped to it, and along an axis that is not a
 * multiple of the edge the last block is shorter.  Each distinct block shape
 * of each patch gets the dense inverse of its block matrix (the stencil
 * restricted to the block's cells), computed once, on the host, by
 * bs_cube_prepare; patches with equal dims, eps and h share them.
 *
 * bs_cube_prepare: builds the inverses, block tables and, for blocks of more
 * than 64 cells, a residual scratch of 8 bytes per cell of the largest group
 * of equally shaped blocks; synchronous (allocates device memory).  Repeated calls with a
 * prepared size return BS_OK at once; bs_set_eps rebuilds every prepared
 * size (a size whose rebuild fails, e.g. for lack of memory, is dropped and
 * must be prepared again).  BS_ERR_INVALID for an edge < 1; BS_ERR_UNSUPPORTED for blocks of
 * more than 512 cells after clipping (8^3 is the paper's largest) or more
 * than 1 GiB of inverses in total. */
bs_status bs_cube_prepare(bs_patchset *ps, int32_t bx, int32_t by, int32_t bz);

/* nsweeps sweeps of cube-block relaxation with a prepared block size: per
 * block, its residual r_b = h^2 f_b - (A u)_b (neighbours outside the block
 * and ghosts included), du_b = Ainv_b r_b, u_b += omega du_b (Algorithm 1 in
 * the residual-correction form).  The blocks' products with their inverses
 * run as one FP64 matrix-core product per block shape (blocks as rows).
 *   BS_JACOBI:     every block from the same iterate, into `work` (the
 *                  second vector), pointer swap; the result ends in u.
 *   BS_COLORED_GS: blocks with (bi+bj+bk) even, then odd, in place.
 *   BS_CHAOTIC_GS: in place, in the same colour-major order (one of the
 *                  orders a chaotic sweep may take; deterministic).
 * prec must be BS_FP64 (BS_ERR_UNSUPPORTED otherwise).  Asynchronous on
 * `stream`; two or more sweeps are captured into a HIP graph on their first
 * call and replayed later, as bs_line_relax.  BS_ERR_INVALID if the block
 * size was not prepared, and for the argument errors of bs_line_relax. */
bs_status bs_cube_relax(bs_patchset *ps, int32_t bx, int32_t by, int32_t bz, bs_scheme scheme, double omega,
                        int32_t nsweeps, bs_precision prec, double *u, const double *f, double *work,
                        hipStream_t stream);

/* Autotuner: time the candidate launch configurations of line sweeps along
 * `axis` for `scheme` (chunk count per line, tile width, one workgroup per
 * tile or a persistent grid) on copies of u -- the caller's buffers are not
 * modified -- and keep the fastest for later bs_line_relax calls on this patch
 * set.  Synchronous; allocates two u-sized scratch buffers for its duration. */
bs_status bs_autotune_line(bs_patchset *ps, int32_t axis, bs_scheme scheme, const double *u, const double *f,
                           hipStream_t stream);

/* The launch configuration bs_line_relax uses for (axis, scheme), written to
 * the caller's host array of six int32:
 *   [5] kernel form: 0 = each line cut into chunks, one wavefront per chunk,
 *       a lane per line; 1 = x-lines of up to 64 cells spread over the lanes
 *       of a 16-lane row, four cells per lane (the default for such x-lines);
 *   [0] form 0: chunks per line; form 1: wavefronts per workgroup;
 *   [1] form 0: register chunk length; form 1: cells per lane (4);
 *   [2] tile width in lanes (y/z lines);
 *   [3] persistent grid size (0: one workgroup per tile);
 *   [4] 1 if it was set by the autotuner. */
bs_status bs_line_config(const bs_patchset *ps, int32_t axis, bs_scheme scheme, int32_t cfg_host[6]);

/* Device workspace needed by bs_relax_backward for these arguments, or 0 on
 * invalid arguments.  `axis` (0..2) is the line axis bs_relax_backward will
 * get: the size (checkpointed states, one recompute segment, the adjoint
 * work fields, and for y/z lines the recomputed sweeps' corrections w)
 * depends on it. */
size_t bs_backward_workspace_bytes(const bs_patchset *ps, int32_t axis, int32_t nsweeps,
                                   int32_t ckpt_every);

/* Adjoint of nsweeps damped Jacobi line sweeps along `axis` (FP64), for a
 * loss L with dL/du_K = grad_uK (u-layout; ghost entries ignored).  States
 * are recomputed from checkpoints taken every ckpt_every sweeps.  Outputs
 * (each may be NULL):
 *   grad_u0  u-layout: interior entries dL/du0; face-ghost entries dL/dghost
 *            (edges and corners 0);
 *   grad_f   f-layout: dL/df;
 *   grad_eps [3*npatch] device doubles: dL/d(eps_x, eps_y, eps_z) per patch.
 * workspace: device memory of at least bs_backward_workspace_bytes bytes.
 * BS_ERR_UNSUPPORTED for a scheme other than Jacobi (only Jacobi has a
 * backward here). */
bs_status bs_relax_backward(bs_patchset *ps, int32_t axis, double omega, int32_t nsweeps,
                            int32_t ckpt_every, const double *u0, const double *f,
                            const double *grad_uK, double *grad_u0, double *grad_f,
                            double *grad_eps, void *workspace, size_t workspace_bytes,
                            hipStream_t stream);

/* Geometric multigrid with the block smoothers (section 1: line and plane
 * smoothers are the components of robust geometric multigrid; section 5:
 * multilevel use).  A cycle object holds the coarse levels of a fine patch
 * set: every patch is coarsened on its own by factors of two (cell width 2h,
 * the same eps) while all its edges are even, down to `levels` levels (0: as
 * many as every patch allows).  One V(nu1, nu2) cycle of bs_vcycle on
 * A u = h^2 f: nu1 sweeps of the smoother; the defect d = h^2 f - A u
 * restricted (mean of the 2x2x2 children) to f_c = R(d / h^2); the cycle
 * applied to the coarse error equation A e = (2h)^2 f_c from e = 0, whose
 * ghosts are zero, or extrapolated on the faces of coarse_bc (the same mask
 * for every patch and coarse level; bs_set_bc's meaning); u += trilinear
 * interpolation of e (across a face of coarse_bc the coarse value is
 * reflected and negated); nu2 sweeps.  The coarsest level takes ncoarse
 * sweeps.  Smoother: kind 0 = line blocks along axis `arg`, kind 1 = plane
 * blocks normal to `arg`, with `scheme` and omega, in FP64.
 *
 * bs_mg_create: synchronous; allocates the levels (their patch sets and
 * three u/f-sized fields each, plus one defect field per level but the
 * coarsest).  The fine set stays the caller's and must outlive the cycle
 * object; its dims, eps and faces are copied: after bs_set_eps or bs_set_bc on
 * it, bs_vcycle returns BS_ERR_INVALID until the object is created again.
 * BS_ERR_INVALID for bad arguments; BS_ERR_UNSUPPORTED for a fine set with
 * links. */
typedef struct bs_mg bs_mg;
bs_status bs_mg_create(bs_patchset *fine, int32_t kind, int32_t arg, bs_scheme scheme, double omega, int32_t nu1,
                       int32_t nu2, int32_t ncoarse, int32_t levels, int32_t coarse_bc, bs_mg **out);
void bs_mg_destroy(bs_mg *mg);
/* Number of levels of the cycle (the fine level included). */
bs_status bs_mg_levels(const bs_mg *mg, int32_t *levels);
/* One V-cycle: u in/out (u layout of the fine set), f (f layout), work (u
 * layout; the Jacobi smoother's second vector, may be NULL for the
 * Gauss-Seidel schemes).  Asynchronous on `stream`.  The first cycle with a
 * given (u, f, work) runs eagerly and builds every table the levels need; the
 * next one is captured into a HIP graph, which later calls replay. */
bs_status bs_vcycle(bs_mg *mg, double *u, const double *f, double *work, hipStream_t stream);

/* Adjoint of nsweeps FP64 sweeps of line blocks (kind 0, along `axis`) or
 * plane blocks (kind 1, normal to `axis`) under BS_JACOBI or BS_COLORED_GS,
 * for a loss L with dL/du_K = grad_uK: the gradients of the differentiable
 * smoother beyond Jacobi lines.  A two-colour sweep is two half-steps
 * u += omega P_c M^{-1} r(u), P_c the projection onto the blocks of colour c
 * (colour 0 first); M is block diagonal, so P_c M^{-1} = M^{-1} P_c, and each
 * half-step is undone in reverse order (colour 1, then colour 0) with
 * lambda = M^{-1} P_c gbar:  dL/df += omega h^2 lambda,  dL/dghost +=
 * omega eps_a lambda (face ghosts),  dL/deps_b -= omega <lambda, D_b u +
 * (dM/deps_b) P_c M^{-1} r(u)>,  gbar -= omega A_int lambda.  States are
 * recomputed from checkpoints taken every ckpt_every sweeps; the workspace
 * (bs_block_backward_workspace_bytes; 0 on invalid arguments) holds them.
 * Outputs and their layouts as bs_relax_backward (each may be NULL).
 * BS_ERR_UNSUPPORTED for BS_CHAOTIC_GS (no unique forward map), for patch sets
 * with links or extrapolated faces, and for lines or planes the forward calls
 * refuse. */
size_t bs_block_backward_workspace_bytes(const bs_patchset *ps, int32_t kind, int32_t axis, bs_scheme scheme,
                                         int32_t nsweeps, int32_t ckpt_every);
bs_status bs_block_backward(bs_patchset *ps, int32_t kind, int32_t axis, bs_scheme scheme, double omega,
                            int32_t nsweeps, int32_t ckpt_every, const double *u0, const double *f,
                            const double *grad_uK, double *grad_u0, double *grad_f, double *grad_eps,
                            void *workspace, size_t workspace_bytes, hipStream_t stream);

/* The same adjoint split at its checkpoints, so that the backward does not
 * run the forward sweeps again (section 2's sweeps; the checkpointing is
 * the differentiable smoother's).  bs_block_forward_ckpt: u in = u0 (u
 * layout, ghosts included), out = u_K after the nsweeps sweeps
 * bs_block_backward differentiates (the ghosts unchanged); it leaves the
 * states at sweeps 0, c, 2c, ... (c = ckpt_every) in `workspace`
 * (bs_block_backward_workspace_bytes bytes, the same arguments).
 * bs_block_backward_ckpt: bs_block_backward from those checkpoints; it
 * takes no u0.  Between the two calls the workspace, f, the patch set's
 * eps and the arguments must stay the same; the backward leaves the
 * checkpoints as they are, so it may run again for another grad_uK.  Errors
 * as bs_block_backward; both are asynchronous on `stream`. */
bs_status bs_block_forward_ckpt(bs_patchset *ps, int32_t kind, int32_t axis, bs_scheme scheme, double omega,
                                int32_t nsweeps, int32_t ckpt_every, double *u, const double *f, void *workspace,
                                size_t workspace_bytes, hipStream_t stream);
bs_status bs_block_backward_ckpt(bs_patchset *ps, int32_t kind, int32_t axis, bs_scheme scheme, double omega,
                                 int32_t nsweeps, int32_t ckpt_every, const double *f, const double *grad_uK,
                                 double *grad_u0, double *grad_f, double *grad_eps, void *workspace,
                                 size_t workspace_bytes, hipStream_t stream);

/* bs_residual for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same result and per-patch norms, bit for bit, with the per-tile partial sums
 * of the norm reduction in a static device array of 65536 doubles (512 KiB)
 * instead of the patch set's own buffer.  Each GPU holds its own copy of the
 * array for the life of the process; its address is looked up on the first
 * call on a device.  Allocates nothing.  Every call on one GPU shares that
 * array: calls that overlap on one GPU (several streams, several host
 * threads) race.  BS_ERR_UNSUPPORTED for a patch set with more than 65536
 * residual tiles (a tile covers at most 256 columns by 64 planes of one
 * patch), BS_ERR_INVALID for the argument errors of bs_residual or when the
 * current device is not the patch set's. */
bs_status bs_residual_noalloc(const bs_patchset *ps, const double *u, const double *f, double *r,
                              double *rnorm2, hipStream_t stream);

/* Message for the last non-OK status returned on this host thread ("" if none). */
const char *bs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BS_H */
