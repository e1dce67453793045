// The patch set owned by the library, and helpers shared by its host files.
#pragma once

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "bs.h"
#include "bs_internal.h"

namespace bs {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { reset(); }
    void reset()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void swap(DevBuf &o)
    {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
    }
};

// A device work list: items of colour 0 first, then colour 1 (colour-split
// lists), or a single run (all lines).
struct WorkList {
    DevBuf buf;
    // the launch runs (colour 0, colour 1) at the start of buf, in dispatch
    // order (may hold empty items, patch < 0, that kernels skip)
    int count[2] = {0, 0};
    // the same items per patch, contiguous, at pp_off[c] in buf: per colour
    // run, per patch, first item (relative to pp_off) and count
    int pp_off[2] = {0, 0};
    std::vector<int> pfirst[2], pcount[2];
};

// Key: kernel kind (0 strided y/z, 1 x), axis, chunk option, tile width, colour
// mode, tiles per even/odd chunk of the chaotic dispatch order (0 otherwise).
using WorkKey = std::tuple<int, int, int, int, int, int>;

// A tuned launch configuration for one (axis, scheme class) of a patch set.
struct LineCfg {
    int popt = -1;    // index into kPOpts
    int Lmax = 0;     // register chunk template (>= every patch's Lr)
    int nwaves = 0;   // wavefronts per workgroup (= P_req)
    int tx = 64;      // strided kernel: lanes along x per row
    int grid = 0;     // persistent grid size (0: one workgroup per work item)
    int form = 0;     // 0: a line's chunks on the wavefronts of a workgroup;
                      // 1: x-lines across the lanes of a 16-lane row (nx <= 64);
                      // 2: the same lines marched along z (nx <= 64; Jacobi, chaotic GS)
    int zc = 0;       // form 2: planes per work item
    int tuned = 0;    // 1: chosen by bs_autotune_line
    int deflt = 0;    // 1: the library's default (not set by a caller or the autotuner)
};

// Geometric cube blocks of one block size: one group per (class of patches
// with equal dims, eps and h; block shape).
struct CubeGroup {
    int nb = 0, nblk = 0, ncol0 = 0;   // cells per block, blocks, colour-0 blocks
    // byte offsets into CubePlan::buf: inverse (nb x nb, row-major), per-cell
    // u / f offsets (nb int32 each), per-block u / f bases (nblk int64 each)
    // in colour order (Gauss-Seidel) and in dispatch order without colours
    // (Jacobi)
    int64_t o_ainv = 0, o_uoff = 0, o_foff = 0, o_ubase = 0, o_fbase = 0, o_jbase = 0, o_jfbase = 0;
    double ex = 0, ey = 0, ez = 0, h2 = 0;
    int64_t sy = 0, sz = 0;
};
struct CubePlan {
    std::vector<CubeGroup> groups;
    DevBuf buf;    // tables and inverses
    DevBuf rbuf;   // block-major residual scratch (largest group of blocks over 64 cells)
    int64_t inv_bytes = 0;
    // device group descriptors and chunk lists, per operand size (16, 32, 64:
    // the small-block kernel; 128, 256: the fused large-block kernel) and list
    // (Jacobi, colour 0, colour 1)
    DevBuf gdesc, chunks;
    int chunk_off[5][3] = {}, chunk_cnt[5][3] = {};
    int fused_max = 256;   // largest block (cells) on the fused kernels; larger: two kernels
};

bs_status fail(bs_status st, const char *fmt, ...);
bs_status cube_rebuild_all(bs_patchset *ps);   // after an eps change
bs_status hip_fail(hipError_t e, const char *what);
bs_status upload(DevBuf &b, const void *src, size_t bytes, const char *what);
bs_status dev_alloc(DevBuf &b, size_t bytes, const char *what);

}  // namespace bs

struct bs_patchset {
    int32_t npatch = 0;
    int device = 0;
    std::vector<int32_t> dims;
    std::vector<double> eps, h;
    std::vector<int64_t> uoff, foff;
    int64_t u_numel = 0, f_numel = 0;
    int32_t max_n[3] = {0, 0, 0};
    std::vector<bs::PatchDesc> desc;
    bs::DevBuf desc_d, tab_d, tab32_d;
    // residual reduction plan
    int32_t nrtiles = 0;    // residual and adjoint tiles
    bs::DevBuf rtile_d, rtile_first_d, rpartial_d;
    // plane solves: sine bases per patch and axis, inverse eigenvalue grids per
    // patch and normal axis (built on first use), and two f-layout scratch fields
    bool plane_ready = false;
    bs::DevBuf plane_tab_d, plane_r_d, plane_t_d;
    bs::DevBuf plane_tab32_d, plane_f1_d, plane_f2_d;   // FP32 copies and float scratch (mixed precision)
    bs::DevBuf plane_tab16_d;                           // BF16 copies of the bases
    int mixed_dlayout = 0;
    int chaotic_chunk = 0;   // tiles per even/odd chunk of the chaotic dispatch order (0: default)
    std::map<std::vector<int>, int> chaotic_chunks;   // per line configuration: tiles per chunk
    // [3 * npatch] each, offsets in doubles: the basis read by the forward
    // transforms (V^T), by the inverse ones (V; the same entries for the
    // symmetric DST-I basis), the inverse eigenvalue grid of the interior
    // planes, and of the first / last plane along the normal when that face
    // is extrapolated (-1 otherwise)
    std::vector<int64_t> basis_off, basis_inv_off, lam_off, lam_lo_off, lam_hi_off;
    std::vector<int8_t> basis_kind;   // [3 * npatch]: 0 DST-I, 1 both ends raised, 2 one end raised
    // cached work lists and tuned configurations
    std::map<bs::WorkKey, std::unique_ptr<bs::WorkList>> lists;
    std::map<std::pair<int, int>, bs::LineCfg> line_cfg;   // (axis, colour_mode) -> cfg
    // cube-block plans, per block size (bx, by, bz), built by bs_cube_prepare
    std::map<std::tuple<int, int, int>, std::unique_ptr<bs::CubePlan>> cube;
    // captured sweep sequences, replayed with one graph launch
    std::map<std::vector<int64_t>, hipGraphExec_t> graphs;
    // boundary conditions and adjacency: per patch the mask of extrapolated
    // faces, the links (a, axis, b) between face-adjacent patches, the face
    // operations of one ghost update (extrapolated faces first) and, per line
    // axis, the lines next to extrapolated faces parallel to them
    std::vector<int32_t> bc;
    std::vector<int32_t> links;
    bs::DevBuf face_ops_d, face_items_d;
    int nfill_items = 0, nface_items = 0;
    bool bline_ready[3] = {false, false, false};
    bs::DevBuf bline_d[3];
    int bline_count[3][2] = {{0, 0}, {0, 0}, {0, 0}};   // colour 0 items, then colour 1
    int bline_maxlen[3] = {0, 0, 0};                     // longest such line per axis
    bs::DevBuf bline_scratch;
    bs::DevBuf bline_fac[3];                             // their LU factors per axis ([t][line])
    hipStream_t capture_stream = nullptr;
    uint64_t gen = 0;   // bumped whenever device tables or captured graphs are replaced
    bool use_graphs = true;
    bool use_pair = true;   // chaotic y/z lines with omega 1: the two-cells-per-lane kernel
    bool line_direct = true;   // Jacobi on y/z lines in the direct form (no copy of u kept for the update)
    bool plane_lr = true;   // FP32 plane chain, normals y, z: the left (non-x) products first and last
    int cube_fused_max = 256;   // cube blocks up to this many cells on the fused kernels (at most 256)
    ~bs_patchset();
};
