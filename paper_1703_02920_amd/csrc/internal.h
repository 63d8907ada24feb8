// Internal declarations of the uvmem library: context layout, work-item
// tables, kernel launchers.  Not part of the public ABI (include/uvmem.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/uvmem.h"

namespace uvm {

// Threads per workgroup of the pixel, visibility and scalar kernels.
constexpr int NTHR = 256;
// Target workgroup counts of the visibility kernels and of the pixel kernels
// (over all channels); a visibility item is a multiple of 2 NTHR
// visibilities, a pixel block a multiple of NTHR pixels.
constexpr int VIS_WGS = 1024;
constexpr int PIX_WGS = 1024;
// Minimum visibilities per adjoint split-K chunk (multiple of 16).
constexpr int ADJ_KMIN = 64;
// Maximum visibilities per split-K chunk of the split-precision adjoint,
// whose chunk sums are FP32 only (bounds their rounding growth).
constexpr int ADJ_KMAX_SPLIT = 32768;
// visibilities per FP32 sum of the 256-tile FP32 adjoint before it is folded
// into FP64 (and the chunk length up to which its partials stay FP32)
constexpr int ADJ_F32_SUM = 8192;
// Partial-sum slots per pixel / visibility item.
constexpr int NPART = 16;
// Trial steps evaluated per line-search pass (two partials each).
constexpr int LS_K = 8;
// Relative tolerance that decides "pixel at the bound I <= M (1 + tol)".
constexpr double BOUND_TOL = 1e-12;
// Gridded model: cells holding more visibilities than this are reduced by a
// wave each before the node gather (bounds the gather's serial loops).
constexpr int GRID_DENSE = 16;
// Default number of line-search passes per CG step after the start in the
// direction's visibility pass (which already settles a step that reaches
// alpha_max); a channel whose search has converged skips the remaining passes.
constexpr int LS_STEPS = 3;

// One workgroup of the persistent split-precision forward model: image block
// (ib, jb) of a channel resident in LDS; the workgroup is number `wg` of the
// `nwg` sharing that block's visibility tiles.
struct FwdPItem {
    int chan;
    int ib;
    int jb;
    int part;
    int wg;
    int nwg;
    long long kbeg;
    long long kend;
};

// One adjoint workgroup: a square pixel tile (ti, tj) of a channel and a
// chunk [kbeg, kend) of its visibilities; `slot` indexes the partial image.
struct AdjItem {
    int chan;
    int ti;
    int tj;
    int slot;
    long long kbeg;
    long long kend;
};

// One visibility-reduction workgroup: [kbeg, kend) inside one channel.
struct VisItem {
    int chan;
    int pad;
    long long kbeg;
    long long kend;
};

// Device-side line-search state of one channel (double[LSS_N]).
enum {
    LSS_PHASE = 0,   // 0 = searching, 3 = done
    LSS_LO,          // largest step known to have phi' < 0
    LSS_HI,          // bracket end with phi'(HI) >= 0 (< 0 means +infinity)
    LSS_FLO, LSS_HLO,   // phi', phi'' at LO
    LSS_FHI, LSS_HHI,   // phi', phi'' at HI (when HI_EVAL)
    LSS_HI_EVAL,     // 1 once phi'(HI) > 0 is known
    LSS_T0,          // LS_K trial steps (ascending) evaluated by the next pass
    LSS_ALPHA = LSS_T0 + LS_K,   // accepted step once done
    LSS_A,           // sum w |Vd|^2
    LSS_B,           // sum w Re(conj(R) Vd)
    LSS_AMAX,        // alpha_max (< 0 means +infinity)
    LSS_STOP,        // 1 if the channel has stopped
    LSS_N = 24
};
static_assert(LSS_STOP < LSS_N, "line-search state overflows its record");
static_assert(2 * LS_K <= NPART, "line-search partials overflow a partial record");

// Per-image flags / CG bookkeeping kept on the device (double).
enum {
    CH_GTD = 0,      // gt . d after projection
    CH_RESTART,      // 1 if the direction was reset to -gt this step
    CH_GG_OLD,       // |gt_old|^2
    CH_STOP,         // 1 once the channel has stopped (zero gradient or zero step)
    CH_E1,           // sum d (ln(I/M) + 1) of the step's direction
    CH_E2,           // sum d^2 / I
    CH_AMAX,         // alpha_max = min over d < 0 of (I - M)/(-d) (INFINITY if none)
    CH_PAD,
    CH_N = 8
};

// Arrival counters of the per-image reductions finished by the last
// workgroup to arrive ([CTR_N][nimg] unsigned, zero between launches).
enum {
    CTR_DIR = 0,     // k_cg_dir: gt . d, alpha_max and the entropy parts of phi', phi''
    CTR_VIS,         // k_cg_vis: a, b, phi'(alpha_max); line-search start
    CTR_LS,          // k_ls_step: phi', phi'' at the trial steps
    CTR_UPD,         // k_cg_update: S and chi^2 of the new image
    CTR_GRAD,        // k_grad: the Polak-Ribiere sums / Phi of an evaluation
    CTR_INIT,        // k_cg_init: |gt|^2
    CTR_N
};

}  // namespace uvm

struct uvmem_ctx {
    int n = 0, np = 0, nchan = 0, mode = 0, prec = 0;
    int nimg = 0;                      // image planes: nchan (cube) or 1 (shared)
    int fwd_model = 0;                 // UVMEM_FWD_DFT or UVMEM_FWD_GRIDDED
    int grad_model = 0;                // UVMEM_GRAD_ADJOINT or UVMEM_GRAD_DFT
    int grid_os = 1;                   // gridded model: Fourier grid side / N
    int grid_lg = 0;                   // gridded model: log2 of the grid side
    hipStream_t stream = nullptr;
    int device = 0;
    double cell = 0.0;
    bool cell_set = false;
    double M = 0.0, lam = 0.0;
    double Mb = 0.0;                   // smallest image value >= M in the image precision (the bound)
    bool prior_set = false;
    bool finalized = false;
    std::string err;

    // host staging (until finalize)
    std::vector<int64_t> nvis;
    std::vector<std::vector<double>> hu, hv;
    std::vector<std::vector<float>> hvis, hw, hbeam;
    std::vector<double> fwhm;
    std::vector<double> cx, cy;        // pointing centres (radians from the image centre)
    std::vector<char> has_uv, has_vis, has_w, has_beam;

    // layout
    std::vector<int64_t> off;          // channel offsets, size nchan+1
    int64_t ztot = 0;
    int ib_rows = 0, n_ib = 0;         // forward i-blocks (image rows per block)
    int jb_cols = 0, n_jb = 1;         // forward j-blocks (image columns per block)
    int n_fparts = 0;                  // forward partials per visibility: n_ib * n_jb
    int adj_tt = 0, adj_nt = 0;        // adjoint tile side, tiles per side
    int n_slots = 0;
    int n_pb = 0;                      // pixel blocks per image plane
    int pix_blk = 0;                   // pixels per pixel block (multiple of NTHR)
    int vis_blk = 0;                   // visibilities per visibility item (multiple of 2 NTHR)
    int ls_steps = 8;                  // line-search passes per CG step
    std::vector<int> h_slot_base;      // split-K slots per channel, nchan+1
    std::vector<int> h_vis_base;       // visibility items per channel, nchan+1
    std::vector<int> h_ivis_base;      // visibility items per image, nimg+1
    std::vector<int> h_ichan_base;     // channels per image, nimg+1
    std::vector<int> h_chan_img;       // image of each channel, nchan
    int n_adj = 0, n_visit = 0;

    // device buffers
    double *d_a = nullptr, *d_b = nullptr;      // u cell, v cell
    double2 *d_vo = nullptr;                    // observed V^o (rotated to the image centre for pointings)
    float *d_w = nullptr;
    void *d_beam = nullptr;                     // real [C][n][n]
    uvm::FwdPItem *d_fwdp = nullptr;
    int n_fwdp = 0;
    uvm::AdjItem *d_adj = nullptr;
    // focus of attention: work lists restricted to the region (the CG's
    // direction forward model and gradient adjoint), their partial count and
    // split-K slot table
    bool has_region = false;
    uvm::FwdPItem *d_fwdp_m = nullptr;
    int n_fwdp_m = 0, n_fparts_m = 0;
    uvm::AdjItem *d_adj_m = nullptr;
    int n_adj_m = 0, n_slots_m = 0;
    int *d_slot_base_m = nullptr;
    uvm::VisItem *d_vis = nullptr;
    int *d_slot_base = nullptr, *d_vis_base = nullptr;
    int *d_ivis_base = nullptr, *d_ichan_base = nullptr, *d_chan_img = nullptr;
    double2 *d_R = nullptr, *d_Vd = nullptr, *d_vpart = nullptr;
    void *d_gpart = nullptr;                    // split-K adjoint partials [slots][Np][Np]: FP64 or FP32
    bool gpart_f32 = false;                     // partials stored as FP32 (split paths; FP32 when every
                                                // chunk is one FP32 sum of at most ADJ_F32_SUM visibilities)
    void *d_bop = nullptr;                      // operand image [C][np][np]
    void *d_g = nullptr, *d_gt = nullptr, *d_dir = nullptr;  // real [nimg][n][n]
    double *d_scal = nullptr;                   // [nimg][NSCAL]
    double *d_chan = nullptr;                   // [nimg][CH_N]
    double *d_ls = nullptr;                     // [nimg][LSS_N] line-search state
    unsigned *d_ctr = nullptr;                  // [CTR_N][nimg] arrival counters
    double *d_ppart = nullptr;                  // [2][nimg][n_pb][NPART] (ping-pong)
    double *d_vispart = nullptr;                // [n_visit][NPART]
    int *d_flag = nullptr;                      // [4]: domain flag, ...
    double *d_wscale = nullptr;                 // [nimg] 1 / sum of the image's weights (0 if none)
    unsigned char *d_mask = nullptr;            // [nimg][N][N] focus-of-attention mask, or null
    std::vector<double> h_wsum;                 // sum of the weights per image
    std::vector<std::vector<unsigned char>> hmask;   // staged masks per image (empty = all free)
    // gridded forward model (Sec. 2.4): twiddles e^{-2 pi i k/L}, k < L/2;
    // row-pass buffer [C][N][L] (adjoint: [C][L][N]); spectrum [C][L][L]
    // (u index major); visibilities sorted by grid cell: per-channel cell
    // offsets [C][L*L + 1] into perm [ztot] (global visibility indices)
    // (visibility perm[j] is the j-th in cell order); bilinear fractions
    // (fx, fy) in that order; the weighted coefficients in that order
    void *d_gtw = nullptr, *d_gx1 = nullptr, *d_ggrid = nullptr;
    int *d_gcell = nullptr, *d_gperm = nullptr;
    double2 *d_gfxy = nullptr, *d_gsc = nullptr;
    // dense cells: per-cell index into the dense list ([C][L*L], -1 if not
    // dense), each dense cell's sorted range, and its four weighted sums
    int *d_gdidx = nullptr;
    int2 *d_gdlist = nullptr;
    double2 *d_gdsum = nullptr;
    int n_gdense = 0;
    size_t bytes_device = 0;

    // CG
    void *cg_I = nullptr;
    bool cg_ready = false;
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    void *graph_I = nullptr;
    hipStream_t cap_stream = nullptr;           // capture stream of the CG graph (made at finalize)
    long long *d_hist_ptr = nullptr;            // device copy of the cg_run history pointer
    long long *d_iter_ctr = nullptr;
    bool hist_in_grad = false;                  // set while a one-image CG step is captured: the
                                                // gradient pass's last workgroup writes the history
    // test hook (UVMEM_TEST_FAIL_ALLOC): index of the finalize allocation
    // that fails, -1 for none; allocations counted so far
    int fail_alloc_at = -1, n_alloc = 0;

    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pend[2];
    double t_ms[2] = {0, 0};
    int64_t t_cnt[2] = {0, 0};
};

namespace uvm {

// ---------------------------------------------------------------- launchers
// All return hipSuccess or the launch error; every launch goes to `st`.

// Forward DFT: vpart[part][k] = the image block's share of V_k (see
// k_dft.hip).  dir != 0: the operand is a CG direction, zero outside a focus
// region, and only the region's blocks are visited (compact partials).
hipError_t launch_forward(const uvmem_ctx *c, const void *bop, hipStream_t st, int dir = 0);
// Adjoint: gpart[slot] tiles of Re F^H (w coef) without the beam factor.
// grad != 0: a gradient, needed inside a focus region only (its own tiles
// and split-K slot table).
hipError_t launch_adjoint(const uvmem_ctx *c, const double2 *coef, const float *w, hipStream_t st, int grad = 0);
// Workgroups of that adjoint kernel resident on one CU at once (occupancy of
// the compiled kernel; at least 1).
int adjoint_wgs_per_cu(const uvmem_ctx *c);
// Gridded forward model and its exact adjoint (k_grid.hip): the forward
// writes the single forward partial vpart[0][k]; the adjoint writes the
// channel's plane gpart[slot_base[c]] (one slot per channel).
hipError_t launch_grid_forward(const uvmem_ctx *c, const void *bop, hipStream_t st);
hipError_t launch_grid_adjoint(const uvmem_ctx *c, const double2 *coef, const float *w, hipStream_t st);

// The FP32 forward on explicit buffers (the allocation-free entry point):
// image blocks ib_rows x jb_cols (128 x 256, 128 x 128 or 64 x 64), work
// items in device memory.
hipError_t launch_forward_f32_raw(int ib_rows, int jb_cols, const FwdPItem *items, int nitems, const double *a,
                                  const double *b, const float *bop, double2 *vpart, int n, int np,
                                  long long ztot, hipStream_t st);
// out[k] = sum over the n_parts forward partials of visibility k, for the
// visibility items in device memory.
hipError_t launch_vis_sum_raw(const VisItem *items, int n_items, const double2 *vpart, int n_parts, long long ztot,
                              double2 *out, hipStream_t st);

// Auxiliary kernels (k_aux.hip).
hipError_t launch_fill(const uvmem_ctx *c, void *img, double value, hipStream_t st);
// Fill a sum-Z complex visibility buffer with (re, im).
hipError_t launch_fill_c(const uvmem_ctx *c, double2 *x, double re, double im, hipStream_t st);
hipError_t launch_prologue(const uvmem_ctx *c, const void *I, int with_entropy, hipStream_t st);
hipError_t launch_vis_sum(const uvmem_ctx *c, int mode, double2 *out, hipStream_t st);
// Per-item max |coef| (slot 2 of the visibility partials) for the scaled
// fp16 adjoint; no-op for the other precisions.
hipError_t launch_coef_max(const uvmem_ctx *c, const double2 *coef, hipStream_t st);
// mode 1 (grad Phi of an evaluation) also writes Phi, chi^2 and S of every
// image to the context's scalars and to user_scal (may be null).
hipError_t launch_grad(const uvmem_ctx *c, const void *I, void *out, int mode, double *user_scal, hipStream_t st);
hipError_t launch_cg_init_dir(const uvmem_ctx *c, const void *I, hipStream_t st);
hipError_t launch_cg_step(const uvmem_ctx *c, void *I, double *user_scal, hipStream_t st);
// The CG step in three phases around the DFT launches (0: before the forward
// model, 1: between forward and adjoint, 2: after the adjoint).
hipError_t launch_cg_phase(const uvmem_ctx *c, void *I, double *user_scal, int phase, hipStream_t st);
hipError_t launch_copy_scal(const uvmem_ctx *c, double *dst, long long *ctr, hipStream_t st);
// Point the graph's history copy at `hist` (may be null) and reset its
// counter, by a one-thread kernel on `st` (no host memory involved).
hipError_t launch_set_hist(const uvmem_ctx *c, double *hist, hipStream_t st);

}  // namespace uvm
