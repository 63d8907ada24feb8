// Host side of the uvmem C ABI: argument checking, staging of the inputs,
// layout and work tables, device allocation, and the hot entry points, which
// only enqueue kernels on the context's stream.
#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <functional>
#include <queue>
#include <vector>

#include "internal.h"

using namespace uvm;

namespace {

int fail(uvmem_ctx *c, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(uvmem_ctx *c, int code, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(c, expr)                                                                       \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail((c), UVMEM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));          \
    } while (0)

size_t real_size(const uvmem_ctx *c) { return c->prec == UVMEM_FP64 ? sizeof(double) : sizeof(float); }

bool valid_chan(uvmem_ctx *c, int chan) { return chan >= 0 && chan < c->nchan; }

// Copy n bytes from a host or device pointer into host memory.
hipError_t fetch(void *dst, const void *src, size_t n) {
    if (n == 0) return hipSuccess;
    hipPointerAttribute_t at;
    hipError_t e = hipPointerGetAttributes(&at, src);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        std::memcpy(dst, src, n);
        return hipSuccess;
    }
    if (at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged)
        return hipMemcpy(dst, src, n, hipMemcpyDeviceToHost);
    std::memcpy(dst, src, n);
    return hipSuccess;
}

template <typename T>
hipError_t dalloc(uvmem_ctx *c, T **p, size_t count) {
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    // test hook: UVMEM_TEST_FAIL_ALLOC=k makes the k-th allocation of a
    // finalize fail as if the device were out of memory
    if (c->fail_alloc_at >= 0 && c->n_alloc++ == c->fail_alloc_at) return hipErrorOutOfMemory;
    hipError_t e = hipMalloc((void **)p, bytes);
    if (e == hipSuccess) {
        c->bytes_device += bytes;
        e = hipMemset(*p, 0, bytes);
    }
    return e;
}

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

// Release every device buffer, graph, stream and event of the context and
// reset the handles, so that a second call (destroy after a failed finalize)
// frees nothing twice.
void free_all(uvmem_ctx *c) {
    dfree(c->d_a); dfree(c->d_b); dfree(c->d_vo); dfree(c->d_w); dfree(c->d_beam);
    dfree(c->d_fwdp); dfree(c->d_adj); dfree(c->d_vis);
    dfree(c->d_slot_base); dfree(c->d_vis_base); dfree(c->d_ivis_base); dfree(c->d_ichan_base);
    dfree(c->d_chan_img);
    dfree(c->d_R); dfree(c->d_Vd); dfree(c->d_vpart); dfree(c->d_gpart); dfree(c->d_bop);
    dfree(c->d_g); dfree(c->d_gt); dfree(c->d_dir);
    dfree(c->d_scal); dfree(c->d_chan); dfree(c->d_ls); dfree(c->d_ctr); dfree(c->d_ppart); dfree(c->d_vispart);
    dfree(c->d_flag); dfree(c->d_hist_ptr); dfree(c->d_iter_ctr);
    dfree(c->d_gtw); dfree(c->d_gx1); dfree(c->d_ggrid); dfree(c->d_gcell); dfree(c->d_gperm);
    dfree(c->d_gfxy); dfree(c->d_gsc); dfree(c->d_gdidx); dfree(c->d_gdlist); dfree(c->d_gdsum);
    dfree(c->d_wscale); dfree(c->d_mask);
    dfree(c->d_fwdp_m); dfree(c->d_adj_m); dfree(c->d_slot_base_m);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    c->graph_I = nullptr;
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->cap_stream = nullptr;
    for (auto &pr : c->pend[0]) { c->ev_pool.push_back(pr.first); c->ev_pool.push_back(pr.second); }
    for (auto &pr : c->pend[1]) { c->ev_pool.push_back(pr.first); c->ev_pool.push_back(pr.second); }
    c->pend[0].clear();
    c->pend[1].clear();
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    c->ev_pool.clear();
    c->bytes_device = 0;
}

// ---------------------------------------------------------------- timing
void harvest(uvmem_ctx *c) {
    for (int w = 0; w < 2; ++w) {
        for (auto &pr : c->pend[w]) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
                c->t_ms[w] += ms;
                c->t_cnt[w] += 1;
            }
            c->ev_pool.push_back(pr.first);
            c->ev_pool.push_back(pr.second);
        }
        c->pend[w].clear();
    }
}

// Launch the forward (which = 0) or adjoint (which = 1) DFT, bracketed by
// events when timing is on.
// flag: the forward operand is a CG direction / the adjoint is a gradient
// (region-restricted work lists under a focus-of-attention mask).
hipError_t timed_dft(uvmem_ctx *c, int which, const void *bop, const double2 *coef, const float *w, int flag) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        if (c->ev_pool.size() < 2) {
            (void)hipStreamSynchronize(c->stream);
            harvest(c);
        }
        if (c->ev_pool.size() >= 2) {
            e0 = c->ev_pool.back(); c->ev_pool.pop_back();
            e1 = c->ev_pool.back(); c->ev_pool.pop_back();
            (void)hipEventRecord(e0, c->stream);
        }
    }
    hipError_t e = which == 0 ? launch_forward(c, bop, c->stream, flag) : launch_adjoint(c, coef, w, c->stream, flag);
    if (e0) {
        (void)hipEventRecord(e1, c->stream);
        c->pend[which].push_back({e0, e1});
    }
    return e;
}

int check_ready(uvmem_ctx *c) {
    if (!c) return UVMEM_EINVAL;
    if (!c->finalized) return fail(c, UVMEM_ESTATE, "context is not finalized");
    return UVMEM_OK;
}

// Completion time of work items with the given costs, dispatched in order
// onto `slots` identical resident-workgroup slots (each item starts on the
// slot that frees first).
double makespan(const std::vector<double> &costs, int slots) {
    std::priority_queue<double, std::vector<double>, std::greater<double>> q;
    for (int i = 0; i < slots; ++i) q.push(0.0);
    double end = 0.0;
    for (double w : costs) {
        const double t = q.top() + w;
        q.pop();
        q.push(t);
        end = std::max(end, t);
    }
    return end;
}

// Schedule choice for the DFT launches.  Candidate workgroup counts are
// multiples of the resident-slot count; each candidate's per-channel splits
// are simulated (longest items first) and the cheapest makespan wins; a
// larger candidate must beat the best so far by 2 % (near-ties go to fewer
// workgroups: fewer split-K partial planes to sum, fewer image-block
// stagings).  Measured against the candidates on six workloads, the pick is
// within 3 % of the fastest of them except on 64 uneven channels, where the
// gains of finer work lists sit near the margin.  `cost(m)` returns the
// items' costs for candidate m.
int pick_schedule(int slots, const std::function<std::vector<double>(int)> &cost) {
    static const int cand[] = {1, 2, 3, 4, 6, 8, 12, 16};
    int best = 1;
    double best_t = 0.0;
    for (int m : cand) {
        std::vector<double> w = cost(m);
        std::sort(w.begin(), w.end(), std::greater<double>());
        const double t = makespan(w, slots);
        if (m == 1 || t < 0.98 * best_t) { best = m; best_t = t; }
    }
    return best;
}

int build_layout(uvmem_ctx *c) {
    const int C = c->nchan;
    c->np = ((c->n + 63) / 64) * 64;
    // persistent forward: image blocks resident in LDS, 128 x 256 where the
    // size allows (FP32 and bf16 also sum at most 256 columns in one FP32
    // accumulator; the blocks are combined in FP64).  FP64 keeps 64 rows (its
    // accumulators take twice the registers) and takes up to 256 columns:
    // each tile's twiddle set-up and row dot then feed four times the products
    // of a 64 x 64 block (512^2 x 1.0M: forward 22.1 -> 17.2 ms)
    if (c->prec == UVMEM_FP64) {
        c->ib_rows = 64;
        c->jb_cols = c->np % 256 == 0 ? 256 : c->np % 128 == 0 ? 128 : 64;
    }
    else if (c->np % 256 == 0) { c->ib_rows = 128; c->jb_cols = 256; }
    else if (c->np % 128 == 0) { c->ib_rows = 128; c->jb_cols = 128; }
    else { c->ib_rows = 64; c->jb_cols = 64; }
    c->n_ib = c->np / c->ib_rows;
    c->n_jb = c->np / c->jb_cols;
    c->n_fparts = c->fwd_model == UVMEM_FWD_GRIDDED ? 1 : c->n_ib * c->n_jb;
    // adjoint pixel tile: 256 x 256 for the FP32 and split kernels where the
    // padded side allows (halves their table work per product), else 128 x 128
    // (FP64 too: its twiddle tables then feed four times the products of a
    // 64 x 64 tile, 512^2 x 1.0M: 22.9 -> 17.5 ms), else 64 x 64
    c->adj_tt = c->np % 128 == 0 ? 128 : 64;
    if (c->prec != UVMEM_FP64 && c->np % 256 == 0) c->adj_tt = 256;
    if (const char *env = std::getenv("UVMEM_ADJ_TILE")) {
        const int t = std::atoi(env);
        if ((t == 64 || t == 128 || (t == 256 && c->prec != UVMEM_FP64)) && c->np % t == 0)
            c->adj_tt = t;
    }
    c->adj_nt = c->np / c->adj_tt;
    c->ls_steps = LS_STEPS;
    if (const char *env = std::getenv("UVMEM_LS_STEPS")) c->ls_steps = std::max(1, std::min(64, std::atoi(env)));
    c->off.assign(C + 1, 0);
    for (int ch = 0; ch < C; ++ch) c->off[ch + 1] = c->off[ch] + c->nvis[ch];
    c->ztot = c->off[C];
    // pixel and visibility kernels: about PIX_WGS / VIS_WGS workgroups in
    // all (enough to spread the streaming over the CUs; few enough that the
    // last workgroup of an image sums a short list of partial records)
    auto roundup = [](int64_t x, int64_t m) { return ((x + m - 1) / m) * m; };
    int64_t pix_wgs = PIX_WGS, vis_wgs = VIS_WGS;
    if (const char *env = std::getenv("UVMEM_PIX_WGS")) pix_wgs = std::max(1L, std::atol(env));
    if (const char *env = std::getenv("UVMEM_VIS_WGS")) vis_wgs = std::max(1L, std::atol(env));
    const int64_t npix = (int64_t)c->n * c->n;
    c->pix_blk = (int)std::max<int64_t>(NTHR, roundup((npix * c->nimg + pix_wgs - 1) / pix_wgs, NTHR));
    c->n_pb = (int)((npix + c->pix_blk - 1) / c->pix_blk);
    c->vis_blk = (int)std::max<int64_t>(2 * NTHR, roundup((c->ztot + vis_wgs - 1) / vis_wgs, 2 * NTHR));
    return UVMEM_OK;
}

}  // namespace

extern "C" {

const char *uvmem_strerror(int code) {
    switch (code) {
    case UVMEM_OK: return "ok";
    case UVMEM_EINVAL: return "invalid argument";
    case UVMEM_ENOMEM: return "out of memory";
    case UVMEM_EDEVICE: return "HIP runtime error";
    case UVMEM_EDOMAIN: return "image pixel <= 0 or NaN";
    case UVMEM_ESTATE: return "call out of order";
    case UVMEM_ETOOBIG: return "sizes exceed the allocation-free scratch";
    default: return "unknown status";
    }
}

const char *uvmem_last_error(const uvmem_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int uvmem_create(uvmem_ctx **out, int n, int n_chan, int mode, int precision, void *hip_stream) {
    if (!out) return UVMEM_EINVAL;
    *out = nullptr;
    if (n < 2 || n > 8192 || (n % 2) != 0) return UVMEM_EINVAL;
    if (n_chan < 1 || n_chan > 65536) return UVMEM_EINVAL;
    if (mode != UVMEM_CUBE && mode != UVMEM_SHARED) return UVMEM_EINVAL;
    if (precision < UVMEM_FP64 || precision > UVMEM_FP16X3) return UVMEM_EINVAL;
    uvmem_ctx *c = new (std::nothrow) uvmem_ctx();
    if (!c) return UVMEM_ENOMEM;
    c->n = n;
    c->nchan = n_chan;
    c->mode = mode;
    c->nimg = mode == UVMEM_SHARED ? 1 : n_chan;
    c->prec = precision;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return UVMEM_EDEVICE;
    }
    c->nvis.assign(n_chan, 0);
    c->hu.resize(n_chan);
    c->hv.resize(n_chan);
    c->hvis.resize(n_chan);
    c->hw.resize(n_chan);
    c->hbeam.resize(n_chan);
    c->fwhm.assign(n_chan, 0.0);
    c->cx.assign(n_chan, 0.0);
    c->hmask.resize(c->nimg);
    c->cy.assign(n_chan, 0.0);
    c->has_uv.assign(n_chan, 0);
    c->has_vis.assign(n_chan, 0);
    c->has_w.assign(n_chan, 0);
    c->has_beam.assign(n_chan, 0);
    *out = c;
    return UVMEM_OK;
}

int uvmem_set_forward_model(uvmem_ctx *c, int model, int oversample, int grad) {
    if (!c) return UVMEM_EINVAL;
    if (c->finalized) return fail(c, UVMEM_ESTATE, "set_forward_model after finalize");
    if (grad != UVMEM_GRAD_ADJOINT && grad != UVMEM_GRAD_DFT) return fail(c, UVMEM_EINVAL, "bad gradient model %d", grad);
    if (model == UVMEM_FWD_DFT) {
        c->fwd_model = model;
        c->grad_model = UVMEM_GRAD_ADJOINT;
        c->grid_os = 1;
        c->grid_lg = 0;
        return UVMEM_OK;
    }
    if (model != UVMEM_FWD_GRIDDED) return fail(c, UVMEM_EINVAL, "bad forward model %d", model);
    const int64_t L = (int64_t)oversample * c->n;
    const int64_t lmax = c->prec == UVMEM_FP64 ? 4096 : 8192;
    if (oversample < 1 || L < 16 || L > lmax || (L & (L - 1)) != 0)
        return fail(c, UVMEM_EINVAL, "gridded model needs oversample * N a power of two in [16, %lld] (got %lld)",
                    (long long)lmax, (long long)L);
    c->fwd_model = model;
    c->grad_model = grad;
    c->grid_os = oversample;
    c->grid_lg = 0;
    while ((1LL << c->grid_lg) < L) ++c->grid_lg;
    return UVMEM_OK;
}

int uvmem_destroy(uvmem_ctx *ctx) {
    if (!ctx) return UVMEM_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (ctx->finalized) (void)hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    delete ctx;
    return UVMEM_OK;
}

int uvmem_set_uv(uvmem_ctx *c, int chan, int64_t nvis, const double *u, const double *v, double cell_rad) {
    if (!c) return UVMEM_EINVAL;
    if (c->finalized) return fail(c, UVMEM_ESTATE, "set_uv after finalize");
    if (!valid_chan(c, chan)) return fail(c, UVMEM_EINVAL, "channel %d out of range", chan);
    if (nvis < 0 || nvis > (int64_t)1 << 40) return fail(c, UVMEM_EINVAL, "bad nvis");
    if (nvis > 0 && (!u || !v)) return fail(c, UVMEM_EINVAL, "null u/v");
    if (!(cell_rad > 0.0) || !std::isfinite(cell_rad)) return fail(c, UVMEM_EINVAL, "bad cell");
    if (c->cell_set && cell_rad != c->cell)
        return fail(c, UVMEM_EINVAL, "cell differs between channels (one pixel grid)");
    // validate into temporaries: the channel's staged data change only on success
    std::vector<double> hu, hv;
    try {
        hu.resize(nvis);
        hv.resize(nvis);
    } catch (...) {
        return fail(c, UVMEM_ENOMEM, "host staging");
    }
    HIPCHK(c, fetch(hu.data(), u, nvis * sizeof(double)));
    HIPCHK(c, fetch(hv.data(), v, nvis * sizeof(double)));
    // at most 4096 cycles per pixel (8192 times the grid's Nyquist limit):
    // keeps the FP64 phases a m, and the FP32 twiddles' quarter-turn counts
    // 4 a m, far inside their exact ranges for any image side
    constexpr double UV_MAX_CYCLES = 4096.0;
    for (int64_t k = 0; k < nvis; ++k) {
        const double uk = hu[k], vk = hv[k];
        if (!std::isfinite(uk) || !std::isfinite(vk))
            return fail(c, UVMEM_EINVAL, "non-finite u/v at %lld", (long long)k);
        if (std::fabs(uk) * cell_rad > UV_MAX_CYCLES || std::fabs(vk) * cell_rad > UV_MAX_CYCLES)
            return fail(c, UVMEM_EINVAL, "u/v at %lld is beyond %g cycles per pixel", (long long)k, UV_MAX_CYCLES);
    }
    c->cell = cell_rad;
    c->cell_set = true;
    // new coordinates invalidate the channel's visibilities and weights
    // (their length may have changed): they must be set again
    c->nvis[chan] = nvis;
    c->hu[chan].swap(hu);
    c->hv[chan].swap(hv);
    std::vector<float>().swap(c->hvis[chan]);
    std::vector<float>().swap(c->hw[chan]);
    c->has_uv[chan] = 1;
    c->has_vis[chan] = nvis == 0;
    c->has_w[chan] = nvis == 0;
    return UVMEM_OK;
}

int uvmem_set_vis(uvmem_ctx *c, int chan, const float *vis) {
    if (!c) return UVMEM_EINVAL;
    if (c->finalized) return fail(c, UVMEM_ESTATE, "set_vis after finalize");
    if (!valid_chan(c, chan)) return fail(c, UVMEM_EINVAL, "channel %d out of range", chan);
    if (!c->has_uv[chan]) return fail(c, UVMEM_ESTATE, "set_vis before set_uv");
    const int64_t nv = c->nvis[chan];
    if (nv > 0 && !vis) return fail(c, UVMEM_EINVAL, "null vis");
    std::vector<float> hvis;
    try { hvis.resize(2 * nv); } catch (...) { return fail(c, UVMEM_ENOMEM, "host staging"); }
    HIPCHK(c, fetch(hvis.data(), vis, 2 * nv * sizeof(float)));
    for (int64_t k = 0; k < 2 * nv; ++k)
        if (!std::isfinite(hvis[k])) return fail(c, UVMEM_EINVAL, "visibility %lld is not finite", (long long)(k / 2));
    c->hvis[chan].swap(hvis);
    c->has_vis[chan] = 1;
    return UVMEM_OK;
}

int uvmem_set_weights(uvmem_ctx *c, int chan, const float *w) {
    if (!c) return UVMEM_EINVAL;
    if (c->finalized) return fail(c, UVMEM_ESTATE, "set_weights after finalize");
    if (!valid_chan(c, chan)) return fail(c, UVMEM_EINVAL, "channel %d out of range", chan);
    if (!c->has_uv[chan]) return fail(c, UVMEM_ESTATE, "set_weights before set_uv");
    const int64_t nv = c->nvis[chan];
    if (nv > 0 && !w) return fail(c, UVMEM_EINVAL, "null weights");
    std::vector<float> hw;
    try { hw.resize(nv); } catch (...) { return fail(c, UVMEM_ENOMEM, "host staging"); }
    HIPCHK(c, fetch(hw.data(), w, nv * sizeof(float)));
    for (int64_t k = 0; k < nv; ++k)
        if (!(hw[k] >= 0.0f) || !std::isfinite(hw[k]))
            return fail(c, UVMEM_EINVAL, "weight %lld is negative or not finite", (long long)k);
    c->hw[chan].swap(hw);
    c->has_w[chan] = 1;
    return UVMEM_OK;
}

int uvmem_set_beam(uvmem_ctx *c, int chan, double fwhm_rad) {
    if (!c) return UVMEM_EINVAL;
    if (c->finalized) return fail(c, UVMEM_ESTATE, "set_beam after finalize");
    if (!valid_chan(c, chan)) return fail(c, UVMEM_EINVAL, "channel %d out of range", chan);
    if (!(fwhm_rad > 0.0) || !std::isfinite(fwhm_rad)) return fail(c, UVMEM_EINVAL, "bad fwhm");
    c->fwhm[chan] = fwhm_rad;
    c->hbeam[chan].clear();
    c->has_beam[chan] = 1;
    return UVMEM_OK;
}

int uvmem_set_beam_image(uvmem_ctx *c, int chan, const float *A) {
    if (!c) return UVMEM_EINVAL;
    if (c->finalized) return fail(c, UVMEM_ESTATE, "set_beam_image after finalize");
    if (!valid_chan(c, chan)) return fail(c, UVMEM_EINVAL, "channel %d out of range", chan);
    if (!A) return fail(c, UVMEM_EINVAL, "null beam image");
    const size_t npix = (size_t)c->n * c->n;
    std::vector<float> hb;
    try { hb.resize(npix); } catch (...) { return fail(c, UVMEM_ENOMEM, "host staging"); }
    HIPCHK(c, fetch(hb.data(), A, npix * sizeof(float)));
    for (size_t p = 0; p < npix; ++p)
        if (!std::isfinite(hb[p])) return fail(c, UVMEM_EINVAL, "non-finite beam value");
    c->hbeam[chan].swap(hb);
    c->fwhm[chan] = 0.0;
    c->has_beam[chan] = 1;
    return UVMEM_OK;
}

int uvmem_set_phase_centre(uvmem_ctx *c, int chan, double x0_rad, double y0_rad) {
    if (!c) return UVMEM_EINVAL;
    if (c->finalized) return fail(c, UVMEM_ESTATE, "set_phase_centre after finalize");
    if (!valid_chan(c, chan)) return fail(c, UVMEM_EINVAL, "bad channel %d", chan);
    if (!std::isfinite(x0_rad) || !std::isfinite(y0_rad)) return fail(c, UVMEM_EINVAL, "non-finite centre");
    c->cx[chan] = x0_rad;
    c->cy[chan] = y0_rad;
    return UVMEM_OK;
}

int uvmem_set_mask(uvmem_ctx *c, int img, const uint8_t *mask) {
    if (!c) return UVMEM_EINVAL;
    if (c->finalized) return fail(c, UVMEM_ESTATE, "set_mask after finalize");
    if (img < 0 || img >= c->nimg) return fail(c, UVMEM_EINVAL, "bad image plane %d", img);
    if (!mask) {
        std::vector<unsigned char>().swap(c->hmask[img]);
        return UVMEM_OK;
    }
    std::vector<unsigned char> hm;
    try { hm.resize((size_t)c->n * c->n); } catch (...) { return fail(c, UVMEM_ENOMEM, "host staging"); }
    HIPCHK(c, fetch(hm.data(), mask, (size_t)c->n * c->n));
    for (auto &x : hm) x = x ? 1 : 0;
    c->hmask[img].swap(hm);
    return UVMEM_OK;
}

int uvmem_set_prior(uvmem_ctx *c, double M, double lambda) {
    if (!c) return UVMEM_EINVAL;
    if (c->finalized) return fail(c, UVMEM_ESTATE, "set_prior after finalize");
    if (!(M > 0.0) || !std::isfinite(M)) return fail(c, UVMEM_EINVAL, "M must be > 0");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(c, UVMEM_EINVAL, "lambda must be >= 0");
    c->M = M;
    c->lam = lambda;
    // the bound I >= M on the image's own number lattice: the smallest value
    // of the image precision that is >= M (M itself in FP64)
    if (c->prec == UVMEM_FP64) {
        c->Mb = M;
    } else {
        float f = (float)M;
        if ((double)f < M) f = std::nextafter(f, INFINITY);
        c->Mb = (double)f;
    }
    c->prior_set = true;
    return UVMEM_OK;
}

extern "C++" {
namespace {
int finalize_impl(uvmem_ctx *c);
}
}

int uvmem_finalize(uvmem_ctx *c) {
    if (!c) return UVMEM_EINVAL;
    if (c->finalized) return fail(c, UVMEM_ESTATE, "finalize called twice");
    // host-side tables may not fit in memory: no exception crosses the ABI
    try {
        return finalize_impl(c);
    } catch (const std::bad_alloc &) {
        free_all(c);
        return fail(c, UVMEM_ENOMEM, "host memory for the finalize tables");
    } catch (...) {
        free_all(c);
        return fail(c, UVMEM_EINVAL, "finalize failed");
    }
}

extern "C++" {
namespace {
int finalize_impl(uvmem_ctx *c) {
    const int C = c->nchan;
    for (int ch = 0; ch < C; ++ch) {
        if (!c->has_uv[ch]) return fail(c, UVMEM_ESTATE, "channel %d has no uv", ch);
        if (!c->has_vis[ch]) return fail(c, UVMEM_ESTATE, "channel %d has no visibilities", ch);
        if (!c->has_w[ch]) return fail(c, UVMEM_ESTATE, "channel %d has no weights", ch);
        if (!c->has_beam[ch]) return fail(c, UVMEM_ESTATE, "channel %d has no beam", ch);
    }
    if (!c->prior_set) return fail(c, UVMEM_ESTATE, "prior not set");
    if (c->fwd_model == UVMEM_FWD_GRIDDED) {
        int64_t z = 0;
        for (int ch = 0; ch < C; ++ch) z += c->nvis[ch];
        const int64_t L = (int64_t)1 << c->grid_lg;
        if (z > (int64_t)INT32_MAX - 1) return fail(c, UVMEM_EINVAL, "gridded model: more than 2^31 visibilities");
        if ((int64_t)C * (L * L + 1) > ((int64_t)1 << 30))
            return fail(c, UVMEM_ENOMEM, "gridded model: cell tables of %d channels x %lld^2 cells too large", C,
                        (long long)L);
    }
    HIPCHK(c, hipSetDevice(c->device));
    c->fail_alloc_at = -1;
    c->n_alloc = 0;
    if (const char *env = std::getenv("UVMEM_TEST_FAIL_ALLOC")) c->fail_alloc_at = std::atoi(env);
    build_layout(c);
    const int n = c->n, np = c->np;
    const size_t npix = (size_t)n * n;
    const size_t rs = real_size(c);

    // ---- work tables
    std::vector<VisItem> vis;
    c->h_vis_base.assign(C + 1, 0);
    for (int ch = 0; ch < C; ++ch) {
        const int64_t b = c->off[ch], e = c->off[ch + 1];
        c->h_vis_base[ch] = (int)vis.size();
        for (int64_t k = b; k < e; k += c->vis_blk)
            vis.push_back(VisItem{ch, 0, (long long)k, (long long)std::min<int64_t>(k + c->vis_blk, e)});
    }
    c->h_vis_base[C] = (int)vis.size();
    // focus of attention: the union of the image planes' masks decides which
    // forward image blocks and adjoint pixel tiles the CG's direction
    // forward model and gradient adjoint visit (outside it the direction is
    // zero and the gradient is not needed)
    std::vector<unsigned char> umask;
    bool region = false;
    if (c->fwd_model == UVMEM_FWD_DFT) {
        umask.assign((size_t)n * n, 0);
        for (int m = 0; m < c->nimg; ++m) {
            if (c->hmask[m].empty()) { umask.assign((size_t)n * n, 1); break; }
            for (size_t p = 0; p < (size_t)n * n; ++p) umask[p] |= c->hmask[m][p];
        }
        for (size_t p = 0; p < umask.size() && !region; ++p) region = !umask[p];
    }
    auto rect_used = [&](int r0, int r1, int c0, int c1) {
        for (int i = r0; i < std::min(r1, n); ++i)
            for (int j = c0; j < std::min(c1, n); ++j)
                if (umask[(size_t)i * n + j]) return true;
        return false;
    };
    // ---- adjoint: split-K chunks.  Resident slots: 256 CUs x the workgroups
    // of the context's adjoint kernel that fit on a CU at once (1 for the
    // 512-thread 256 x 256 tiles, 2-3 for the 256-thread 128 x 128 and 64 x
    // 64 tiles, from the compiled kernel's occupancy).  A channel of Z_c
    // visibilities is cut into ceil(Z_c / klen) equal chunks (multiples of 16)
    // and every chunk covers the used pixel tiles; the split kernel's chunks
    // are also bounded because it sums a chunk in FP32 only.
    const bool split = c->prec == UVMEM_BF16X3 || c->prec == UVMEM_FP16X3;
    const int adj_slots = 256 * adjoint_wgs_per_cu(c);
    auto chunks_of = [&](int64_t nv, int64_t klen, int64_t &len) {
        const int64_t nch = (nv + klen - 1) / klen;
        len = nch ? ((nv + nch - 1) / nch + 15) / 16 * 16 : 0;
        return nch;
    };
    // the gridded model's own adjoint writes one plane per channel
    const bool grid_adj = c->fwd_model == UVMEM_FWD_GRIDDED && c->grad_model == UVMEM_GRAD_ADJOINT;
    auto build_adj = [&](const std::vector<char> &tile_used, std::vector<AdjItem> &adj,
                         std::vector<int> &slot_base) {
        int tiles = 0;
        for (char t : tile_used) tiles += t ? 1 : 0;
        auto adj_klen = [&](int64_t target) {
            int64_t klen = (c->ztot * std::max(tiles, 1) + target - 1) / target;
            klen = std::max<int64_t>(klen, ADJ_KMIN);
            if (split) klen = std::min<int64_t>(klen, ADJ_KMAX_SPLIT);
            return ((klen + 15) / 16) * 16;
        };
        constexpr double ADJ_OVERHEAD = 64.0;   // per-workgroup set-up and tile store, in visibilities
        const int adj_m = pick_schedule(adj_slots, [&](int m) {
            std::vector<double> w;
            const int64_t klen = adj_klen((int64_t)adj_slots * m);
            for (int ch = 0; ch < C; ++ch) {
                int64_t len;
                const int64_t nch = chunks_of(c->nvis[ch], klen, len);
                for (int64_t x = 0; x < nch; ++x) {
                    const double z = (double)std::min<int64_t>(len, c->nvis[ch] - x * len);
                    for (int t = 0; t < tiles; ++t) w.push_back(z + ADJ_OVERHEAD);
                }
            }
            return w;
        });
        int64_t klen = adj_klen((int64_t)adj_slots * adj_m);
        if (const char *env = std::getenv("UVMEM_ADJ_WGS")) klen = adj_klen(std::max(1L, std::atol(env)));
        slot_base.assign(C + 1, 0);
        int slot = 0;
        for (int ch = 0; ch < C; ++ch) {
            const int64_t b = c->off[ch], e = c->off[ch + 1];
            slot_base[ch] = slot;
            if (grid_adj) {
                ++slot;
                continue;
            }
            int64_t len;
            chunks_of(e - b, klen, len);
            for (int64_t k = b; k < e; k += len, ++slot)
                for (int ti = 0; ti < c->adj_nt; ++ti)
                    for (int tj = 0; tj < c->adj_nt; ++tj)
                        if (tile_used[(size_t)ti * c->adj_nt + tj])
                            adj.push_back(AdjItem{ch, ti, tj, slot, (long long)k,
                                                  (long long)std::min<int64_t>(k + len, e)});
        }
        slot_base[C] = slot;
        // longest chunks first (the slot of an item fixes its place in the
        // split-K sum, so the order of the items is free)
        std::stable_sort(adj.begin(), adj.end(), [](const AdjItem &x, const AdjItem &y) {
            return x.kend - x.kbeg > y.kend - y.kbeg;
        });
        return slot;
    };
    std::vector<AdjItem> adj, adj_m;
    std::vector<int> slot_base_m;
    const int ntile = c->adj_nt * c->adj_nt;
    int slot = build_adj(std::vector<char>(ntile, 1), adj, c->h_slot_base);
    int slots_m = 0;
    if (region) {
        std::vector<char> used(ntile, 0);
        for (int ti = 0; ti < c->adj_nt; ++ti)
            for (int tj = 0; tj < c->adj_nt; ++tj)
                used[(size_t)ti * c->adj_nt + tj] =
                    rect_used(ti * c->adj_tt, (ti + 1) * c->adj_tt, tj * c->adj_tt, (tj + 1) * c->adj_tt);
        slots_m = build_adj(used, adj_m, slot_base_m);
    }
    // ---- persistent forward: one resident workgroup per CU; the
    // (channel, image block) pairs are shared by g_c workgroups each, with
    // g_c = ceil(Z_c / L) for the per-workgroup visibility count L chosen by
    // the same simulation.  part_of[b] is the forward partial that block b
    // writes, -1 for a block left out.
    auto build_fwd = [&](const std::vector<int> &part_of, std::vector<FwdPItem> &fwdp) {
        int nblk = 0;
        for (int x : part_of) nblk += x >= 0 ? 1 : 0;
        if (c->ztot == 0 || nblk == 0) return;
        // image-block staging and start-up per workgroup, in visibilities: on
        // 64 uneven channels 256 kept the lists at 1,536 workgroups while
        // 3,072-4,096 ran the forward 4-5 % faster; 128 picks 3,072 there and
        // leaves single-channel workloads at one workgroup per CU
        constexpr double FWD_OVERHEAD = 128.0;
        auto shares = [&](int64_t wgs, int ch) {
            const int64_t nv = c->nvis[ch];
            const int64_t L = std::max<int64_t>(16, (c->ztot * nblk + wgs - 1) / wgs);
            const int64_t tl = (nv + 15) / 16;   // 16-visibility wave tiles
            return std::max<int64_t>(1, std::min<int64_t>((nv + L - 1) / L, (tl + 7) / 8));
        };
        int fwd_m = pick_schedule(256, [&](int m) {
            std::vector<double> w;
            for (int ch = 0; ch < C; ++ch) {
                if (c->nvis[ch] == 0) continue;
                const int64_t g = shares(256LL * m, ch);
                for (int b = 0; b < nblk; ++b)
                    for (int64_t x = 0; x < g; ++x) w.push_back((double)c->nvis[ch] / (double)g + FWD_OVERHEAD);
            }
            return w;
        });
        int64_t wgs = 256LL * fwd_m;
        if (const char *env = std::getenv("UVMEM_FWD_WGS")) wgs = std::max(1L, std::atol(env));
        for (int ch = 0; ch < C; ++ch) {
            if (c->nvis[ch] == 0) continue;
            const int64_t g = shares(wgs, ch);
            for (int ib = 0; ib < c->n_ib; ++ib)
                for (int jb = 0; jb < c->n_jb; ++jb) {
                    const int part = part_of[(size_t)ib * c->n_jb + jb];
                    if (part < 0) continue;
                    for (int64_t x = 0; x < g; ++x)
                        fwdp.push_back(FwdPItem{ch, ib, jb, part, (int)x, (int)g, (long long)c->off[ch],
                                                (long long)c->off[ch + 1]});
                }
        }
        std::stable_sort(fwdp.begin(), fwdp.end(), [&](const FwdPItem &x, const FwdPItem &y) {
            return (double)c->nvis[x.chan] / x.nwg > (double)c->nvis[y.chan] / y.nwg;
        });
    };
    std::vector<FwdPItem> fwdp, fwdp_m;
    c->n_fparts_m = 0;
    if (c->fwd_model == UVMEM_FWD_DFT) {
        const int nblk = c->n_ib * c->n_jb;
        std::vector<int> part_of(nblk);
        for (int b = 0; b < nblk; ++b) part_of[b] = b;
        build_fwd(part_of, fwdp);
        if (region) {
            for (int ib = 0; ib < c->n_ib; ++ib)
                for (int jb = 0; jb < c->n_jb; ++jb)
                    part_of[(size_t)ib * c->n_jb + jb] =
                        rect_used(ib * c->ib_rows, (ib + 1) * c->ib_rows, jb * c->jb_cols, (jb + 1) * c->jb_cols)
                            ? c->n_fparts_m++
                            : -1;
            build_fwd(part_of, fwdp_m);
        }
    }
    // the 256-tile FP32 adjoint folds at most ADJ_F32_SUM visibilities per
    // FP32 sum; when no chunk is longer, its partials are single FP32 sums and are
    // stored as such (half the traffic of the split-K planes)
    int64_t maxchunk = 0;
    for (auto &x : adj) maxchunk = std::max<int64_t>(maxchunk, x.kend - x.kbeg);
    for (auto &x : adj_m) maxchunk = std::max<int64_t>(maxchunk, x.kend - x.kbeg);
    c->gpart_f32 = split || (c->prec == UVMEM_FP32 && c->adj_tt == 256 && !grid_adj && maxchunk <= ADJ_F32_SUM);
    c->n_fwdp = (int)fwdp.size();
    c->n_fwdp_m = (int)fwdp_m.size();
    c->n_adj_m = (int)adj_m.size();
    c->n_slots_m = slots_m;
    c->has_region = region;
    // image planes: channel ranges, visibility-item ranges, channel -> image
    const int IMG = c->nimg;
    c->h_ichan_base.assign(IMG + 1, 0);
    c->h_ivis_base.assign(IMG + 1, 0);
    c->h_chan_img.assign(C, 0);
    for (int m = 0; m <= IMG; ++m) c->h_ichan_base[m] = IMG == C ? m : (m == 0 ? 0 : C);
    for (int m = 0; m <= IMG; ++m) c->h_ivis_base[m] = c->h_vis_base[c->h_ichan_base[m]];
    for (int ch = 0; ch < C; ++ch) c->h_chan_img[ch] = IMG == C ? ch : 0;
    c->n_slots = slot;
    c->n_adj = (int)adj.size();
    c->n_visit = (int)vis.size();

    // ---- host-side conversions
    std::vector<double> a(c->ztot), bb(c->ztot);
    std::vector<double> vo(2 * c->ztot);
    std::vector<float> w(c->ztot);
    for (int ch = 0; ch < C; ++ch) {
        const int64_t o = c->off[ch];
        for (int64_t k = 0; k < c->nvis[ch]; ++k) {
            a[o + k] = c->hu[ch][k] * c->cell;
            bb[o + k] = c->hv[ch][k] * c->cell;
            if (c->cx[ch] != 0.0 || c->cy[ch] != 0.0) {
                // phase reference moved from the pointing centre to the image
                // centre: V^o e^{-2 pi i (u x0 + v y0)}, phase reduced mod 1
                const double ph = c->hu[ch][k] * c->cx[ch] + c->hv[ch][k] * c->cy[ch];
                const double f = ph - std::nearbyint(ph);
                const double cs = std::cos(2.0 * M_PI * f), sn = std::sin(2.0 * M_PI * f);
                const double re = c->hvis[ch][2 * k], im = c->hvis[ch][2 * k + 1];
                vo[2 * (o + k)] = re * cs + im * sn;
                vo[2 * (o + k) + 1] = im * cs - re * sn;
            } else {
                vo[2 * (o + k)] = c->hvis[ch][2 * k];
                vo[2 * (o + k) + 1] = c->hvis[ch][2 * k + 1];
            }
            w[o + k] = c->hw[ch][k];
        }
    }
    // ---- gridded model: twiddles (FP64, rounded to the transform type) and
    // the visibilities sorted by grid cell (counting sort per channel, stable,
    // so each cell keeps increasing visibility order).  The cell of a
    // visibility is computed exactly as the kernels do: floor(a L), mod L.
    const bool gridded = c->fwd_model == UVMEM_FWD_GRIDDED;
    const int GL = gridded ? 1 << c->grid_lg : 0;
    const size_t gcells = (size_t)GL * GL;
    std::vector<char> gtw;
    std::vector<int> gcell, gperm;
    std::vector<double> gfxy;
    std::vector<int> gdidx, gdlist;
    if (gridded) {
        const size_t csz = 2 * rs;
        gtw.resize((size_t)(GL / 2) * csz);
        for (int k = 0; k < GL / 2; ++k) {
            const double ang = -2.0 * M_PI * (double)k / (double)GL;
            const double re = std::cos(ang), im = std::sin(ang);
            if (rs == 8) {
                reinterpret_cast<double *>(gtw.data())[2 * k] = re;
                reinterpret_cast<double *>(gtw.data())[2 * k + 1] = im;
            } else {
                reinterpret_cast<float *>(gtw.data())[2 * k] = (float)re;
                reinterpret_cast<float *>(gtw.data())[2 * k + 1] = (float)im;
            }
        }
        gcell.assign((size_t)C * (gcells + 1), 0);
        gperm.assign(c->ztot, 0);
        std::vector<int> cellof(c->ztot);
        for (int ch = 0; ch < C; ++ch) {
            int *cs = gcell.data() + (size_t)ch * (gcells + 1);
            std::vector<int> cnt(gcells, 0);
            for (int64_t k = c->off[ch]; k < c->off[ch + 1]; ++k) {
                const long long px = (long long)std::floor(a[k] * (double)GL);
                const long long py = (long long)std::floor(bb[k] * (double)GL);
                const int cell = (int)((px & (GL - 1)) * GL + (py & (GL - 1)));
                cellof[k] = cell;
                ++cnt[cell];
            }
            int64_t pos = c->off[ch];
            for (size_t t = 0; t < gcells; ++t) {
                cs[t] = (int)pos;
                pos += cnt[t];
            }
            cs[gcells] = (int)pos;
            std::vector<int> fill(cs, cs + gcells);
            for (int64_t k = c->off[ch]; k < c->off[ch + 1]; ++k) gperm[fill[cellof[k]]++] = (int)k;
        }
        gdidx.assign((size_t)C * gcells, -1);
        for (int ch = 0; ch < C; ++ch) {
            const int *cs = gcell.data() + (size_t)ch * (gcells + 1);
            for (size_t t = 0; t < gcells; ++t)
                if (cs[t + 1] - cs[t] > GRID_DENSE) {
                    gdidx[(size_t)ch * gcells + t] = (int)(gdlist.size() / 2);
                    gdlist.push_back(cs[t]);
                    gdlist.push_back(cs[t + 1]);
                }
        }
        c->n_gdense = (int)(gdlist.size() / 2);
        gfxy.resize(2 * (size_t)c->ztot);
        for (int64_t j = 0; j < c->ztot; ++j) {
            const int64_t k = gperm[j];
            const double gx = a[k] * (double)GL, gy = bb[k] * (double)GL;
            gfxy[2 * j] = gx - std::floor(gx);
            gfxy[2 * j + 1] = gy - std::floor(gy);
        }
    }

    c->h_wsum.assign(c->nimg, 0.0);
    for (int ch = 0; ch < C; ++ch)
        for (int64_t k = 0; k < c->nvis[ch]; ++k) c->h_wsum[c->nimg == C ? ch : 0] += (double)c->hw[ch][k];
    std::vector<double> wscale(c->nimg);
    for (int m = 0; m < c->nimg; ++m) wscale[m] = c->h_wsum[m] > 0.0 ? 1.0 / c->h_wsum[m] : 0.0;
    bool any_mask = false;
    for (auto &mk : c->hmask) any_mask = any_mask || !mk.empty();
    std::vector<unsigned char> mask;
    if (any_mask) {
        mask.assign((size_t)c->nimg * npix, 1);
        for (int m = 0; m < c->nimg; ++m)
            if (!c->hmask[m].empty()) std::memcpy(mask.data() + (size_t)m * npix, c->hmask[m].data(), npix);
    }

    std::vector<char> beam(C * npix * rs);
    for (int ch = 0; ch < C; ++ch) {
        for (size_t p = 0; p < npix; ++p) {
            double A;
            if (!c->hbeam[ch].empty()) {
                A = c->hbeam[ch][p];
            } else {
                const double x = (double)((int)(p % n) - n / 2) * c->cell - c->cx[ch];
                const double y = (double)((int)(p / n) - n / 2) * c->cell - c->cy[ch];
                A = std::exp(-4.0 * std::log(2.0) * (x * x + y * y) / (c->fwhm[ch] * c->fwhm[ch]));
            }
            if (rs == 8) reinterpret_cast<double *>(beam.data())[ch * npix + p] = A;
            else reinterpret_cast<float *>(beam.data())[ch * npix + p] = (float)A;
        }
    }

    // ---- device allocation
    hipError_t e = hipSuccess;
    auto ok = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    ok(dalloc(c, &c->d_a, c->ztot));
    ok(dalloc(c, &c->d_b, c->ztot));
    ok(dalloc(c, &c->d_vo, c->ztot));
    ok(dalloc(c, &c->d_w, c->ztot));
    ok(dalloc(c, (char **)&c->d_beam, C * npix * rs));
    ok(dalloc(c, &c->d_fwdp, fwdp.size()));
    ok(dalloc(c, &c->d_adj, adj.size()));
    ok(dalloc(c, &c->d_vis, vis.size()));
    ok(dalloc(c, &c->d_slot_base, C + 1));
    ok(dalloc(c, &c->d_vis_base, C + 1));
    ok(dalloc(c, &c->d_ivis_base, IMG + 1));
    ok(dalloc(c, &c->d_ichan_base, IMG + 1));
    ok(dalloc(c, &c->d_chan_img, C));
    ok(dalloc(c, &c->d_R, c->ztot));
    ok(dalloc(c, &c->d_Vd, c->ztot));
    ok(dalloc(c, &c->d_vpart, (size_t)c->n_fparts * c->ztot));
    ok(dalloc(c, (char **)&c->d_gpart,
              (size_t)std::max(c->n_slots, c->n_slots_m) * np * np * (c->gpart_f32 ? sizeof(float) : sizeof(double))));
    if (region) {
        ok(dalloc(c, &c->d_fwdp_m, fwdp_m.size()));
        ok(dalloc(c, &c->d_adj_m, adj_m.size()));
        ok(dalloc(c, &c->d_slot_base_m, C + 1));
    }
    ok(dalloc(c, (char **)&c->d_bop, (size_t)C * np * np * rs));
    ok(dalloc(c, (char **)&c->d_g, IMG * npix * rs));
    ok(dalloc(c, (char **)&c->d_gt, IMG * npix * rs));
    ok(dalloc(c, (char **)&c->d_dir, IMG * npix * rs));
    ok(dalloc(c, &c->d_scal, (size_t)IMG * UVMEM_NSCAL));
    ok(dalloc(c, &c->d_chan, (size_t)IMG * CH_N));
    ok(dalloc(c, &c->d_ls, (size_t)IMG * LSS_N));
    ok(dalloc(c, &c->d_ctr, (size_t)CTR_N * IMG));
    ok(dalloc(c, &c->d_ppart, (size_t)2 * IMG * c->n_pb * NPART));
    ok(dalloc(c, &c->d_vispart, (size_t)std::max(c->n_visit, 1) * NPART));
    ok(dalloc(c, &c->d_flag, 4));
    ok(dalloc(c, &c->d_hist_ptr, 1));
    ok(dalloc(c, &c->d_iter_ctr, 1));
    ok(dalloc(c, &c->d_wscale, (size_t)c->nimg));
    if (any_mask) ok(dalloc(c, &c->d_mask, mask.size()));
    if (gridded) {
        ok(dalloc(c, (char **)&c->d_gtw, gtw.size()));
        ok(dalloc(c, (char **)&c->d_gx1, (size_t)C * n * GL * 2 * rs));
        ok(dalloc(c, (char **)&c->d_ggrid, (size_t)C * gcells * 2 * rs));
        ok(dalloc(c, &c->d_gcell, gcell.size()));
        ok(dalloc(c, &c->d_gperm, gperm.size()));
        ok(dalloc(c, &c->d_gfxy, c->ztot));
        ok(dalloc(c, &c->d_gsc, c->ztot));
        ok(dalloc(c, &c->d_gdidx, gdidx.size()));
        ok(dalloc(c, &c->d_gdlist, (size_t)c->n_gdense));
        ok(dalloc(c, &c->d_gdsum, (size_t)c->n_gdense * 4));
    }
    if (e != hipSuccess) {
        free_all(c);
        (void)hipGetLastError();
        return fail(c, e == hipErrorOutOfMemory ? UVMEM_ENOMEM : UVMEM_EDEVICE, "device allocation: %s",
                    hipGetErrorString(e));
    }
    auto up = [&](void *dst, const void *src, size_t bytes) {
        if (bytes && e == hipSuccess) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    up(c->d_a, a.data(), a.size() * 8);
    up(c->d_b, bb.data(), bb.size() * 8);
    up(c->d_vo, vo.data(), vo.size() * 8);
    up(c->d_w, w.data(), w.size() * 4);
    up(c->d_beam, beam.data(), beam.size());
    up(c->d_fwdp, fwdp.data(), fwdp.size() * sizeof(FwdPItem));
    up(c->d_adj, adj.data(), adj.size() * sizeof(AdjItem));
    up(c->d_vis, vis.data(), vis.size() * sizeof(VisItem));
    up(c->d_slot_base, c->h_slot_base.data(), (C + 1) * sizeof(int));
    up(c->d_vis_base, c->h_vis_base.data(), (C + 1) * sizeof(int));
    up(c->d_ivis_base, c->h_ivis_base.data(), (IMG + 1) * sizeof(int));
    up(c->d_ichan_base, c->h_ichan_base.data(), (IMG + 1) * sizeof(int));
    up(c->d_chan_img, c->h_chan_img.data(), C * sizeof(int));
    up(c->d_wscale, wscale.data(), wscale.size() * sizeof(double));
    if (region) {
        up(c->d_fwdp_m, fwdp_m.data(), fwdp_m.size() * sizeof(FwdPItem));
        up(c->d_adj_m, adj_m.data(), adj_m.size() * sizeof(AdjItem));
        up(c->d_slot_base_m, slot_base_m.data(), (C + 1) * sizeof(int));
    }
    if (any_mask) up(c->d_mask, mask.data(), mask.size());
    if (gridded) {
        up(c->d_gtw, gtw.data(), gtw.size());
        up(c->d_gcell, gcell.data(), gcell.size() * sizeof(int));
        up(c->d_gperm, gperm.data(), gperm.size() * sizeof(int));
        up(c->d_gfxy, gfxy.data(), gfxy.size() * sizeof(double));
        up(c->d_gdidx, gdidx.data(), gdidx.size() * sizeof(int));
        up(c->d_gdlist, gdlist.data(), gdlist.size() * sizeof(int));
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        free_all(c);
        (void)hipGetLastError();
        return fail(c, UVMEM_EDEVICE, "upload: %s", hipGetErrorString(e));
    }
    e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_all(c);
        (void)hipGetLastError();
        return fail(c, UVMEM_EDEVICE, "finalize: %s", hipGetErrorString(e));
    }
    // release host staging
    for (int ch = 0; ch < C; ++ch) {
        std::vector<double>().swap(c->hu[ch]);
        std::vector<double>().swap(c->hv[ch]);
        std::vector<float>().swap(c->hvis[ch]);
        std::vector<float>().swap(c->hw[ch]);
        std::vector<float>().swap(c->hbeam[ch]);
    }
    c->finalized = true;
    return UVMEM_OK;
}
}  // namespace
}  // extern "C++"

int uvmem_phi_and_grad(uvmem_ctx *c, const void *I, void *grad, double *scal) {
    int s = check_ready(c);
    if (s) return s;
    if (!I || !grad) return fail(c, UVMEM_EINVAL, "null image or gradient");
    HIPCHK(c, launch_prologue(c, I, 1, c->stream));
    HIPCHK(c, timed_dft(c, 0, c->d_bop, nullptr, nullptr, 0));
    HIPCHK(c, launch_vis_sum(c, 1, nullptr, c->stream));
    HIPCHK(c, timed_dft(c, 1, nullptr, c->d_R, c->d_w, 1));
    HIPCHK(c, launch_grad(c, I, grad, 1, scal, c->stream));
    return UVMEM_OK;
}

int uvmem_forward(uvmem_ctx *c, const void *I, void *vis) {
    int s = check_ready(c);
    if (s) return s;
    if (!I || (!vis && c->ztot)) return fail(c, UVMEM_EINVAL, "null image or output");
    HIPCHK(c, launch_prologue(c, I, 0, c->stream));
    HIPCHK(c, timed_dft(c, 0, c->d_bop, nullptr, nullptr, 0));
    HIPCHK(c, launch_vis_sum(c, 0, (double2 *)vis, c->stream));
    return UVMEM_OK;
}

int uvmem_adjoint(uvmem_ctx *c, const void *coef, void *img) {
    int s = check_ready(c);
    if (s) return s;
    if ((!coef && c->ztot) || !img) return fail(c, UVMEM_EINVAL, "null coefficients or output");
    HIPCHK(c, launch_coef_max(c, (const double2 *)coef, c->stream));
    HIPCHK(c, timed_dft(c, 1, nullptr, (const double2 *)coef, nullptr, 0));
    HIPCHK(c, launch_grad(c, nullptr, img, 0, nullptr, c->stream));
    return UVMEM_OK;
}

int uvmem_get_residual(uvmem_ctx *c, void *res) {
    int s = check_ready(c);
    if (s) return s;
    if (!res && c->ztot) return fail(c, UVMEM_EINVAL, "null output");
    if (c->ztot)
        HIPCHK(c, hipMemcpyAsync(res, c->d_R, c->ztot * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
    return UVMEM_OK;
}

int uvmem_dirty_image(uvmem_ctx *c, void *dirty, void *psf) {
    int s = check_ready(c);
    if (s) return s;
    if (dirty) {
        HIPCHK(c, launch_coef_max(c, c->d_vo, c->stream));
        HIPCHK(c, launch_adjoint(c, c->d_vo, c->d_w, c->stream));
        HIPCHK(c, launch_grad(c, nullptr, dirty, 3, nullptr, c->stream));
    }
    if (psf) {
        HIPCHK(c, launch_fill_c(c, c->d_Vd, 1.0, 0.0, c->stream));
        HIPCHK(c, launch_coef_max(c, c->d_Vd, c->stream));
        HIPCHK(c, launch_adjoint(c, c->d_Vd, c->d_w, c->stream));
        HIPCHK(c, launch_grad(c, nullptr, psf, 3, nullptr, c->stream));
    }
    return UVMEM_OK;
}

int uvmem_noise(const uvmem_ctx *c, double *sigma_d) {
    if (!c || !sigma_d) return UVMEM_EINVAL;
    if (!c->finalized) return UVMEM_ESTATE;
    for (int m = 0; m < c->nimg; ++m) sigma_d[m] = c->h_wsum[m] > 0.0 ? 1.0 / std::sqrt(c->h_wsum[m]) : INFINITY;
    return UVMEM_OK;
}

extern "C++" {
namespace {
// Elliptical Gaussian fitted to the main lobe of one PSF plane: the pixels
// with PSF >= 1/2 connected to the centre pixel (4-neighbours), least
// squares of -ln PSF = A dx^2 + B dx dy + C dy^2 (the peak is 1 at the
// centre by construction).  Returns false when the lobe is too small or the
// fitted form is not positive definite.
template <typename R>
bool fit_beam_plane(const R *psf, int n, double cell, double &bmaj, double &bmin, double &bpa) {
    const int c0 = n / 2;
    std::vector<char> seen((size_t)n * n, 0);
    std::vector<int> stack{c0 * n + c0};
    seen[(size_t)c0 * n + c0] = 1;
    double S[3][3] = {{0}}, t[3] = {0};
    int count = 0;
    while (!stack.empty()) {
        const int p = stack.back();
        stack.pop_back();
        const int i = p / n, j = p % n;
        const double val = (double)psf[p];
        if (!(val >= 0.5)) continue;
        if (val > 0.0 && (i != c0 || j != c0)) {
            const double dx = j - c0, dy = i - c0;
            const double phi[3] = {dx * dx, dx * dy, dy * dy};
            const double y = -std::log(val);
            for (int a = 0; a < 3; ++a) {
                t[a] += phi[a] * y;
                for (int b = 0; b < 3; ++b) S[a][b] += phi[a] * phi[b];
            }
            ++count;
        }
        const int nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
        for (auto &q : nb) {
            if (q[0] < 0 || q[0] >= n || q[1] < 0 || q[1] >= n) continue;
            const size_t id = (size_t)q[0] * n + q[1];
            if (!seen[id]) { seen[id] = 1; stack.push_back((int)id); }
        }
    }
    if (count < 3) return false;
    // 3 x 3 solve by Cramer's rule
    auto det3 = [](const double m[3][3]) {
        return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
               m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
    };
    const double D = det3(S);
    if (!(std::fabs(D) > 0.0)) return false;
    double x[3];
    for (int k = 0; k < 3; ++k) {
        double M[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) M[a][b] = b == k ? t[a] : S[a][b];
        x[k] = det3(M) / D;
    }
    const double A = x[0], B = x[1], Cq = x[2];
    const double mid = 0.5 * (A + Cq), rad = std::sqrt(0.25 * (A - Cq) * (A - Cq) + 0.25 * B * B);
    const double lmin = mid - rad, lmax = mid + rad;
    if (!(lmin > 0.0)) return false;
    // major axis: eigenvector of the smaller eigenvalue
    double ex = 0.5 * B, ey = lmin - A;
    if (std::fabs(ex) + std::fabs(ey) < 1e-300 * (std::fabs(A) + std::fabs(Cq))) { ex = lmin - Cq; ey = 0.5 * B; }
    if (std::fabs(ex) + std::fabs(ey) == 0.0) { ex = A <= Cq ? 1.0 : 0.0; ey = A <= Cq ? 0.0 : 1.0; }
    bmaj = 2.0 * std::sqrt(std::log(2.0) / lmin) * cell;
    bmin = 2.0 * std::sqrt(std::log(2.0) / lmax) * cell;
    double ang = std::atan2(ex, ey) * 180.0 / M_PI;   // from +y towards +x
    while (ang > 90.0) ang -= 180.0;
    while (ang <= -90.0) ang += 180.0;
    bpa = ang;
    return true;
}
}  // namespace
}  // extern "C++"

int uvmem_fit_beam(uvmem_ctx *c, const void *psf, double *bmaj, double *bmin, double *bpa) {
    int s = check_ready(c);
    if (s) return s;
    if (!psf || !bmaj || !bmin || !bpa) return fail(c, UVMEM_EINVAL, "null argument");
    const size_t npix = (size_t)c->n * c->n;
    std::vector<char> host(c->nimg * npix * real_size(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(host.data(), psf, host.size(), hipMemcpyDeviceToHost));
    for (int m = 0; m < c->nimg; ++m) {
        const bool okf = c->prec == UVMEM_FP64
            ? fit_beam_plane(reinterpret_cast<const double *>(host.data()) + m * npix, c->n, c->cell, bmaj[m],
                             bmin[m], bpa[m])
            : fit_beam_plane(reinterpret_cast<const float *>(host.data()) + m * npix, c->n, c->cell, bmaj[m],
                             bmin[m], bpa[m]);
        if (!okf) return fail(c, UVMEM_EDOMAIN, "image %d: PSF main lobe cannot be fitted", m);
    }
    return UVMEM_OK;
}

int uvmem_cg_init(uvmem_ctx *c, void *I, int init_to_floor) {
    int s = check_ready(c);
    if (s) return s;
    if (!I) return fail(c, UVMEM_EINVAL, "null image");
    if (init_to_floor) HIPCHK(c, launch_fill(c, I, c->Mb, c->stream));
    s = uvmem_phi_and_grad(c, I, c->d_g, nullptr);
    if (s) return s;
    HIPCHK(c, launch_cg_init_dir(c, I, c->stream));
    c->cg_I = I;
    c->cg_ready = true;
    return UVMEM_OK;
}

int uvmem_cg_step(uvmem_ctx *c, void *I, double *scal) {
    int s = check_ready(c);
    if (s) return s;
    if (!c->cg_ready) return fail(c, UVMEM_ESTATE, "cg_step before cg_init");
    if (I != c->cg_I) return fail(c, UVMEM_EINVAL, "cg_step image differs from cg_init's");
    HIPCHK(c, launch_cg_phase(c, I, scal, 0, c->stream));
    HIPCHK(c, timed_dft(c, 0, c->d_bop, nullptr, nullptr, 1));
    HIPCHK(c, launch_cg_phase(c, I, scal, 1, c->stream));
    HIPCHK(c, timed_dft(c, 1, nullptr, c->d_R, c->d_w, 1));
    HIPCHK(c, launch_cg_phase(c, I, scal, 2, c->stream));
    return UVMEM_OK;
}

int uvmem_cg_run(uvmem_ctx *c, void *I, int iters, double *hist, int use_graph) {
    int s = check_ready(c);
    if (s) return s;
    if (!c->cg_ready) return fail(c, UVMEM_ESTATE, "cg_run before cg_init");
    if (I != c->cg_I) return fail(c, UVMEM_EINVAL, "cg_run image differs from cg_init's");
    if (iters < 0) return fail(c, UVMEM_EINVAL, "negative iteration count");
    const size_t stride = (size_t)c->nimg * UVMEM_NSCAL;
    if (!use_graph) {
        for (int t = 0; t < iters; ++t) {
            s = uvmem_cg_step(c, I, hist ? hist + t * stride : nullptr);
            if (s) return s;
        }
        return UVMEM_OK;
    }
    if (!c->graph_exec || c->graph_I != I) {
        // first graph call on this image: capture one step (and the history
        // copy) on the capture stream made at finalize and instantiate it
        if (c->graph_exec) { (void)hipGraphExecDestroy(c->graph_exec); c->graph_exec = nullptr; }
        if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
        c->graph_I = nullptr;
        hipStream_t cap = c->cap_stream;
        // graph launches go to the context's stream, so a replay still runs
        // after the work queued there before it
        // with one image the gradient pass's last workgroup writes the
        // history row itself (one launch less per replay)
        c->hist_in_grad = c->nimg == 1;
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) e = launch_cg_step(c, I, nullptr, cap);
        if (e == hipSuccess && !c->hist_in_grad) e = launch_copy_scal(c, nullptr, c->d_iter_ctr, cap);
        c->hist_in_grad = false;
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cap, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            c->graph_exec = nullptr;
            return fail(c, UVMEM_EDEVICE, "graph capture: %s", hipGetErrorString(e));
        }
        c->graph = g;
        c->graph_I = I;
    }
    // point the history copy at the caller's buffer and reset the counter:
    // a kernel argument carries the pointer, so nothing waits for the host
    HIPCHK(c, launch_set_hist(c, hist, c->stream));
    for (int t = 0; t < iters; ++t) HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
    return UVMEM_OK;
}

namespace {
struct StateHeader {
    uint64_t magic;
    int32_t n, nchan, prec, mode;
    int32_t fwd_model, grid_lg, grad_model, pad;
    int64_t ztot;
};
const uint64_t STATE_MAGIC = 0x33534d454d5655ull;  // "UVMEMS3"
}  // namespace

int uvmem_cg_get_state(uvmem_ctx *c, void *blob, size_t *bytes) {
    int s = check_ready(c);
    if (s) return s;
    if (!bytes) return fail(c, UVMEM_EINVAL, "null size");
    const size_t img = (size_t)c->nimg * c->n * c->n * real_size(c);
    const size_t need = sizeof(StateHeader) + 3 * img + c->ztot * sizeof(double2) +
                        (size_t)c->nimg * (UVMEM_NSCAL + CH_N) * sizeof(double);
    if (!blob) { *bytes = need; return UVMEM_OK; }
    if (*bytes < need) return fail(c, UVMEM_EINVAL, "state buffer too small (%zu < %zu)", *bytes, need);
    if (!c->cg_ready) return fail(c, UVMEM_ESTATE, "no CG state");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    char *p = (char *)blob;
    StateHeader h{STATE_MAGIC, c->n, c->nchan, c->prec, c->mode, c->fwd_model, c->grid_lg, c->grad_model, 0, c->ztot};
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    HIPCHK(c, hipMemcpy(p, c->d_dir, img, hipMemcpyDeviceToHost)); p += img;
    HIPCHK(c, hipMemcpy(p, c->d_gt, img, hipMemcpyDeviceToHost)); p += img;
    HIPCHK(c, hipMemcpy(p, c->d_g, img, hipMemcpyDeviceToHost)); p += img;
    if (c->ztot) HIPCHK(c, hipMemcpy(p, c->d_R, c->ztot * sizeof(double2), hipMemcpyDeviceToHost));
    p += c->ztot * sizeof(double2);
    HIPCHK(c, hipMemcpy(p, c->d_scal, c->nimg * UVMEM_NSCAL * sizeof(double), hipMemcpyDeviceToHost));
    p += c->nimg * UVMEM_NSCAL * sizeof(double);
    HIPCHK(c, hipMemcpy(p, c->d_chan, c->nimg * CH_N * sizeof(double), hipMemcpyDeviceToHost));
    *bytes = need;
    return UVMEM_OK;
}

int uvmem_cg_set_state(uvmem_ctx *c, const void *blob, size_t bytes) {
    int s = check_ready(c);
    if (s) return s;
    if (!blob) return fail(c, UVMEM_EINVAL, "null state");
    if (!c->cg_ready) return fail(c, UVMEM_ESTATE, "cg_set_state before cg_init");
    const size_t img = (size_t)c->nimg * c->n * c->n * real_size(c);
    const size_t need = sizeof(StateHeader) + 3 * img + c->ztot * sizeof(double2) +
                        (size_t)c->nimg * (UVMEM_NSCAL + CH_N) * sizeof(double);
    if (bytes < need) return fail(c, UVMEM_EINVAL, "state blob too small");
    StateHeader h;
    std::memcpy(&h, blob, sizeof h);
    if (h.magic != STATE_MAGIC || h.n != c->n || h.nchan != c->nchan || h.prec != c->prec || h.mode != c->mode ||
        h.fwd_model != c->fwd_model || h.grid_lg != c->grid_lg || h.grad_model != c->grad_model ||
        h.ztot != c->ztot)
        return fail(c, UVMEM_EINVAL, "state blob does not match this context");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const char *p = (const char *)blob + sizeof h;
    HIPCHK(c, hipMemcpy(c->d_dir, p, img, hipMemcpyHostToDevice)); p += img;
    HIPCHK(c, hipMemcpy(c->d_gt, p, img, hipMemcpyHostToDevice)); p += img;
    HIPCHK(c, hipMemcpy(c->d_g, p, img, hipMemcpyHostToDevice)); p += img;
    if (c->ztot) HIPCHK(c, hipMemcpy(c->d_R, p, c->ztot * sizeof(double2), hipMemcpyHostToDevice));
    p += c->ztot * sizeof(double2);
    HIPCHK(c, hipMemcpy(c->d_scal, p, c->nimg * UVMEM_NSCAL * sizeof(double), hipMemcpyHostToDevice));
    p += c->nimg * UVMEM_NSCAL * sizeof(double);
    HIPCHK(c, hipMemcpy(c->d_chan, p, c->nimg * CH_N * sizeof(double), hipMemcpyHostToDevice));
    return UVMEM_OK;
}

int uvmem_check(uvmem_ctx *c) {
    int s = check_ready(c);
    if (s) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int flag[4] = {0, 0, 0, 0};
    HIPCHK(c, hipMemcpy(flag, c->d_flag, sizeof flag, hipMemcpyDeviceToHost));
    if (flag[0]) {
        int zero[4] = {0, 0, 0, 0};
        HIPCHK(c, hipMemcpy(c->d_flag, zero, sizeof zero, hipMemcpyHostToDevice));
        return fail(c, UVMEM_EDOMAIN, "an image pixel was <= 0 or NaN");
    }
    HIPCHK(c, hipGetLastError());
    return UVMEM_OK;
}

int uvmem_timing_enable(uvmem_ctx *c, int enable) {
    if (!c) return UVMEM_EINVAL;
    if (enable && c->ev_pool.empty()) {
        for (int i = 0; i < 512; ++i) {
            hipEvent_t e;
            HIPCHK(c, hipEventCreate(&e));
            c->ev_pool.push_back(e);
        }
    }
    c->timing = enable != 0;
    return UVMEM_OK;
}

int uvmem_timing_read(uvmem_ctx *c, int which, double *total_ms, int64_t *count, int reset) {
    if (!c || which < 0 || which > 1) return UVMEM_EINVAL;
    if (c->finalized) HIPCHK(c, hipStreamSynchronize(c->stream));
    harvest(c);
    if (total_ms) *total_ms = c->t_ms[which];
    if (count) *count = c->t_cnt[which];
    if (reset) {
        c->t_ms[which] = 0.0;
        c->t_cnt[which] = 0;
    }
    return UVMEM_OK;
}

int uvmem_info(const uvmem_ctx *c, int64_t *out, int nout) {
    if (!c || !out) return UVMEM_EINVAL;
    const int64_t vals[] = {c->n, c->np, c->nchan, c->prec, c->ztot, c->n_fparts, c->adj_tt, c->n_slots,
                            c->n_fwdp, c->n_adj, c->n_visit, (int64_t)c->bytes_device, c->n_pb, c->pix_blk,
                            c->vis_blk, c->nimg, c->fwd_model,
                            c->fwd_model == UVMEM_FWD_GRIDDED ? (int64_t)1 << c->grid_lg : 0, c->grad_model,
                            c->n_fwdp_m, c->n_adj_m};
    const int nv = (int)(sizeof vals / sizeof vals[0]);
    for (int i = 0; i < nout && i < nv; ++i) out[i] = vals[i];
    return UVMEM_OK;
}

int uvmem_chan_range(const uvmem_ctx *c, int chan, int64_t *offset, int64_t *nvis) {
    if (!c || chan < 0 || chan >= c->nchan) return UVMEM_EINVAL;
    int64_t o = 0;
    for (int ch = 0; ch < chan; ++ch) o += c->nvis[ch];
    if (offset) *offset = o;
    if (nvis) *nvis = c->nvis[chan];
    return UVMEM_OK;
}

}  // extern "C"
