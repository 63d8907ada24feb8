// Streaming kernels around the DFT contractions: attenuation prologue,
// visibility sums (residual, chi^2, line-search scalars), gradient
// finalisation with the entropy term, and the projected-CG step.
//
// Every reduction is FP64 and has a fixed order: a workgroup sums its
// elements in a fixed thread/stride pattern, then across waves in LDS; the
// per-channel totals sum the workgroup partials in index order.  Consumers
// that need a per-channel total recompute it from the partials themselves
// (every workgroup of the channel gets the same bits), which keeps each CG
// phase to one launch without atomics.
#include <cmath>
#include <type_traits>

#include "internal.h"

namespace uvm {
namespace {

// ---------------------------------------------------------------- reductions
// Sum K doubles over the workgroup; every thread receives the totals.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K]) {
    __shared__ double red[K][NTHR / 64];
#pragma unroll
    for (int x = 0; x < K; ++x) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[x] += __shfl_xor(v[x], o, 64);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int x = 0; x < K; ++x) red[x][wave] = v[x];
    }
    __syncthreads();
#pragma unroll
    for (int x = 0; x < K; ++x) v[x] = (red[x][0] + red[x][1]) + (red[x][2] + red[x][3]);
}

__device__ __forceinline__ double block_min(double v) {
    __shared__ double red[NTHR / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

// Partial records are written and read at device coherence (relaxed
// agent-scope atomic stores and loads: they bypass the caches that are not
// coherent between the chiplets), so that the workgroup that finishes a
// reduction in the same launch reads every other workgroup's record.
__device__ __forceinline__ void coh_store(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void coh_store(float *p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double coh_load(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum slot `s` (K slots starting at s0) of n_items partial records of NPART
// doubles starting at `base`, in index order (strided per thread, then the
// fixed workgroup reduction).
template <int K>
__device__ __forceinline__ void sum_partials(const double *base, int n_items, int s0, double (&out)[K]) {
#pragma unroll
    for (int x = 0; x < K; ++x) out[x] = 0.0;
    for (int it = threadIdx.x; it < n_items; it += NTHR) {
#pragma unroll
        for (int x = 0; x < K; ++x) out[x] += coh_load(base + (size_t)it * NPART + s0 + x);
    }
    block_sum<K>(out);
}

// Two record sets in one pass, their loads issued together (one memory round
// trip instead of two): slots [s0, s0 + K) of na records at `a` and slots
// [s1, s1 + L) of nb records at `b`, each summed in index order exactly as
// sum_partials does.  Past a set's end a thread reads a stand-in record of
// the other set (never of an empty one) and adds -0.0, an exact identity.
template <int K, int L>
__device__ __forceinline__ void sum_partials2(const double *a, int na, int s0, double (&oa)[K], const double *b,
                                              int nb, int s1, double (&ob)[L]) {
    double v[K + L];
#pragma unroll
    for (int x = 0; x < K + L; ++x) v[x] = 0.0;
    const int nmax = na > nb ? na : nb;
    for (int it = threadIdx.x; it < nmax; it += NTHR) {
        const bool oka = it < na, okb = it < nb;
        const double *ra = oka ? a + (size_t)it * NPART + s0 : b + (size_t)it * NPART + s1;
        const double *rb = okb ? b + (size_t)it * NPART + s1 : ra;
        double la[K], lb[L];
#pragma unroll
        for (int x = 0; x < K; ++x) la[x] = coh_load(ra + (oka ? x : 0));
#pragma unroll
        for (int x = 0; x < L; ++x) lb[x] = coh_load(rb + (okb ? x : 0));
#pragma unroll
        for (int x = 0; x < K; ++x) v[x] += oka ? la[x] : -0.0;
#pragma unroll
        for (int x = 0; x < L; ++x) v[K + x] += okb ? lb[x] : -0.0;
    }
    block_sum<K + L>(v);
#pragma unroll
    for (int x = 0; x < K; ++x) oa[x] = v[x];
#pragma unroll
    for (int x = 0; x < L; ++x) ob[x] = v[K + x];
}

// Sums of slots [0, K) and minima of slots [K, K + MN) of n_items records,
// one pass over the records (the sums in the order of sum_partials).
template <int K, int MN>
__device__ __forceinline__ void sum_min_partials(const double *base, int n_items, double (&sums)[K],
                                                 double (&mins)[MN]) {
#pragma unroll
    for (int x = 0; x < K; ++x) sums[x] = 0.0;
#pragma unroll
    for (int x = 0; x < MN; ++x) mins[x] = INFINITY;
    for (int it = threadIdx.x; it < n_items; it += NTHR) {
        double l[K + MN];
#pragma unroll
        for (int x = 0; x < K + MN; ++x) l[x] = coh_load(base + (size_t)it * NPART + x);
#pragma unroll
        for (int x = 0; x < K; ++x) sums[x] += l[x];
#pragma unroll
        for (int x = 0; x < MN; ++x) mins[x] = fmin(mins[x], l[K + x]);
    }
    block_sum<K>(sums);
#pragma unroll
    for (int x = 0; x < MN; ++x) mins[x] = block_min(mins[x]);
}

// Arrival at the end of a partial-sum pass, once thread 0 has stored this
// workgroup's partial record (coh_store): returns true (in every thread) in
// exactly one workgroup per image and launch, the last to arrive at `ctr`,
// which may then read every record of the image (coh_load) and finish the
// image's reduction in a fixed order.  Thread 0 waits for its record's store
// to complete before it counts itself in, so the last arrival finds every
// record in place.  The counter only elects that workgroup (the sums never
// depend on arrival order) and is left at zero for the next launch; no
// workgroup waits for another.
__device__ __forceinline__ bool arrive_last(unsigned *ctr, unsigned expected) {
    __shared__ unsigned s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);   // this workgroup's record stored
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const unsigned t = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const bool last = t + 1 == expected;
        if (last) __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = last ? 1u : 0u;
    }
    __syncthreads();
    return s_last != 0;
}

// ---------------------------------------------------------------- fill
template <typename R>
__global__ void k_fill(R *__restrict__ x, R value, long long count) {
    long long i = (long long)blockIdx.x * NTHR + threadIdx.x;
    long long stride = (long long)gridDim.x * NTHR;
    for (; i < count; i += stride) x[i] = value;
}

// ---------------------------------------------------------------- prologue
// B = A o I written into the padded operand image; optional entropy partial
// S = sum I ln(I/M) and the domain flag (I <= 0 or NaN).
template <typename R>
__global__ __launch_bounds__(NTHR) void k_prologue(const R *__restrict__ I, const R *__restrict__ beam,
                                                   R *__restrict__ bop, const int *__restrict__ ichan_base,
                                                   double *__restrict__ ppart,
                                                   int *__restrict__ flag, int n, int np, int n_pb, int pb_len,
                                                   double M, int with_entropy) {
    const int c = blockIdx.x / n_pb, pb = blockIdx.x % n_pb;   // image plane, pixel block
    const long long npix = (long long)n * n;
    const R *Ic = I + (size_t)c * npix;
    const int ch0 = ichan_base[c], ch1 = ichan_base[c + 1];   // the channels that see this image
    double s[1] = {0.0};
    int bad = 0;
    for (int r = 0; r < pb_len / NTHR; ++r) {
        long long p = (long long)pb * pb_len + r * NTHR + threadIdx.x;
        if (p >= npix) break;
        const int i = (int)(p / n), j = (int)(p % n);
        const R x = Ic[p];
        for (int ch = ch0; ch < ch1; ++ch)
            bop[(size_t)ch * np * np + (size_t)i * np + j] = beam[(size_t)ch * npix + p] * x;
        if (with_entropy) {
            const double xd = (double)x;
            if (!(xd > 0.0)) bad = 1;
            else s[0] += xd * log(xd / M);
        }
    }
    if (with_entropy) {
        if (bad) atomicOr(flag, 1);
        block_sum<1>(s);
        if (threadIdx.x == 0) coh_store(ppart + ((size_t)c * n_pb + pb) * NPART + 0, s[0]);
    }
}

// ---------------------------------------------------------------- visibilities
// mode 0: out[k] = V_k (model visibilities)
// mode 1: R_k = V_k - Vo_k -> R; partial[0] = sum w |R|^2
// mode 2: Vd_k = V_k -> Vd; partial[0] = sum w |Vd|^2, partial[1] = sum w Re(conj(R) Vd)
// mode 3: R_k += alpha_c Vd_k; partial[0] = sum w |R|^2
// mode 4: R is a caller's coefficient vector, only read (w may be null)
// with_max (modes 1, 3, 4): partial[2] = max over the item of w max(|Re R|, |Im R|)
// One visibility item (index `item`); `alpha` is the step length of mode 3.
__device__ __forceinline__ void vis_item(const VisItem it, int item, const double2 *__restrict__ vpart,
                                         int n_parts, long long ztot, const double2 *__restrict__ vo,
                                         const float *__restrict__ w, double2 *__restrict__ R,
                                         double2 *__restrict__ Vd, double2 *__restrict__ out,
                                         double *__restrict__ vispart, int mode, int with_max, double alpha) {
    double acc[2] = {0.0, 0.0};
    double cmax = 0.0;   // max |Re|, |Im| of the adjoint's coefficients w R (mode 4: R alone)
    constexpr int U = 2;   // visibilities per thread and round, loads issued together
    for (long long k0 = it.kbeg; k0 < it.kend; k0 += U * NTHR) {
        // the loads that do not depend on the forward partials are issued
        // first, then every block's partials (four blocks in flight), which
        // are summed in block order; indices past the item's end are clamped
        // and null arrays replaced by the partials, so that no load sits
        // behind a branch (values loaded that way are never used)
        const double2 *anyv = vpart ? vpart : R;
        const float *wsrc = w ? w : reinterpret_cast<const float *>(anyv);
        const double2 *lsrc = mode == 1 ? vo : mode >= 2 ? R : anyv;
        const double2 *l2src = mode == 3 ? Vd : anyv;
        double ww[U];
        double2 ld[U], ld2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long k = k0 + threadIdx.x + (long long)u * NTHR;
            const long long kc = k < it.kend ? k : it.kend - 1;
            const float wr = wsrc[kc];
            ww[u] = w ? (double)wr : 1.0;
            ld[u] = lsrc[kc];
            ld2[u] = l2src[kc];
        }
        double2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = make_double2(0.0, 0.0);
        if (mode < 3) {
            constexpr int PB = 4;
            for (int ib0 = 0; ib0 < n_parts; ib0 += PB) {
                double2 pv[PB][U];
#pragma unroll
                for (int b = 0; b < PB; ++b)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const long long k = k0 + threadIdx.x + (long long)u * NTHR;
                        const long long kc = k < it.kend ? k : it.kend - 1;
                        const int ibc = ib0 + b < n_parts ? ib0 + b : n_parts - 1;
                        pv[b][u] = vpart[(size_t)ibc * ztot + kc];
                    }
                // blocks past the last add -0.0, an exact identity (no branch
                // between the loads and the sums)
#pragma unroll
                for (int b = 0; b < PB; ++b) {
                    const bool okb = ib0 + b < n_parts;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        v[u].x += okb ? pv[b][u].x : -0.0;
                        v[u].y += okb ? pv[b][u].y : -0.0;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long k = k0 + threadIdx.x + (long long)u * NTHR;
            if (k >= it.kend) continue;
            const double wv = ww[u];
            if (mode == 0) {
                out[k] = v[u];
            } else if (mode == 1) {
                const double2 o = ld[u];
                const double2 r = make_double2(v[u].x - (double)o.x, v[u].y - (double)o.y);
                R[k] = r;
                acc[0] += wv * (r.x * r.x + r.y * r.y);
                cmax = fmax(cmax, wv * fmax(fabs(r.x), fabs(r.y)));
            } else if (mode == 2) {
                Vd[k] = v[u];
                const double2 r = ld[u];
                acc[0] += wv * (v[u].x * v[u].x + v[u].y * v[u].y);
                acc[1] += wv * (r.x * v[u].x + r.y * v[u].y);
            } else if (mode == 3) {
                const double2 d = ld2[u];
                double2 r = ld[u];
                r.x += alpha * d.x;
                r.y += alpha * d.y;
                R[k] = r;
                acc[0] += wv * (r.x * r.x + r.y * r.y);
                cmax = fmax(cmax, wv * fmax(fabs(r.x), fabs(r.y)));
            } else {
                const double2 r = ld[u];
                cmax = fmax(cmax, wv * fmax(fabs(r.x), fabs(r.y)));
            }
        }
    }
    if (mode != 0 && mode != 4) {
        block_sum<2>(acc);
        if (threadIdx.x == 0) {
            coh_store(vispart + (size_t)item * NPART + 0, acc[0]);
            coh_store(vispart + (size_t)item * NPART + 1, acc[1]);
        }
    }
    if (with_max && mode != 0 && mode != 2) {
        cmax = -block_min(-cmax);
        if (threadIdx.x == 0) coh_store(vispart + (size_t)item * NPART + 2, cmax);
    }
}

__device__ void ls_init(double *st, double a, double b, double e1, double e2, double amax, bool stop,
                        bool am_eval, double f_am, double h_am);

// Visibility pass over the context's items (modes 0, 1, 3 and 4 above).
__global__ __launch_bounds__(NTHR) void k_vis(const VisItem *__restrict__ items,
                                              const double2 *__restrict__ vpart, int n_parts, long long ztot,
                                              const double2 *__restrict__ vo, const float *__restrict__ w,
                                              double2 *__restrict__ R, double2 *__restrict__ Vd,
                                              double2 *__restrict__ out, const double *__restrict__ scal,
                                              double *__restrict__ vispart, const int *__restrict__ chan_img,
                                              int mode, int with_max) {
    const VisItem it = items[blockIdx.x];
    const int img = chan_img ? chan_img[it.chan] : 0;
    const double alpha = mode == 3 ? scal[(size_t)img * UVMEM_NSCAL + UVMEM_S_ALPHA] : 0.0;
    vis_item(it, blockIdx.x, vpart, n_parts, ztot, vo, w, R, Vd, out, vispart, mode, with_max, alpha);
}

// ---------------------------------------------------------------- gradient
// G = sum over the channel's split-K slots of gpart (fixed order);
// mode 0: out = A o G (adjoint only)
// mode 1: out = A o G + lambda (ln(I/M) + 1)            (grad Phi)
// mode 2: as 1 into g; gt = g with zeros on the active set; partials
//         [0] = gt_new . gt_new, [1] = gt_new . gt_old; gt updated in place.
// mode 3: out = scale_img x G without the attenuation (dirty image / PSF).
// With a focus-of-attention mask, pixels outside it are not free: modes 1
// and 2 write 0 there (gradient and projected gradient).
// Image totals finished by the last workgroup of an image (modes 1 and 2):
//   mode 1: Phi, chi^2 (from the visibility pass's partials) and S (from the
//           prologue's partials) into the scalars and, if given, `user`;
//   mode 2: the Polak-Ribiere beta (clipped at 0), |gt|^2 and the iteration
//           count; all scalars copied to `user`.
struct GradTail {
    unsigned *ctr;
    const double *vispart;
    const int *ivis_base;
    const double *pp_S;
    double *scal;
    double *chan;
    double *user;
    // graph replays of a one-image CG step: the history buffer's address and
    // the replay counter (the scalars go to row *hist_ctr); null otherwise
    const long long *hist_ptr;
    long long *hist_ctr;
};

template <typename R, int RP, typename PT>
__global__ __launch_bounds__(NTHR) void k_grad(const PT *__restrict__ gpart, const int *__restrict__ slot_base,
                                               const int *__restrict__ ichan_base,
                                               const R *__restrict__ beam, const R *__restrict__ I,
                                               R *__restrict__ out, R *__restrict__ gt,
                                               double *__restrict__ ppart, const double *__restrict__ img_scale,
                                               const unsigned char *__restrict__ mask, int n, int np, int n_pb,
                                               int pb_len, double M, double Mb, double lam, int mode,
                                               GradTail tail) {
    const int c = blockIdx.x / n_pb, pb = blockIdx.x % n_pb;
    const long long npix = (long long)n * n;
    const int ch0 = ichan_base[c], ch1 = ichan_base[c + 1];   // the channels that see this image
    const size_t np2 = (size_t)np * np;
    double acc[2] = {0.0, 0.0};
    // groups of RP pixels per thread; fixed-order sum over the slots with
    // 8 slots x RP pixels of independent loads in flight
    for (int g0 = 0; g0 < pb_len; g0 += RP * NTHR) {
        size_t off[RP];
        bool okp[RP];
#pragma unroll
        for (int r = 0; r < RP; ++r) {
            const long long p = (long long)pb * pb_len + g0 + r * NTHR + threadIdx.x;
            okp[r] = g0 + r * NTHR < pb_len && p < npix;
            const long long pc = okp[r] ? p : 0;
            off[r] = (size_t)(pc / n) * np + (size_t)(pc % n);
        }
        // per-pixel inputs of the epilogue and the first channel's beam,
        // loaded ahead of the slot sums, unconditionally (from a stand-in
        // array where one is absent or unused, so that no load sits behind a
        // branch; such values are never used)
        const R *Isrc = mode == 1 || mode == 2 ? I : gt;
        const unsigned char *msrc = mask ? mask : reinterpret_cast<const unsigned char *>(gt);
        const size_t bbase = (size_t)(ch0 < ch1 ? ch0 : 0) * npix;
        R xI[RP], xgt[RP], bm0[RP];
        unsigned char mk[RP];
#pragma unroll
        for (int r = 0; r < RP; ++r) {
            const long long p = (long long)pb * pb_len + g0 + r * NTHR + threadIdx.x;
            const long long pc = okp[r] ? p : 0;
            const size_t q = (size_t)c * npix + pc;
            xI[r] = Isrc[q];
            xgt[r] = gt[q];
            mk[r] = msrc[q];
            bm0[r] = beam[bbase + pc];
        }
        // grad chi^2 = sum over the image's channels of A_ch o (sum of the
        // channel's slots)
        double AG[RP];
#pragma unroll
        for (int r = 0; r < RP; ++r) AG[r] = 0.0;
        for (int ch = ch0; ch < ch1; ++ch) {
            const int s0 = slot_base[ch], s1 = slot_base[ch + 1];
            double Gs[RP];
#pragma unroll
            for (int r = 0; r < RP; ++r) Gs[r] = 0.0;
            int s = s0;
            // UL slots x RP pixels of independent loads in flight (32 slots
            // when a thread owns one pixel), then batches of 8; the sum
            // stays in slot order
            constexpr int UL = RP == 1 ? 32 : 8;
            auto batch = [&](auto ul) {
                constexpr int B = decltype(ul)::value;
                double v[RP][B];
#pragma unroll
                for (int r = 0; r < RP; ++r)
#pragma unroll
                    for (int u = 0; u < B; ++u) v[r][u] = (double)gpart[(size_t)(s + u) * np2 + off[r]];
#pragma unroll
                for (int r = 0; r < RP; ++r)
#pragma unroll
                    for (int u = 0; u < B; ++u) Gs[r] += v[r][u];
                s += B;
            };
            while (s + UL <= s1) batch(std::integral_constant<int, UL>());
            if constexpr (UL > 8)
                while (s + 8 <= s1) batch(std::integral_constant<int, 8>());
            for (; s < s1; ++s) {
#pragma unroll
                for (int r = 0; r < RP; ++r) Gs[r] += (double)gpart[(size_t)s * np2 + off[r]];
            }
#pragma unroll
            for (int r = 0; r < RP; ++r) {
                const long long p = (long long)pb * pb_len + g0 + r * NTHR + threadIdx.x;
                const double A = mode == 3 ? 1.0 : ch == ch0 ? (double)bm0[r] : (double)beam[(size_t)ch * npix + p];
                if (okp[r]) AG[r] += A * Gs[r];
            }
        }
#pragma unroll
        for (int r = 0; r < RP; ++r) {
            if (!okp[r]) continue;
            const long long p = (long long)pb * pb_len + g0 + r * NTHR + threadIdx.x;
            const size_t q = (size_t)c * npix + p;
            double gv = AG[r];
            if (mode == 3) gv *= img_scale[c];
            if (mode == 1 || mode == 2) {
                const double x = (double)xI[r];
                gv += lam * (log(x / M) + 1.0);
                if (mask && !mk[r]) gv = 0.0;
            }
            const R gr = (R)gv;
            out[q] = gr;
            if (mode == 2) {
                const double x = (double)xI[r];
                const bool act = (x <= Mb * (1.0 + BOUND_TOL)) && ((double)gr > 0.0);
                const double gnew = act ? 0.0 : (double)gr;
                const double gold = (double)xgt[r];
                gt[q] = (R)gnew;
                acc[0] += gnew * gnew;
                acc[1] += gnew * gold;
            }
        }
    }
    if (mode == 2) {
        block_sum<2>(acc);
        if (threadIdx.x == 0) {
            coh_store(ppart + ((size_t)c * n_pb + pb) * NPART + 0, acc[0]);
            coh_store(ppart + ((size_t)c * n_pb + pb) * NPART + 1, acc[1]);
        }
    }
    if ((mode != 1 && mode != 2) || !arrive_last(tail.ctr + c, (unsigned)n_pb)) return;
    double *sc = tail.scal + (size_t)c * UVMEM_NSCAL;
    if (mode == 1) {
        double x2[1], S[1];
        const int v0 = tail.ivis_base[c], v1 = tail.ivis_base[c + 1];
        sum_partials2<1, 1>(tail.vispart + (size_t)v0 * NPART, v1 - v0, 0, x2,
                            tail.pp_S + (size_t)c * n_pb * NPART, n_pb, 0, S);
        if (threadIdx.x == 0) {
            const double chi2 = 0.5 * x2[0];
            sc[UVMEM_S_PHI] = chi2 + lam * S[0];
            sc[UVMEM_S_CHI2] = chi2;
            sc[UVMEM_S_S] = S[0];
            if (tail.user) {
                double *u = tail.user + (size_t)c * UVMEM_NSCAL;
                u[UVMEM_S_PHI] = sc[UVMEM_S_PHI];
                u[UVMEM_S_CHI2] = chi2;
                u[UVMEM_S_S] = S[0];
            }
        }
        return;
    }
    double gg[2];
    sum_partials<2>(ppart + (size_t)c * n_pb * NPART, n_pb, 0, gg);
    if (threadIdx.x == 0) {
        double *ch = tail.chan + (size_t)c * CH_N;
        const double gold = ch[CH_GG_OLD];
        const bool stop = ch[CH_STOP] != 0.0;
        double beta = 0.0;
        if (!stop && gold > 0.0) beta = fmax(0.0, (gg[0] - gg[1]) / gold);
        sc[UVMEM_S_BETA] = beta;
        sc[UVMEM_S_GNORM2] = gg[0];
        if (sc[UVMEM_S_ALPHA] != 0.0) sc[UVMEM_S_ITER] += 1.0;
        if (tail.user) {
            for (int x = 0; x < UVMEM_NSCAL; ++x) tail.user[(size_t)c * UVMEM_NSCAL + x] = sc[x];
        }
        if (tail.hist_ptr) {
            double *hb = reinterpret_cast<double *>(tail.hist_ptr[0]);
            const long long t = tail.hist_ctr[0];
            if (hb) {
                for (int x = 0; x < UVMEM_NSCAL; ++x) hb[t * UVMEM_NSCAL + x] = sc[x];
            }
            tail.hist_ctr[0] = t + 1;
        }
    }
}

// ---------------------------------------------------------------- CG
// Initial projected gradient gt = g off the active set, partial |gt|^2; the
// last workgroup of an image starts its CG bookkeeping.
template <typename R>
__global__ __launch_bounds__(NTHR) void k_cg_init(const R *__restrict__ I, const R *__restrict__ g,
                                                  R *__restrict__ gt, R *__restrict__ dir,
                                                  double *__restrict__ ppart, int n, int n_pb, int pb_len, double Mb,
                                                  unsigned *__restrict__ ctr, double *__restrict__ scal,
                                                  double *__restrict__ chan) {
    const int c = blockIdx.x / n_pb, pb = blockIdx.x % n_pb;
    const long long npix = (long long)n * n;
    double acc[1] = {0.0};
    for (int r = 0; r < pb_len / NTHR; ++r) {
        const long long p = (long long)pb * pb_len + r * NTHR + threadIdx.x;
        if (p >= npix) break;
        const size_t q = (size_t)c * npix + p;
        const double x = (double)I[q], gv = (double)g[q];
        const bool act = (x <= Mb * (1.0 + BOUND_TOL)) && (gv > 0.0);
        const double gn = act ? 0.0 : gv;
        gt[q] = (R)gn;
        dir[q] = (R)0;
        acc[0] += gn * gn;
    }
    block_sum<1>(acc);
    if (threadIdx.x == 0) coh_store(ppart + ((size_t)c * n_pb + pb) * NPART + 0, acc[0]);
    if (!arrive_last(ctr + c, (unsigned)n_pb)) return;
    double gg[1];
    sum_partials<1>(ppart + (size_t)c * n_pb * NPART, n_pb, 0, gg);
    if (threadIdx.x == 0) {
        double *sc = scal + (size_t)c * UVMEM_NSCAL;
        sc[UVMEM_S_ALPHA] = 0.0;
        sc[UVMEM_S_BETA] = 0.0;
        sc[UVMEM_S_GNORM2] = gg[0];
        sc[UVMEM_S_ALPHA_MAX] = 0.0;
        sc[UVMEM_S_ITER] = 0.0;
        double *ch = chan + (size_t)c * CH_N;
        for (int x = 0; x < CH_N; ++x) ch[x] = 0.0;
        ch[CH_GG_OLD] = gg[0];
        ch[CH_STOP] = gg[0] == 0.0 ? 1.0 : 0.0;
    }
}

// Steps 1-3: d <- -gt + beta d, projected onto the feasible directions at the
// bound (d = 0 on the active set, d >= 0 on the other bound pixels), stored
// with B = A o d for the forward model; partials of gt . d and, for this
// direction and for the restart direction -gt, of the entropy parts of
// phi'(0) - b and phi''(0) - a and of alpha_max.  The last workgroup of an
// image takes step 2: restart with d = -gt when gt . d >= 0 (it then rewrites
// the image's d and B itself, which a restart alone needs), stop when the
// projected gradient is zero; it keeps the chosen direction's totals and
// starts the line search of an image that has no visibilities.
template <typename R>
__global__ __launch_bounds__(NTHR) void k_cg_dir(const R *__restrict__ I, const R *__restrict__ g,
                                                 const R *__restrict__ gt, R *__restrict__ dir,
                                                 const R *__restrict__ beam, R *__restrict__ bop,
                                                 const int *__restrict__ ichan_base,
                                                 const double *__restrict__ scal, double *__restrict__ chan,
                                                 double *__restrict__ ppart, int n, int np, int n_pb, int pb_len,
                                                 double M, double Mb, double lam, unsigned *__restrict__ ctr,
                                                 const int *__restrict__ ivis_base, double *__restrict__ ls) {
    const int c = blockIdx.x / n_pb, pb = blockIdx.x % n_pb;
    const long long npix = (long long)n * n;
    const double beta = scal[(size_t)c * UVMEM_NSCAL + UVMEM_S_BETA];
    const bool stop = chan[(size_t)c * CH_N + CH_STOP] != 0.0;
    const int ch0 = ichan_base[c], ch1 = ichan_base[c + 1];   // the channels that see this image
    // [0] gt . d; entropy parts [1], [2] of d and [3], [4] of -gt
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double am_d = INFINITY, am_s = INFINITY;
    for (int r = 0; r < pb_len / NTHR; ++r) {
        const long long p = (long long)pb * pb_len + r * NTHR + threadIdx.x;
        if (p >= npix) break;
        const size_t q = (size_t)c * npix + p;
        const double x = (double)I[q], gv = (double)g[q], gtv = (double)gt[q];
        // the first channel's beam with the other loads (the stores below
        // would otherwise hold it back)
        const R bm0 = ch0 < ch1 ? beam[(size_t)ch0 * npix + p] : R(0);
        double d = -gtv + beta * (double)dir[q];
        const bool atb = x <= Mb * (1.0 + BOUND_TOL);
        if (atb && gv > 0.0) d = 0.0;
        else if (atb) d = fmax(d, 0.0);
        if (stop) d = 0.0;
        const R dr = (R)d;
        // device-coherent stores: a restart rewrites these pixels from the
        // last workgroup, which may run on another chiplet, and no cache may
        // keep an older copy to write back after it
        coh_store(dir + q, dr);
        const int i = (int)(p / n), j = (int)(p % n);
        for (int ch = ch0; ch < ch1; ++ch)
            coh_store(bop + (size_t)ch * np * np + (size_t)i * np + j,
                      (ch == ch0 ? bm0 : beam[(size_t)ch * npix + p]) * dr);
        d = (double)dr;
        const double s = stop ? 0.0 : -gtv;
        const double lg = log(x / M) + 1.0;
        acc[0] += gtv * d;
        acc[1] += d * lg;
        acc[2] += d * d / x;
        acc[3] += s * lg;
        acc[4] += s * s / x;
        if (d < 0.0) am_d = fmin(am_d, (x - Mb) / (-d));
        if (s < 0.0) am_s = fmin(am_s, (x - Mb) / (-s));
    }
    block_sum<5>(acc);
    am_d = block_min(am_d);
    am_s = block_min(am_s);
    if (threadIdx.x == 0) {
        double *pp = ppart + ((size_t)c * n_pb + pb) * NPART;
        for (int m = 0; m < 5; ++m) coh_store(pp + m, acc[m]);
        coh_store(pp + 5, am_d);
        coh_store(pp + 6, am_s);
    }
    if (!arrive_last(ctr + c, (unsigned)n_pb)) return;
    double t[5];
    double amm[2];
    sum_min_partials<5, 2>(ppart + (size_t)c * n_pb * NPART, n_pb, t, amm);
    const double am0 = amm[0], am1 = amm[1];
    const double gg = scal[(size_t)c * UVMEM_NSCAL + UVMEM_S_GNORM2];
    const bool restart = t[0] >= 0.0;
    const bool stop_now = stop || gg == 0.0;
    if (threadIdx.x == 0) {
        double *ch = chan + (size_t)c * CH_N;
        if (stop_now) ch[CH_STOP] = 1.0;
        ch[CH_RESTART] = restart ? 1.0 : 0.0;
        ch[CH_GTD] = restart ? -gg : t[0];
        ch[CH_GG_OLD] = gg;
        ch[CH_E1] = restart ? t[3] : t[1];
        ch[CH_E2] = restart ? t[4] : t[2];
        ch[CH_AMAX] = restart ? am1 : am0;
        // no visibility workgroup will start this image's line search
        if (ivis_base[c + 1] == ivis_base[c])
            ls_init(ls + (size_t)c * LSS_N, 0.0, 0.0, lam * ch[CH_E1], lam * ch[CH_E2], ch[CH_AMAX], stop_now,
                    false, 0.0, 0.0);
    }
    // a stopped image's direction is zero already (gt = 0 or stop)
    if (!restart || stop_now) return;
    for (long long p = threadIdx.x; p < npix; p += NTHR) {
        const size_t q = (size_t)c * npix + p;
        const R dr = (R)(-(double)gt[q]);
        coh_store(dir + q, dr);
        const int i = (int)(p / n), j = (int)(p % n);
        for (int ch = ch0; ch < ch1; ++ch)
            coh_store(bop + (size_t)ch * np * np + (size_t)i * np + j, beam[(size_t)ch * npix + p] * dr);
    }
}

// ---- line search: exact minimisation of the convex phi on [0, alpha_max]
//   phi'(al)  = b + a al + lambda sum d (ln((I + al d)/M) + 1)
//   phi''(al) = a + lambda sum d^2 / (I + al d)
// The entropy part of phi' increases with al, so phi'(al) >= phi'(0) + a al
// and the minimiser lies below -phi'(0)/a: that bounds a search without
// alpha_max.  The start knows phi', phi'' at 0 and, from the direction's
// visibility pass, at alpha_max, which settles a step that reaches alpha_max
// without any pass.  Each pass evaluates phi', phi'' at LS_K trial steps
// inside the bracket [LO, HI] and keeps the smallest bracket.  With HI
// evaluated the trials are the root of the cubic Hermite interpolant of phi'
// on the bracket, the Newton steps from both ends, the secant step and points
// 1e-3 and 1e-6 of the bracket either side of the cubic's root; with HI an
// unevaluated bound, a geometric ladder from the Newton step to HI; with no
// bound, factors of 4 from the Newton step.  A bracket narrowed to 1e-13 (or
// the last pass) accepts the cubic's root.  The state is advanced identically
// by every workgroup of the channel.
enum { PH_SEARCH = 0, PH_DONE = 3 };
static_assert(LS_K == 8, "the bracket proposal fills eight trial steps");

__device__ __forceinline__ void ls_finish(double *st, double al) {
    st[LSS_PHASE] = PH_DONE;
    st[LSS_ALPHA] = al;
#pragma unroll
    for (int m = 0; m < LS_K; ++m) st[LSS_T0 + m] = al;
}

// Root in [lo, hi] of the cubic Hermite interpolant p of phi' from its values
// f0 < 0 < f1 and slopes h0, h1 at the ends, by Newton's method on the unit
// parameter s of the bracket, safeguarded by bisection of the sub-bracket on
// which p changes sign.
__device__ double hermite_root(double lo, double hi, double f0, double f1, double h0, double h1) {
    const double w = hi - lo, d0 = h0 * w, d1 = h1 * w;
    double sl = 0.0, sh = 1.0;
    double s = f0 / (f0 - f1);
    if (!(s > 0.0 && s < 1.0)) s = 0.5;
    for (int it = 0; it < 64; ++it) {
        const double s2 = s * s, s3 = s2 * s;
        const double p = (2.0 * s3 - 3.0 * s2 + 1.0) * f0 + (s3 - 2.0 * s2 + s) * d0 + (3.0 * s2 - 2.0 * s3) * f1 +
                         (s3 - s2) * d1;
        if (p == 0.0) break;
        if (p < 0.0) sl = s;
        else sh = s;
        const double dp = 6.0 * (s2 - s) * (f0 - f1) + (3.0 * s2 - 4.0 * s + 1.0) * d0 + (3.0 * s2 - 2.0 * s) * d1;
        double sn = dp != 0.0 ? s - p / dp : 0.5 * (sl + sh);
        if (!(sn > sl && sn < sh)) sn = 0.5 * (sl + sh);
        if (sn == s) break;
        s = sn;
    }
    return fmin(fmax(lo + s * w, lo), hi);
}

__device__ __forceinline__ double ls_cubic(const double *st) {
    return hermite_root(st[LSS_LO], st[LSS_HI], st[LSS_FLO], st[LSS_FHI], st[LSS_HLO], st[LSS_HHI]);
}

__device__ void ls_propose(double *st) {
    const double lo = st[LSS_LO], hi = st[LSS_HI];
    const double tn = lo - st[LSS_FLO] / st[LSS_HLO];   // > lo (FLO < 0, HLO > 0)
    double t[LS_K];
    if (hi < 0.0) {
        double x = (tn > lo && isfinite(tn)) ? tn : (lo > 0.0 ? 2.0 * lo : 1.0);
        for (int m = 0; m < LS_K; ++m, x *= 4.0) t[m] = x;
    } else if (st[LSS_HI_EVAL] == 0.0) {
        const double t0 = (tn > lo && tn < hi) ? tn : lo + 0.5 * (hi - lo);
        const double r = log(hi / t0) / (LS_K - 1);
        for (int m = 0; m < LS_K - 1; ++m) t[m] = t0 * exp(r * m);
        t[LS_K - 1] = hi;
    } else {
        const double w = hi - lo;
        const double rc = ls_cubic(st);
        t[0] = rc;
        t[1] = tn;
        t[2] = hi - st[LSS_FHI] / st[LSS_HHI];
        t[3] = lo - st[LSS_FLO] * w / (st[LSS_FHI] - st[LSS_FLO]);
        t[4] = rc - 1e-3 * w;
        t[5] = rc + 1e-3 * w;
        t[6] = rc - 1e-6 * w;
        t[7] = rc + 1e-6 * w;
        for (int m = 0; m < LS_K; ++m)
            if (!(t[m] > lo && t[m] < hi)) t[m] = lo + (m + 1) * w / (LS_K + 1);
    }
    for (int i = 1; i < LS_K; ++i)   // ascending (insertion sort)
        for (int j = i; j > 0 && t[j] < t[j - 1]; --j) {
            const double x = t[j]; t[j] = t[j - 1]; t[j - 1] = x;
        }
#pragma unroll
    for (int m = 0; m < LS_K; ++m) st[LSS_T0 + m] = t[m];
}

// Start from a, b, e1 = lambda sum d (ln(I/M) + 1), e2 = lambda sum d^2/I
// (so phi'(0) = b + e1, phi''(0) = a + e2), alpha_max and, when am_eval, the
// entropy parts f_am, h_am of phi', phi'' at alpha_max.
__device__ void ls_init(double *st, double a, double b, double e1, double e2, double amax, bool stop,
                        bool am_eval, double f_am, double h_am) {
    st[LSS_A] = a;
    st[LSS_B] = b;
    st[LSS_AMAX] = isfinite(amax) ? amax : -1.0;
    st[LSS_STOP] = stop ? 1.0 : 0.0;
    st[LSS_LO] = 0.0;
    st[LSS_HI] = isfinite(amax) ? amax : -1.0;
    st[LSS_FLO] = b + e1;
    st[LSS_HLO] = a + e2;
    st[LSS_FHI] = 0.0;
    st[LSS_HHI] = 0.0;
    st[LSS_HI_EVAL] = 0.0;
    st[LSS_PHASE] = PH_SEARCH;
    if (stop || !(st[LSS_FLO] < 0.0) || !(st[LSS_HLO] > 0.0) || (isfinite(amax) && amax <= 0.0)) {
        ls_finish(st, 0.0);
        return;
    }
    if (isfinite(amax) && am_eval) {
        const double fa = b + a * amax + f_am;
        if (fa <= 0.0) {   // phi' <= 0 on all of [0, alpha_max]
            ls_finish(st, amax);
            return;
        }
        st[LSS_FHI] = fa;
        st[LSS_HHI] = a + h_am;
        st[LSS_HI_EVAL] = 1.0;
    } else if (!isfinite(amax) && a > 0.0) {
        st[LSS_HI] = -st[LSS_FLO] / a;
    }
    ls_propose(st);
}

// Advance the state with phi'(T_m) = f[m], phi''(T_m) = h[m].
__device__ void ls_update(double *st, const double *f, const double *h) {
    if ((int)st[LSS_PHASE] == PH_DONE) return;
    int m = 0;
    while (m < LS_K && f[m] <= 0.0) ++m;
    if (m > 0 && f[m - 1] == 0.0) { ls_finish(st, st[LSS_T0 + m - 1]); return; }
    if (m > 0) {
        st[LSS_LO] = st[LSS_T0 + m - 1];
        st[LSS_FLO] = f[m - 1];
        st[LSS_HLO] = h[m - 1];
    }
    if (m < LS_K) {
        st[LSS_HI] = st[LSS_T0 + m];
        st[LSS_FHI] = f[m];
        st[LSS_HHI] = h[m];
        st[LSS_HI_EVAL] = 1.0;
    } else if (st[LSS_HI] >= 0.0 && st[LSS_HI_EVAL] == 0.0 && st[LSS_T0 + LS_K - 1] == st[LSS_HI]) {
        // phi'(HI) <= 0 at an unevaluated end: HI is alpha_max, the minimiser
        // on [0, alpha_max], or the bound -phi'(0)/a, where phi' >= 0, so the
        // root up to rounding
        ls_finish(st, st[LSS_HI]);
        return;
    }
    const double lo = st[LSS_LO], hi = st[LSS_HI];
    if (st[LSS_HI_EVAL] != 0.0 && hi - lo <= 1e-13 * hi) {
        ls_finish(st, ls_cubic(st));
        return;
    }
    ls_propose(st);
}

// Accepted step when the pass budget ran out: the cubic's root in the
// bracket, or the largest step known to descend.
__device__ double ls_fallback(const double *st) {
    return st[LSS_HI_EVAL] != 0.0 ? ls_cubic(st) : st[LSS_LO];
}

// Sum the LS_K (phi' entropy part, phi'' entropy part) partials of a channel
// and turn them into phi', phi'' at the trial steps.
__device__ __forceinline__ void ls_eval(const double *st, const double *pp, int n_pb, double lam,
                                        double *f, double *h) {
    double e[2 * LS_K];
    sum_partials<2 * LS_K>(pp, n_pb, 0, e);
#pragma unroll
    for (int m = 0; m < LS_K; ++m) {
        const double t = st[LSS_T0 + m];
        f[m] = st[LSS_B] + st[LSS_A] * t + lam * e[2 * m];
        h[m] = st[LSS_A] + lam * e[2 * m + 1];
    }
}

// Step 5: Vd and the partials of a = sum w |Vd|^2 and b = sum w Re(conj(R) Vd)
// (the first n_visit workgroups, one visibility item each), and the entropy
// parts of phi', phi'' at alpha_max (pixel workgroups of the images that have
// visibilities; zero without a finite alpha_max).  The last workgroup of an
// image starts its line search from these totals and the direction pass's.
template <typename R>
__global__ __launch_bounds__(NTHR) void k_cg_vis(const VisItem *__restrict__ items, int n_visit,
                                                 const double2 *__restrict__ vpart, int n_parts, long long ztot,
                                                 const float *__restrict__ w, double2 *__restrict__ Rv,
                                                 double2 *__restrict__ Vd, double *__restrict__ vispart,
                                                 const int *__restrict__ chan_img, const int *__restrict__ ivis_base,
                                                 const R *__restrict__ I, const R *__restrict__ dir,
                                                 double *__restrict__ ppart, int n, int n_pb, int pb_len, double M,
                                                 double lam, const double *__restrict__ chan,
                                                 double *__restrict__ ls, unsigned *__restrict__ ctr) {
    int img;
    if ((int)blockIdx.x < n_visit) {
        const VisItem it = items[blockIdx.x];
        img = chan_img[it.chan];
        vis_item(it, blockIdx.x, vpart, n_parts, ztot, nullptr, w, Rv, Vd, nullptr, vispart, 2, 0, 0.0);
    } else {
        const int blk = (int)blockIdx.x - n_visit;
        img = blk / n_pb;
        const int pb = blk % n_pb;
        const long long npix = (long long)n * n;
        // the thread's first pixel, loaded ahead of the image's scalars
        // (pixel 0 stands in past the end)
        const long long p_1 = (long long)pb * pb_len + threadIdx.x;
        const size_t q_1 = (size_t)img * npix + (p_1 < npix ? p_1 : 0);
        const R d_1 = dir[q_1], x_1 = I[q_1];
        if (ivis_base[img + 1] == ivis_base[img]) return;   // started by the direction pass
        const double *chc = chan + (size_t)img * CH_N;
        const double am = chc[CH_AMAX];
        double acc[2] = {0.0, 0.0};
        if (isfinite(am) && chc[CH_STOP] == 0.0) {
            for (int r = 0; r < pb_len / NTHR; ++r) {
                const long long p = (long long)pb * pb_len + r * NTHR + threadIdx.x;
                if (p >= npix) break;
                const size_t q = (size_t)img * npix + p;
                const double d = r == 0 ? (double)d_1 : (double)dir[q];
                if (d == 0.0) continue;
                const double x = (r == 0 ? (double)x_1 : (double)I[q]) + am * d;
                acc[0] += d * (log(x / M) + 1.0);
                acc[1] += d * d / x;
            }
        }
        block_sum<2>(acc);
        if (threadIdx.x == 0) {
            coh_store(ppart + ((size_t)img * n_pb + pb) * NPART + 0, acc[0]);
            coh_store(ppart + ((size_t)img * n_pb + pb) * NPART + 1, acc[1]);
        }
    }
    const int v0 = ivis_base[img], v1 = ivis_base[img + 1];
    if (!arrive_last(ctr + img, (unsigned)(v1 - v0 + n_pb))) return;
    double ab[2], fh[2];
    sum_partials2<2, 2>(vispart + (size_t)v0 * NPART, v1 - v0, 0, ab, ppart + (size_t)img * n_pb * NPART, n_pb, 0,
                        fh);
    if (threadIdx.x == 0) {
        const double *ch = chan + (size_t)img * CH_N;
        ls_init(ls + (size_t)img * LSS_N, ab[0], ab[1], lam * ch[CH_E1], lam * ch[CH_E2], ch[CH_AMAX],
                ch[CH_STOP] != 0.0, true, lam * fh[0], lam * fh[1]);
    }
}

// Pass of the line search: every workgroup of an image reads the state and
// evaluates the phi', phi'' partials at its LS_K trial steps; the last
// workgroup to arrive advances the state with the totals (in the last pass,
// a search that has not converged takes its fallback step).  A converged
// search makes the whole image skip the pass.
template <typename R>
__global__ __launch_bounds__(NTHR) void k_ls_step(const R *__restrict__ I, const R *__restrict__ dir,
                                                  double *__restrict__ ls, double *__restrict__ ppart,
                                                  int n, int n_pb, int pb_len, double M, double lam, int last_pass,
                                                  unsigned *__restrict__ ctr) {
    const int c = blockIdx.x / n_pb, pb = blockIdx.x % n_pb;
    const long long npix = (long long)n * n;
    // the thread's first pixel, loaded ahead of the state (pixel 0 stands in
    // past the end)
    const long long p_1 = (long long)pb * pb_len + threadIdx.x;
    const size_t q_1 = (size_t)c * npix + (p_1 < npix ? p_1 : 0);
    const R d_1 = dir[q_1], x_1 = I[q_1];
    __shared__ double st[LSS_N];
    double *lsc = ls + (size_t)c * LSS_N;
    if (threadIdx.x < LSS_N) st[threadIdx.x] = lsc[threadIdx.x];
    __syncthreads();
    if ((int)st[LSS_PHASE] == PH_DONE) return;
    double tr[LS_K];
#pragma unroll
    for (int m = 0; m < LS_K; ++m) tr[m] = st[LSS_T0 + m];
    double acc[2 * LS_K];
#pragma unroll
    for (int m = 0; m < 2 * LS_K; ++m) acc[m] = 0.0;
    for (int r = 0; r < pb_len / NTHR; ++r) {
        const long long p = (long long)pb * pb_len + r * NTHR + threadIdx.x;
        if (p >= npix) break;
        const size_t q = (size_t)c * npix + p;
        const double d = r == 0 ? (double)d_1 : (double)dir[q];
        if (d == 0.0) continue;
        const double x0 = r == 0 ? (double)x_1 : (double)I[q];
#pragma unroll
        for (int m = 0; m < LS_K; ++m) {
            const double x = x0 + tr[m] * d;
            acc[2 * m] += d * (log(x / M) + 1.0);
            acc[2 * m + 1] += d * d / x;
        }
    }
    block_sum<2 * LS_K>(acc);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int m = 0; m < 2 * LS_K; ++m) coh_store(ppart + ((size_t)c * n_pb + pb) * NPART + m, acc[m]);
    }
    if (!arrive_last(ctr + c, (unsigned)n_pb)) return;
    double f[LS_K], h[LS_K];
    ls_eval(st, ppart + (size_t)c * n_pb * NPART, n_pb, lam, f, h);
    if (threadIdx.x == 0) {
        ls_update(st, f, h);
        if (last_pass && (int)st[LSS_PHASE] != PH_DONE) ls_finish(st, ls_fallback(st));
    }
    __syncthreads();
    if (threadIdx.x < LSS_N) lsc[threadIdx.x] = st[threadIdx.x];
}

// Step 8: I <- max(I + alpha d, M) with the accepted step and the entropy
// partial of the new image (pixel workgroups); R <- R + alpha Vd and its
// chi^2 partials (visibility workgroups, one item each).  The last
// workgroup of an image stores Phi, chi^2, S, alpha and alpha_max.
template <typename R>
__global__ __launch_bounds__(NTHR) void k_cg_update(R *__restrict__ I, const R *__restrict__ dir,
                                                    const double *__restrict__ ls, double *__restrict__ pp_out,
                                                    double *__restrict__ scal, double *__restrict__ chan,
                                                    int *__restrict__ flag,
                                                    int n, int n_pb, int pb_len, double M, double Mb, double lam,
                                                    const VisItem *__restrict__ vitems, const float *__restrict__ w,
                                                    double2 *__restrict__ Rv, const double2 *__restrict__ Vd,
                                                    double *__restrict__ vispart, const int *__restrict__ chan_img,
                                                    const int *__restrict__ ivis_base, int n_pixwg, int with_max,
                                                    unsigned *__restrict__ ctr) {
    const bool visw = (int)blockIdx.x >= n_pixwg;
    const int vi = (int)blockIdx.x - n_pixwg;
    const VisItem vit = visw ? vitems[vi] : VisItem{};
    const int c = visw ? chan_img[vit.chan] : (int)blockIdx.x / n_pb, pb = visw ? -1 : (int)blockIdx.x % n_pb;
    const long long npix = (long long)n * n;
    const double *lsc = ls + (size_t)c * LSS_N;
    const double al = lsc[LSS_ALPHA];
    if (visw) {
        vis_item(vit, vi, nullptr, 0, 0, nullptr, w, Rv, const_cast<double2 *>(Vd), nullptr, vispart, 3, with_max, al);
    } else {
        double acc[1] = {0.0};
        int bad = 0;
        for (int r = 0; r < pb_len / NTHR; ++r) {
            const long long p = (long long)pb * pb_len + r * NTHR + threadIdx.x;
            if (p >= npix) break;
            const size_t q = (size_t)c * npix + p;
            // I and d are loaded together, before the step is known (selects,
            // not a branch, so that the load of d is not deferred behind it)
            const double x0 = (double)I[q], dv = (double)dir[q];
            const R xr = (R)fmax(x0 + al * dv, Mb);
            const bool moved = al != 0.0;
            double x = moved ? (double)xr : x0;
            if (moved) I[q] = xr;
            if (!(x > 0.0)) bad = 1;
            else acc[0] += x * log(x / M);
        }
        if (bad) atomicOr(flag, 1);
        block_sum<1>(acc);
        if (threadIdx.x == 0) coh_store(pp_out + ((size_t)c * n_pb + pb) * NPART + 0, acc[0]);
    }
    const int v0 = ivis_base[c], v1 = ivis_base[c + 1];
    if (!arrive_last(ctr + c, (unsigned)(n_pb + v1 - v0))) return;
    double x2[1], S[1];
    sum_partials2<1, 1>(vispart + (size_t)v0 * NPART, v1 - v0, 0, x2, pp_out + (size_t)c * n_pb * NPART, n_pb, 0,
                        S);
    if (threadIdx.x == 0) {
        double *sc = scal + (size_t)c * UVMEM_NSCAL;
        const double chi2 = 0.5 * x2[0];
        sc[UVMEM_S_PHI] = chi2 + lam * S[0];
        sc[UVMEM_S_CHI2] = chi2;
        sc[UVMEM_S_S] = S[0];
        sc[UVMEM_S_ALPHA] = al;
        sc[UVMEM_S_ALPHA_MAX] = lsc[LSS_AMAX] < 0.0 ? INFINITY : lsc[LSS_AMAX];
        if (al == 0.0) chan[(size_t)c * CH_N + CH_STOP] = 1.0;
    }
}

// History copy for graph replays: dst = *hist_ptr + ctr * (C * NSCAL).
__global__ void k_copy_hist(const double *__restrict__ scal, const long long *__restrict__ hist_ptr,
                            long long *__restrict__ ctr, int count) {
    double *base = reinterpret_cast<double *>(hist_ptr[0]);
    const long long t = ctr[0];
    if (base) {
        for (int x = threadIdx.x; x < count; x += blockDim.x) base[t * count + x] = scal[x];
    }
    __syncthreads();
    if (threadIdx.x == 0) ctr[0] = t + 1;
}

__global__ void k_set_hist(long long *__restrict__ hist_ptr, long long *__restrict__ ctr, long long hist) {
    if (threadIdx.x == 0) {
        hist_ptr[0] = hist;
        ctr[0] = 0;
    }
}

template <typename R> inline R *P(void *p) { return reinterpret_cast<R *>(p); }
template <typename R> inline const R *CP(const void *p) { return reinterpret_cast<const R *>(p); }

inline int pix_grid(const uvmem_ctx *c) { return c->nimg * c->n_pb; }
// Partial records of the pixel passes: buffer 0 holds the prologue's entropy
// partials until the evaluation's gradient pass has read them; every CG pass
// writes buffer 1 and its last workgroups read it in the same launch.
inline double *pp(const uvmem_ctx *c, int buf) {
    return c->d_ppart + (size_t)buf * c->nimg * c->n_pb * NPART;
}
inline unsigned *ctr(const uvmem_ctx *c, int site) { return c->d_ctr + (size_t)site * c->nimg; }
// The fp16 split adjoint scales its coefficients by the channel's max |w R|,
// which the visibility pass leaves in slot 2 of its partial records.
inline int adj_scaled(const uvmem_ctx *c) { return c->prec == UVMEM_FP16X3 ? 1 : 0; }

template <typename R>
hipError_t t_prologue(const uvmem_ctx *c, const void *I, int with_entropy, hipStream_t st) {
    hipLaunchKernelGGL(k_prologue<R>, dim3(pix_grid(c)), dim3(NTHR), 0, st, CP<R>(I), CP<R>(c->d_beam),
                       P<R>(c->d_bop), c->d_ichan_base, pp(c, 0), c->d_flag, c->n, c->np, c->n_pb, c->pix_blk, c->M,
                       with_entropy);
    return hipGetLastError();
}

// k_grad with 4 pixels per thread and round when the pixel blocks are long
// enough, else 1 (more workgroups, fewer loads in flight per thread); the
// split-K partials are FP32 for the split precisions, else FP64
template <typename R, typename PT>
void grad_launch_t(const uvmem_ctx *c, const void *I, void *out, double *ppart, int mode, double *user,
                   hipStream_t st) {
    const PT *gp = static_cast<const PT *>(c->d_gpart);
    // gradients (modes 1, 2) follow the region-restricted adjoint and its slots
    const int *slots = (mode == 1 || mode == 2) && c->has_region ? c->d_slot_base_m : c->d_slot_base;
    const bool hist = mode == 2 && c->hist_in_grad;
    const GradTail tail{ctr(c, CTR_GRAD), c->d_vispart, c->d_ivis_base, pp(c, 0), c->d_scal, c->d_chan, user,
                        hist ? c->d_hist_ptr : nullptr, hist ? c->d_iter_ctr : nullptr};
    if (c->pix_blk >= 4 * NTHR)
        hipLaunchKernelGGL((k_grad<R, 4, PT>), dim3(pix_grid(c)), dim3(NTHR), 0, st, gp, slots,
                           c->d_ichan_base, CP<R>(c->d_beam), CP<R>(I), P<R>(out), P<R>(c->d_gt), ppart,
                           c->d_wscale, c->d_mask, c->n, c->np, c->n_pb, c->pix_blk, c->M, c->Mb, c->lam, mode, tail);
    else
        hipLaunchKernelGGL((k_grad<R, 1, PT>), dim3(pix_grid(c)), dim3(NTHR), 0, st, gp, slots,
                           c->d_ichan_base, CP<R>(c->d_beam), CP<R>(I), P<R>(out), P<R>(c->d_gt), ppart,
                           c->d_wscale, c->d_mask, c->n, c->np, c->n_pb, c->pix_blk, c->M, c->Mb, c->lam, mode, tail);
}

template <typename R>
void grad_launch(const uvmem_ctx *c, const void *I, void *out, double *ppart, int mode, double *user,
                 hipStream_t st) {
    if (c->gpart_f32)
        grad_launch_t<R, float>(c, I, out, ppart, mode, user, st);
    else
        grad_launch_t<R, double>(c, I, out, ppart, mode, user, st);
}

template <typename R>
hipError_t t_cg_init_dir(const uvmem_ctx *c, const void *I, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_init<R>, dim3(pix_grid(c)), dim3(NTHR), 0, st, CP<R>(I), CP<R>(c->d_g),
                       P<R>(c->d_gt), P<R>(c->d_dir), pp(c, 1), c->n, c->n_pb, c->pix_blk, c->Mb,
                       ctr(c, CTR_INIT), c->d_scal, c->d_chan);
    return hipGetLastError();
}

// The CG step in three phases around the DFT launches (phase 0: before the
// forward model, 1: between forward and adjoint, 2: after the adjoint).
template <typename R>
hipError_t t_cg_phase(const uvmem_ctx *c, void *I, double *user, int phase, hipStream_t st) {
    const dim3 gp(pix_grid(c)), blk(NTHR);
    if (phase == 0) {
        // 1-3. direction update and projection, restart test and stop, B = A o d,
        // alpha_max and the entropy parts of phi'(0), phi''(0)
        hipLaunchKernelGGL(k_cg_dir<R>, gp, blk, 0, st, CP<R>(I), CP<R>(c->d_g), CP<R>(c->d_gt), P<R>(c->d_dir),
                           CP<R>(c->d_beam), P<R>(c->d_bop), c->d_ichan_base, c->d_scal, c->d_chan, pp(c, 1), c->n,
                           c->np, c->n_pb, c->pix_blk, c->M, c->Mb, c->lam, ctr(c, CTR_DIR), c->d_ivis_base,
                           c->d_ls);
        return hipGetLastError();
    }
    if (phase == 1) {
        // 5. Vd, the quadratic coefficients a, b of chi^2 along d and phi'
        // at alpha_max; the line search starts from them
        if (c->n_visit)
            hipLaunchKernelGGL(k_cg_vis<R>, dim3(c->n_visit + pix_grid(c)), blk, 0, st, c->d_vis, c->n_visit,
                               c->d_vpart, c->has_region ? c->n_fparts_m : c->n_fparts, (long long)c->ztot,
                               c->d_w, c->d_R, c->d_Vd, c->d_vispart, c->d_chan_img, c->d_ivis_base, CP<R>(I),
                               CP<R>(c->d_dir), pp(c, 1), c->n, c->n_pb, c->pix_blk, c->M, c->lam, c->d_chan,
                               c->d_ls, ctr(c, CTR_VIS));
        // 6-7. line-search passes (the last one accepts a step)
        const int L = c->ls_steps;
        for (int t = 0; t < L; ++t)
            hipLaunchKernelGGL(k_ls_step<R>, gp, blk, 0, st, CP<R>(I), CP<R>(c->d_dir), c->d_ls, pp(c, 1), c->n,
                               c->n_pb, c->pix_blk, c->M, c->lam, t == L - 1 ? 1 : 0, ctr(c, CTR_LS));
        // 8-9. I <- max(I + alpha d, M) and its entropy partial (pixel
        // workgroups); R <- R + alpha Vd and the chi^2 partials (visibility
        // workgroups); Phi of the new image
        hipLaunchKernelGGL(k_cg_update<R>, dim3(pix_grid(c) + c->n_visit), blk, 0, st, P<R>(I), CP<R>(c->d_dir),
                           c->d_ls, pp(c, 1), c->d_scal, c->d_chan, c->d_flag, c->n, c->n_pb, c->pix_blk, c->M,
                           c->Mb, c->lam, c->d_vis, c->d_w, c->d_R, c->d_Vd, c->d_vispart, c->d_chan_img,
                           c->d_ivis_base, pix_grid(c), adj_scaled(c), ctr(c, CTR_UPD));
        return hipGetLastError();
    }
    // 10-12. gradient at the new point, projected gradient, beta and the scalars
    grad_launch<R>(c, I, c->d_g, pp(c, 1), 2, user, st);
    return hipGetLastError();
}

}  // namespace

__global__ void k_fill_c(double2 *__restrict__ x, double2 value, long long count) {
    long long i = (long long)blockIdx.x * NTHR + threadIdx.x;
    const long long stride = (long long)gridDim.x * NTHR;
    for (; i < count; i += stride) x[i] = value;
}

hipError_t launch_fill_c(const uvmem_ctx *c, double2 *x, double re, double im, hipStream_t st) {
    const long long count = c->ztot;
    if (count == 0) return hipSuccess;
    const int blocks = (int)std::min<long long>((count + NTHR - 1) / NTHR, 4096);
    hipLaunchKernelGGL(k_fill_c, dim3(blocks), dim3(NTHR), 0, st, x, make_double2(re, im), count);
    return hipGetLastError();
}

hipError_t launch_fill(const uvmem_ctx *c, void *img, double value, hipStream_t st) {
    const long long count = (long long)c->nimg * c->n * c->n;
    const int blocks = (int)std::min<long long>((count + NTHR - 1) / NTHR, 4096);
    if (c->prec == UVMEM_FP64)
        hipLaunchKernelGGL(k_fill<double>, dim3(blocks), dim3(NTHR), 0, st, P<double>(img), value, count);
    else
        hipLaunchKernelGGL(k_fill<float>, dim3(blocks), dim3(NTHR), 0, st, P<float>(img), (float)value, count);
    return hipGetLastError();
}

hipError_t launch_prologue(const uvmem_ctx *c, const void *I, int with_entropy, hipStream_t st) {
    return c->prec == UVMEM_FP64 ? t_prologue<double>(c, I, with_entropy, st)
                                 : t_prologue<float>(c, I, with_entropy, st);
}

hipError_t launch_vis_sum(const uvmem_ctx *c, int mode, double2 *out, hipStream_t st) {
    if (c->n_visit == 0) return hipSuccess;
    hipLaunchKernelGGL(k_vis, dim3(c->n_visit), dim3(NTHR), 0, st, c->d_vis, c->d_vpart, c->n_fparts,
                       (long long)c->ztot, c->d_vo, c->d_w, c->d_R, c->d_Vd, out, c->d_scal, c->d_vispart,
                       c->d_chan_img, mode, adj_scaled(c));
    return hipGetLastError();
}

hipError_t launch_vis_sum_raw(const VisItem *items, int n_items, const double2 *vpart, int n_parts, long long ztot,
                              double2 *out, hipStream_t st) {
    if (n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(k_vis, dim3(n_items), dim3(NTHR), 0, st, items, vpart, n_parts, ztot,
                       (const double2 *)nullptr, (const float *)nullptr, (double2 *)nullptr, (double2 *)nullptr,
                       out, (const double *)nullptr, (double *)nullptr, (const int *)nullptr, 0, 0);
    return hipGetLastError();
}

hipError_t launch_coef_max(const uvmem_ctx *c, const double2 *coef, hipStream_t st) {
    if (c->n_visit == 0 || !adj_scaled(c)) return hipSuccess;
    hipLaunchKernelGGL(k_vis, dim3(c->n_visit), dim3(NTHR), 0, st, c->d_vis, c->d_vpart, c->n_fparts,
                       (long long)c->ztot, c->d_vo, (const float *)nullptr, const_cast<double2 *>(coef), c->d_Vd,
                       (double2 *)nullptr, c->d_scal, c->d_vispart, c->d_chan_img, 4, 1);
    return hipGetLastError();
}

hipError_t launch_grad(const uvmem_ctx *c, const void *I, void *out, int mode, double *user_scal, hipStream_t st) {
    if (c->prec == UVMEM_FP64) grad_launch<double>(c, I, out, pp(c, 1), mode, user_scal, st);
    else grad_launch<float>(c, I, out, pp(c, 1), mode, user_scal, st);
    return hipGetLastError();
}

hipError_t launch_cg_init_dir(const uvmem_ctx *c, const void *I, hipStream_t st) {
    return c->prec == UVMEM_FP64 ? t_cg_init_dir<double>(c, I, st) : t_cg_init_dir<float>(c, I, st);
}

hipError_t launch_copy_scal(const uvmem_ctx *c, double *, long long *ctr, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_hist, dim3(1), dim3(NTHR), 0, st, c->d_scal,
                       reinterpret_cast<const long long *>(c->d_hist_ptr), ctr, c->nimg * UVMEM_NSCAL);
    return hipGetLastError();
}

hipError_t launch_set_hist(const uvmem_ctx *c, double *hist, hipStream_t st) {
    hipLaunchKernelGGL(k_set_hist, dim3(1), dim3(64), 0, st, c->d_hist_ptr, c->d_iter_ctr,
                       (long long)(uintptr_t)hist);
    return hipGetLastError();
}

hipError_t launch_cg_phase(const uvmem_ctx *c, void *I, double *user, int phase, hipStream_t st) {
    return c->prec == UVMEM_FP64 ? t_cg_phase<double>(c, I, user, phase, st)
                                 : t_cg_phase<float>(c, I, user, phase, st);
}

hipError_t launch_cg_step(const uvmem_ctx *c, void *I, double *user, hipStream_t st) {
    hipError_t e;
    if ((e = launch_cg_phase(c, I, user, 0, st)) != hipSuccess) return e;
    if ((e = launch_forward(c, c->d_bop, st, 1)) != hipSuccess) return e;
    if ((e = launch_cg_phase(c, I, user, 1, st)) != hipSuccess) return e;
    if ((e = launch_adjoint(c, c->d_R, c->d_w, st, 1)) != hipSuccess) return e;
    return launch_cg_phase(c, I, user, 2, st);
}

}  // namespace uvm
