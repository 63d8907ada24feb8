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

#include "internal.h"

namespace uvm {
namespace {

constexpr int NTHR = 256;

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

// Sum slot `s` (K slots starting at s0) of n_items partial records of NPART
// doubles starting at `base`, in index order (strided per thread, then the
// fixed workgroup reduction).
template <int K>
__device__ __forceinline__ void sum_partials(const double *base, int n_items, int s0, double (&out)[K]) {
#pragma unroll
    for (int x = 0; x < K; ++x) out[x] = 0.0;
    for (int it = threadIdx.x; it < n_items; it += NTHR) {
#pragma unroll
        for (int x = 0; x < K; ++x) out[x] += base[(size_t)it * NPART + s0 + x];
    }
    block_sum<K>(out);
}

__device__ __forceinline__ double min_partials(const double *base, int n_items, int s) {
    double m = INFINITY;
    for (int it = threadIdx.x; it < n_items; it += NTHR) m = fmin(m, base[(size_t)it * NPART + s]);
    return block_min(m);
}

// ---------------------------------------------------------------- operand store
// The DFT operand image: plain (SPLIT = 0, element type R) or split into
// bf16 hi and lo halves (SPLIT = 1; lo at element offset lo_off).
template <typename R, int SPLIT>
__device__ __forceinline__ void store_op(void *bop, size_t idx, size_t lo_off, R v) {
    if constexpr (SPLIT == 0) {
        reinterpret_cast<R *>(bop)[idx] = v;
    } else {
        __bf16 *h = reinterpret_cast<__bf16 *>(bop);
        const float x = (float)v;
        const __bf16 hh = (__bf16)x;
        h[idx] = hh;
        h[lo_off + idx] = (__bf16)(x - (float)hh);
    }
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
template <typename R, int SPLIT>
__global__ __launch_bounds__(NTHR) void k_prologue(const R *__restrict__ I, const R *__restrict__ beam,
                                                   void *__restrict__ bop, size_t lo_off,
                                                   double *__restrict__ ppart,
                                                   int *__restrict__ flag, int n, int np, int n_pb,
                                                   double M, int with_entropy) {
    const int c = blockIdx.x / n_pb, pb = blockIdx.x % n_pb;
    const long long npix = (long long)n * n;
    const R *Ic = I + (size_t)c * npix;
    const R *Ac = beam + (size_t)c * npix;
    const size_t cb = (size_t)c * np * np;
    double s[1] = {0.0};
    int bad = 0;
    for (int r = 0; r < PIX_BLK / NTHR; ++r) {
        long long p = (long long)pb * PIX_BLK + r * NTHR + threadIdx.x;
        if (p >= npix) break;
        const int i = (int)(p / n), j = (int)(p % n);
        const R x = Ic[p];
        store_op<R, SPLIT>(bop, cb + (size_t)i * np + j, lo_off, Ac[p] * x);
        if (with_entropy) {
            const double xd = (double)x;
            if (!(xd > 0.0)) bad = 1;
            else s[0] += xd * log(xd / M);
        }
    }
    if (with_entropy) {
        if (bad) atomicOr(flag, 1);
        block_sum<1>(s);
        if (threadIdx.x == 0) ppart[((size_t)c * n_pb + pb) * NPART + 0] = s[0];
    }
}

// ---------------------------------------------------------------- visibilities
// mode 0: out[k] = V_k (model visibilities)
// mode 1: R_k = V_k - Vo_k -> R; partial[0] = sum w |R|^2
// mode 2: Vd_k = V_k -> Vd; partial[0] = sum w |Vd|^2, partial[1] = sum w Re(conj(R) Vd)
// mode 3: R_k += alpha_c Vd_k; partial[0] = sum w |R|^2
__global__ __launch_bounds__(NTHR) void k_vis(const VisItem *__restrict__ items,
                                              const double2 *__restrict__ vpart, int n_ib, long long ztot,
                                              const float2 *__restrict__ vo, const float *__restrict__ w,
                                              double2 *__restrict__ R, double2 *__restrict__ Vd,
                                              double2 *__restrict__ out, const double *__restrict__ scal,
                                              double *__restrict__ vispart, int mode) {
    const VisItem it = items[blockIdx.x];
    double acc[2] = {0.0, 0.0};
    const double alpha = mode == 3 ? scal[(size_t)it.chan * UVMEM_NSCAL + UVMEM_S_ALPHA] : 0.0;
    for (long long k = it.kbeg + threadIdx.x; k < it.kend; k += NTHR) {
        double2 v = make_double2(0.0, 0.0);
        if (mode != 3) {
            for (int ib = 0; ib < n_ib; ++ib) {
                const double2 p = vpart[(size_t)ib * ztot + k];
                v.x += p.x;
                v.y += p.y;
            }
        }
        const double ww = (double)w[k];
        if (mode == 0) {
            out[k] = v;
        } else if (mode == 1) {
            const float2 o = vo[k];
            const double2 r = make_double2(v.x - (double)o.x, v.y - (double)o.y);
            R[k] = r;
            acc[0] += ww * (r.x * r.x + r.y * r.y);
        } else if (mode == 2) {
            Vd[k] = v;
            const double2 r = R[k];
            acc[0] += ww * (v.x * v.x + v.y * v.y);
            acc[1] += ww * (r.x * v.x + r.y * v.y);
        } else {
            const double2 d = Vd[k];
            double2 r = R[k];
            r.x += alpha * d.x;
            r.y += alpha * d.y;
            R[k] = r;
            acc[0] += ww * (r.x * r.x + r.y * r.y);
        }
    }
    if (mode != 0) {
        block_sum<2>(acc);
        if (threadIdx.x == 0) {
            vispart[(size_t)blockIdx.x * NPART + 0] = acc[0];
            vispart[(size_t)blockIdx.x * NPART + 1] = acc[1];
        }
    }
}

// ---------------------------------------------------------------- gradient
// G = sum over the channel's split-K slots of gpart (fixed order);
// mode 0: out = A o G (adjoint only)
// mode 1: out = A o G + lambda (ln(I/M) + 1)            (grad Phi)
// mode 2: as 1 into g; gt = g with zeros on the active set; partials
//         [0] = gt_new . gt_new, [1] = gt_new . gt_old; gt updated in place.
template <typename R>
__global__ __launch_bounds__(NTHR) void k_grad(const double *__restrict__ gpart, const int *__restrict__ slot_base,
                                               const R *__restrict__ beam, const R *__restrict__ I,
                                               R *__restrict__ out, R *__restrict__ gt,
                                               double *__restrict__ ppart, int n, int np, int n_pb,
                                               double M, double Mb, double lam, int mode) {
    const int c = blockIdx.x / n_pb, pb = blockIdx.x % n_pb;
    const long long npix = (long long)n * n;
    const int s0 = slot_base[c], s1 = slot_base[c + 1];
    const size_t np2 = (size_t)np * np;
    double acc[2] = {0.0, 0.0};
    for (int r = 0; r < PIX_BLK / NTHR; ++r) {
        const long long p = (long long)pb * PIX_BLK + r * NTHR + threadIdx.x;
        if (p >= npix) break;
        const int i = (int)(p / n), j = (int)(p % n);
        // fixed-order sum over the slots, eight independent loads in flight
        const double *gp = gpart + (size_t)i * np + j;
        double G = 0.0;
        int s = s0;
        for (; s + 8 <= s1; s += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = gp[(size_t)(s + u) * np2];
#pragma unroll
            for (int u = 0; u < 8; ++u) G += v[u];
        }
        for (; s < s1; ++s) G += gp[(size_t)s * np2];
        const size_t q = (size_t)c * npix + p;
        double gv = (double)beam[q] * G;
        if (mode >= 1) {
            const double x = (double)I[q];
            gv += lam * (log(x / M) + 1.0);
        }
        const R gr = (R)gv;
        out[q] = gr;
        if (mode == 2) {
            const double x = (double)I[q];
            const bool act = (x <= Mb * (1.0 + BOUND_TOL)) && ((double)gr > 0.0);
            const double gnew = act ? 0.0 : (double)gr;
            const double gold = (double)gt[q];
            gt[q] = (R)gnew;
            acc[0] += gnew * gnew;
            acc[1] += gnew * gold;
        }
    }
    if (mode == 2) {
        block_sum<2>(acc);
        if (threadIdx.x == 0) {
            ppart[((size_t)c * n_pb + pb) * NPART + 0] = acc[0];
            ppart[((size_t)c * n_pb + pb) * NPART + 1] = acc[1];
        }
    }
}

// ---------------------------------------------------------------- per-channel scalars
// Phi, chi^2, S of a plain evaluation.
__global__ __launch_bounds__(NTHR) void k_chan_phi(const double *__restrict__ vispart, const int *__restrict__ vis_base,
                                                   const double *__restrict__ ppart, int n_pb, double lam,
                                                   double *__restrict__ scal, double *__restrict__ user) {
    const int c = blockIdx.x;
    double x2[1], S[1];
    sum_partials<1>(vispart + (size_t)vis_base[c] * NPART, vis_base[c + 1] - vis_base[c], 0, x2);
    sum_partials<1>(ppart + (size_t)c * n_pb * NPART, n_pb, 0, S);
    if (threadIdx.x == 0) {
        const double chi2 = 0.5 * x2[0];
        double *sc = scal + (size_t)c * UVMEM_NSCAL;
        sc[UVMEM_S_PHI] = chi2 + lam * S[0];
        sc[UVMEM_S_CHI2] = chi2;
        sc[UVMEM_S_S] = S[0];
        if (user) {
            user[(size_t)c * UVMEM_NSCAL + UVMEM_S_PHI] = sc[UVMEM_S_PHI];
            user[(size_t)c * UVMEM_NSCAL + UVMEM_S_CHI2] = chi2;
            user[(size_t)c * UVMEM_NSCAL + UVMEM_S_S] = S[0];
        }
    }
}

// ---------------------------------------------------------------- CG
// Initial projected gradient gt = g off the active set, partial |gt|^2.
template <typename R>
__global__ __launch_bounds__(NTHR) void k_cg_init(const R *__restrict__ I, const R *__restrict__ g,
                                                  R *__restrict__ gt, R *__restrict__ dir,
                                                  double *__restrict__ ppart, int n, int n_pb, double Mb) {
    const int c = blockIdx.x / n_pb, pb = blockIdx.x % n_pb;
    const long long npix = (long long)n * n;
    double acc[1] = {0.0};
    for (int r = 0; r < PIX_BLK / NTHR; ++r) {
        const long long p = (long long)pb * PIX_BLK + r * NTHR + threadIdx.x;
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
    if (threadIdx.x == 0) ppart[((size_t)c * n_pb + pb) * NPART + 0] = acc[0];
}

__global__ __launch_bounds__(NTHR) void k_chan_cg_init(const double *__restrict__ ppart, int n_pb,
                                                       double *__restrict__ scal, double *__restrict__ chan) {
    const int c = blockIdx.x;
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
        ch[CH_GTD] = 0.0;
        ch[CH_RESTART] = 0.0;
        ch[CH_GG_OLD] = gg[0];
        ch[CH_STOP] = gg[0] == 0.0 ? 1.0 : 0.0;
    }
}

// Step 1: d <- -gt + beta d, projected onto the feasible directions at the
// bound (d = 0 on the active set, d >= 0 on the other bound pixels); partial
// gt . d.
template <typename R>
__global__ __launch_bounds__(NTHR) void k_cg_dir(const R *__restrict__ I, const R *__restrict__ g,
                                                 const R *__restrict__ gt, R *__restrict__ dir,
                                                 const double *__restrict__ scal, const double *__restrict__ chan,
                                                 double *__restrict__ ppart, int n, int n_pb, double Mb) {
    const int c = blockIdx.x / n_pb, pb = blockIdx.x % n_pb;
    const long long npix = (long long)n * n;
    const double beta = scal[(size_t)c * UVMEM_NSCAL + UVMEM_S_BETA];
    const bool stop = chan[(size_t)c * CH_N + CH_STOP] != 0.0;
    double acc[1] = {0.0};
    for (int r = 0; r < PIX_BLK / NTHR; ++r) {
        const long long p = (long long)pb * PIX_BLK + r * NTHR + threadIdx.x;
        if (p >= npix) break;
        const size_t q = (size_t)c * npix + p;
        const double x = (double)I[q], gv = (double)g[q], gtv = (double)gt[q];
        double d = -gtv + beta * (double)dir[q];
        const bool atb = x <= Mb * (1.0 + BOUND_TOL);
        if (atb && gv > 0.0) d = 0.0;
        else if (atb) d = fmax(d, 0.0);
        if (stop) d = 0.0;
        const R dr = (R)d;
        dir[q] = dr;
        acc[0] += gtv * (double)dr;
    }
    block_sum<1>(acc);
    if (threadIdx.x == 0) ppart[((size_t)c * n_pb + pb) * NPART + 0] = acc[0];
}

// Step 2: restart test per channel.
__global__ __launch_bounds__(NTHR) void k_chan_gtd(const double *__restrict__ ppart, int n_pb,
                                                   const double *__restrict__ scal, double *__restrict__ chan) {
    const int c = blockIdx.x;
    double gtd[1];
    sum_partials<1>(ppart + (size_t)c * n_pb * NPART, n_pb, 0, gtd);
    if (threadIdx.x == 0) {
        double *ch = chan + (size_t)c * CH_N;
        const double gg = scal[(size_t)c * UVMEM_NSCAL + UVMEM_S_GNORM2];
        if (gg == 0.0) ch[CH_STOP] = 1.0;
        const bool restart = gtd[0] >= 0.0;
        ch[CH_RESTART] = restart ? 1.0 : 0.0;
        ch[CH_GTD] = restart ? -gg : gtd[0];
        ch[CH_GG_OLD] = gg;
    }
}

// Step 3: apply the restart, stage B = A o d for the forward model, and the
// partials of alpha_max, phi'(0) - b and phi''(0) - a (entropy parts).
template <typename R, int SPLIT>
__global__ __launch_bounds__(NTHR) void k_cg_dir2(const R *__restrict__ I, const R *__restrict__ gt,
                                                  R *__restrict__ dir, const R *__restrict__ beam,
                                                  void *__restrict__ bop, size_t lo_off,
                                                  const double *__restrict__ chan,
                                                  double *__restrict__ ppart, int n, int np, int n_pb,
                                                  double M, double Mb) {
    const int c = blockIdx.x / n_pb, pb = blockIdx.x % n_pb;
    const long long npix = (long long)n * n;
    const bool restart = chan[(size_t)c * CH_N + CH_RESTART] != 0.0;
    const bool stop = chan[(size_t)c * CH_N + CH_STOP] != 0.0;
    const size_t cb = (size_t)c * np * np;
    double amax = INFINITY;
    double acc[2] = {0.0, 0.0};
    for (int r = 0; r < PIX_BLK / NTHR; ++r) {
        const long long p = (long long)pb * PIX_BLK + r * NTHR + threadIdx.x;
        if (p >= npix) break;
        const size_t q = (size_t)c * npix + p;
        double d = (double)dir[q];
        if (restart) d = -(double)gt[q];
        if (stop) d = 0.0;
        const R dr = (R)d;
        d = (double)dr;
        dir[q] = dr;
        const int i = (int)(p / n), j = (int)(p % n);
        store_op<R, SPLIT>(bop, cb + (size_t)i * np + j, lo_off, beam[q] * dr);
        const double x = (double)I[q];
        if (d < 0.0) amax = fmin(amax, (x - Mb) / (-d));
        acc[0] += d * (log(x / M) + 1.0);
        acc[1] += d * d / x;
    }
    amax = block_min(amax);
    block_sum<2>(acc);
    if (threadIdx.x == 0) {
        double *pp = ppart + ((size_t)c * n_pb + pb) * NPART;
        pp[0] = acc[0];
        pp[1] = acc[1];
        pp[2] = amax;
    }
}

// ---- line search: exact minimisation of the convex phi on [0, alpha_max]
//   phi'(al)  = b + a al + lambda sum d (ln((I + al d)/M) + 1)
//   phi''(al) = a + lambda sum d^2 / (I + al d)
// State machine shared by all workgroups of a channel (see update_ls).
enum { PH_CHECK = 0, PH_GROW = 1, PH_NEWTON = 2, PH_DONE = 3 };

__device__ __forceinline__ void ls_finish(double *st, double al) {
    st[LSS_PHASE] = PH_DONE;
    st[LSS_ALPHA] = al;
    st[LSS_TRY] = al;
}

// Advance the state given phi'(try) = f1 and phi''(try) = f2.
__device__ void update_ls(double *st, double f1, double f2) {
    const int ph = (int)st[LSS_PHASE];
    const double t = st[LSS_TRY];
    if (ph == PH_DONE) return;
    if (ph == PH_CHECK) {
        if (f1 <= 0.0) { ls_finish(st, t); return; }
        st[LSS_HI] = t;
        st[LSS_PHASE] = PH_NEWTON;
        // restart Newton from the root of the chi^2 part when inside the bracket
        const double a = st[LSS_A], b = st[LSS_B];
        double nxt = 0.5 * (st[LSS_LO] + st[LSS_HI]);
        if (a > 0.0) {
            const double gsx = -b / a;
            if (gsx > st[LSS_LO] && gsx < st[LSS_HI]) nxt = gsx;
        }
        st[LSS_TRY] = nxt;
        return;
    }
    if (f1 == 0.0) { ls_finish(st, t); return; }
    if (f1 > 0.0) st[LSS_HI] = t; else st[LSS_LO] = t;
    if (ph == PH_GROW && f1 < 0.0) {
        double nxt = f2 > 0.0 ? t - f1 / f2 : 2.0 * t;
        if (!(nxt > t) || !isfinite(nxt)) nxt = 2.0 * t;
        st[LSS_TRY] = nxt;
        return;
    }
    st[LSS_PHASE] = PH_NEWTON;
    const double lo = st[LSS_LO], hi = st[LSS_HI];
    double nxt = f2 > 0.0 ? t - f1 / f2 : 0.5 * (lo + hi);
    if (!(nxt > lo && nxt < hi)) nxt = 0.5 * (lo + hi);
    if (fabs(nxt - t) <= 1e-13 * fabs(nxt)) { ls_finish(st, nxt); return; }
    st[LSS_TRY] = nxt;
}

// Step 6: initialise the line search of each channel.
__global__ __launch_bounds__(NTHR) void k_chan_ls_init(const double *__restrict__ vispart, const int *__restrict__ vis_base,
                                                       const double *__restrict__ ppart, int n_pb, double lam,
                                                       const double *__restrict__ chan, double *__restrict__ ls) {
    const int c = blockIdx.x;
    double ab[2], ent[2];
    sum_partials<2>(vispart + (size_t)vis_base[c] * NPART, vis_base[c + 1] - vis_base[c], 0, ab);
    sum_partials<2>(ppart + (size_t)c * n_pb * NPART, n_pb, 0, ent);
    const double amax = min_partials(ppart + (size_t)c * n_pb * NPART, n_pb, 2);
    if (threadIdx.x == 0) {
        double *st = ls + (size_t)c * LSS_N;
        const double a = ab[0], b = ab[1];
        const bool stop = chan[(size_t)c * CH_N + CH_STOP] != 0.0;
        st[LSS_A] = a;
        st[LSS_B] = b;
        st[LSS_AMAX] = isfinite(amax) ? amax : -1.0;
        st[LSS_LO] = 0.0;
        st[LSS_HI] = isfinite(amax) ? amax : -1.0;
        st[LSS_STOP] = stop ? 1.0 : 0.0;
        const double f1 = b + lam * ent[0];     // phi'(0)
        const double f2 = a + lam * ent[1];     // phi''(0)
        if (stop || !(f1 < 0.0)) {
            ls_finish(st, 0.0);
        } else if (isfinite(amax)) {
            st[LSS_PHASE] = PH_CHECK;
            st[LSS_TRY] = amax;
        } else {
            st[LSS_PHASE] = PH_GROW;
            double t = f2 > 0.0 ? -f1 / f2 : 1.0;
            if (!(t > 0.0) || !isfinite(t)) t = 1.0;
            st[LSS_TRY] = t;
        }
    }
}

// Reads the previous state and partials (if any), advances the state (all
// workgroups of the channel compute the same bits; workgroup 0 stores it) and
// evaluates phi' and phi'' partials at the new trial step.
template <typename R>
__global__ __launch_bounds__(NTHR) void k_ls_step(const R *__restrict__ I, const R *__restrict__ dir,
                                                  const double *__restrict__ ls_prev, double *__restrict__ ls_next,
                                                  const double *__restrict__ pp_prev, double *__restrict__ pp_next,
                                                  int n, int n_pb, double M, double lam, int first) {
    const int c = blockIdx.x / n_pb, pb = blockIdx.x % n_pb;
    const long long npix = (long long)n * n;
    __shared__ double st[LSS_N];
    if (threadIdx.x < LSS_N) st[threadIdx.x] = ls_prev[(size_t)c * LSS_N + threadIdx.x];
    __syncthreads();
    if (!first && (int)st[LSS_PHASE] != PH_DONE) {
        double e[2];
        sum_partials<2>(pp_prev + (size_t)c * n_pb * NPART, n_pb, 0, e);
        if (threadIdx.x == 0) {
            const double t = st[LSS_TRY];
            update_ls(st, st[LSS_B] + st[LSS_A] * t + lam * e[0], st[LSS_A] + lam * e[1]);
        }
    }
    __syncthreads();
    if (pb == 0 && threadIdx.x < LSS_N) ls_next[(size_t)c * LSS_N + threadIdx.x] = st[threadIdx.x];
    if ((int)st[LSS_PHASE] == PH_DONE) return;
    const double al = st[LSS_TRY];
    double acc[2] = {0.0, 0.0};
    for (int r = 0; r < PIX_BLK / NTHR; ++r) {
        const long long p = (long long)pb * PIX_BLK + r * NTHR + threadIdx.x;
        if (p >= npix) break;
        const size_t q = (size_t)c * npix + p;
        const double d = (double)dir[q];
        const double x = (double)I[q] + al * d;
        acc[0] += d * (log(x / M) + 1.0);
        acc[1] += d * d / x;
    }
    block_sum<2>(acc);
    if (threadIdx.x == 0) {
        pp_next[((size_t)c * n_pb + pb) * NPART + 0] = acc[0];
        pp_next[((size_t)c * n_pb + pb) * NPART + 1] = acc[1];
    }
}

// Step 8: final line-search update, then I <- max(I + alpha d, M) and the
// entropy partial of the new image.
template <typename R>
__global__ __launch_bounds__(NTHR) void k_cg_update(R *__restrict__ I, const R *__restrict__ dir,
                                                    const double *__restrict__ ls_prev, const double *__restrict__ pp_prev,
                                                    double *__restrict__ pp_out, double *__restrict__ scal,
                                                    double *__restrict__ chan, int *__restrict__ flag,
                                                    int n, int n_pb, double M, double Mb, double lam) {
    const int c = blockIdx.x / n_pb, pb = blockIdx.x % n_pb;
    const long long npix = (long long)n * n;
    __shared__ double st[LSS_N];
    if (threadIdx.x < LSS_N) st[threadIdx.x] = ls_prev[(size_t)c * LSS_N + threadIdx.x];
    __syncthreads();
    if ((int)st[LSS_PHASE] != PH_DONE) {
        double e[2];
        sum_partials<2>(pp_prev + (size_t)c * n_pb * NPART, n_pb, 0, e);
        if (threadIdx.x == 0) {
            const double t = st[LSS_TRY];
            update_ls(st, st[LSS_B] + st[LSS_A] * t + lam * e[0], st[LSS_A] + lam * e[1]);
            if ((int)st[LSS_PHASE] != PH_DONE) {
                // not converged within the fixed budget: take the bracketed trial
                double al = st[LSS_TRY];
                if (st[LSS_HI] >= 0.0) al = fmin(al, st[LSS_HI]);
                al = fmax(al, st[LSS_LO]);
                ls_finish(st, al);
            }
        }
    }
    __syncthreads();
    const double al = st[LSS_ALPHA];
    if (pb == 0 && threadIdx.x == 0) {
        double *sc = scal + (size_t)c * UVMEM_NSCAL;
        sc[UVMEM_S_ALPHA] = al;
        sc[UVMEM_S_ALPHA_MAX] = st[LSS_AMAX] < 0.0 ? INFINITY : st[LSS_AMAX];
        if (al == 0.0) chan[(size_t)c * CH_N + CH_STOP] = 1.0;
    }
    double acc[1] = {0.0};
    int bad = 0;
    for (int r = 0; r < PIX_BLK / NTHR; ++r) {
        const long long p = (long long)pb * PIX_BLK + r * NTHR + threadIdx.x;
        if (p >= npix) break;
        const size_t q = (size_t)c * npix + p;
        double x = (double)I[q];
        if (al != 0.0) {
            x = fmax(x + al * (double)dir[q], Mb);
            const R xr = (R)x;
            I[q] = xr;
            x = (double)xr;
        }
        if (!(x > 0.0)) bad = 1;
        else acc[0] += x * log(x / M);
    }
    if (bad) atomicOr(flag, 1);
    block_sum<1>(acc);
    if (threadIdx.x == 0) pp_out[((size_t)c * n_pb + pb) * NPART + 0] = acc[0];
}

// Step 12: Polak-Ribiere beta (clipped at 0) and the per-channel scalars.
__global__ __launch_bounds__(NTHR) void k_chan_beta(const double *__restrict__ vispart, const int *__restrict__ vis_base,
                                                    const double *__restrict__ pp_S, const double *__restrict__ pp_g,
                                                    int n_pb, double lam, double *__restrict__ scal,
                                                    double *__restrict__ chan, double *__restrict__ user) {
    const int c = blockIdx.x;
    double x2[1], S[1], gg[2];
    sum_partials<1>(vispart + (size_t)vis_base[c] * NPART, vis_base[c + 1] - vis_base[c], 0, x2);
    sum_partials<1>(pp_S + (size_t)c * n_pb * NPART, n_pb, 0, S);
    sum_partials<2>(pp_g + (size_t)c * n_pb * NPART, n_pb, 0, gg);
    if (threadIdx.x == 0) {
        double *sc = scal + (size_t)c * UVMEM_NSCAL;
        double *ch = chan + (size_t)c * CH_N;
        const double chi2 = 0.5 * x2[0];
        const double gold = ch[CH_GG_OLD];
        const bool stop = ch[CH_STOP] != 0.0;
        double beta = 0.0;
        if (!stop && gold > 0.0) beta = fmax(0.0, (gg[0] - gg[1]) / gold);
        sc[UVMEM_S_PHI] = chi2 + lam * S[0];
        sc[UVMEM_S_CHI2] = chi2;
        sc[UVMEM_S_S] = S[0];
        sc[UVMEM_S_BETA] = beta;
        sc[UVMEM_S_GNORM2] = gg[0];
        if (sc[UVMEM_S_ALPHA] != 0.0) sc[UVMEM_S_ITER] += 1.0;
        if (user) {
            for (int x = 0; x < UVMEM_NSCAL; ++x) user[(size_t)c * UVMEM_NSCAL + x] = sc[x];
        }
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

template <typename R> inline R *P(void *p) { return reinterpret_cast<R *>(p); }
template <typename R> inline const R *CP(const void *p) { return reinterpret_cast<const R *>(p); }

inline int pix_grid(const uvmem_ctx *c) { return c->nchan * c->n_pb; }
inline double *pp(const uvmem_ctx *c, int buf) {
    return c->d_ppart + (size_t)buf * c->nchan * c->n_pb * NPART;
}
inline double *lsb(const uvmem_ctx *c, int buf) { return c->d_ls + (size_t)buf * c->nchan * LSS_N; }

inline size_t lo_off(const uvmem_ctx *c) { return (size_t)c->nchan * c->np * c->np; }

template <typename R, int SPLIT>
hipError_t t_prologue(const uvmem_ctx *c, const void *I, int with_entropy, hipStream_t st) {
    hipLaunchKernelGGL((k_prologue<R, SPLIT>), dim3(pix_grid(c)), dim3(NTHR), 0, st, CP<R>(I), CP<R>(c->d_beam),
                       c->d_bop, lo_off(c), pp(c, 0), c->d_flag, c->n, c->np, c->n_pb, c->M, with_entropy);
    return hipGetLastError();
}

template <typename R>
hipError_t t_grad(const uvmem_ctx *c, const void *I, void *out, int mode, hipStream_t st) {
    hipLaunchKernelGGL(k_grad<R>, dim3(pix_grid(c)), dim3(NTHR), 0, st, c->d_gpart, c->d_slot_base,
                       CP<R>(c->d_beam), CP<R>(I), P<R>(out), P<R>(c->d_gt), pp(c, 1), c->n, c->np, c->n_pb,
                       c->M, c->Mb, c->lam, mode);
    return hipGetLastError();
}

template <typename R>
hipError_t t_cg_init_dir(const uvmem_ctx *c, const void *I, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_init<R>, dim3(pix_grid(c)), dim3(NTHR), 0, st, CP<R>(I), CP<R>(c->d_g),
                       P<R>(c->d_gt), P<R>(c->d_dir), pp(c, 0), c->n, c->n_pb, c->Mb);
    hipLaunchKernelGGL(k_chan_cg_init, dim3(c->nchan), dim3(NTHR), 0, st, pp(c, 0), c->n_pb, c->d_scal,
                       c->d_chan);
    return hipGetLastError();
}

template <typename R, int SPLIT>
hipError_t t_cg_step(const uvmem_ctx *c, void *I, double *user, hipStream_t st);

}  // namespace

hipError_t launch_fill(const uvmem_ctx *c, void *img, double value, hipStream_t st) {
    const long long count = (long long)c->nchan * c->n * c->n;
    const int blocks = (int)std::min<long long>((count + NTHR - 1) / NTHR, 4096);
    if (c->prec == UVMEM_FP64)
        hipLaunchKernelGGL(k_fill<double>, dim3(blocks), dim3(NTHR), 0, st, P<double>(img), value, count);
    else
        hipLaunchKernelGGL(k_fill<float>, dim3(blocks), dim3(NTHR), 0, st, P<float>(img), (float)value, count);
    return hipGetLastError();
}

hipError_t launch_prologue(const uvmem_ctx *c, const void *I, int with_entropy, hipStream_t st) {
    if (c->prec == UVMEM_FP64) return t_prologue<double, 0>(c, I, with_entropy, st);
    if (c->prec == UVMEM_BF16X3) return t_prologue<float, 1>(c, I, with_entropy, st);
    return t_prologue<float, 0>(c, I, with_entropy, st);
}

hipError_t launch_vis_sum(const uvmem_ctx *c, int mode, double2 *out, hipStream_t st) {
    if (c->n_visit == 0) return hipSuccess;
    hipLaunchKernelGGL(k_vis, dim3(c->n_visit), dim3(NTHR), 0, st, c->d_vis, c->d_vpart, c->n_ib,
                       (long long)c->ztot, c->d_vo, c->d_w, c->d_R, c->d_Vd, out, c->d_scal, c->d_vispart, mode);
    return hipGetLastError();
}

hipError_t launch_grad(const uvmem_ctx *c, const void *I, void *out, int mode, hipStream_t st) {
    return c->prec == UVMEM_FP64 ? t_grad<double>(c, I, out, mode, st) : t_grad<float>(c, I, out, mode, st);
}

hipError_t launch_chan_phi(const uvmem_ctx *c, double *user_scal, hipStream_t st) {
    hipLaunchKernelGGL(k_chan_phi, dim3(c->nchan), dim3(NTHR), 0, st, c->d_vispart, c->d_vis_base, pp(c, 0),
                       c->n_pb, c->lam, c->d_scal, user_scal);
    return hipGetLastError();
}

hipError_t launch_cg_init_dir(const uvmem_ctx *c, const void *I, hipStream_t st) {
    return c->prec == UVMEM_FP64 ? t_cg_init_dir<double>(c, I, st) : t_cg_init_dir<float>(c, I, st);
}

hipError_t launch_copy_scal(const uvmem_ctx *c, double *, long long *ctr, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_hist, dim3(1), dim3(NTHR), 0, st, c->d_scal,
                       reinterpret_cast<const long long *>(c->d_hist_ptr), ctr, c->nchan * UVMEM_NSCAL);
    return hipGetLastError();
}

namespace {
template <typename R, int SPLIT>
hipError_t t_cg_step(const uvmem_ctx *c, void *I, double *user, hipStream_t st) {
    hipError_t e;
    const dim3 gp(pix_grid(c)), gc(c->nchan), blk(NTHR);
    // 1. direction update and projection; partial gt.d
    hipLaunchKernelGGL(k_cg_dir<R>, gp, blk, 0, st, CP<R>(I), CP<R>(c->d_g), CP<R>(c->d_gt), P<R>(c->d_dir),
                       c->d_scal, c->d_chan, pp(c, 0), c->n, c->n_pb, c->Mb);
    // 2. restart test
    hipLaunchKernelGGL(k_chan_gtd, gc, blk, 0, st, pp(c, 0), c->n_pb, c->d_scal, c->d_chan);
    // 3. restart, B = A o d, alpha_max and entropy parts of phi'(0), phi''(0)
    hipLaunchKernelGGL((k_cg_dir2<R, SPLIT>), gp, blk, 0, st, CP<R>(I), CP<R>(c->d_gt), P<R>(c->d_dir),
                       CP<R>(c->d_beam), c->d_bop, lo_off(c), c->d_chan, pp(c, 1), c->n, c->np, c->n_pb, c->M,
                       c->Mb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // 4. Vd = F(d)
    return hipSuccess;
}
}  // namespace

// The CG step is split so that the host can bracket the DFT launches with
// timing events: cg_phase(c, I, user, phase, st) with phase 0 = before the
// forward model, 1 = between forward and adjoint, 2 = after the adjoint.
hipError_t launch_cg_phase(const uvmem_ctx *c, void *I, double *user, int phase, hipStream_t st);

hipError_t launch_cg_step(const uvmem_ctx *c, void *I, double *user, hipStream_t st) {
    hipError_t e;
    if ((e = launch_cg_phase(c, I, user, 0, st)) != hipSuccess) return e;
    if ((e = launch_forward(c, c->d_bop, st)) != hipSuccess) return e;
    if ((e = launch_cg_phase(c, I, user, 1, st)) != hipSuccess) return e;
    if ((e = launch_adjoint(c, c->d_R, c->d_w, st)) != hipSuccess) return e;
    return launch_cg_phase(c, I, user, 2, st);
}

namespace {
template <typename R, int SPLIT>
hipError_t t_cg_phase(const uvmem_ctx *c, void *I, double *user, int phase, hipStream_t st) {
    const dim3 gp(pix_grid(c)), gc(c->nchan), blk(NTHR);
    if (phase == 0) return t_cg_step<R, SPLIT>(c, I, user, st);
    if (phase == 1) {
        // 5. Vd and the quadratic coefficients a, b of chi^2 along d
        if (c->n_visit)
            hipLaunchKernelGGL(k_vis, dim3(c->n_visit), blk, 0, st, c->d_vis, c->d_vpart, c->n_ib,
                               (long long)c->ztot, c->d_vo, c->d_w, c->d_R, c->d_Vd, (double2 *)nullptr,
                               c->d_scal, c->d_vispart, 2);
        // 6. line-search initialisation
        hipLaunchKernelGGL(k_chan_ls_init, gc, blk, 0, st, c->d_vispart, c->d_vis_base, pp(c, 1), c->n_pb,
                           c->lam, c->d_chan, lsb(c, 0));
        // 7. fixed number of Newton / bisection evaluations
        for (int t = 0; t < LS_STEPS; ++t) {
            // launch t: state S^t-1 from ls[t%2] (S^0 from the initialisation),
            // partials P^t-1 from pp[(t+1)%2]; writes S^t to ls[(t+1)%2] and
            // P^t (phi', phi'' at the new trial) to pp[t%2]
            hipLaunchKernelGGL(k_ls_step<R>, gp, blk, 0, st, CP<R>(I), CP<R>(c->d_dir), lsb(c, t % 2),
                               lsb(c, (t + 1) % 2), pp(c, (t + 1) % 2), pp(c, t % 2), c->n, c->n_pb, c->M,
                               c->lam, t == 0 ? 1 : 0);
        }
        const int last = (LS_STEPS - 1) % 2;   // pp buffer holding the last partials
        // 8. final update of the step, I <- max(I + alpha d, M), entropy partial
        hipLaunchKernelGGL(k_cg_update<R>, gp, blk, 0, st, P<R>(I), CP<R>(c->d_dir), lsb(c, 1 - last),
                           pp(c, last), pp(c, 1 - last), c->d_scal, c->d_chan, c->d_flag, c->n, c->n_pb, c->M,
                           c->Mb, c->lam);
        // 9. R <- R + alpha Vd, chi^2 partials
        if (c->n_visit)
            hipLaunchKernelGGL(k_vis, dim3(c->n_visit), blk, 0, st, c->d_vis, c->d_vpart, c->n_ib,
                               (long long)c->ztot, c->d_vo, c->d_w, c->d_R, c->d_Vd, (double2 *)nullptr,
                               c->d_scal, c->d_vispart, 3);
        return hipGetLastError();
    }
    // 11. gradient at the new point, projected gradient, PR partials
    const int last = (LS_STEPS - 1) % 2;
    hipLaunchKernelGGL(k_grad<R>, gp, blk, 0, st, c->d_gpart, c->d_slot_base, CP<R>(c->d_beam), CP<R>(I),
                       P<R>(c->d_g), P<R>(c->d_gt), pp(c, last), c->n, c->np, c->n_pb, c->M, c->Mb, c->lam, 2);
    // 12. beta and scalars
    hipLaunchKernelGGL(k_chan_beta, gc, blk, 0, st, c->d_vispart, c->d_vis_base, pp(c, 1 - last), pp(c, last),
                       c->n_pb, c->lam, c->d_scal, c->d_chan, user);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_cg_phase(const uvmem_ctx *c, void *I, double *user, int phase, hipStream_t st) {
    if (c->prec == UVMEM_FP64) return t_cg_phase<double, 0>(c, I, user, phase, st);
    if (c->prec == UVMEM_BF16X3) return t_cg_phase<float, 1>(c, I, user, phase, st);
    return t_cg_phase<float, 0>(c, I, user, phase, st);
}

}  // namespace uvm
