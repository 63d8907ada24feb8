// Separable direct-DFT contractions on CDNA4 matrix cores (gfx950).
//
// Forward model (Eq. fft discretised at the measured (u, v)):
//   V_k = sum_i E_v[k,i] T[k,i],   T[k,i] = sum_j E_u[k,j] B[i,j],
//   E_u[k,j] = exp(-2 pi i a_k (j - N/2)),  E_v[k,i] = exp(-2 pi i b_k (i - N/2)),
//   a_k = u_k cell, b_k = v_k cell, B = A o I.
// The exponent of Eq. fft factorises over the two image axes, so the N^2-term
// sum per visibility becomes one complex-by-real matrix product over j (on
// MFMA) followed by a length-N row dot over i.
//
// Adjoint (Eq. chi2gradient / Alg. 3 without the beam factor, applied later):
//   G[i,j] = sum_k Re( P[k,i] conj(E_u[k,j]) ),  P[k,i] = c_k conj(E_v[k,i]),
//          = sum_k P_re[k,i] cos(2 pi a_k m_j) - P_im[k,i] sin(2 pi a_k m_j)
// a real matrix product with the visibilities as the contraction dimension,
// split over visibility chunks (split-K); chunk partials are summed in a fixed
// order by the gradient kernel, so results are bitwise reproducible.
//
// Phases are formed and reduced modulo one cycle in FP64 (t = a_k m); the FP64
// kernels take sincospi of the reduced phase, the FP32 ones cos and sin from
// the quadrant and remainder of 4 t (see cisphase), the split ones the
// hardware sine and cosine.
#include <cstdlib>

#include "internal.h"

namespace uvm {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;

// v_mfma_f32_16x16x4_f32: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// it holds D[4 (l/16) + r][l%16] in accumulator register r.
template <> struct Mfma<float> {
    typedef floatx4 acc;
    static __device__ __forceinline__ acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int g, int r) { return 4 * g + r; }
    static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
};

// v_mfma_f64_16x16x4_f64: same A/B lane layout as FP32, but lane l holds
// D[4 r + l/16][l%16] in accumulator register r (checked on gfx950).
template <> struct Mfma<double> {
    typedef doublex4 acc;
    static __device__ __forceinline__ acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int g, int r) { return 4 * r + g; }
    static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
};

__device__ __forceinline__ void cis2pi(double f, double &c, double &s) { sincospi(2.0 * f, &s, &c); }
__device__ __forceinline__ void cis2pi(float f, float &c, float &s) { sincospif(2.0f * f, &s, &c); }

// Reduced phase frac(a * m) in [-1/2, 1/2], formed in FP64.
__device__ __forceinline__ double phase(double a, int m) {
    double t = a * (double)m;
    return t - rint(t);
}

// cos and sin of 2 pi frac(a m).  FP64: sincospi of the reduced phase.
// FP32: u = 4 a m quarter turns (FP64) splits into the quadrant j = rint(u)
// and r = u - j in [-1/2, 1/2] (exact); cos and sin of (pi / 2) r come from
// minimax polynomials in r^2 fitted on [0, 1/2] (the sine's leading
// coefficient pi / 2 carried as a float plus a correction), then the result
// is rotated by j quarter turns.  Against FP64 cos and sin: within 1.01 ulp
// of those of the float remainder (sine polynomial 0.76 ulp, cosine 1.01),
// within 1.32 ulp of those of the FP64 phase (the float remainder's own
// rounding adds up to half an ulp).  The quadrant needs |a m| < 2^29 turns.
__device__ __forceinline__ void cisphase(double a, int m, double &c, double &s) { cis2pi(phase(a, m), c, s); }
__device__ __forceinline__ void cisphase(double a, int m, float &c, float &s) {
    const double u = a * (double)(4 * m);
    const double jd = rint(u);
    const float r = (float)(u - jd);
    const int j = (int)jd;
    const float z = r * r;
    float q = fmaf(z, -0x1.2edef6p-8f, 0x1.466626p-4f);
    q = fmaf(z, q, -0x1.4abbcep-1f);
    q = fmaf(z, q, -0x1.777a5cp-25f);
    const float sn = fmaf(r, 0x1.921fb6p+0f, r * q);
    float p = fmaf(z, 0x1.d9de14p-11f, -0x1.55c6a0p-6f);
    p = fmaf(z, p, 0x1.03c1e2p-2f);
    p = fmaf(z, p, -0x1.3bd3ccp+0f);
    const float cs = fmaf(z, p, 1.0f);
    const bool odd = (j & 1) != 0;
    const float cc = odd ? sn : cs, ss = odd ? cs : sn;
    c = ((j + 1) & 2) ? -cc : cc;
    s = (j & 2) ? -ss : ss;
}

// Sum over each 16-lane row of the wave with DPP lane moves instead of LDS
// permutes: quad swaps (xor 1, xor 2), then the half-row and row mirrors,
// which pair lanes in the same groups as an xor butterfly over 4 and 8, so
// every lane of the row ends with the same, identically rounded sum.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
__device__ __forceinline__ T row16_sum(T v) {
    v += dpp_mov<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_mov<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_mov<0x141>(v);   // row_half_mirror
    v += dpp_mov<0x140>(v);   // row_mirror
    return v;
}

template <typename T> struct C2T;
template <> struct C2T<float> { typedef float2 type; };
template <> struct C2T<double> { typedef double2 type; };

template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef float4 type; };
template <> struct Vec4<double> { typedef double4 type; };

// Column contraction of one 16-visibility tile of the forward against KT
// 16-row slices of the LDS image block, starting at slice t0:
//   acc[t][k][q'] = sum_j E_u[k][j] B[16 (t0 + t) + q'][j]  (real, imaginary)
// with E_u[k][j0 + 16 m + 4 g + s] = E(j0 + 16 m - N/2) E(4 g + s).
template <typename T, int KT, int JB, int LDB>
__device__ __forceinline__ void fwd_contract(const T (*sB)[LDB], int t0, double ak, int j0, int half, int q,
                                             int g, typename Mfma<T>::acc (&accR)[KT],
                                             typename Mfma<T>::acc (&accI)[KT]) {
    typedef typename Vec4<T>::type T4;
    T fc[4], fs[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) cisphase(ak, 4 * g + s, fc[s], fs[s]);
#pragma unroll
    for (int t = 0; t < KT; ++t) {
        accR[t] = Mfma<T>::zero();
        accI[t] = Mfma<T>::zero();
    }
    // coarse factors E(a_k (j0 + js - N/2)) of four 16-column steps: lane
    // group g computes step 4 u + g, the others read it by lane exchange
    for (int js0 = 0; js0 < JB; js0 += 64) {
        T cc4, sc4;
        cisphase(ak, j0 + js0 + 16 * g - half, cc4, sc4);
#pragma unroll 2
        for (int m = 0; m < 4; ++m) {
            const int js = js0 + 16 * m;
            const T cc = __shfl(cc4, q + 16 * m, 64), sc = __shfl(sc4, q + 16 * m, 64);
            T cr[4], ci[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                cr[s] = cc * fc[s] - sc * fs[s];
                ci[s] = -(sc * fc[s] + cc * fs[s]);
            }
            T4 bv[KT];
#pragma unroll
            for (int t = 0; t < KT; ++t) bv[t] = *reinterpret_cast<const T4 *>(&sB[16 * (t0 + t) + q][js + 4 * g]);
#pragma unroll
            for (int t = 0; t < KT; ++t) {
                accR[t] = Mfma<T>::mma(cr[0], bv[t].x, accR[t]);
                accI[t] = Mfma<T>::mma(ci[0], bv[t].x, accI[t]);
                accR[t] = Mfma<T>::mma(cr[1], bv[t].y, accR[t]);
                accI[t] = Mfma<T>::mma(ci[1], bv[t].y, accI[t]);
                accR[t] = Mfma<T>::mma(cr[2], bv[t].z, accR[t]);
                accI[t] = Mfma<T>::mma(ci[2], bv[t].z, accI[t]);
                accR[t] = Mfma<T>::mma(cr[3], bv[t].w, accR[t]);
                accI[t] = Mfma<T>::mma(ci[3], bv[t].w, accI[t]);
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Forward, FP32 / FP64, persistent.  A workgroup of eight waves keeps the
// image block [i0, i0 + IB) x [j0, j0 + JB) in LDS and streams 16-visibility
// tiles through its waves.  Twiddles come from FP64-reduced phases
// (cisphase): E_u[k][j0 + 16 m + 4 g + s] = E(j0 + 16 m - N/2) E(4 g + s);
// the row dot uses E_v = E(i0 + q - N/2) E(16 t), the second factors in a
// per-wave FP64 LDS table, accumulated in FP64.
template <typename T, int IB, int JB>
__global__ __launch_bounds__(512, 1) void k_forward_p(const FwdPItem *__restrict__ items,
                                                      const double *__restrict__ a,
                                                      const double *__restrict__ b,
                                                      const T *__restrict__ bop, double2 *__restrict__ vpart,
                                                      int n, int np, long long ztot) {
    typedef typename Mfma<T>::acc acc_t;
    typedef typename Vec4<T>::type T4;
    constexpr int NT = IB / 16;
    // rows padded by 8 floats (row stride = 8 mod 128 words): the 128-bit
    // operand reads of 32 lanes (16 rows x two 4-column groups) then cover
    // distinct banks; a 4-float pad measured one bank conflict per read
    constexpr int PADC = 8;
    __shared__ __attribute__((aligned(16))) T sB[IB][JB + PADC];
    // coarse row factors in FP64 (converted once when stored); one pad
    // entry per row, so that the four rows a read touches (4 g + r) start
    // in different banks
    __shared__ double2 sCo[8][16][NT + 1];

    const FwdPItem it = items[blockIdx.x];
    const int i0 = it.ib * IB, j0 = it.jb * JB;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int q = lane & 15, g = lane >> 4;
    const int half = n / 2;
    {
        const T *B = bop + (size_t)it.chan * np * np;
        constexpr int VROW = JB / 4;
        for (int x = tid; x < IB * VROW; x += 512) {
            const int row = x / VROW, c4 = x % VROW;
            *reinterpret_cast<T4 *>(&sB[row][4 * c4]) =
                *reinterpret_cast<const T4 *>(B + (size_t)(i0 + row) * np + j0 + 4 * c4);
        }
    }
    __syncthreads();
    const long long nk = it.kend - it.kbeg;
    const long long ntiles = (nk + 15) / 16;
    // tile wave * nwg + wg of each round: a round's leftover tiles go to one
    // wave of distinct workgroups, so no CU carries them on all its SIMDs.
    // With eight 16-row slices per block and at most two leftover tiles per
    // workgroup, the eight waves share each leftover tile instead, a slice
    // each (a single wave would keep one SIMD busy for a whole tile after
    // the others have finished).
    const long long stride = 8LL * it.nwg;
    const long long nfull = ntiles / stride * stride;
    const bool share = NT == 8 && ntiles > nfull && (ntiles - nfull + it.nwg - 1) / it.nwg <= 2;
    const long long tend = share ? nfull : ntiles;
    // the coordinates a tile needs, loaded one tile ahead: the eight waves
    // reach their tile boundaries together, so a load issued at the boundary
    // would stall them all at once
    constexpr int NCO = 16 * NT / 64;   // coarse-table entries per lane
    static_assert(16 * NT % 64 == 0, "image blocks of 64 or 128 rows");
    struct TileK {
        double ak, bco[NCO], br[4];
    };
    auto load_k = [&](long long tile, TileK &tk) {
        const long long k0 = it.kbeg + 16 * tile;
        const long long nv = it.kend - k0;   // <= 0 past the last tile
        tk.ak = q < nv ? a[k0 + q] : 0.0;
#pragma unroll
        for (int m = 0; m < NCO; ++m) {
            const int kk = (lane + 64 * m) / NT;
            tk.bco[m] = kk < nv ? b[k0 + kk] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int kk = Mfma<T>::drow(g, r);
            tk.br[r] = kk < nv ? b[k0 + kk] : 0.0;
        }
    };
    TileK cur;
    load_k((long long)wave * it.nwg + it.wg, cur);
    for (long long tile = (long long)wave * it.nwg + it.wg; tile < tend; tile += stride) {
        const long long k0 = it.kbeg + 16 * tile;
        const int nvalid = (int)(it.kend - k0 < 16 ? it.kend - k0 : 16);
        const TileK tk = cur;
        load_k(tile + stride, cur);
        acc_t accR[NT], accI[NT];
        fwd_contract<T, NT, JB>(sB, 0, tk.ak, j0, half, q, g, accR, accI);
        // per-wave coarse factors E(16 b_k t) of the tile's 16 rows
#pragma unroll
        for (int m = 0; m < NCO; ++m) {
            const int e = lane + 64 * m;
            const int kk = e / NT, t = e % NT;
            T c, sn;
            cisphase(tk.bco[m], 16 * t, c, sn);
            sCo[wave][kk][t] = make_double2((double)c, (double)sn);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int kk = Mfma<T>::drow(g, r);
            const bool ok = kk < nvalid;
            const double bk = tk.br[r];
            T fcq, fsq;
            cisphase(bk, i0 + q - half, fcq, fsq);
            // conj(E_v) T = conj(fine) sum_t conj(coarse_t) T_t, in FP64
            double wr = 0.0, wi = 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double2 co = sCo[wave][kk][t];
                const double tr = (double)accR[t][r], ti = (double)accI[t][r];
                wr += co.x * tr + co.y * ti;
                wi += co.x * ti - co.y * tr;
            }
            const double fc = (double)fcq, fs = (double)fsq;
            double vr = fc * wr + fs * wi, vi = fc * wi - fs * wr;
            vr = row16_sum(vr);
            vi = row16_sum(vi);
            if (q == 0 && ok) vpart[(size_t)it.part * ztot + k0 + kk] = make_double2(vr, vi);
        }
        __builtin_amdgcn_wave_barrier();
    }
    if constexpr (NT == 8) {
        if (!share) return;
        // wave w contracts rows [i0 + 16 w, i0 + 16 w + 16) of the tile with
        // the row twiddle E(b_k (i0 + 16 w + q - N/2)) formed directly; the
        // eight slice sums are added in slice order
        __shared__ double2 sSl[8][16];
        for (long long tile = nfull + it.wg; tile < ntiles; tile += it.nwg) {
            const long long k0 = it.kbeg + 16 * tile;
            const int nvalid = (int)(it.kend - k0 < 16 ? it.kend - k0 : 16);
            const double ak = q < nvalid ? a[k0 + q] : 0.0;
            acc_t accR[1], accI[1];
            fwd_contract<T, 1, JB>(sB, wave, ak, j0, half, q, g, accR, accI);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int kk = Mfma<T>::drow(g, r);
                const double bk = kk < nvalid ? b[k0 + kk] : 0.0;
                T ce, se;
                cisphase(bk, i0 + 16 * wave + q - half, ce, se);
                const double cd = (double)ce, sd = (double)se;
                const double tr = (double)accR[0][r], ti = (double)accI[0][r];
                const double vr = row16_sum(cd * tr + sd * ti);
                const double vi = row16_sum(cd * ti - sd * tr);
                if (q == 0) sSl[wave][kk] = make_double2(vr, vi);
            }
            __syncthreads();
            if (tid < nvalid) {
                double vr = 0.0, vi = 0.0;
#pragma unroll
                for (int w = 0; w < 8; ++w) {
                    vr += sSl[w][tid].x;
                    vi += sSl[w][tid].y;
                }
                vpart[(size_t)it.part * ztot + k0 + tid] = make_double2(vr, vi);
            }
            __syncthreads();
        }
    }
}

// ----------------------------------------------------------------------------
// Adjoint.  Workgroup tile TT x TT pixels (TT = 2 WT), 2 x 2 waves of WT x WT.
// Per 16-visibility super-step the workgroup writes to LDS, for k in the step,
//   Hv[k][q] = c_k w_k exp(+2 pi i b_k (i0 + q - N/2)),  Gv[k][t] = exp(+2 pi i b_k 16 t)
//   Fu[k][q] = exp(+2 pi i a_k (j0 + q - N/2)),          Gu[k][t] = exp(+2 pi i a_k 16 t)
// so that P[k][i0 + 16 t + q] = Hv[k][q] Gv[k][t] and the cos/sin operand at
// column j0 + 16 t + q is Fu[k][q] Gu[k][t] (one product per operand of two
// factors from cisphase).  MFMA #s of lane group g contracts visibility
// 4 g + s of the step.  FP32 accumulators are folded into FP64 ones every
// FLUSH super-steps.
// ----------------------------------------------------------------------------

template <typename T, int WT>
__global__ __launch_bounds__(256) void k_adjoint(const AdjItem *__restrict__ items,
                                                 const double *__restrict__ a,
                                                 const double *__restrict__ b,
                                                 const double2 *__restrict__ coef,
                                                 const float *__restrict__ w,
                                                 double *__restrict__ gpart, int n, int np) {
    typedef typename Mfma<T>::acc acc_t;
    typedef typename C2T<T>::type C2;
    constexpr int TT = 2 * WT;
    constexpr int NT = WT / 16;
    constexpr int NC = TT / 16;
    constexpr int FLUSH = 16;
    __shared__ C2 sHv[2][16][16], sFu[2][16][16], sGv[2][16][NC], sGu[2][16][NC];
    // FP64 fold of the FP32 sums, one slot per (wave, tile, register, lane):
    // each lane reads and writes only its own slots
    constexpr int NACC = sizeof(T) == 4 ? 4 * NT * NT * 4 * 64 : 1;
    __shared__ double sAcc[NACC];

    const AdjItem it = items[blockIdx.x];
    const int i0 = it.ti * TT, j0 = it.tj * TT;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int q = lane & 15, g = lane >> 4;
    const int ci0 = (wave >> 1) * NT;   // wave's first coarse i-tile
    const int cj0 = (wave & 1) * NT;    // wave's first coarse j-tile
    const int half = n / 2;

    acc_t acc[NT][NT];
    auto slot = [&](int x, int y, int r) { return (((wave * NT + x) * NT + y) * 4 + r) * 64 + lane; };
#pragma unroll
    for (int x = 0; x < NT; ++x)
#pragma unroll
        for (int y = 0; y < NT; ++y) {
            acc[x][y] = Mfma<T>::zero();
            if constexpr (sizeof(T) == 4) {
#pragma unroll
                for (int r = 0; r < 4; ++r) sAcc[slot(x, y, r)] = 0.0;
            }
        }

    // this thread's table tasks: fine (k = tid >> 4, q = tid & 15) and, for
    // tid < 32 NC, one coarse entry (axis `which`, k2, t2); the visibility data
    // of the next step are loaded while the current step computes
    const int fkk = tid >> 4, fqq = tid & 15;
    const bool has_c = tid < 32 * NC;
    const int which = tid / (16 * NC);
    const int ck2 = (tid % (16 * NC)) / NC, ct2 = tid % NC;
    struct Pre {
        double a, b, cab;
        double2 c;
        float w;
    };
    // branch-free prefetch: indices past the chunk end are clamped to its last
    // visibility and their weight is zeroed (so the step's tables are zero)
    const double *cab_src = which ? a : b;
    auto fetch = [&](long long kb, Pre &p) {
        const long long k = kb + fkk, kc = kb + ck2;
        const long long kl = k < it.kend ? k : it.kend - 1;
        const long long kcl = kc < it.kend ? kc : it.kend - 1;
        p.a = a[kl];
        p.b = b[kl];
        p.c = coef[kl];
        const float wv = w ? w[kl] : 1.f;
        p.w = k < it.kend ? wv : 0.f;
        p.cab = cab_src[kcl];
    };
    // twiddle tables of the step starting at kb from its prefetched data, into
    // buffer `buf` (branch-free: entries past the chunk end are zero)
    auto gen = [&](int buf, long long kb, const Pre &p) {
        T c, s;
        cisphase(p.b, i0 + fqq - half, c, s);
        const double cr = (double)p.w * p.c.x, cim = (double)p.w * p.c.y;
        C2 hv, fu;
        hv.x = (T)(cr * (double)c - cim * (double)s);
        hv.y = (T)(cr * (double)s + cim * (double)c);
        cisphase(p.a, j0 + fqq - half, c, s);
        const bool live = kb + fkk < it.kend;
        fu.x = live ? c : (T)0;
        fu.y = live ? s : (T)0;
        sHv[buf][fkk][fqq] = hv;
        sFu[buf][fkk][fqq] = fu;
        if (has_c) {
            cisphase(p.cab, 16 * ct2, c, s);
            C2 *dst = which ? &sGu[buf][ck2][ct2] : &sGv[buf][ck2][ct2];
            *dst = C2{c, s};
        }
    };
    Pre cur, nxt;
    fetch(it.kbeg, cur);
    gen(0, it.kbeg, cur);
    fetch(it.kbeg + 16, cur);       // cur now holds the data of the second step
    __syncthreads();
    int buf = 0;
    // outer loop: groups of FLUSH steps whose FP32 sums are folded into FP64
    // (FP64 operands accumulate directly; one group covers the whole chunk)
    const long long group = sizeof(T) == 4 ? 16LL * FLUSH : (it.kend - it.kbeg);
    for (long long kg = it.kbeg; kg < it.kend; kg += group) {
        const long long kg_end = kg + group < it.kend ? kg + group : it.kend;
        for (long long kb = kg; kb < kg_end; kb += 16) {
            // data two steps ahead; tables one step ahead into the other buffer
            fetch(kb + 32, nxt);
            gen(buf ^ 1, kb + 16, cur);
            // ---- contract this step on matrix cores
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int kk = 4 * g + s;
                const C2 h = sHv[buf][kk][q];
                const C2 f = sFu[buf][kk][q];
                T pr[NT], pn[NT], ec[NT], es[NT];
#pragma unroll
                for (int x = 0; x < NT; ++x) {
                    const C2 gv = sGv[buf][kk][ci0 + x];
                    pr[x] = h.x * gv.x - h.y * gv.y;
                    pn[x] = -(h.x * gv.y + h.y * gv.x);
                }
#pragma unroll
                for (int y = 0; y < NT; ++y) {
                    const C2 gu = sGu[buf][kk][cj0 + y];
                    ec[y] = f.x * gu.x - f.y * gu.y;
                    es[y] = f.x * gu.y + f.y * gu.x;
                }
#pragma unroll
                for (int x = 0; x < NT; ++x)
#pragma unroll
                    for (int y = 0; y < NT; ++y) {
                        acc[x][y] = Mfma<T>::mma(pr[x], ec[y], acc[x][y]);
                        acc[x][y] = Mfma<T>::mma(pn[x], es[y], acc[x][y]);
                    }
            }
            // interleave the next step's loads, table work and this step's
            // operand arithmetic between the matrix-core instructions
#pragma unroll
            for (int i = 0; i < 8 * NT * NT; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
                __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);   // up to three VALU
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
            }
            __syncthreads();
            buf ^= 1;
            cur = nxt;
        }
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int x = 0; x < NT; ++x)
#pragma unroll
                for (int y = 0; y < NT; ++y) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) sAcc[slot(x, y, r)] += (double)acc[x][y][r];
                    acc[x][y] = Mfma<T>::zero();
                }
        }
    }
    double *out = gpart + (size_t)it.slot * np * np;
#pragma unroll
    for (int x = 0; x < NT; ++x)
#pragma unroll
        for (int y = 0; y < NT; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + 16 * (ci0 + x) + Mfma<T>::drow(g, r);
                const int j = j0 + 16 * (cj0 + y) + q;
                out[(size_t)i * np + j] = sizeof(T) == 4 ? sAcc[slot(x, y, r)] : (double)acc[x][y][r];
            }
}

// ----------------------------------------------------------------------------
// Adjoint, FP32, 256 x 256 workgroup tile, eight waves of 64 (i) x 128 (j).
// Same tables and products as k_adjoint, but one super-step's tables (16
// visibilities: fine and coarse factors of both axes, 1024 correctly
// rounded twiddles) now feed 2048 matrix instructions instead of 512, and
// each wave forms 12 operands per 64 products instead of 8 per 32.  The FP32
// sums (at most ADJ_F32_SUM visibilities each) are folded every FLUSH super-steps
// into the workgroup's own FP64 partial tile in global memory
// (read-modify-write of a region no other workgroup touches; 512 KiB would
// not fit in LDS); a chunk of at most FLUSH super-steps writes it once.
// ----------------------------------------------------------------------------
// F32OUT: every chunk is at most FLUSH super-steps, so the single fold stores
// the FP32 sums directly into FP32 partial planes.
template <bool F32OUT>
__global__ __launch_bounds__(512, 1) void k_adjoint_w(const AdjItem *__restrict__ items,
                                                      const double *__restrict__ a,
                                                      const double *__restrict__ b,
                                                      const double2 *__restrict__ coef,
                                                      const float *__restrict__ w,
                                                      void *__restrict__ gpart_v, int n, int np) {
    typedef Mfma<float>::acc acc_t;
    constexpr int TT = 256, NTI = 4, NTJ = 8, FLUSH = ADJ_F32_SUM / 16;
    // [buf][table][k][q or t]: tables 0 Hv, 1 Fu (fine), 2 Gv, 3 Gu (coarse);
    // rows padded to 20 entries so that the rows 4 g + s read by the four
    // lane groups fall in different banks
    __shared__ float2 sT[2][4][16][20];

    const AdjItem it = items[blockIdx.x];
    const int i0 = it.ti * TT, j0 = it.tj * TT;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int q = lane & 15, g = lane >> 4;
    const int ci0 = (wave >> 1) * NTI;   // wave's first coarse i-tile (0, 4, 8, 12)
    const int cj0 = (wave & 1) * NTJ;    // wave's first coarse j-tile (0, 8)
    const int half = n / 2;

    // table tasks: thread tid fills entry (k, e) = (tid >> 4 & 15, tid & 15)
    // of the fine table (tid < 256: Hv, else Fu) and of the coarse table
    // (tid < 256: Gv, else Gu) of the same axis
    const int tk = (tid >> 4) & 15, te = tid & 15;
    const bool vaxis = tid < 256;
    const double *ab = vaxis ? b : a;
    struct Pre {
        double x;
        double2 c;
        float w;
    };
    auto fetch = [&](long long kb, Pre &p) {
        const long long k = kb + tk;
        const long long kl = k < it.kend ? k : it.kend - 1;
        p.x = ab[kl];
        p.c = vaxis ? coef[kl] : make_double2(0.0, 0.0);
        const float wv = w ? w[kl] : 1.f;
        p.w = k < it.kend ? wv : 0.f;
    };
    auto gen = [&](int buf, const Pre &p) {
        float c, s;
        cisphase(p.x, (vaxis ? i0 : j0) + te - half, c, s);
        float2 fine;
        if (vaxis) {
            const double cr = (double)p.w * p.c.x, cim = (double)p.w * p.c.y;
            fine.x = (float)(cr * (double)c - cim * (double)s);
            fine.y = (float)(cr * (double)s + cim * (double)c);
        } else {
            fine.x = p.w != 0.f ? c : 0.f;
            fine.y = p.w != 0.f ? s : 0.f;
        }
        sT[buf][vaxis ? 0 : 1][tk][te] = fine;
        cisphase(p.x, 16 * te, c, s);
        sT[buf][vaxis ? 2 : 3][tk][te] = float2{c, s};
    };

    acc_t acc[NTI][NTJ];
#pragma unroll
    for (int x = 0; x < NTI; ++x)
#pragma unroll
        for (int y = 0; y < NTJ; ++y) acc[x][y] = Mfma<float>::zero();
    double *out = reinterpret_cast<double *>(gpart_v) + (size_t)it.slot * np * np;
    float *out32 = reinterpret_cast<float *>(gpart_v) + (size_t)it.slot * np * np;
    bool first = true;
    // fold the FP32 sums into the FP64 tile, one 16 x 16 tile (4 values per
    // lane) at a time: the accumulators already hold 128 registers
    auto fold = [&]() {
#pragma unroll
        for (int x = 0; x < NTI; ++x)
#pragma unroll
            for (int y = 0; y < NTJ; ++y) {
                const size_t e0 = (size_t)(i0 + 16 * (ci0 + x) + 4 * g) * np + j0 + 16 * (cj0 + y) + q;
                if constexpr (F32OUT) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) out32[e0 + (size_t)r * np] = acc[x][y][r];
                    acc[x][y] = Mfma<float>::zero();
                    continue;
                }
                double *o = out + e0;
                double v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = first ? 0.0 : o[(size_t)r * np];
#pragma unroll
                for (int r = 0; r < 4; ++r) o[(size_t)r * np] = v[r] + (double)acc[x][y][r];
                acc[x][y] = Mfma<float>::zero();
            }
        first = false;
    };

    Pre cur, nxt;
    fetch(it.kbeg, cur);
    gen(0, cur);
    fetch(it.kbeg + 16, cur);
    __syncthreads();
    int buf = 0;
    int steps = 0;
    for (long long kb = it.kbeg; kb < it.kend; kb += 16) {
        fetch(kb + 32, nxt);
        gen(buf ^ 1, cur);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int kk = 4 * g + s;
            const float2 h = sT[buf][0][kk][q];
            const float2 f = sT[buf][1][kk][q];
            float pr[NTI], pn[NTI], ec[NTJ], es[NTJ];
#pragma unroll
            for (int x = 0; x < NTI; ++x) {
                const float2 gv = sT[buf][2][kk][ci0 + x];
                pr[x] = h.x * gv.x - h.y * gv.y;
                pn[x] = -(h.x * gv.y + h.y * gv.x);
            }
#pragma unroll
            for (int y = 0; y < NTJ; ++y) {
                const float2 gu = sT[buf][3][kk][cj0 + y];
                ec[y] = f.x * gu.x - f.y * gu.y;
                es[y] = f.x * gu.y + f.y * gu.x;
            }
#pragma unroll
            for (int x = 0; x < NTI; ++x)
#pragma unroll
                for (int y = 0; y < NTJ; ++y) {
                    acc[x][y] = Mfma<float>::mma(pr[x], ec[y], acc[x][y]);
                    acc[x][y] = Mfma<float>::mma(pn[x], es[y], acc[x][y]);
                }
        }
        __syncthreads();
        buf ^= 1;
        cur = nxt;
        if (++steps == FLUSH) {
            fold();
            steps = 0;
        }
    }
    if (steps > 0 || first) fold();
}

// ----------------------------------------------------------------------------
// Split precision (16-bit hi + lo, three products per real product):
//   x y ~= x_h y_h + x_h y_l + x_l y_h,  x_h = RN_16(x), x_l = RN_16(x - x_h),
// on v_mfma_f32_16x16x32_{bf16,f16} (lane l supplies A[l%16][8 (l/16) + e] and
// B[8 (l/16) + e][l%16], e = 0..7; it holds D[4 (l/16) + r][l%16]) with FP32
// accumulation, folded into FP64 periodically.  The dropped x_l y_l term and
// the representation error leave ~2^-16 relative error per product.
// ----------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// 16-bit operand formats of the split path.  bf16 keeps the FP32 exponent
// range (no scaling); fp16 has 11-bit halves (hi + lo ~ 22 bits) but a narrow
// range, so its operands are scaled by powers of two to a magnitude <= 1
// (v_mfma_f32_16x16x32_f16 has the same lane layout as the bf16 form).
template <typename H> struct Half16;
template <> struct Half16<__bf16> {
    typedef bf16x8 h8;
    static constexpr bool scaled = false;
    static __device__ __forceinline__ floatx4 mma(h8 a, h8 b, floatx4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Half16<_Float16> {
    typedef f16x8 h8;
    static constexpr bool scaled = true;
    static __device__ __forceinline__ floatx4 mma(h8 a, h8 b, floatx4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

template <typename H>
__device__ __forceinline__ void split16(float x, H &h, H &l) {
    h = (H)x;
    l = (H)(x - (float)h);
}

// Split eight floats into hi and lo vectors, two values per conversion
// instruction (v_cvt_pk_{bf16,f16}_f32).
typedef float float2v __attribute__((ext_vector_type(2)));
template <typename H>
__device__ __forceinline__ void split8(const float (&x)[8], typename Half16<H>::h8 &hi,
                                       typename Half16<H>::h8 &lo) {
    typedef H h2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const float2v v = {x[2 * m], x[2 * m + 1]};
        const h2 hh = __builtin_convertvector(v, h2);
        const float2v back = __builtin_convertvector(hh, float2v);
        const float2v d = {v.x - back.x, v.y - back.y};
        const h2 ll = __builtin_convertvector(d, h2);
        hi[2 * m] = hh.x;
        hi[2 * m + 1] = hh.y;
        lo[2 * m] = ll.x;
        lo[2 * m + 1] = ll.y;
    }
}

// 2^-e with e chosen so that m 2^-e < 1 (1 for m = 0 or not finite).
__device__ __forceinline__ float pow2_scale(float m) {
    if (!(m > 0.f) || !isfinite(m)) return 1.f;
    return ldexpf(1.f, -(ilogbf(m) + 1));
}

// Hardware sine/cosine of 2 pi f for f in revolutions (|f| <= 1/2).
__device__ __forceinline__ void cis2pi_hw(float f, float &c, float &s) {
    s = __builtin_amdgcn_sinf(f);
    c = __builtin_amdgcn_cosf(f);
}

// Forward, split precision, persistent.  A workgroup of eight waves holds the
// image block rows [i0, i0 + IB) x columns [j0, j0 + JB) in LDS for its
// whole life (16-bit hi and lo halves, fp16 scaled by a power of
// two to the block's maximum) and streams 16-visibility tiles through its waves:
// tile t of the block goes to wave (t mod 8 nwg) / nwg of workgroup t mod nwg.  For a tile the
// wave forms the E_u operand of each 32-column step from a coarse factor and
// eight fine factors (hardware sin/cos of FP64-reduced phases), contracts the
// block on matrix cores, then does the row dot with E_v and writes the
// block's partial V_k.
template <typename H, int IB, int JB, int NV>
__global__ __launch_bounds__(512, 1) void k_forward_h16p(const FwdPItem *__restrict__ items,
                                                         const double *__restrict__ a,
                                                         const double *__restrict__ b,
                                                         const float *__restrict__ bop,
                                                         double2 *__restrict__ vpart, int n, int np,
                                                         long long ztot) {
    typedef typename Half16<H>::h8 h8;
    constexpr int NT = IB / 16;
    constexpr int KSTEPS = JB / 32;
    // 8-element column group cg of row r is stored at group cg ^ (r & SWM):
    // the 16 rows read by one matrix-core operand load then fall into
    // distinct LDS banks
    constexpr int NCG = JB / 8;
    constexpr int SWM = NCG >= 16 ? 15 : NCG - 1;
    __shared__ __attribute__((aligned(16))) H sH[IB][JB];
    __shared__ __attribute__((aligned(16))) H sL[IB][JB];
    __shared__ float sMax[8];

    const FwdPItem it = items[blockIdx.x];
    const int i0 = it.ib * IB, j0 = it.jb * JB;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int q = lane & 15, g = lane >> 4;
    const int half = n / 2;
    // stage the block: (scale,) split into hi and lo halves
    const float *Bc = bop + (size_t)it.chan * np * np;
    constexpr int VROW = JB / 4;
    float scale = 1.f;
    if constexpr (Half16<H>::scaled) {
        float m = 0.f;
        for (int x = tid; x < IB * VROW; x += 512) {
            const int row = x / VROW, c4 = x % VROW;
            const float4 v = *reinterpret_cast<const float4 *>(Bc + (size_t)(i0 + row) * np + j0 + 4 * c4);
            m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
        if (lane == 0) sMax[wave] = m;
        __syncthreads();
        m = sMax[0];
#pragma unroll
        for (int x = 1; x < 8; ++x) m = fmaxf(m, sMax[x]);
        scale = pow2_scale(m);
    }
    for (int x = tid; x < IB * NCG; x += 512) {
        const int row = x / NCG, cg = x % NCG;
        const float *src = Bc + (size_t)(i0 + row) * np + j0 + 8 * cg;
        const float4 v0 = *reinterpret_cast<const float4 *>(src);
        const float4 v1 = *reinterpret_cast<const float4 *>(src + 4);
        const float vv[8] = {v0.x * scale, v0.y * scale, v0.z * scale, v0.w * scale,
                             v1.x * scale, v1.y * scale, v1.z * scale, v1.w * scale};
        h8 hv, lv;
        split8<H>(vv, hv, lv);
        const int o = 8 * (cg ^ (row & SWM));
        *reinterpret_cast<h8 *>(&sH[row][o]) = hv;
        *reinterpret_cast<h8 *>(&sL[row][o]) = lv;
    }
    __syncthreads();
    const float unscale = 1.f / scale;
    // a wave's tile: NV groups of 16 visibilities that share every image
    // fragment read from LDS
    constexpr int TV = 16 * NV;
    const long long nk = it.kend - it.kbeg;
    const long long ntiles = (nk + TV - 1) / TV;
    // tile wave * nwg + wg of each round: a round's leftover tiles go to one
    // wave of distinct workgroups, so no CU carries them on all its SIMDs
    const long long stride = 8LL * it.nwg;
    for (long long tile = (long long)wave * it.nwg + it.wg; tile < ntiles; tile += stride) {
        const long long k0 = it.kbeg + TV * tile;
        const int nvalid = (int)(it.kend - k0 < TV ? it.kend - k0 : TV);
        double ak[NV];
        float fc[NV][8], fs[NV][8];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            ak[v] = 16 * v + q < nvalid ? a[k0 + 16 * v + q] : 0.0;
#pragma unroll
            for (int e = 0; e < 8; ++e) cis2pi_hw((float)phase(ak[v], e), fc[v][e], fs[v][e]);
        }
        floatx4 accR[NV][NT], accI[NV][NT];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                accR[v][t] = floatx4{0.f, 0.f, 0.f, 0.f};
                accI[v][t] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
        // E_u operand of group v, 32-column step ks: E(a_k (j0 + 32 ks + 8 g - N/2)) E(a_k e)
        auto twiddle = [&](int ks, int v, h8 &th, h8 &tl, h8 &uh, h8 &ul) {
            float cc, sc;
            cis2pi_hw((float)phase(ak[v], j0 + 32 * ks + 8 * g - half), cc, sc);
            float cv[8], nsv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                cv[e] = cc * fc[v][e] - sc * fs[v][e];
                nsv[e] = (-sc) * fc[v][e] - cc * fs[v][e];
            }
            split8<H>(cv, th, tl);
            split8<H>(nsv, uh, ul);
        };
#pragma unroll 2
        for (int ks = 0; ks < KSTEPS; ++ks) {
            h8 rh[NV], rl[NV], ih[NV], il[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) twiddle(ks, v, rh[v], rl[v], ih[v], il[v]);
            const int o = 8 * ((4 * ks + g) ^ (q & SWM));
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const h8 bhv = *reinterpret_cast<const h8 *>(&sH[16 * t + q][o]);
                const h8 blv = *reinterpret_cast<const h8 *>(&sL[16 * t + q][o]);
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    accR[v][t] = Half16<H>::mma(rh[v], bhv, accR[v][t]);
                    accI[v][t] = Half16<H>::mma(ih[v], bhv, accI[v][t]);
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    accR[v][t] = Half16<H>::mma(rh[v], blv, accR[v][t]);
                    accI[v][t] = Half16<H>::mma(ih[v], blv, accI[v][t]);
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    accR[v][t] = Half16<H>::mma(rl[v], bhv, accR[v][t]);
                    accI[v][t] = Half16<H>::mma(il[v], bhv, accI[v][t]);
                }
            }
        }
        // row dot: E_v[k][i0 + 16 t + q] = E(b_k (i0 + q - N/2)) E(16 b_k)^t
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int kk = 16 * v + 4 * g + r;
                const bool ok = kk < nvalid;
                const double bk = ok ? b[k0 + kk] : 0.0;
                float ec, es, sc16, ss16;
                cis2pi_hw((float)phase(bk, i0 + q - half), ec, es);
                cis2pi_hw((float)phase(bk, 16), sc16, ss16);
                // W = sum_t conj(rho)^t T_t by Horner's rule (rho = E(16 b_k)),
                // then V = conj(E(b_k (i0 + q - N/2))) W
                float wr = accR[v][NT - 1][r], wi = accI[v][NT - 1][r];
#pragma unroll
                for (int t = NT - 2; t >= 0; --t) {
                    const float nr = accR[v][t][r] + sc16 * wr + ss16 * wi;
                    wi = accI[v][t][r] + sc16 * wi - ss16 * wr;
                    wr = nr;
                }
                float vr = ec * wr + es * wi, vi = ec * wi - es * wr;
                vr = row16_sum(vr);
                vi = row16_sum(vi);
                if (q == 0 && ok)
                    vpart[(size_t)it.part * ztot + k0 + kk] =
                        make_double2((double)vr * (double)unscale, (double)vi * (double)unscale);
            }
    }
}

// Adjoint, split precision.  Per 32-visibility step the workgroup builds
// fine/coarse twiddle tables (hardware sin/cos of FP64-reduced phases):
//   Hv[q][k] = conj(w_k c_k exp(+2 pi i b_k (i0 + q - N/2))),  Gv[t][k] = exp(-2 pi i b_k 16 t)
//   Fu[q][k] = exp(+2 pi i a_k (j0 + q - N/2)),                Gu[t][k] = exp(+2 pi i a_k 16 t)
// (the P side conjugated, so that Hv Gv = (Re P, -Im P) directly), then the
// pre-split operand tiles P[i][k] = Hv Gv and E[j][k] = Fu Gu (cos, sin) in
// LDS (one thread per operand row), and the
// waves contract them on matrix cores.  The visibility data of the next
// step are loaded into registers while the current step computes.
template <typename H, int WT>
__global__ __launch_bounds__(256, 2) void k_adjoint_h16(const AdjItem *__restrict__ items,
                                                        const double *__restrict__ a,
                                                        const double *__restrict__ b,
                                                        const double2 *__restrict__ coef,
                                                        const float *__restrict__ w,
                                                        const double *__restrict__ vispart,
                                                        const int *__restrict__ vis_base,
                                                        float *__restrict__ gpart, int n, int np) {
    typedef typename Half16<H>::h8 h8;
    constexpr int TT = 2 * WT;
    constexpr int NT = WT / 16;
    constexpr int NC = TT / 16;
    constexpr int KS = 32;
    constexpr int KT = KS + 2;     // padded table rows (float2)
    constexpr int KP = KS;         // operand rows: 4 groups of 8, XOR-swizzled (see swz)
    __shared__ __attribute__((aligned(16))) float2 sHv[16][KT], sFu[16][KT], sGv[NC][KT], sGu[NC][KT];
    __shared__ __attribute__((aligned(16))) H sP[4][TT][KP];   // re_h, re_l, -im_h, -im_l
    __shared__ __attribute__((aligned(16))) H sE[4][TT][KP];   // cos_h, cos_l, sin_h, sin_l
    __shared__ double sRed[4];
    // group kg of row r is stored at group kg ^ ((r >> 1) & 3): eight
    // consecutive rows then hit distinct LDS banks for 16-byte accesses
    auto swz = [](int r, int kg) { return 8 * (kg ^ ((r >> 1) & 3)); };

    const AdjItem it = items[blockIdx.x];
    const int i0 = it.ti * TT, j0 = it.tj * TT;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int q = lane & 15, g = lane >> 4;
    const int wi = (wave >> 1) * WT, wj = (wave & 1) * WT;
    const int half = n / 2;
    // fp16: coefficients scaled by 2^-e so that max |w c| of the channel
    // (slot 2 of its visibility partials) is below one
    float scale = 1.f;
    if constexpr (Half16<H>::scaled) {
        double m = 0.0;
        for (int x = vis_base[it.chan] + tid; x < vis_base[it.chan + 1]; x += 256)
            m = fmax(m, vispart[(size_t)x * NPART + 2]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
        if (lane == 0) sRed[wave] = m;
        __syncthreads();
        m = fmax(fmax(sRed[0], sRed[1]), fmax(sRed[2], sRed[3]));
        scale = pow2_scale((float)m);
    }

    // table tasks of this thread: fine (k = tid>>4 and tid>>4 + 16, q = tid&15),
    // coarse (k = tid / NC8, t = tid % NC8 for both axes when tid < KS*NC)
    const int fk0 = tid >> 4, fq = tid & 15;
    const int ck = tid / NC, ct = tid % NC;
    const bool has_c = tid < KS * NC;

    struct Pre {
        double a0, b0, a1, b1, ac, bc;
        double2 c0, c1;
        float w0, w1;
    };
    auto fetch = [&](long long kb, Pre &p) {
        const long long k0 = kb + fk0, k1 = kb + fk0 + 16, kc = kb + ck;
        p.a0 = p.b0 = p.a1 = p.b1 = p.ac = p.bc = 0.0;
        p.c0 = p.c1 = make_double2(0.0, 0.0);
        p.w0 = p.w1 = 0.f;
        if (k0 < it.kend) { p.a0 = a[k0]; p.b0 = b[k0]; p.c0 = coef[k0]; p.w0 = w ? w[k0] : 1.f; }
        if (k1 < it.kend) { p.a1 = a[k1]; p.b1 = b[k1]; p.c1 = coef[k1]; p.w1 = w ? w[k1] : 1.f; }
        if (has_c && kc < it.kend) { p.ac = a[kc]; p.bc = b[kc]; }
    };

    floatx4 acc[NT][NT];
#pragma unroll
    for (int x = 0; x < NT; ++x)
#pragma unroll
        for (int y = 0; y < NT; ++y) acc[x][y] = floatx4{0.f, 0.f, 0.f, 0.f};

    Pre cur, nxt;
    fetch(it.kbeg, cur);
    for (long long kb = it.kbeg; kb < it.kend; kb += KS) {
        if (kb + KS < it.kend) fetch(kb + KS, nxt);
        // ---- twiddle tables (zero coefficients / unit coarse factors past the end)
        {
            float c, s;
            cis2pi_hw((float)phase(cur.b0, i0 + fq - half), c, s);
            float cr = scale * (float)((double)cur.w0 * cur.c0.x), ci = scale * (float)((double)cur.w0 * cur.c0.y);
            sHv[fq][fk0] = make_float2(cr * c - ci * s, -(cr * s + ci * c));
            cis2pi_hw((float)phase(cur.a0, j0 + fq - half), c, s);
            sFu[fq][fk0] = make_float2(c, s);
            cis2pi_hw((float)phase(cur.b1, i0 + fq - half), c, s);
            cr = scale * (float)((double)cur.w1 * cur.c1.x);
            ci = scale * (float)((double)cur.w1 * cur.c1.y);
            sHv[fq][fk0 + 16] = make_float2(cr * c - ci * s, -(cr * s + ci * c));
            cis2pi_hw((float)phase(cur.a1, j0 + fq - half), c, s);
            sFu[fq][fk0 + 16] = make_float2(c, s);
            if (has_c) {
                cis2pi_hw((float)phase(cur.bc, 16 * ct), c, s);
                sGv[ct][ck] = make_float2(c, -s);
                cis2pi_hw((float)phase(cur.ac, 16 * ct), c, s);
                sGu[ct][ck] = make_float2(c, s);
            }
        }
        __syncthreads();
        // ---- pre-split operand rows: thread -> (operand, row)
        for (int x = tid; x < 2 * TT; x += 256) {
            const int dim = x / TT, row = x % TT;
            const int qq = row & 15, t = row >> 4;
            const float2 *f = dim == 0 ? sHv[qq] : sFu[qq];
            const float2 *gc = dim == 0 ? sGv[t] : sGu[t];
            H (*dst)[TT][KP] = dim == 0 ? sP : sE;
#pragma unroll
            for (int kg = 0; kg < KS / 8; ++kg) {
                h8 v0, v1, v2, v3;
                float re[8], im[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float2 fv = f[8 * kg + e], gv = gc[8 * kg + e];
                    re[e] = fv.x * gv.x - fv.y * gv.y;
                    im[e] = fv.x * gv.y + fv.y * gv.x;
                }
                split8<H>(re, v0, v1);
                split8<H>(im, v2, v3);
                const int o = swz(row, kg);
                *reinterpret_cast<h8 *>(&dst[0][row][o]) = v0;
                *reinterpret_cast<h8 *>(&dst[1][row][o]) = v1;
                *reinterpret_cast<h8 *>(&dst[2][row][o]) = v2;
                *reinterpret_cast<h8 *>(&dst[3][row][o]) = v3;
            }
        }
        __syncthreads();
        // ---- contract on matrix cores
        h8 ech[NT], ecl[NT], esh[NT], esl[NT];
#pragma unroll
        for (int y = 0; y < NT; ++y) {
            const int r = wj + 16 * y + q;
            const int o = swz(r, g);
            ech[y] = *reinterpret_cast<const h8 *>(&sE[0][r][o]);
            ecl[y] = *reinterpret_cast<const h8 *>(&sE[1][r][o]);
            esh[y] = *reinterpret_cast<const h8 *>(&sE[2][r][o]);
            esl[y] = *reinterpret_cast<const h8 *>(&sE[3][r][o]);
        }
#pragma unroll
        for (int x = 0; x < NT; ++x) {
            const int r = wi + 16 * x + q;
            const int o = swz(r, g);
            const h8 prh = *reinterpret_cast<const h8 *>(&sP[0][r][o]);
            const h8 prl = *reinterpret_cast<const h8 *>(&sP[1][r][o]);
            const h8 pih = *reinterpret_cast<const h8 *>(&sP[2][r][o]);
            const h8 pil = *reinterpret_cast<const h8 *>(&sP[3][r][o]);
#pragma unroll
            for (int y = 0; y < NT; ++y) {
                acc[x][y] = Half16<H>::mma(prh, ech[y], acc[x][y]);
                acc[x][y] = Half16<H>::mma(pih, esh[y], acc[x][y]);
                acc[x][y] = Half16<H>::mma(prh, ecl[y], acc[x][y]);
                acc[x][y] = Half16<H>::mma(pih, esl[y], acc[x][y]);
                acc[x][y] = Half16<H>::mma(prl, ech[y], acc[x][y]);
                acc[x][y] = Half16<H>::mma(pil, esh[y], acc[x][y]);
            }
        }
        __syncthreads();
        cur = nxt;
    }
    float *out = gpart + (size_t)it.slot * np * np;
    const float inv = 1.f / scale;   // a power of two: exact
#pragma unroll
    for (int x = 0; x < NT; ++x)
#pragma unroll
        for (int y = 0; y < NT; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wi + 16 * x + 4 * g + r;
                const int j = j0 + wj + 16 * y + q;
                out[(size_t)i * np + j] = acc[x][y][r] * inv;
            }
}

// Adjoint, split precision, 256 x 256 pixel tile, eight waves of 128 (i) x 64
// (j), software-pipelined over steps of 16 visibilities.  The real and
// imaginary parts of a step are concatenated along the contraction
// dimension, so one v_mfma_f32_16x16x32 covers the step's 16 visibilities:
//   G[i][j] += sum_{k'} A[i][k'] B[k'][j],
//   A[i][k] = Re P[k][i], A[i][16 + k] = -Im P[k][i]   (P = w c conj E_v)
//   B[k][j] = cos 2 pi a_k m_j, B[16 + k][j] = sin 2 pi a_k m_j,
// three products per pair (hi hi, hi lo, lo hi).  Per step and workgroup:
//   tables  -- fine and coarse factors of both axes (one hardware sin/cos per
//              entry, 1,024 entries: two per thread),
//   operands -- one 32-element row per thread, P (threads 0-255) or E
//              (256-511), formed from the tables and split into hi and lo,
//   products -- 96 matrix instructions per wave.
// The operand rows of step s + 1 and the tables of step s + 2 are formed
// while the matrix cores contract step s: operands and tables are
// double-buffered in LDS, so one workgroup barrier per step orders them.
// The visibility data of a table step are loaded three steps ahead (held in
// registers for a whole step) and the tables are formed last in the step,
// which covers the latency of loads that miss the caches.
// Chunk sums are FP32 and the partial tile is stored in FP32.
template <typename H>
__global__ __launch_bounds__(512, 1) void k_adjoint_h16s(const AdjItem *__restrict__ items,
                                                         const double *__restrict__ a,
                                                         const double *__restrict__ b,
                                                         const double2 *__restrict__ coef,
                                                         const float *__restrict__ w,
                                                         const double *__restrict__ vispart,
                                                         const int *__restrict__ vis_base,
                                                         float *__restrict__ gpart, int n, int np) {
    typedef typename Half16<H>::h8 h8;
    constexpr int TT = 256;
    constexpr int KV = 16;         // visibilities per step
    constexpr int KP = 2 * KV;     // contraction length per step (re, im)
    constexpr int NR = 8;          // 16-row blocks per wave (128 rows)
    constexpr int NCB = 4;         // 16-column blocks per wave (64 columns)
    constexpr int TR = KV + 2;     // table row stride in float2 (16-byte aligned rows)
    // operands: [buffer][hi, lo][row: P 0-255, E 256-511][KP], 16-byte
    // chunks XOR-swizzled by (row >> 1) & 3
    __shared__ __attribute__((aligned(16))) H sOp[2][2][2 * TT][KP];
    // tables: [buffer][axis: v (P side), u (E side)][fine, coarse][index][k]
    __shared__ __attribute__((aligned(16))) float2 sTab[2][2][2][16][TR];
    __shared__ double sRed[8];
    auto swz = [](int r, int c) { return 8 * (c ^ ((r >> 1) & 3)); };

    const AdjItem it = items[blockIdx.x];
    const int i0 = it.ti * TT, j0 = it.tj * TT;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int q = lane & 15, g = lane >> 4;
    const int wi = (wave >> 2) * 128, wj = (wave & 3) * 64;
    const int half = n / 2;
    float scale = 1.f;
    if constexpr (Half16<H>::scaled) {
        double m = 0.0;
        for (int x = vis_base[it.chan] + tid; x < vis_base[it.chan + 1]; x += 512)
            m = fmax(m, vispart[(size_t)x * NPART + 2]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
        if (lane == 0) sRed[wave] = m;
        __syncthreads();
        m = sRed[0];
#pragma unroll
        for (int x = 1; x < 8; ++x) m = fmax(m, sRed[x]);
        scale = pow2_scale((float)m);
    }

    // table task: axis tax (0: v / P side, 1: u / E side), index tix, visibility tk of the step
    const int tax = tid >> 8, tix = (tid >> 4) & 15, tk = tid & 15;
    const double *xsrc = tax == 0 ? b : a;
    const int origin = (tax == 0 ? i0 : j0) + tix - half;
    struct Pre {
        double x;
        double2 c;
        float w;
    };
    auto fetch = [&](long long kb, Pre &p) {
        const long long k = kb + tk;
        p.x = 0.0;
        p.c = make_double2(0.0, 0.0);
        p.w = 0.f;
        if (k < it.kend) {
            p.x = xsrc[k];
            if (tax == 0) {
                p.c = coef[k];
                p.w = w ? w[k] : 1.f;
            }
        }
    };
    // fine[idx][k] = conj(s w_k c_k E(b_k (i0 + idx - N/2))) or E(a_k (j0 + idx - N/2));
    // coarse[idx][k] = conj E(16 b_k idx) or E(16 a_k idx)   (E(x) = exp(2 pi i x))
    auto gen = [&](int tb, const Pre &p) {
        float c, sn;
        cis2pi_hw((float)phase(p.x, origin), c, sn);
        float2 fine;
        if (tax == 0) {
            const float cr = scale * (float)((double)p.w * p.c.x);
            const float ci = scale * (float)((double)p.w * p.c.y);
            fine = make_float2(cr * c - ci * sn, -(cr * sn + ci * c));
        } else {
            fine = make_float2(c, sn);
        }
        sTab[tb][tax][0][tix][tk] = fine;
        cis2pi_hw((float)phase(p.x, 16 * tix), c, sn);
        sTab[tb][tax][1][tix][tk] = make_float2(c, tax == 0 ? -sn : sn);
    };
    // operand row of this thread: side fside (0: P, 1: E), row frow of that side
    const int fside = tid >> 8, frow = tid & 255;
    const int fq = frow & 15, ft = frow >> 4;
    const int orow = fside * TT + frow;
    // half a row: visibilities 8 hk .. 8 hk + 7, both parts (chunks hk and 2 + hk)
    auto form_half = [&](int tb, int ob, int hk) {
        const float2 *fr = &sTab[tb][fside][0][fq][8 * hk];
        const float2 *cr = &sTab[tb][fside][1][ft][8 * hk];
        float re[8], im[8];
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
            const float4 f2 = *reinterpret_cast<const float4 *>(fr + e);
            const float4 c2 = *reinterpret_cast<const float4 *>(cr + e);
            re[e] = f2.x * c2.x - f2.y * c2.y;
            im[e] = f2.x * c2.y + f2.y * c2.x;
            re[e + 1] = f2.z * c2.z - f2.w * c2.w;
            im[e + 1] = f2.z * c2.w + f2.w * c2.z;
        }
        h8 rh, rl, ih, il;
        split8<H>(re, rh, rl);
        split8<H>(im, ih, il);
        *reinterpret_cast<h8 *>(&sOp[ob][0][orow][swz(orow, hk)]) = rh;
        *reinterpret_cast<h8 *>(&sOp[ob][1][orow][swz(orow, hk)]) = rl;
        *reinterpret_cast<h8 *>(&sOp[ob][0][orow][swz(orow, 2 + hk)]) = ih;
        *reinterpret_cast<h8 *>(&sOp[ob][1][orow][swz(orow, 2 + hk)]) = il;
    };

    floatx4 acc[NR][NCB];
#pragma unroll
    for (int x = 0; x < NR; ++x)
#pragma unroll
        for (int y = 0; y < NCB; ++y) acc[x][y] = floatx4{0.f, 0.f, 0.f, 0.f};

    const long long kb0 = it.kbeg;
    const int nsteps = (int)((it.kend - it.kbeg + KV - 1) / KV);
    Pre pre, pre2;
    fetch(kb0, pre);
    gen(0, pre);
    fetch(kb0 + KV, pre);
    fetch(kb0 + 2 * KV, pre2);
    __syncthreads();
    form_half(0, 0, 0);
    form_half(0, 0, 1);
    gen(1, pre);
    pre = pre2;
    __syncthreads();
    // One basic block per step (no branches), so that the scheduler can
    // spread the operand formation of step s + 1 and the table work of step
    // s + 2 between the matrix instructions of step s.  In the last steps
    // they form rows from stale tables or zero data into buffers that are
    // never read again.
    for (int s = 0; s < nsteps; ++s) {
        const int ob = s & 1;
        fetch(kb0 + (long long)(s + 3) * KV, pre2);
        // E fragments of this wave's four column blocks
        h8 eh[NCB], el[NCB];
#pragma unroll
        for (int y = 0; y < NCB; ++y) {
            const int r = TT + wj + 16 * y + q;
            eh[y] = *reinterpret_cast<const h8 *>(&sOp[ob][0][r][swz(r, g)]);
            el[y] = *reinterpret_cast<const h8 *>(&sOp[ob][1][r][swz(r, g)]);
        }
        // the eight row blocks, the P fragments of the next block loaded
        // while this one contracts
        h8 ph, pl;
        {
            const int r = wi + q;
            ph = *reinterpret_cast<const h8 *>(&sOp[ob][0][r][swz(r, g)]);
            pl = *reinterpret_cast<const h8 *>(&sOp[ob][1][r][swz(r, g)]);
        }
#pragma unroll
        for (int x = 0; x < NR; ++x) {
            const h8 ch = ph, cl = pl;
            if (x + 1 < NR) {
                const int r = wi + 16 * (x + 1) + q;
                ph = *reinterpret_cast<const h8 *>(&sOp[ob][0][r][swz(r, g)]);
                pl = *reinterpret_cast<const h8 *>(&sOp[ob][1][r][swz(r, g)]);
            }
#pragma unroll
            for (int y = 0; y < NCB; ++y) acc[x][y] = Half16<H>::mma(ch, eh[y], acc[x][y]);
#pragma unroll
            for (int y = 0; y < NCB; ++y) acc[x][y] = Half16<H>::mma(ch, el[y], acc[x][y]);
#pragma unroll
            for (int y = 0; y < NCB; ++y) acc[x][y] = Half16<H>::mma(cl, eh[y], acc[x][y]);
            if (x == 1) form_half(ob ^ 1, ob ^ 1, 0);
            if (x == 4) form_half(ob ^ 1, ob ^ 1, 1);
            if (x == 7) gen(ob, pre);
        }
        pre = pre2;
        __syncthreads();
    }
    float *out = gpart + (size_t)it.slot * np * np;
    const float inv = 1.f / scale;   // a power of two: exact
#pragma unroll
    for (int x = 0; x < NR; ++x)
#pragma unroll
        for (int y = 0; y < NCB; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wi + 16 * x + 4 * g + r;
                const int j = j0 + wj + 16 * y + q;
                out[(size_t)i * np + j] = acc[x][y][r] * inv;
            }
}

// 32 x 32 x 16 forms of the split-precision products (v_mfma_f32_32x32x16_{bf16,
// f16}): lane l supplies A[l % 32][8 (l / 32) + e] and B[8 (l / 32) + e][l % 32],
// e = 0..7, and holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] in accumulator
// register r (checked on gfx950).  They issue twice the products per cycle of
// the 16 x 16 x 32 forms on this hardware.
typedef float floatx16 __attribute__((ext_vector_type(16)));
template <typename H> struct Half32;
template <> struct Half32<__bf16> {
    static __device__ __forceinline__ floatx16 mma(bf16x8 a, bf16x8 b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Half32<_Float16> {
    static __device__ __forceinline__ floatx16 mma(f16x8 a, f16x8 b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

// Forward, split precision, persistent, 32 x 32 x 16 products.  As
// k_forward_h16p, a workgroup of eight waves holds an IB x JB image block
// (hi and lo halves, fp16 scaled by a power of two to the block maximum) in
// LDS and streams visibility tiles through its waves, here 32 visibilities
// per wave tile.  The image rows are the A operand and the twiddles the B
// operand, so the products come out transposed, T[k][i] in D[i][k]: lane l
// holds visibility l % 32 of the tile for 16 rows of each 32-row tile.  Per
// 16-column step the lane forms its eight twiddles E(a_k (j - N/2)) from a
// coarse factor and eight fine ones (hardware sin/cos of FP64-reduced
// phases) and splits them; then the row dot
//   V_k = sum_i conj E(b_k (i - N/2)) T[k][i]
// is summed in the lane over its 64 rows with the row factor split as
// E(b_k (i0 - N/2 + 4 h)) E(b_k r) E(8 b_k a) E(32 b_k t) (h = l / 32, row
// 32 t + 8 a + 4 h + r), and the two lanes of a visibility are added.
template <typename H, int IB, int JB>
__global__ __launch_bounds__(512, 1) void k_forward_h16m(const FwdPItem *__restrict__ items,
                                                         const double *__restrict__ a,
                                                         const double *__restrict__ b,
                                                         const float *__restrict__ bop,
                                                         double2 *__restrict__ vpart, int n, int np,
                                                         long long ztot) {
    typedef typename Half16<H>::h8 h8;
    constexpr int NT = IB / 32;        // 32-row tiles of the block
    constexpr int KSTEPS = JB / 16;
    constexpr int NCG = JB / 8;
    constexpr int SWM = NCG >= 16 ? 15 : NCG - 1;
    __shared__ __attribute__((aligned(16))) H sH[IB][JB];
    __shared__ __attribute__((aligned(16))) H sL[IB][JB];
    __shared__ float sMax[8];

    const FwdPItem it = items[blockIdx.x];
    const int i0 = it.ib * IB, j0 = it.jb * JB;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int l32 = lane & 31, hk = lane >> 5;
    const int half = n / 2;
    const float *Bc = bop + (size_t)it.chan * np * np;
    constexpr int VROW = JB / 4;
    float scale = 1.f;
    if constexpr (Half16<H>::scaled) {
        float m = 0.f;
        for (int x = tid; x < IB * VROW; x += 512) {
            const int row = x / VROW, c4 = x % VROW;
            const float4 v = *reinterpret_cast<const float4 *>(Bc + (size_t)(i0 + row) * np + j0 + 4 * c4);
            m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
        if (lane == 0) sMax[wave] = m;
        __syncthreads();
        m = sMax[0];
#pragma unroll
        for (int x = 1; x < 8; ++x) m = fmaxf(m, sMax[x]);
        scale = pow2_scale(m);
    }
    for (int x = tid; x < IB * NCG; x += 512) {
        const int row = x / NCG, cg = x % NCG;
        const float *src = Bc + (size_t)(i0 + row) * np + j0 + 8 * cg;
        const float4 v0 = *reinterpret_cast<const float4 *>(src);
        const float4 v1 = *reinterpret_cast<const float4 *>(src + 4);
        const float vv[8] = {v0.x * scale, v0.y * scale, v0.z * scale, v0.w * scale,
                             v1.x * scale, v1.y * scale, v1.z * scale, v1.w * scale};
        h8 hv, lv;
        split8<H>(vv, hv, lv);
        const int o = 8 * (cg ^ (row & SWM));
        *reinterpret_cast<h8 *>(&sH[row][o]) = hv;
        *reinterpret_cast<h8 *>(&sL[row][o]) = lv;
    }
    __syncthreads();
    const double unscale = 1.0 / (double)scale;
    constexpr int TV = 32;
    const long long nk = it.kend - it.kbeg;
    const long long ntiles = (nk + TV - 1) / TV;
    // tile wave * nwg + wg of each round: a round's leftover tiles go to one
    // wave of distinct workgroups, so no CU carries them on all its SIMDs
    const long long stride = 8LL * it.nwg;
    // With at most two leftover tiles per workgroup after the full rounds,
    // the eight waves share each leftover tile, a 1/8 of its columns each
    // (one wave alone would keep one SIMD busy for a whole tile after the
    // others have finished); the eight partial visibilities are added in
    // wave order.
    const long long nfull = ntiles / stride * stride;
    const bool share = KSTEPS % 8 == 0 && ntiles > nfull && (ntiles - nfull + it.nwg - 1) / it.nwg <= 2;
    const long long tend = share ? nfull : ntiles;
    // T[k][i] over the column steps [ks0, ks1) of the lane's visibility
    auto contract = [&](double ak, int ks0, int ks1, floatx16 (&accR)[NT], floatx16 (&accI)[NT]) {
        float fc[8], fs[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) cis2pi_hw((float)phase(ak, e), fc[e], fs[e]);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                accR[t][r] = 0.f;
                accI[t][r] = 0.f;
            }
#pragma unroll 2
        for (int ks = ks0; ks < ks1; ++ks) {
            // twiddles of columns j0 + 16 ks + 8 h + e: E(a_k (j0 + 16 ks + 8 h - N/2)) E(a_k e)
            float cc, sc;
            cis2pi_hw((float)phase(ak, j0 + 16 * ks + 8 * hk - half), cc, sc);
            float cv[8], nsv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                cv[e] = cc * fc[e] - sc * fs[e];
                nsv[e] = (-sc) * fc[e] - cc * fs[e];   // negations fold into the operand modifiers
            }
            h8 th, tl, uh, ul;
            split8<H>(cv, th, tl);
            split8<H>(nsv, uh, ul);
            const int o = 8 * ((2 * ks + hk) ^ (l32 & SWM));
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const h8 bh = *reinterpret_cast<const h8 *>(&sH[32 * t + l32][o]);
                const h8 bl = *reinterpret_cast<const h8 *>(&sL[32 * t + l32][o]);
                accR[t] = Half32<H>::mma(bh, th, accR[t]);
                accI[t] = Half32<H>::mma(bh, uh, accI[t]);
                accR[t] = Half32<H>::mma(bh, tl, accR[t]);
                accI[t] = Half32<H>::mma(bh, ul, accI[t]);
                accR[t] = Half32<H>::mma(bl, th, accR[t]);
                accI[t] = Half32<H>::mma(bl, uh, accI[t]);
            }
        }
    };
    // row dot of the lane's visibility over its 64 rows, the two lanes of a
    // visibility added (unscaled)
    auto row_dot = [&](double bk, const floatx16 (&accR)[NT], const floatx16 (&accI)[NT], double &vr,
                       double &vi) {
        float f1c[4], f1s[4], f2c[4], f2s[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            cis2pi_hw((float)phase(bk, r), f1c[r], f1s[r]);
            cis2pi_hw((float)phase(bk, 8 * r), f2c[r], f2s[r]);
        }
        float c32, s32, cb, sb;
        cis2pi_hw((float)phase(bk, 32), c32, s32);
        cis2pi_hw((float)phase(bk, i0 + 4 * hk - half), cb, sb);
        // W = sum_t conj(E(32 b_k))^t W_t by Horner's rule, W_t = sum_a conj
        // E(8 b_k a) sum_r conj E(b_k r) T_t[4 a + r]
        float wr = 0.f, wi = 0.f;
#pragma unroll
        for (int t = NT - 1; t >= 0; --t) {
            float tr = 0.f, ti = 0.f;
#pragma unroll
            for (int aa = 0; aa < 4; ++aa) {
                float ur = 0.f, ui = 0.f;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float xr = accR[t][4 * aa + r], xi = accI[t][4 * aa + r];
                    ur += f1c[r] * xr + f1s[r] * xi;
                    ui += f1c[r] * xi - f1s[r] * xr;
                }
                tr += f2c[aa] * ur + f2s[aa] * ui;
                ti += f2c[aa] * ui - f2s[aa] * ur;
            }
            const float nr = tr + c32 * wr + s32 * wi;
            wi = ti + c32 * wi - s32 * wr;
            wr = nr;
        }
        vr = (double)(cb * wr + sb * wi);
        vi = (double)(cb * wi - sb * wr);
        vr += __shfl_xor(vr, 32, 64);
        vi += __shfl_xor(vi, 32, 64);
    };
    for (long long tile = (long long)wave * it.nwg + it.wg; tile < tend; tile += stride) {
        const long long k0 = it.kbeg + TV * tile;
        const int nvalid = (int)(it.kend - k0 < TV ? it.kend - k0 : TV);
        const bool ok = l32 < nvalid;
        const double ak = ok ? a[k0 + l32] : 0.0;
        const double bk = ok ? b[k0 + l32] : 0.0;
        floatx16 accR[NT], accI[NT];
        contract(ak, 0, KSTEPS, accR, accI);
        double vr, vi;
        row_dot(bk, accR, accI, vr, vi);
        if (hk == 0 && ok) vpart[(size_t)it.part * ztot + k0 + l32] = make_double2(vr * unscale, vi * unscale);
    }
    if (!share) return;
    __shared__ double2 sSl[8][TV];
    constexpr int KPW = KSTEPS / 8;   // column steps per wave
    for (long long tile = nfull + it.wg; tile < ntiles; tile += it.nwg) {
        const long long k0 = it.kbeg + TV * tile;
        const int nvalid = (int)(it.kend - k0 < TV ? it.kend - k0 : TV);
        const bool ok = l32 < nvalid;
        const double ak = ok ? a[k0 + l32] : 0.0;
        const double bk = ok ? b[k0 + l32] : 0.0;
        floatx16 accR[NT], accI[NT];
        contract(ak, KPW * wave, KPW * (wave + 1), accR, accI);
        double vr, vi;
        row_dot(bk, accR, accI, vr, vi);
        if (hk == 0) sSl[wave][l32] = make_double2(vr, vi);
        __syncthreads();
        if (tid < nvalid) {
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                sr += sSl[w][tid].x;
                si += sSl[w][tid].y;
            }
            vpart[(size_t)it.part * ztot + k0 + tid] = make_double2(sr * unscale, si * unscale);
        }
        __syncthreads();
    }
}

template <typename T>
hipError_t fwd_dispatch(const uvmem_ctx *c, const void *bop, hipStream_t st, const FwdPItem *items, int nitems) {
    if (nitems == 0) return hipSuccess;
    const dim3 grid(nitems), blk(512);
    if constexpr (sizeof(T) == 4) {
        if (c->ib_rows == 128 && c->jb_cols == 256) {
            hipLaunchKernelGGL((k_forward_p<T, 128, 256>), grid, blk, 0, st, items, c->d_a, c->d_b,
                               (const T *)bop, c->d_vpart, c->n, c->np, (long long)c->ztot);
            return hipGetLastError();
        }
        if (c->ib_rows == 128 && c->jb_cols == 128) {
            hipLaunchKernelGGL((k_forward_p<T, 128, 128>), grid, blk, 0, st, items, c->d_a, c->d_b,
                               (const T *)bop, c->d_vpart, c->n, c->np, (long long)c->ztot);
            return hipGetLastError();
        }
    } else {
        if (c->ib_rows == 64 && c->jb_cols == 256) {
            hipLaunchKernelGGL((k_forward_p<T, 64, 256>), grid, blk, 0, st, items, c->d_a, c->d_b,
                               (const T *)bop, c->d_vpart, c->n, c->np, (long long)c->ztot);
            return hipGetLastError();
        }
        if (c->ib_rows == 64 && c->jb_cols == 128) {
            hipLaunchKernelGGL((k_forward_p<T, 64, 128>), grid, blk, 0, st, items, c->d_a, c->d_b,
                               (const T *)bop, c->d_vpart, c->n, c->np, (long long)c->ztot);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_forward_p<T, 64, 64>), grid, blk, 0, st, items, c->d_a, c->d_b, (const T *)bop,
                       c->d_vpart, c->n, c->np, (long long)c->ztot);
    return hipGetLastError();
}

template <typename T>
hipError_t adj_dispatch(const uvmem_ctx *c, const double2 *coef, const float *w, hipStream_t st,
                        const AdjItem *items, int nitems) {
    if (nitems == 0) return hipSuccess;
    if constexpr (sizeof(T) == 4) {
        if (c->adj_tt == 256) {
            if (c->gpart_f32)
                hipLaunchKernelGGL(k_adjoint_w<true>, dim3(nitems), dim3(512), 0, st, items, c->d_a, c->d_b, coef, w,
                                   c->d_gpart, c->n, c->np);
            else
                hipLaunchKernelGGL(k_adjoint_w<false>, dim3(nitems), dim3(512), 0, st, items, c->d_a, c->d_b, coef,
                                   w, c->d_gpart, c->n, c->np);
            return hipGetLastError();
        }
    }
    if (c->adj_tt == 128)
        hipLaunchKernelGGL((k_adjoint<T, 64>), dim3(nitems), dim3(256), 0, st, items, c->d_a,
                           c->d_b, coef, w, (double *)c->d_gpart, c->n, c->np);
    else
        hipLaunchKernelGGL((k_adjoint<T, 32>), dim3(nitems), dim3(256), 0, st, items, c->d_a,
                           c->d_b, coef, w, (double *)c->d_gpart, c->n, c->np);
    return hipGetLastError();
}

template <typename H, int NV>
hipError_t fwd_h16_t(const uvmem_ctx *c, const float *B, hipStream_t st, const FwdPItem *items, int nitems) {
    const dim3 grid(nitems), blk(512);
    if (c->ib_rows == 128 && c->jb_cols == 256)
        hipLaunchKernelGGL((k_forward_h16m<H, 128, 256>), grid, blk, 0, st, items, c->d_a, c->d_b, B,
                           c->d_vpart, c->n, c->np, (long long)c->ztot);
    else if (c->ib_rows == 128 && c->jb_cols == 128)
        hipLaunchKernelGGL((k_forward_h16m<H, 128, 128>), grid, blk, 0, st, items, c->d_a, c->d_b, B,
                           c->d_vpart, c->n, c->np, (long long)c->ztot);
    else
        hipLaunchKernelGGL((k_forward_h16p<H, 64, 64, NV>), grid, blk, 0, st, items, c->d_a, c->d_b, B,
                           c->d_vpart, c->n, c->np, (long long)c->ztot);
    return hipGetLastError();
}

// One 16-visibility group per wave tile: two groups (one LDS image read for
// twice the matrix-core work) measured slower on 256^2 (register pressure).
template <typename H>
hipError_t fwd_h16(const uvmem_ctx *c, const void *bop, hipStream_t st, const FwdPItem *items, int nitems) {
    if (nitems == 0) return hipSuccess;
    return fwd_h16_t<H, 1>(c, reinterpret_cast<const float *>(bop), st, items, nitems);
}

template <typename H>
hipError_t adj_h16(const uvmem_ctx *c, const double2 *coef, const float *w, hipStream_t st, const AdjItem *items,
                   int nitems) {
    if (nitems == 0) return hipSuccess;
    if (c->adj_tt == 256)
        hipLaunchKernelGGL((k_adjoint_h16s<H>), dim3(nitems), dim3(512), 0, st, items, c->d_a, c->d_b,
                           coef, w, c->d_vispart, c->d_vis_base, (float *)c->d_gpart, c->n, c->np);
    else if (c->adj_tt == 128)
        hipLaunchKernelGGL((k_adjoint_h16<H, 64>), dim3(nitems), dim3(256), 0, st, items, c->d_a, c->d_b,
                           coef, w, c->d_vispart, c->d_vis_base, (float *)c->d_gpart, c->n, c->np);
    else
        hipLaunchKernelGGL((k_adjoint_h16<H, 32>), dim3(nitems), dim3(256), 0, st, items, c->d_a, c->d_b,
                           coef, w, c->d_vispart, c->d_vis_base, (float *)c->d_gpart, c->n, c->np);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_forward_f32_raw(int ib_rows, int jb_cols, const FwdPItem *items, int nitems, const double *a,
                                  const double *b, const float *bop, double2 *vpart, int n, int np,
                                  long long ztot, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    const dim3 grid(nitems), blk(512);
    if (ib_rows == 128 && jb_cols == 256)
        hipLaunchKernelGGL((k_forward_p<float, 128, 256>), grid, blk, 0, st, items, a, b, bop, vpart, n, np, ztot);
    else if (ib_rows == 128 && jb_cols == 128)
        hipLaunchKernelGGL((k_forward_p<float, 128, 128>), grid, blk, 0, st, items, a, b, bop, vpart, n, np, ztot);
    else if (ib_rows == 64 && jb_cols == 64)
        hipLaunchKernelGGL((k_forward_p<float, 64, 64>), grid, blk, 0, st, items, a, b, bop, vpart, n, np, ztot);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_forward(const uvmem_ctx *c, const void *bop, hipStream_t st, int dir) {
    if (c->fwd_model == UVMEM_FWD_GRIDDED) return launch_grid_forward(c, bop, st);
    // the direction of a region-restricted CG is zero outside the region
    const bool rg = dir && c->has_region;
    const FwdPItem *it = rg ? c->d_fwdp_m : c->d_fwdp;
    const int ni = rg ? c->n_fwdp_m : c->n_fwdp;
    if (c->prec == UVMEM_FP64) return fwd_dispatch<double>(c, bop, st, it, ni);
    if (c->prec == UVMEM_BF16X3) return fwd_h16<__bf16>(c, bop, st, it, ni);
    if (c->prec == UVMEM_FP16X3) return fwd_h16<_Float16>(c, bop, st, it, ni);
    return fwd_dispatch<float>(c, bop, st, it, ni);
}

// Workgroups of the adjoint kernel that this context launches which fit on
// one CU at once (registers, LDS and waves of the compiled kernel), at
// least 1.
int adjoint_wgs_per_cu(const uvmem_ctx *c) {
    int nb = 0;
    hipError_t e = hipSuccess;
    const bool split = c->prec == UVMEM_BF16X3 || c->prec == UVMEM_FP16X3;
    if (split) {
        if (c->adj_tt == 256)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adjoint_h16s<__bf16>, 512, 0);
        else if (c->adj_tt == 128)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adjoint_h16<__bf16, 64>, 256, 0);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adjoint_h16<__bf16, 32>, 256, 0);
    } else if (c->prec == UVMEM_FP64) {
        if (c->adj_tt == 128)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adjoint<double, 64>, 256, 0);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adjoint<double, 32>, 256, 0);
    } else if (c->adj_tt == 256) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adjoint_w<true>, 512, 0);
    } else if (c->adj_tt == 128) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adjoint<float, 64>, 256, 0);
    } else {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adjoint<float, 32>, 256, 0);
    }
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_adjoint(const uvmem_ctx *c, const double2 *coef, const float *w, hipStream_t st, int grad) {
    if (c->fwd_model == UVMEM_FWD_GRIDDED && c->grad_model == UVMEM_GRAD_ADJOINT)
        return launch_grid_adjoint(c, coef, w, st);
    // a gradient of a region-restricted problem is needed inside the region only
    const bool rg = grad && c->has_region;
    const AdjItem *it = rg ? c->d_adj_m : c->d_adj;
    const int ni = rg ? c->n_adj_m : c->n_adj;
    if (c->prec == UVMEM_FP64) return adj_dispatch<double>(c, coef, w, st, it, ni);
    if (c->prec == UVMEM_BF16X3) return adj_h16<__bf16>(c, coef, w, st, it, ni);
    if (c->prec == UVMEM_FP16X3) return adj_h16<_Float16>(c, coef, w, st, it, ni);
    return adj_dispatch<float>(c, coef, w, st, it, ni);
}

}  // namespace uvm
