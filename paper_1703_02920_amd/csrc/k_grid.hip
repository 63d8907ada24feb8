// Gridded forward model of the paper's GPU objective (Sec. 2.4, Alg. 1) and
// its exact adjoint, for gfx950.
//
// Forward, per channel c (grid side L = oversample * N, a power of two,
// du = 1 / (L cell)):
//   B = A_c o I (staged by the prologue, zero-padded to L x L here),
//   Vhat[p][q] = e^{+2 pi i (p + q)(N/2)/L} sum_{i,j} B_ij e^{-2 pi i (p j + q i)/L}
//     (2-D DFT, then the modulation that puts the phase centre at pixel N/2),
//   V_k = bilinear interpolation of Vhat at (u_k/du, v_k/du) = (a_k L, b_k L),
//     wrapping modulo L.
// The spectrum is stored transposed, [p][q] (u index major), so that both
// transform passes read and write whole rows.  Adjoint (the transpose of the
// above, real part): each grid node gathers w_k c_k times its bilinear
// weight from the visibilities of the four cells around it (visibilities
// sorted by cell at set-up: a fixed summation order, no atomics), takes the
// conjugate modulation, and two inverse passes give Re sum H e^{+...} on the
// first N rows and columns: the channel's plane of the split-K partial
// buffer, which the gradient kernel multiplies by A_c.
//
// Transform: decimation in time on P sequences of length L held in LDS,
// inputs placed at bit-reversed positions, radix-2 stages fused in pairs
// (one barrier per pair); twiddles e^{-2 pi i k / L}, k < L/2, from a table
// built in FP64 at set-up.
// FP64 transforms for the FP64 precision, FP32 otherwise.

#include "internal.h"

namespace uvm {
namespace {

template <typename T> struct Cx;
template <> struct Cx<float> { using t = float2; };
template <> struct Cx<double> { using t = double2; };

template <typename T> using V2 = typename Cx<T>::t;

constexpr int GT = 256;   // threads per workgroup of the grid kernels

__device__ __forceinline__ int bitrev(int e, int lg) { return (int)(__brev((unsigned)e) >> (32 - lg)); }

// Workgroups are dispatched to the 8 XCDs round-robin (block b on XCD b % 8);
// the column passes renumber them so that each XCD works through one
// contiguous run of column groups, whose partial cache lines then meet in
// that XCD's L2.  Identity unless the grid is a multiple of 8.
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
    return (nblocks & 7) ? b : (b & 7) * (nblocks >> 3) + (b >> 3);
}

// e^{+2 pi i m / L} for an integer m in [0, L) from the table of e^{-2 pi i k / L}.
template <typename T>
__device__ __forceinline__ V2<T> expi_pos(const V2<T> *__restrict__ tw, int m, int L) {
    const int h = L >> 1;
    V2<T> t = tw[m < h ? m : m - h];
    V2<T> r;
    r.x = m < h ? t.x : -t.x;
    r.y = m < h ? -t.y : t.y;
    return r;
}

template <typename T>
__device__ __forceinline__ V2<T> cmul(V2<T> w, V2<T> x) {
    V2<T> t;
    t.x = w.x * x.x - w.y * x.y;
    t.y = w.x * x.y + w.y * x.x;
    return t;
}

template <typename T>
__device__ __forceinline__ void bfly(V2<T> &x0, V2<T> &x1, V2<T> w) {
    const V2<T> t = cmul<T>(w, x1);
    V2<T> y0, y1;
    y0.x = x0.x + t.x;
    y0.y = x0.y + t.y;
    y1.x = x0.x - t.x;
    y1.y = x0.y - t.y;
    x0 = y0;
    x1 = y1;
}

template <typename T, int DIR>
__device__ __forceinline__ V2<T> twid(const V2<T> *__restrict__ tw, int idx) {
    V2<T> w = tw[idx];
    if (DIR > 0) w.y = -w.y;
    return w;
}

// Stages of the in-place transform of s[r * L + e], r < P (inputs already at
// bit-reversed positions).  DIR = -1: e^{-}, +1: e^{+}.  Radix-2 stage st
// (span 2h, h = 2^(st-1)) combines s[i] and s[i + h] with W_{2h}^j; pairs of
// stages run as one radix-4 pass over four elements per thread (the same
// butterflies, half the LDS round trips and barriers), and an odd last
// stage runs alone.
template <typename T, int DIR>
__device__ void fft_stages(V2<T> *s, int P, int lg, const V2<T> *__restrict__ tw) {
    const int L = 1 << lg;
    int st = 1;
    for (; st + 1 <= lg; st += 2) {
        const int h = 1 << (st - 1);
        const int nq = P * (L >> 2);
        for (int b = threadIdx.x; b < nq; b += GT) {
            const int r = b >> (lg - 2);
            const int k = b & ((L >> 2) - 1);
            const int j = k & (h - 1);
            const int i0 = r * L + ((k >> (st - 1)) << (st + 1)) + j;
            V2<T> a0 = s[i0], a1 = s[i0 + h], a2 = s[i0 + 2 * h], a3 = s[i0 + 3 * h];
            const V2<T> w1 = twid<T, DIR>(tw, j * (L >> st));
            bfly<T>(a0, a1, w1);
            bfly<T>(a2, a3, w1);
            bfly<T>(a0, a2, twid<T, DIR>(tw, j * (L >> (st + 1))));
            bfly<T>(a1, a3, twid<T, DIR>(tw, (j + h) * (L >> (st + 1))));
            s[i0] = a0;
            s[i0 + h] = a1;
            s[i0 + 2 * h] = a2;
            s[i0 + 3 * h] = a3;
        }
        __syncthreads();
    }
    if (st == lg) {
        const int h = 1 << (st - 1);
        const int nb = P * (L >> 1);
        for (int b = threadIdx.x; b < nb; b += GT) {
            const int r = b >> (lg - 1);
            const int k = b & ((L >> 1) - 1);
            const int j = k & (h - 1);
            const int i0 = r * L + ((k >> (st - 1)) << st) + j;
            V2<T> x0 = s[i0], x1 = s[i0 + h];
            bfly<T>(x0, x1, twid<T, DIR>(tw, j * (L >> st)));
            s[i0] = x0;
            s[i0 + h] = x1;
        }
        __syncthreads();
    }
}

// Forward pass 1: rows i < N of B_c (stride np), zero-padded to L:
// x1[c][i][p] = sum_j B[i][j] e^{-2 pi i p j / L}.  P rows per workgroup.
template <typename T, typename R>
__global__ __launch_bounds__(GT) void k_grid_rows_fwd(const R *__restrict__ bop, int n, int np, int lg, int P,
                                                      const V2<T> *__restrict__ tw, V2<T> *__restrict__ x1) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    V2<T> *s = reinterpret_cast<V2<T> *>(smem);
    const int L = 1 << lg;
    const int bpc = (n + P - 1) / P;
    const int c = blockIdx.x / bpc, i0 = (blockIdx.x % bpc) * P;
    const R *B = bop + (size_t)c * np * np;
    for (int x = threadIdx.x; x < P * L; x += GT) {
        const int r = x >> lg, e = x & (L - 1), i = i0 + r;
        V2<T> v;
        v.x = (e < n && i < n) ? (T)B[(size_t)i * np + e] : (T)0;
        v.y = (T)0;
        s[r * L + bitrev(e, lg)] = v;
    }
    __syncthreads();
    fft_stages<T, -1>(s, P, lg, tw);
    for (int x = threadIdx.x; x < P * L; x += GT) {
        const int r = x >> lg, p = x & (L - 1), i = i0 + r;
        if (i < n) x1[((size_t)c * n + i) * L + p] = s[r * L + p];
    }
}

// Forward pass 2: P adjacent columns p of x1 (rows i < N, zero beyond),
// transformed along i and modulated: grid[c][p][q].
template <typename T>
__global__ __launch_bounds__(GT) void k_grid_cols_fwd(const V2<T> *__restrict__ x1, int n, int lg, int P,
                                                      const V2<T> *__restrict__ tw, V2<T> *__restrict__ grid) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    V2<T> *s = reinterpret_cast<V2<T> *>(smem);
    const int L = 1 << lg;
    const int bpc = L / P;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int c = blk / bpc, p0 = (blk % bpc) * P;
    const V2<T> *X = x1 + (size_t)c * n * L;
    for (int x = threadIdx.x; x < P * L; x += GT) {
        const int r = x % P, i = x / P;
        V2<T> v;
        if (i < n) v = X[(size_t)i * L + p0 + r];
        else { v.x = (T)0; v.y = (T)0; }
        s[r * L + bitrev(i, lg)] = v;
    }
    __syncthreads();
    fft_stages<T, -1>(s, P, lg, tw);
    const int hn = n >> 1;
    V2<T> *G = grid + (size_t)c * L * L;
    for (int x = threadIdx.x; x < P * L; x += GT) {
        const int r = x >> lg, q = x & (L - 1), p = p0 + r;
        const int m = (int)(((long long)(p + q) * hn) & (L - 1));
        const V2<T> f = expi_pos<T>(tw, m, L);
        const V2<T> v = s[r * L + q];
        V2<T> o;
        o.x = v.x * f.x - v.y * f.y;
        o.y = v.x * f.y + v.y * f.x;
        G[(size_t)p * L + q] = o;
    }
}

// Lower grid node (mod L) and bilinear fractions of a visibility.
__device__ __forceinline__ void grid_node(double a, double b, int L, int &p0, int &q0, double &fx, double &fy) {
    const double gx = a * (double)L, gy = b * (double)L;
    const double px = floor(gx), py = floor(gy);
    fx = gx - px;
    fy = gy - py;
    p0 = (int)((long long)px & (long long)(L - 1));
    q0 = (int)((long long)py & (long long)(L - 1));
}

// Forward pass 3: V_k by bilinear interpolation, one workgroup per
// visibility item; written as the single forward partial.
template <typename T>
__global__ __launch_bounds__(GT) void k_grid_interp(const VisItem *__restrict__ items, const double *__restrict__ a,
                                                    const double *__restrict__ b, const V2<T> *__restrict__ grid,
                                                    int lg, double2 *__restrict__ vout) {
    const VisItem it = items[blockIdx.x];
    const int L = 1 << lg;
    const V2<T> *G = grid + (size_t)it.chan * L * L;
    for (long long k = it.kbeg + threadIdx.x; k < it.kend; k += GT) {
        int p0, q0;
        double fx, fy;
        grid_node(a[k], b[k], L, p0, q0, fx, fy);
        const int p1 = (p0 + 1) & (L - 1), q1 = (q0 + 1) & (L - 1);
        const V2<T> g00 = G[(size_t)p0 * L + q0], g10 = G[(size_t)p1 * L + q0];
        const V2<T> g01 = G[(size_t)p0 * L + q1], g11 = G[(size_t)p1 * L + q1];
        const double w00 = (1.0 - fx) * (1.0 - fy), w10 = fx * (1.0 - fy), w01 = (1.0 - fx) * fy, w11 = fx * fy;
        double2 v;
        v.x = w00 * (double)g00.x + w10 * (double)g10.x + w01 * (double)g01.x + w11 * (double)g11.x;
        v.y = w00 * (double)g00.y + w10 * (double)g10.y + w01 * (double)g01.y + w11 * (double)g11.y;
        vout[k] = v;
    }
}

// Adjoint pass 0: the weighted coefficients w_k coef_k in cell-sorted
// order (w may be null), so that pass 1 reads contiguous ranges.
__global__ __launch_bounds__(GT) void k_grid_sort_coef(const int *__restrict__ perm, const double2 *__restrict__ coef,
                                                       const float *__restrict__ w, long long ztot,
                                                       double2 *__restrict__ sorted) {
    const long long j = (long long)blockIdx.x * GT + threadIdx.x;
    if (j >= ztot) return;
    const int k = perm[j];
    const double ww = w ? (double)w[k] : 1.0;
    const double2 cf = coef[k];
    sorted[j] = make_double2(ww * cf.x, ww * cf.y);
}

// Adjoint pass 1a: the four weighted sums of each dense cell (more than
// GRID_DENSE visibilities) -- its shares for the nodes (p0, q0), (p0+1, q0),
// (p0, q0+1), (p0+1, q0+1) -- one wave per cell, lanes striding over the
// cell's sorted range, then a fixed butterfly reduction.
__global__ __launch_bounds__(GT) void k_grid_dense(const int2 *__restrict__ dlist, int ndense,
                                                   const double2 *__restrict__ fxy,
                                                   const double2 *__restrict__ sorted, double2 *__restrict__ dsum) {
    const int lane = threadIdx.x & 63;
    const int cidx = blockIdx.x * (GT / 64) + (threadIdx.x >> 6);
    if (cidx >= ndense) return;   // the whole wave leaves together
    const int2 rg = dlist[cidx];
    double acc[8];
#pragma unroll
    for (int x = 0; x < 8; ++x) acc[x] = 0.0;
    for (int j = rg.x + lane; j < rg.y; j += 64) {
        const double2 f = fxy[j], cf = sorted[j];
        const double w[4] = {(1.0 - f.x) * (1.0 - f.y), f.x * (1.0 - f.y), (1.0 - f.x) * f.y, f.x * f.y};
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            acc[2 * d] += w[d] * cf.x;
            acc[2 * d + 1] += w[d] * cf.y;
        }
    }
#pragma unroll
    for (int x = 0; x < 8; ++x)
        for (int o = 32; o > 0; o >>= 1) acc[x] += __shfl_xor(acc[x], o, 64);
    if (lane == 0)
        for (int d = 0; d < 4; ++d) dsum[(size_t)cidx * 4 + d] = make_double2(acc[2 * d], acc[2 * d + 1]);
}

// Adjoint pass 1: H[c][p][q] = e^{-2 pi i (p+q)(N/2)/L} sum over the four
// cells around node (p, q) of bilinear weight x (w coef), reading the
// cell-sorted coefficients and the bilinear fractions stored in the same
// order at set-up.
template <typename T>
__global__ __launch_bounds__(GT) void k_grid_gather(const int *__restrict__ cell_start,
                                                    const double2 *__restrict__ fxy,
                                                    const double2 *__restrict__ sorted,
                                                    const int *__restrict__ didx, const double2 *__restrict__ dsum,
                                                    int n, int lg, int nchan, const V2<T> *__restrict__ tw,
                                                    V2<T> *__restrict__ hgrid) {
    const int L = 1 << lg;
    const long long cells = (long long)L * L;
    const long long t = (long long)blockIdx.x * GT + threadIdx.x;
    if (t >= cells * nchan) return;
    const int c = (int)(t / cells);
    const int cell = (int)(t % cells);
    const int p = cell >> lg, q = cell & (L - 1);
    const int *cs = cell_start + (size_t)c * (cells + 1);
    int jb[4], je[4], di[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int src = ((p - (d & 1)) & (L - 1)) * L + ((q - (d >> 1)) & (L - 1));
        jb[d] = cs[src];
        je[d] = cs[src + 1];
        di[d] = didx[(size_t)c * cells + src];
    }
    // sums in sorted order; four visibilities' loads issued together
    double hx = 0.0, hy = 0.0;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int dp = d & 1, dq = d >> 1;
        if (di[d] >= 0) {   // a dense cell: its share for this node, summed in pass 1a
            const double2 v = dsum[(size_t)di[d] * 4 + d];
            hx += v.x;
            hy += v.y;
            continue;
        }
        int j = jb[d];
        for (; j + 4 <= je[d]; j += 4) {
            double2 f[4], cf[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                f[u] = fxy[j + u];
                cf[u] = sorted[j + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double wt = (dp ? f[u].x : 1.0 - f[u].x) * (dq ? f[u].y : 1.0 - f[u].y);
                hx += wt * cf[u].x;
                hy += wt * cf[u].y;
            }
        }
        for (; j < je[d]; ++j) {
            const double2 f = fxy[j];
            const double wt = (dp ? f.x : 1.0 - f.x) * (dq ? f.y : 1.0 - f.y);
            const double2 cf = sorted[j];
            hx += wt * cf.x;
            hy += wt * cf.y;
        }
    }
    const int m = (int)(((long long)(p + q) * (n >> 1)) & (L - 1));
    const V2<T> f = expi_pos<T>(tw, m, L);   // conjugated below
    V2<T> o;
    o.x = (T)(hx * (double)f.x + hy * (double)f.y);
    o.y = (T)(hy * (double)f.x - hx * (double)f.y);
    hgrid[(size_t)c * cells + cell] = o;
}

// Adjoint pass 2: P rows p of H, inverse transform along q, outputs i < N:
// y[c][p][i].
template <typename T>
__global__ __launch_bounds__(GT) void k_grid_rows_inv(const V2<T> *__restrict__ hgrid, int n, int lg, int P,
                                                      const V2<T> *__restrict__ tw, V2<T> *__restrict__ y) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    V2<T> *s = reinterpret_cast<V2<T> *>(smem);
    const int L = 1 << lg;
    const int bpc = L / P;
    const int c = blockIdx.x / bpc, p0 = (blockIdx.x % bpc) * P;
    const V2<T> *H = hgrid + ((size_t)c * L + p0) * L;
    for (int x = threadIdx.x; x < P * L; x += GT) {
        const int r = x >> lg, q = x & (L - 1);
        s[r * L + bitrev(q, lg)] = H[(size_t)r * L + q];
    }
    __syncthreads();
    fft_stages<T, 1>(s, P, lg, tw);
    for (int x = threadIdx.x; x < P * n; x += GT) {
        const int r = x / n, i = x % n;
        y[((size_t)c * L + p0 + r) * n + i] = s[r * L + i];
    }
}

// Adjoint pass 3: P image rows i (columns of y), inverse transform along p,
// outputs j < N, real part into the channel's plane of the partial buffer.
template <typename T, typename PT>
__global__ __launch_bounds__(GT) void k_grid_cols_inv(const V2<T> *__restrict__ y, int n, int np, int lg, int P,
                                                      const V2<T> *__restrict__ tw, const int *__restrict__ slot_base,
                                                      PT *__restrict__ gpart) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    V2<T> *s = reinterpret_cast<V2<T> *>(smem);
    const int L = 1 << lg;
    const int bpc = (n + P - 1) / P;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int c = blk / bpc, i0 = (blk % bpc) * P;
    const V2<T> *Y = y + (size_t)c * L * n;
    for (int x = threadIdx.x; x < P * L; x += GT) {
        const int r = x % P, pp = x / P, i = i0 + r;
        V2<T> v;
        if (i < n) v = Y[(size_t)pp * n + i];
        else { v.x = (T)0; v.y = (T)0; }
        s[r * L + bitrev(pp, lg)] = v;
    }
    __syncthreads();
    fft_stages<T, 1>(s, P, lg, tw);
    PT *out = gpart + (size_t)slot_base[c] * np * np;
    for (int x = threadIdx.x; x < P * n; x += GT) {
        const int r = x / n, j = x % n, i = i0 + r;
        if (i < n) out[(size_t)i * np + j] = (PT)s[r * L + j].x;
    }
}

// Sequences per workgroup: enough butterflies for the workgroup (rows), or
// adjacent columns for wider loads (columns), within 64 KiB of LDS and
// keeping at least 256 workgroups where the grid allows.
int seqs_rows(int L, size_t esz) {
    const int cap = (int)std::max<size_t>(1, 65536 / ((size_t)L * esz));
    return std::max(1, std::min(std::min(cap, L), 512 / L));
}

int seqs_cols(int L, size_t esz, int nchan) {
    const int cap = (int)std::max<size_t>(1, 65536 / ((size_t)L * esz));
    int P = std::min(8, cap);
    while (P > 1 && (long long)nchan * L / P < 256) P >>= 1;
    return P;
}

template <typename T>
hipError_t grid_fwd_t(const uvmem_ctx *c, const void *bop, hipStream_t st) {
    const int n = c->n, lg = c->grid_lg, L = 1 << lg, C = c->nchan;
    const V2<T> *tw = reinterpret_cast<const V2<T> *>(c->d_gtw);
    V2<T> *x1 = reinterpret_cast<V2<T> *>(c->d_gx1);
    V2<T> *grid = reinterpret_cast<V2<T> *>(c->d_ggrid);
    const size_t esz = sizeof(V2<T>);
    const int pr = seqs_rows(L, esz), pc = seqs_cols(L, esz, C);
    hipLaunchKernelGGL((k_grid_rows_fwd<T, T>), dim3(C * ((n + pr - 1) / pr)), dim3(GT), pr * L * esz, st,
                       reinterpret_cast<const T *>(bop), n, c->np, lg, pr, tw, x1);
    hipLaunchKernelGGL((k_grid_cols_fwd<T>), dim3(C * (L / pc)), dim3(GT), pc * L * esz, st, x1, n, lg, pc, tw,
                       grid);
    if (c->n_visit > 0)
        hipLaunchKernelGGL((k_grid_interp<T>), dim3(c->n_visit), dim3(GT), 0, st, c->d_vis, c->d_a, c->d_b, grid, lg,
                           c->d_vpart);
    return hipGetLastError();
}

template <typename T, typename PT>
hipError_t grid_adj_t(const uvmem_ctx *c, const double2 *coef, const float *w, hipStream_t st) {
    const int n = c->n, lg = c->grid_lg, L = 1 << lg, C = c->nchan;
    const V2<T> *tw = reinterpret_cast<const V2<T> *>(c->d_gtw);
    V2<T> *y = reinterpret_cast<V2<T> *>(c->d_gx1);
    V2<T> *hgrid = reinterpret_cast<V2<T> *>(c->d_ggrid);
    const size_t esz = sizeof(V2<T>);
    const long long cells = (long long)L * L * C;
    if (c->ztot > 0)
        hipLaunchKernelGGL(k_grid_sort_coef, dim3((unsigned)((c->ztot + GT - 1) / GT)), dim3(GT), 0, st, c->d_gperm,
                           coef, w, (long long)c->ztot, c->d_gsc);
    if (c->n_gdense > 0)
        hipLaunchKernelGGL(k_grid_dense, dim3((c->n_gdense + GT / 64 - 1) / (GT / 64)), dim3(GT), 0, st, c->d_gdlist,
                           c->n_gdense, c->d_gfxy, c->d_gsc, c->d_gdsum);
    hipLaunchKernelGGL((k_grid_gather<T>), dim3((unsigned)((cells + GT - 1) / GT)), dim3(GT), 0, st, c->d_gcell,
                       c->d_gfxy, c->d_gsc, c->d_gdidx, c->d_gdsum, n, lg, C, tw, hgrid);
    const int pr = seqs_rows(L, esz), pc = seqs_cols(L, esz, C);
    hipLaunchKernelGGL((k_grid_rows_inv<T>), dim3(C * (L / pr)), dim3(GT), pr * L * esz, st, hgrid, n, lg, pr, tw, y);
    hipLaunchKernelGGL((k_grid_cols_inv<T, PT>), dim3(C * ((n + pc - 1) / pc)), dim3(GT), pc * L * esz, st, y, n,
                       c->np, lg, pc, tw, c->d_slot_base, reinterpret_cast<PT *>(c->d_gpart));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_grid_forward(const uvmem_ctx *c, const void *bop, hipStream_t st) {
    if (c->prec == UVMEM_FP64) return grid_fwd_t<double>(c, bop, st);
    return grid_fwd_t<float>(c, bop, st);
}

hipError_t launch_grid_adjoint(const uvmem_ctx *c, const double2 *coef, const float *w, hipStream_t st) {
    if (c->prec == UVMEM_FP64) return grid_adj_t<double, double>(c, coef, w, st);
    if (c->gpart_f32) return grid_adj_t<float, float>(c, coef, w, st);
    return grid_adj_t<float, double>(c, coef, w, st);
}

}  // namespace uvm
