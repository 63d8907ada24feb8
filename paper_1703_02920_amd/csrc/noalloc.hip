// Allocation-free variant of the forward model (uvmem_forward_noalloc): the
// same FP32 matrix-core forward as a context's uvmem_forward, for callers
// that cannot allocate device memory.  Every buffer the launch needs beyond
// the caller's inputs and output -- the reduced coordinates, the attenuated
// operand image, the per-block partial visibilities and the work tables --
// lives in one file-scope device array of fixed size.  Each GPU holds its own
// copy of that array (its address is looked up once per device); calls that
// overlap on one GPU share it and race.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "internal.h"

using namespace uvm;

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)UVMEM_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
void *g_scratch[MAX_DEVICES];
hipError_t g_scratch_err[MAX_DEVICES];
std::once_flag g_scratch_once[MAX_DEVICES];

// Device address of this device's scratch array (looked up on the first call
// on each device, with that device current).
hipError_t scratch_address(int dev, void **ptr) {
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::call_once(g_scratch_once[dev], [dev]() {
        void *p = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch[dev] = g_scratch_err[dev] == hipSuccess ? p : nullptr;
    });
    *ptr = g_scratch[dev];
    return g_scratch_err[dev];
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Reduced coordinates a = u cell, b = v cell (FP64, as a context computes
// them), the forward work items (block (ib, jb) of the image, workgroup x of
// the g sharing its visibility tiles) and the visibility items of the
// partial sum.
__global__ void k_noalloc_setup(const double *__restrict__ u, const double *__restrict__ v, double cell,
                                long long nvis, double *__restrict__ a, double *__restrict__ b,
                                FwdPItem *__restrict__ items, int n_items, int n_jb, int g,
                                VisItem *__restrict__ vitems, int n_visit, long long vis_blk) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < nvis; k += stride) {
        a[k] = u[k] * cell;
        b[k] = v[k] * cell;
    }
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n_items; t += stride) {
        const int blk = (int)(t / g), x = (int)(t % g);
        items[t] = FwdPItem{0, blk / n_jb, blk % n_jb, blk, x, g, 0LL, nvis};
    }
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n_visit; t += stride) {
        const long long k0 = t * vis_blk;
        vitems[t] = VisItem{0, 0, k0, std::min(k0 + vis_blk, nvis)};
    }
}

// Operand image B = A o I on the padded np x np grid, zero outside the image
// (every element written: the scratch keeps the previous call's contents).
__global__ void k_noalloc_prologue(const float *__restrict__ I, const float *__restrict__ beam,
                                   float *__restrict__ bop, int n, int np) {
    const long long total = (long long)np * np;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += stride) {
        const int i = (int)(p / np), j = (int)(p % np);
        float x = 0.f;
        if (i < n && j < n) {
            const size_t q = (size_t)i * n + j;
            x = beam ? beam[q] * I[q] : I[q];
        }
        bop[p] = x;
    }
}

}  // namespace

extern "C" int uvmem_forward_noalloc(int n, double cell_rad, int64_t nvis, const double *u, const double *v,
                                     const float *beam, const float *I, double *vis, void *hip_stream) {
    if (n < 2 || n > 8192 || (n % 2) != 0) return UVMEM_EINVAL;
    if (nvis < 0 || !(cell_rad > 0.0) || !std::isfinite(cell_rad)) return UVMEM_EINVAL;
    if (!I || (nvis > 0 && (!u || !v || !vis))) return UVMEM_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    // layout as a context with this image side chooses for FP32
    const int np = (n + 63) / 64 * 64;
    int ib = 64, jb = 64;
    if (np % 256 == 0) { ib = 128; jb = 256; }
    else if (np % 128 == 0) { ib = 128; jb = 128; }
    const int n_ib = np / ib, n_jb = np / jb, nblk = n_ib * n_jb;
    // one workgroup per CU in all: g workgroups share each block's tiles
    const long long z = nvis;
    const long long L = std::max<long long>(16, (z * nblk + 255) / 256);
    const long long tiles = (z + 15) / 16;
    const int g = (int)std::max<long long>(1, std::min<long long>((z + L - 1) / L, (tiles + 7) / 8));
    const long long n_items = (long long)nblk * g;
    const long long vis_blk = std::max<long long>(2 * NTHR, ((z + VIS_WGS - 1) / VIS_WGS + 2 * NTHR - 1) /
                                                                (2 * NTHR) * (2 * NTHR));
    const long long n_visit = (z + vis_blk - 1) / vis_blk;
    // scratch layout
    const size_t o_a = 0;
    const size_t o_b = o_a + align256(sizeof(double) * (size_t)z);
    const size_t o_bop = o_b + align256(sizeof(double) * (size_t)z);
    const size_t o_vp = o_bop + align256(sizeof(float) * (size_t)np * np);
    const size_t o_it = o_vp + align256(sizeof(double2) * (size_t)nblk * (size_t)z);
    const size_t o_vi = o_it + align256(sizeof(FwdPItem) * (size_t)n_items);
    const size_t need = o_vi + align256(sizeof(VisItem) * (size_t)n_visit);
    if (need > SCRATCH_BYTES) return UVMEM_ETOOBIG;
    if (z == 0) return UVMEM_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return UVMEM_EDEVICE;
    void *base = nullptr;
    if (scratch_address(dev, &base) != hipSuccess || !base) return UVMEM_EDEVICE;
    unsigned char *s = static_cast<unsigned char *>(base);
    double *a = reinterpret_cast<double *>(s + o_a);
    double *b = reinterpret_cast<double *>(s + o_b);
    float *bop = reinterpret_cast<float *>(s + o_bop);
    double2 *vpart = reinterpret_cast<double2 *>(s + o_vp);
    FwdPItem *items = reinterpret_cast<FwdPItem *>(s + o_it);
    VisItem *vitems = reinterpret_cast<VisItem *>(s + o_vi);
    const long long setup_n = std::max<long long>(z, std::max(n_items, n_visit));
    const int setup_blocks = (int)std::min<long long>((setup_n + NTHR - 1) / NTHR, 2048);
    hipLaunchKernelGGL(k_noalloc_setup, dim3(setup_blocks), dim3(NTHR), 0, st, u, v, cell_rad, z, a, b, items,
                       (int)n_items, n_jb, g, vitems, (int)n_visit, vis_blk);
    if (hipGetLastError() != hipSuccess) return UVMEM_EDEVICE;
    const int pro_blocks = (int)std::min<long long>(((long long)np * np + NTHR - 1) / NTHR, 2048);
    hipLaunchKernelGGL(k_noalloc_prologue, dim3(pro_blocks), dim3(NTHR), 0, st, I, beam, bop, n, np);
    if (hipGetLastError() != hipSuccess) return UVMEM_EDEVICE;
    if (launch_forward_f32_raw(ib, jb, items, (int)n_items, a, b, bop, vpart, n, np, z, st) != hipSuccess)
        return UVMEM_EDEVICE;
    if (launch_vis_sum_raw(vitems, (int)n_visit, vpart, nblk, z, reinterpret_cast<double2 *>(vis), st) !=
        hipSuccess)
        return UVMEM_EDEVICE;
    return UVMEM_OK;
}
