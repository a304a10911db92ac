// Allocation-free diagnostics: lb_stats_noalloc computes what lb_stats returns
// (per-component mass, fluid momentum, mass removed by particles, fluid node
// count, health) for a lone handle or for every system of a batch, into the
// caller's device memory, on the handle's stream, without waiting and without
// any allocation. The per-block partial sums live in `scratch`, a file-scope
// device array that each GPU holds until the process ends; its device address
// is taken once per device (hipGetSymbolAddress, with that device current) at
// the entry point's first call there, and only that address is ever passed to
// kernels. Every partial is rewritten by each call before it is read, so the
// array needs no clearing; calls that overlap on one GPU race on it.
#include <mutex>

#include "lbe_internal.h"

namespace lbe {
namespace {

constexpr int kNB = 256;  // partial blocks per system (256 threads each, grid-stride over the nodes)
constexpr size_t kScratchDoubles = (size_t)LB_NOALLOC_MAX_SYSTEMS * kNB * 8;

__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on GPU dev (taken once, with dev current).
hipError_t scratch_of(int dev, double** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        g_scratch[dev] = (double*)p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

// Partial sums of block b (of kNB) of system s over its nodes n = b * 256 +
// t, b * 256 + t + kNB * 256, ...: masses, momentum, fluid count (sums) and
// the health flag (max), into part8[0..7]. Populations copy c, owner copy o.
template <class P>
__device__ void stats_partial(const SysDev& d, int c, int o, int b, double* __restrict__ part8) {
    using S = typename P::S;
    const Box& bx = d.box;
    const int64_t N = bx.N;
    const S* f = (const S*)d.f[c];
    const uint32_t* owner = d.owner[o];
    const uint32_t* bmask = d.bmask[c];
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t n = (int64_t)b * 256 + threadIdx.x; n < N; n += (int64_t)kNB * 256) {
        if (owner[n] != OWN_FLUID) continue;
        acc[5] += 1.0;
        const uint32_t bm = bmask[n];
        const uint32_t pl = (uint32_t)bx.nx * (uint32_t)bx.ny;
        const int z = (int)((uint32_t)n / pl);
        const uint32_t rem = (uint32_t)n - (uint32_t)z * pl;
        const int y = (int)(rem / (uint32_t)bx.nx), x = (int)(rem - (uint32_t)y * (uint32_t)bx.nx);
#pragma unroll
        for (int cc = 0; cc < 2; cc++) {
            double r = 0.0;
#pragma unroll
            for (int i = 0; i < Q; i++) {
                // population i sits in plane ibar at n - c_i when bit i of the bounce mask is set
                const bool up = (bm >> i) & 1u;
                const int64_t m = up ? (int64_t)upstream(bx.nx, bx.ny, bx.nz, x, y, z, i) : n;
                const double v = pop64<P>(f[(size_t)(cc * Q + (up ? opp(i) : i)) * N + m], wq(i) * bx.rref[cc]);
                r += v;
                acc[2] += v * cx(i);
                acc[3] += v * cy(i);
                acc[4] += v * cz(i);
            }
            acc[cc] += r;
            if (!(r >= 0.0)) acc[6] = 1.0;
        }
    }
    __shared__ double sh[7][256];
#pragma unroll
    for (int k = 0; k < 7; k++) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int k = 0; k < 6; k++) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
            sh[6][threadIdx.x] = fmax(sh[6][threadIdx.x], sh[6][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 7) part8[threadIdx.x] = sh[threadIdx.x][0];
}

// Batch: block (b, s) of system s; lone handle: the descriptor by value.
template <class P>
__global__ __launch_bounds__(256) void k_stats_nb_batch(const SysDev* __restrict__ sd, int c, double* __restrict__ sc) {
    const int s = blockIdx.y, b = blockIdx.x;
    stats_partial<P>(sd[s], c, c, b, sc + ((size_t)s * kNB + b) * 8);
}
template <class P>
__global__ __launch_bounds__(256) void k_stats_nb_one(SysDev d, int c, int o, double* __restrict__ sc) {
    stats_partial<P>(d, c, o, blockIdx.x, sc + (size_t)blockIdx.x * 8);
}

// Totals of system s in the order lb_stats forms them: partials in block
// order; mass removed = placement removal + sum over particles, in index order,
// of (killed + last step's killed) - (filled + last step's filled).
__device__ void stats_final(const SysDev& d, const double* __restrict__ sc, double* __restrict__ out) {
    double t[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int b = 0; b < kNB; b++) {
        for (int k = 0; k < 6; k++) t[k] += sc[(size_t)b * 8 + k];
        t[6] = fmax(t[6], sc[(size_t)b * 8 + 6]);
    }
    double removed = d.counters[0];
    for (int p = 0; p < d.np; p++)
        removed += (d.part[KMASS * d.cap + p] + d.kpart[(size_t)8 * p + 6]) -
                   (d.part[FMASS * d.cap + p] + d.kpart[(size_t)8 * p + 7]);
    out[0] = t[0];
    out[1] = t[1];
    out[2] = t[2];
    out[3] = t[3];
    out[4] = t[4];
    out[5] = removed;
    out[6] = t[5];
    out[7] = t[6];
}
__global__ void k_stats_final_batch(const SysDev* __restrict__ sd, int nsys, const double* __restrict__ sc,
                                    double* __restrict__ out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nsys) stats_final(sd[s], sc + (size_t)s * kNB * 8, out + (size_t)s * 8);
}
__global__ void k_stats_final_one(SysDev d, const double* __restrict__ sc, double* __restrict__ out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) stats_final(d, sc, out);
}

#define LBE_NA_DISPATCH(prec, CALL)                          \
    switch (prec) {                                          \
        case LB_FP64: { using P = PolF64; CALL; } break;     \
        case LB_FP32: { using P = PolF32; CALL; } break;     \
        case LB_FP16_DEV: { using P = PolF16; CALL; } break; \
        default: { using P = PolBF16; CALL; } break;         \
    }

}  // namespace
}  // namespace lbe

using namespace lbe;

extern "C" int lb_stats_noalloc(lb_handle* h, double* dev_out) {
    if (!h || !dev_out) return LB_EINVAL;
    if (h->parent) return fail(h, LB_ESTATE, "call lb_stats_noalloc on the batch handle (it covers every system)");
    if (h->device < 0 || h->device >= kMaxDevices) return fail(h, LB_EINVAL, "device index out of range");
    double* sc = nullptr;
    LBE_HIP_OR_FAIL(h, scratch_of(h->device, &sc));
    if (h->batch) {
        const int n = lb_batch_size(h);
        if (n > LB_NOALLOC_MAX_SYSTEMS)
            return fail(h, LB_EINVAL,
                        "batch of " + std::to_string(n) + " systems exceeds the allocation-free scratch (" +
                            std::to_string(LB_NOALLOC_MAX_SYSTEMS) + " systems)");
        // no table upload here (it would synchronise the stream): a batch
        // changed since its last step is refused
        const SysDev* d_sys = nullptr;
        int nsys = 0, parity = 0;
        const int rc = batch_sys(h, &d_sys, &nsys, &parity, false);
        if (rc != LB_OK) return rc;
        LBE_NA_DISPATCH(h->prm.precision, hipLaunchKernelGGL(k_stats_nb_batch<P>, dim3(kNB, nsys), dim3(256), 0,
                                                              h->stream, d_sys, parity, sc));
        LBE_HIP_OR_FAIL(h, hipGetLastError());
        hipLaunchKernelGGL(k_stats_final_batch, dim3((nsys + 63) / 64), dim3(64), 0, h->stream, d_sys, nsys, sc,
                           dev_out);
        LBE_HIP_OR_FAIL(h, hipGetLastError());
        return LB_OK;
    }
    if (!h->inited) return fail(h, LB_ESTATE, "fields not initialised");
    const SysDev d = sys_dev(h);
    LBE_NA_DISPATCH(h->prm.precision, hipLaunchKernelGGL(k_stats_nb_one<P>, dim3(kNB), dim3(256), 0, h->stream, d,
                                                          h->cur, h->ocur, sc));
    LBE_HIP_OR_FAIL(h, hipGetLastError());
    hipLaunchKernelGGL(k_stats_final_one, dim3(1), dim3(64), 0, h->stream, d, sc, dev_out);
    LBE_HIP_OR_FAIL(h, hipGetLastError());
    return LB_OK;
}
