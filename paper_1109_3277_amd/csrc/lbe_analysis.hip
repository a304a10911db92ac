// Lateral domain size of the order parameter phi~ = rho_A - rho_B (Sec. 4,
// Eq. (12)): L_i = 2 pi / sqrt(<k_i^2>), <k_i^2> = sum_k k_i^2 S(k) / sum_k S(k),
// S(k) = |phi'_k|^2 / N with phi' = phi~ - <phi~>, L = (L_x + L_y + L_z) / 3.
//
// The 3-D transform is never formed. For a fixed k_i, Parseval's theorem over
// the other two axes turns sum over those axes of |phi'_k|^2 into (N / n_i)
// times the sum, over the lines along axis i, of |A(k_i)|^2, A the 1-D
// transform of a line; and sum_k |phi'_k|^2 = N sum_n phi'(n)^2. Hence
//   <k_i^2> = sum_lines sum_{k_i} k_i^2 |A(k_i)|^2 / (n_i sum_n phi'(n)^2),
// three passes of 1-D transforms, each reading the staged field once.
//
// Passes (all on the handle's stream, all sums in a fixed order):
//  1. k_order_param: phi~ per node from the populations, read through the
//     bounce masks (0 on particle and wall nodes, which hold no fluid), into
//     the staging plane (the idle population copy), with block partials of
//     sum phi~.
//  2. k_ds_mean: <phi~>.
//  3. k_line_moments<axis>: groups of lines along the axis; two real lines
//     are transformed together as one complex line z = a + i b. For weights
//     w_n even in the wave number, sum_n w_n |Z_n|^2 = sum_n w_n (|A_n|^2 +
//     |B_n|^2), so a pair needs no unpacking. Power-of-two lengths run an
//     in-place radix-2 FFT in LDS (bit-reversed load); other lengths a direct
//     DFT from an LDS twiddle table. The x pass also sums phi'^2.
//  4. k_ds_final: <k_i^2>, L_i and L.
#include <math.h>

#include <algorithm>

#include "lbe_internal.h"

namespace lbe {
namespace {

constexpr int kLineComplex = 2048;  // complex values of a group's lines in LDS (32 KB)
constexpr int kMaxPairs = 8;        // line pairs per group at most
constexpr int kDsThreads = 256;

// Slots of the per-block partials (red[b * 8 + slot]).
enum { DS_SUM = 0, DS_SQ = 1, DS_MX = 2 };

template <class P>
__global__ __launch_bounds__(kDsThreads) void k_order_param(Box bx, const typename P::S* __restrict__ f,
                                                            const uint32_t* __restrict__ owner,
                                                            const uint32_t* __restrict__ bmask,
                                                            double* __restrict__ phi, double* __restrict__ red) {
    const int64_t N = bx.N;
    double acc[1] = {0.0};
    for (int64_t n = (int64_t)blockIdx.x * kDsThreads + threadIdx.x; n < N; n += (int64_t)gridDim.x * kDsThreads) {
        double v = 0.0;
        if (owner[n] == OWN_FLUID) {
            const uint32_t bm = bmask[n];
            int x, y, z;
            node_xyz(bx, (uint32_t)n, x, y, z);
            double r[2] = {0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 2; c++) {
#pragma unroll
                for (int i = 0; i < Q; i++) {
                    int pi;
                    uint32_t m;
                    pop_src(bx, (uint32_t)n, x, y, z, bm, i, pi, m);
                    r[c] += pop64<P>(f[(size_t)(c * Q + pi) * N + m], wq(i) * bx.rref[c]);
                }
            }
            v = r[0] - r[1];
        }
        phi[n] = v;
        acc[0] += v;
    }
    double tot[1];
    block_sum<1>(acc, tot);
    if (threadIdx.x == 0) red[(size_t)blockIdx.x * 8 + DS_SUM] = tot[0];
}

// Ordered sums of the block partials by one block: thread t adds partials
// t, t + 256, ... in turn, then the fixed tree of block_sum.
template <int K>
__device__ void partial_sums(const double* __restrict__ red, int nblocks, const int (&slot)[K], double (&tot)[K]) {
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; k++) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kDsThreads)
#pragma unroll
        for (int k = 0; k < K; k++) acc[k] += red[(size_t)b * 8 + slot[k]];
    block_sum<K>(acc, tot);
}

__global__ __launch_bounds__(kDsThreads) void k_ds_mean(double* __restrict__ red, int nblocks, double N) {
    const int slot[1] = {DS_SUM};
    double tot[1];
    partial_sums<1>(red, nblocks, slot, tot);
    if (threadIdx.x == 0) red[(size_t)nblocks * 8] = tot[0] / N;
}

// Lines along axis AX (0: x, 1: y, 2: z) of length La, in groups of 2 * np
// lines: consecutive rows for AX = 0, consecutive x at one (y or z) for the
// others. Every block walks groups blockIdx.x, blockIdx.x + gridDim.x, ... in
// order and writes one partial.
template <int AX>
__global__ __launch_bounds__(kDsThreads) void k_line_moments(Box bx, const double* __restrict__ phi,
                                                             const double* __restrict__ mean_of_phi,
                                                             double* __restrict__ red, int np, int fft_bits) {
    extern __shared__ double2 lds[];
    const int nx = bx.nx, ny = bx.ny, nz = bx.nz;
    const int La = AX == 0 ? nx : (AX == 1 ? ny : nz);
    const int G = 2 * np;
    const bool fft = fft_bits >= 0;
    const int ntw = fft ? La / 2 : La;
    double2* data = lds;                      // np lines of La complex values
    double2* tw = lds + (size_t)np * La;      // exp(-2 pi i m / La)
    double* datad = (double*)data;
    const double mean = *mean_of_phi;
    for (int m = threadIdx.x; m < ntw; m += kDsThreads) {
        double s, c;
        sincospi(-2.0 * (double)m / (double)La, &s, &c);
        tw[m] = make_double2(c, s);
    }
    // lines and groups
    const int64_t nlines = AX == 0 ? (int64_t)ny * nz : (AX == 1 ? (int64_t)nx * nz : (int64_t)nx * ny);
    const int gx = (nx + G - 1) / G;  // groups across x (AX = 1, 2)
    const int64_t ngroups = AX == 0 ? (nlines + G - 1) / G : (int64_t)gx * (AX == 1 ? nz : ny);
    double acc[2] = {0.0, 0.0};  // sum w |Z|^2, sum phi'^2 (x pass)
    for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        __syncthreads();  // the previous group's reads of LDS are done (and the twiddles are written)
        const int total = G * La;
        for (int e = threadIdx.x; e < total; e += kDsThreads) {
            int g, j;
            bool ok;
            size_t node;
            if (AX == 0) {
                g = e / La;
                j = e - g * La;
                const int64_t r = grp * G + g;
                ok = r < nlines;
                node = (size_t)r * nx + j;
            } else {
                g = e % G;
                j = e / G;
                const int64_t q = grp / gx;  // z (AX = 1) or y (AX = 2)
                const int x = (int)(grp - q * gx) * G + g;
                ok = x < nx;
                node = AX == 1 ? (size_t)x + (size_t)nx * ((size_t)j + (size_t)ny * q)
                               : (size_t)x + (size_t)nx * ((size_t)q + (size_t)ny * j);
            }
            double v = 0.0;
            if (ok) {
                v = phi[node] - mean;
                if (AX == 0) acc[1] += v * v;
            }
            const int jj = fft ? (int)(__brev((unsigned)j) >> (32 - fft_bits)) : j;
            datad[2 * ((size_t)(g >> 1) * La + jj) + (g & 1)] = v;
        }
        __syncthreads();
        if (fft) {
            const int halfL = La >> 1;
            for (int s = 0, half = 1; half < La; s++, half <<= 1) {
                const int tstride = halfL >> s;  // La / (2 half)
                for (int q = threadIdx.x; q < np * halfL; q += kDsThreads) {
                    const int p = q / halfL;
                    const int r = q - p * halfL;
                    const int pos = r & (half - 1);
                    const int i0 = p * La + ((r >> s) << (s + 1)) + pos;
                    const int i1 = i0 + half;
                    const double2 w = tw[pos * tstride];
                    const double2 b = data[i1];
                    const double2 a = data[i0];
                    const double vr = b.x * w.x - b.y * w.y;
                    const double vi = b.x * w.y + b.y * w.x;
                    data[i0] = make_double2(a.x + vr, a.y + vi);
                    data[i1] = make_double2(a.x - vr, a.y - vi);
                }
                __syncthreads();
            }
            for (int e = threadIdx.x; e < np * La; e += kDsThreads) {
                const int n = e % La;
                const int ns = n <= La / 2 ? n : n - La;
                const double k = 2.0 * M_PI * (double)ns / (double)La;
                const double2 z = data[e];
                acc[0] += k * k * (z.x * z.x + z.y * z.y);
            }
        } else {
            for (int e = threadIdx.x; e < np * La; e += kDsThreads) {
                const int p = e / La;
                const int n = e - p * La;
                const double2* zl = data + (size_t)p * La;
                double zr = 0.0, zi = 0.0;
                int idx = 0;  // (n * j) mod La
                for (int j = 0; j < La; j++) {
                    const double2 a = zl[j];
                    const double2 w = tw[idx];
                    zr += a.x * w.x - a.y * w.y;
                    zi += a.x * w.y + a.y * w.x;
                    idx += n;
                    if (idx >= La) idx -= La;
                }
                const int ns = n <= La / 2 ? n : n - La;
                const double k = 2.0 * M_PI * (double)ns / (double)La;
                acc[0] += k * k * (zr * zr + zi * zi);
            }
        }
    }
    double tot[2];
    block_sum<2>(acc, tot);
    if (threadIdx.x == 0) {
        red[(size_t)blockIdx.x * 8 + DS_MX + AX] = tot[0];
        if (AX == 0) red[(size_t)blockIdx.x * 8 + DS_SQ] = tot[1];
    }
}

// out: L_x, L_y, L_z, L, <k_x^2>, <k_y^2>, <k_z^2>, sum_k S(k) (= sum phi'^2).
__global__ __launch_bounds__(kDsThreads) void k_ds_final(Box bx, double* __restrict__ red, int nblocks) {
    const int slot[4] = {DS_SQ, DS_MX, DS_MX + 1, DS_MX + 2};
    double tot[4];
    partial_sums<4>(red, nblocks, slot, tot);
    if (threadIdx.x != 0) return;
    const double sq = tot[0], m[3] = {tot[1], tot[2], tot[3]};
    const int n[3] = {bx.nx, bx.ny, bx.nz};
    double* out = red + (size_t)nblocks * 8;
    double Ls = 0.0;
    for (int d = 0; d < 3; d++) {
        const double k2 = m[d] / ((double)n[d] * sq);
        const double L = sq > 0.0 ? (m[d] > 0.0 ? 2.0 * M_PI / sqrt(k2) : INFINITY) : NAN;
        out[d] = L;
        out[4 + d] = sq > 0.0 ? k2 : NAN;
        Ls += L;
    }
    out[3] = Ls / 3.0;
    out[7] = sq;
}

#define LBE_AN_DISPATCH(prec, CALL)                          \
    switch (prec) {                                          \
        case LB_FP64: { using P = PolF64; CALL; } break;     \
        case LB_FP32: { using P = PolF32; CALL; } break;     \
        case LB_FP16_DEV: { using P = PolF16; CALL; } break; \
        default: { using P = PolBF16; CALL; } break;         \
    }

// Group shape of the lines along an axis of length La: line pairs per group
// and log2(La) for a power of two (-1: direct DFT).
void line_shape(int La, int* np, int* bits) {
    *np = std::max(1, std::min(kMaxPairs, kLineComplex / La));
    *bits = -1;
    if ((La & (La - 1)) == 0 && La >= 2) {
        int b = 0;
        while ((1 << b) < La) b++;
        *bits = b;
    }
}

template <int AX>
hipError_t launch_lines(lb_handle* h, const double* phi) {
    const int La = AX == 0 ? h->box.nx : (AX == 1 ? h->box.ny : h->box.nz);
    int np, bits;
    line_shape(La, &np, &bits);
    const int ntw = bits >= 0 ? La / 2 : La;
    const size_t lds = ((size_t)np * La + (size_t)ntw) * sizeof(double2);
    hipLaunchKernelGGL(k_line_moments<AX>, dim3(kRedBlocks), dim3(kDsThreads), lds, h->stream, h->box, phi,
                       h->b.red + (size_t)kRedBlocks * 8, h->b.red, np, bits);
    return hipGetLastError();
}

}  // namespace
}  // namespace lbe

using namespace lbe;

extern "C" int lb_domain_size(lb_handle* h, double out[8]) {
    if (!h || !out) return LB_EINVAL;
    if (h->batch) return fail(h, LB_ESTATE, "per-system call on a batch handle: use lb_batch_system");
    if (!h->inited) return fail(h, LB_ESTATE, "fields not initialised");
    const int L3[3] = {h->box.nx, h->box.ny, h->box.nz};
    for (int d = 0; d < 3; d++)
        if (L3[d] > LB_DOMAIN_MAX_LINE)
            return fail(h, LB_EINVAL, "box side " + std::to_string(L3[d]) + " exceeds the domain-size limit of " +
                                          std::to_string(LB_DOMAIN_MAX_LINE));
    // phi~ is staged in the idle population copy (rewritten by the next step's
    // streaming before anything reads it)
    double* phi = (double*)h->b.f[1 - h->cur];
    LBE_AN_DISPATCH(h->prm.precision,
                    hipLaunchKernelGGL(k_order_param<P>, dim3(kRedBlocks), dim3(kDsThreads), 0, h->stream, h->box,
                                       (const typename P::S*)h->b.f[h->cur], h->b.owner[h->ocur], h->b.bmask[h->cur],
                                       phi, h->b.red));
    LBE_HIP_OR_FAIL(h, hipGetLastError());
    hipLaunchKernelGGL(k_ds_mean, dim3(1), dim3(kDsThreads), 0, h->stream, h->b.red, kRedBlocks, (double)h->box.N);
    LBE_HIP_OR_FAIL(h, hipGetLastError());
    LBE_HIP_OR_FAIL(h, launch_lines<0>(h, phi));
    LBE_HIP_OR_FAIL(h, launch_lines<1>(h, phi));
    LBE_HIP_OR_FAIL(h, launch_lines<2>(h, phi));
    hipLaunchKernelGGL(k_ds_final, dim3(1), dim3(kDsThreads), 0, h->stream, h->box, h->b.red, kRedBlocks);
    LBE_HIP_OR_FAIL(h, hipGetLastError());
    LBE_HIP_OR_FAIL(h, hipMemcpyAsync(out, h->b.red + (size_t)kRedBlocks * 8, 8 * sizeof(double),
                                      hipMemcpyDeviceToHost, h->stream));
    LBE_HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    return LB_OK;
}
