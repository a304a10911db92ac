// Fluid kernels of liblbe (gfx950): densities, shell fill, the fused
// force + collision + streaming + moving bounce-back step, initialisation,
// field readout and deterministic FP64 reductions.
//
// Layout in HBM: populations f[c][i][n] (structure of arrays, x fastest, one
// plane of N values per (component, velocity)), two copies (current / next);
// effective masses Psi[c][n]; owner map uint32 per node. One thread per node, tiles
// of 64x4 (or 32x8) nodes of one xy-plane per 256-thread block, tiles of
// neighbouring z on the same XCD.
#include "lbe_internal.h"

namespace lbe {

// Workgroups are dispatched round-robin over the 8 XCDs. Remap the block index
// so each XCD walks a contiguous range of tiles (whole z-slabs): the rows a
// tile reads from its y / z neighbours then sit in the same L2.
__device__ inline int xcd_remap(int b, int nb) {
    if ((nb & 7) != 0) return b;
    int per = nb >> 3;
    return (b & 7) * per + (b >> 3);
}

template <class R>
__device__ inline R feq_i(int i, R rho, R ux, R uy, R uz, R uu) {
    R cu = R(cx(i)) * ux + R(cy(i)) * uy + R(cz(i)) * uz;
    return R(wq(i)) * rho * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
}

// Wave64 reduction of per-lane particle force / torque contributions keyed by
// particle index, then one set of FP64 atomics per particle touched by the
// wave. Every lane of the wave must call this.
__device__ inline void wave_flush(int pid, const double* acc, double* part, int cap) {
    const int lane = __lane_id();
    unsigned long long pend = __ballot(pid >= 0);
    while (pend) {
        const int leader = __ffsll((long long)pend) - 1;
        const int p = __shfl(pid, leader, 64);
        const bool mine = (pid == p);
        double v[6];
#pragma unroll
        for (int k = 0; k < 6; k++) v[k] = mine ? acc[k] : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
            for (int k = 0; k < 6; k++) v[k] += __shfl_xor(v[k], off, 64);
        }
        if (lane == leader) {
            unsafeAtomicAdd(part + FX * cap + p, v[0]);
            unsafeAtomicAdd(part + FY * cap + p, v[1]);
            unsafeAtomicAdd(part + FZ * cap + p, v[2]);
            unsafeAtomicAdd(part + TX * cap + p, v[3]);
            unsafeAtomicAdd(part + TY * cap + p, v[4]);
            unsafeAtomicAdd(part + TZ * cap + p, v[5]);
        }
        if (mine) pid = -1;
        pend = __ballot(pid >= 0);
    }
}

__device__ inline void flush_direct(int pid, const double* acc, double* part, int cap) {
    unsafeAtomicAdd(part + FX * cap + pid, acc[0]);
    unsafeAtomicAdd(part + FY * cap + pid, acc[1]);
    unsafeAtomicAdd(part + FZ * cap + pid, acc[2]);
    unsafeAtomicAdd(part + TX * cap + pid, acc[3]);
    unsafeAtomicAdd(part + TY * cap + pid, acc[4]);
    unsafeAtomicAdd(part + TZ * cap + pid, acc[5]);
}

// ---------------------------------------------------------------- S1
// rho^c(n) = sum_i f_i^c(n) on fluid nodes, stored as the effective mass
// Psi^c(n) of Eq. (3), the only form the force stencil reads; health flag on
// NaN / rho < 0.
template <class P, bool SOLID>
__global__ __launch_bounds__(256) void k_density(Box bx, const typename P::S* __restrict__ f,
                                                 typename P::R* __restrict__ psi,
                                                 const uint32_t* __restrict__ owner, int* __restrict__ health) {
    using R = typename P::R;
    const int64_t N = bx.N;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    if (SOLID && owner[n] != OWN_FLUID) return;
    const R ref0 = R(bx.rref[0]), ref1 = R(bx.rref[1]);
    R r0 = R(0), r1 = R(0);
#pragma unroll
    for (int i = 0; i < Q; i++) {
        r0 += P::ld(f + (size_t)i * N + n, R(wq(i)) * ref0);
        r1 += P::ld(f + (size_t)(Q + i) * N + n, R(wq(i)) * ref1);
    }
    psi[n] = psi_of(r0, bx.psi_kind);
    psi[N + n] = psi_of(r1, bx.psi_kind);
    if (!(r0 >= R(0)) || !(r1 >= R(0))) atomicOr(health, 1);
}

// ---------------------------------------------------------------- S2
// Eq. (10): a solid node with fluid neighbours takes their mean density; the
// particle colour is added to A if positive, its magnitude to B if negative.
// Densities are recovered from the stored Psi (rho = -log(1 - Psi) for the
// exponential form) and the result is stored as Psi again.
template <class R>
__device__ inline R rho_of_psi(R p, int kind) {
    return kind == 0 ? p : -log1p(-p);
}

template <class R>
__global__ __launch_bounds__(256) void k_shell(Box bx, R* __restrict__ rho, const uint32_t* __restrict__ owner,
                                               const double* __restrict__ part, int cap) {
    const int64_t N = bx.N;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const uint32_t o = owner[n];
    if (o == OWN_FLUID) return;
    const int nx = bx.nx, ny = bx.ny, nz = bx.nz;
    const int x = (int)(n % nx);
    const int y = (int)((n / nx) % ny);
    const int z = (int)(n / ((int64_t)nx * ny));
    R s0 = R(0), s1 = R(0);
    int k = 0;
#pragma unroll
    for (int i = 1; i < Q; i++) {
        const int64_t m = wrapc(x + cx(i), nx) + (int64_t)nx * (wrapc(y + cy(i), ny) + (int64_t)ny * wrapc(z + cz(i), nz));
        if (owner[m] == OWN_FLUID) {
            s0 += rho_of_psi(rho[m], bx.psi_kind);
            s1 += rho_of_psi(rho[N + m], bx.psi_kind);
            k++;
        }
    }
    if (k == 0) {
        rho[n] = R(0);
        rho[N + n] = R(0);
        return;
    }
    R a = s0 / R(k), b = s1 / R(k);
    const double dr = (o < OWN_WALL) ? part[DRHO * cap + o] : 0.0;
    if (dr > 0.0) a += R(dr);
    else if (dr < 0.0) b += R(-dr);
    rho[n] = psi_of(a, bx.psi_kind);
    rho[N + n] = psi_of(b, bx.psi_kind);
}

// ---------------------------------------------------------------- S3-S6
// Per fluid node: Shan-Chen force (Eq. (3)) from neighbour Psi, BGK collision
// (Eq. (2)) with the common-velocity shift u^eq_c = u' + tau F^c/rho^c, then
// push streaming (Eq. (1)); links into solid nodes bounce back with
// C = 6 w_i rho^c (u_b . c_ibar) (Eq. (4)) and add (2 f*_i + C) c_i and its
// torque about the particle centre to the particle (Eq. (5)).
template <class P, bool SOLID>
__global__ __launch_bounds__(256) void k_fused(Box bx, const typename P::S* __restrict__ fs,
                                               typename P::S* __restrict__ fd,
                                               const typename P::R* __restrict__ psi,
                                               const uint32_t* __restrict__ owner, double* __restrict__ part,
                                               int cap, int BX, int BY, int tiles_x, int tiles_y) {
    using R = typename P::R;
    const int nx = bx.nx, ny = bx.ny, nz = bx.nz;
    const int64_t N = bx.N;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int txy = tiles_x * tiles_y;
    const int z = tile / txy;
    const int rem = tile - z * txy;
    const int ty = rem / tiles_x;
    const int tx = rem - ty * tiles_x;
    const int lx = threadIdx.x % BX, ly = threadIdx.x / BX;
    const int x = tx * BX + lx, y = ty * BY + ly;

    int pid = -1;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};

    const bool active = (x < nx) && (y < ny);
    const int64_t n = active ? (x + (int64_t)nx * (y + (int64_t)ny * z)) : 0;
    const bool fluid = active && (!SOLID || owner[n] == OWN_FLUID);
    if (fluid) {
        // neighbour coordinates, indexed by velocity component 0, +1, -1
        const int xs[3] = {x, x + 1 == nx ? 0 : x + 1, x == 0 ? nx - 1 : x - 1};
        const int64_t ys[3] = {(int64_t)y * nx, (int64_t)(y + 1 == ny ? 0 : y + 1) * nx,
                               (int64_t)(y == 0 ? ny - 1 : y - 1) * nx};
        const int64_t pl = (int64_t)nx * ny;
        const int64_t zs[3] = {(int64_t)z * pl, (int64_t)(z + 1 == nz ? 0 : z + 1) * pl,
                               (int64_t)(z == 0 ? nz - 1 : z - 1) * pl};
#define LBE_SEL(c) ((c) == 0 ? 0 : ((c) > 0 ? 1 : 2))
#define LBE_NB(i) (xs[LBE_SEL(cx(i))] + ys[LBE_SEL(cy(i))] + zs[LBE_SEL(cz(i))])

        const R ref0 = R(bx.rref[0]), ref1 = R(bx.rref[1]);
        R f0[Q], f1[Q];
#pragma unroll
        for (int i = 0; i < Q; i++) {
            f0[i] = P::ld(fs + (size_t)i * N + n, R(wq(i)) * ref0);
            f1[i] = P::ld(fs + (size_t)(Q + i) * N + n, R(wq(i)) * ref1);
        }
        R r0 = R(0), r1 = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
        for (int i = 0; i < Q; i++) {
            r0 += f0[i];
            r1 += f1[i];
            const R s = f0[i] + f1[i];
            if (cx(i) > 0) jx += s;
            if (cx(i) < 0) jx -= s;
            if (cy(i) > 0) jy += s;
            if (cy(i) < 0) jy -= s;
            if (cz(i) > 0) jz += s;
            if (cz(i) < 0) jz -= s;
        }
        // neighbour sums S^c = sum_i Psi^c(n + c_i) c_i
        const int kind = bx.psi_kind;
        R s0x = R(0), s0y = R(0), s0z = R(0), s1x = R(0), s1y = R(0), s1z = R(0);
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const int64_t m = LBE_NB(i);
            const R p0 = psi[m];
            const R p1 = psi[N + m];
            if (cx(i) > 0) { s0x += p0; s1x += p1; }
            if (cx(i) < 0) { s0x -= p0; s1x -= p1; }
            if (cy(i) > 0) { s0y += p0; s1y += p1; }
            if (cy(i) < 0) { s0y -= p0; s1y -= p1; }
            if (cz(i) > 0) { s0z += p0; s1z += p1; }
            if (cz(i) < 0) { s0z -= p0; s1z -= p1; }
        }
        const R tau = R(bx.tau);
        const R rt = r0 + r1;
        const R ux = jx / rt, uy = jy / rt, uz = jz / rt;
        const R k0 = -R(bx.g) * psi_ratio(r0, kind);
        const R k1 = -R(bx.g) * psi_ratio(r1, kind);
        const R ax = R(bx.ax), ay = R(bx.ay), az = R(bx.az);
        const R u0x = ux + tau * (k0 * s1x + ax), u0y = uy + tau * (k0 * s1y + ay), u0z = uz + tau * (k0 * s1z + az);
        const R u1x = ux + tau * (k1 * s0x + ax), u1y = uy + tau * (k1 * s0y + ay), u1z = uz + tau * (k1 * s0z + az);
        const R uu0 = u0x * u0x + u0y * u0y + u0z * u0z;
        const R uu1 = u1x * u1x + u1y * u1y + u1z * u1z;
        const R om = R(1) / tau;
#pragma unroll
        for (int i = 0; i < Q; i++) {
            f0[i] = f0[i] - om * (f0[i] - feq_i(i, r0, u0x, u0y, u0z, uu0));
            f1[i] = f1[i] - om * (f1[i] - feq_i(i, r1, u1x, u1y, u1z, uu1));
        }
        // streaming and bounce-back
        P::st(fd + n, f0[0], R(wq(0)) * ref0);
        P::st(fd + (size_t)Q * N + n, f1[0], R(wq(0)) * ref1);
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const int64_t m = LBE_NB(i);
            bool solid = false;
            uint32_t o = OWN_FLUID;
            if (SOLID) {
                o = owner[m];
                solid = (o != OWN_FLUID);
            }
            if (!solid) {
                P::st(fd + (size_t)i * N + m, f0[i], R(wq(i)) * ref0);
                P::st(fd + (size_t)(Q + i) * N + m, f1[i], R(wq(i)) * ref1);
            } else {
                double ubx = 0.0, uby = 0.0, ubz = 0.0, rx = 0.0, ry = 0.0, rz = 0.0;
                const bool isp = (o < OWN_WALL);
                if (isp) {
                    rx = minimg(((double)x + 0.5 * cx(i)) - part[PX * cap + o], nx);
                    ry = minimg(((double)y + 0.5 * cy(i)) - part[PY * cap + o], ny);
                    rz = minimg(((double)z + 0.5 * cz(i)) - part[PZ * cap + o], nz);
                    const double wx = part[WX * cap + o], wy = part[WY * cap + o], wz = part[WZ * cap + o];
                    ubx = part[VX * cap + o] + (wy * rz - wz * ry);
                    uby = part[VY * cap + o] + (wz * rx - wx * rz);
                    ubz = part[VZ * cap + o] + (wx * ry - wy * rx);
                }
                // u_b . c_ibar = -(u_b . c_i)
                const double cub = -(ubx * cx(i) + uby * cy(i) + ubz * cz(i));
                const R C0 = R(6.0 * wq(i) * cub) * r0;
                const R C1 = R(6.0 * wq(i) * cub) * r1;
                const int b = opp(i);
                P::st(fd + (size_t)b * N + n, f0[i] + C0, R(wq(b)) * ref0);
                P::st(fd + (size_t)(Q + b) * N + n, f1[i] + C1, R(wq(b)) * ref1);
                if (isp) {
                    const double mag = 2.0 * ((double)f0[i] + (double)f1[i]) + ((double)C0 + (double)C1);
                    const double dFx = mag * cx(i), dFy = mag * cy(i), dFz = mag * cz(i);
                    if (pid != (int)o) {
                        if (pid >= 0) flush_direct(pid, acc, part, cap);
                        pid = (int)o;
#pragma unroll
                        for (int k = 0; k < 6; k++) acc[k] = 0.0;
                    }
                    acc[0] += dFx;
                    acc[1] += dFy;
                    acc[2] += dFz;
                    acc[3] += ry * dFz - rz * dFy;
                    acc[4] += rz * dFx - rx * dFz;
                    acc[5] += rx * dFy - ry * dFx;
                }
            }
        }
#undef LBE_NB
#undef LBE_SEL
    }
    if (SOLID) wave_flush(pid, acc, part, cap);
}

// ---------------------------------------------------------------- init
template <class P>
__global__ __launch_bounds__(256) void k_init(Box bx, typename P::S* __restrict__ f, const double* __restrict__ ra,
                                              const double* __restrict__ rb, const double* __restrict__ u,
                                              const uint32_t* __restrict__ owner) {
    using R = typename P::R;
    const int64_t N = bx.N;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const bool fluid = owner[n] == OWN_FLUID;
    const double ux = u ? u[3 * n] : 0.0, uy = u ? u[3 * n + 1] : 0.0, uz = u ? u[3 * n + 2] : 0.0;
    const double uu = ux * ux + uy * uy + uz * uz;
    const double rr[2] = {ra[n], rb[n]};
#pragma unroll
    for (int c = 0; c < 2; c++) {
        const R ref = R(bx.rref[c]);
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const double v = fluid ? feq_i<double>(i, rr[c], ux, uy, uz, uu) : 0.0;
            P::st(f + (size_t)(c * Q + i) * N + n, R(v), R(wq(i)) * ref);
        }
    }
}

// ---------------------------------------------------------------- readout
template <class P>
__global__ __launch_bounds__(256) void k_fields(Box bx, const typename P::S* __restrict__ f,
                                                const uint32_t* __restrict__ owner, double* __restrict__ out) {
    using R = typename P::R;
    const int64_t N = bx.N;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double r[2] = {0.0, 0.0}, j[3] = {0.0, 0.0, 0.0};
    const bool fluid = owner[n] == OWN_FLUID;
    if (fluid) {
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const R ref = R(bx.rref[c]);
#pragma unroll
            for (int i = 0; i < Q; i++) {
                const double v = (double)P::ld(f + (size_t)(c * Q + i) * N + n, R(wq(i)) * ref);
                r[c] += v;
                j[0] += v * cx(i);
                j[1] += v * cy(i);
                j[2] += v * cz(i);
            }
        }
    }
    out[n] = r[0];
    out[N + n] = r[1];
    const double rt = r[0] + r[1];
#pragma unroll
    for (int k = 0; k < 3; k++) out[2 * N + 3 * n + k] = (fluid && rt != 0.0) ? j[k] / rt : 0.0;
}

// Deterministic reduction: fixed grid, per-block LDS tree, then one ordered pass.
template <class P>
__global__ __launch_bounds__(256) void k_stats_partial(Box bx, const typename P::S* __restrict__ f,
                                                       const uint32_t* __restrict__ owner, double* __restrict__ red) {
    using R = typename P::R;
    const int64_t N = bx.N;
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        if (owner[n] != OWN_FLUID) continue;
        acc[5] += 1.0;
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const R ref = R(bx.rref[c]);
            double r = 0.0;
#pragma unroll
            for (int i = 0; i < Q; i++) {
                const double v = (double)P::ld(f + (size_t)(c * Q + i) * N + n, R(wq(i)) * ref);
                r += v;
                acc[2] += v * cx(i);
                acc[3] += v * cy(i);
                acc[4] += v * cz(i);
            }
            acc[c] += r;
            if (!(r >= 0.0)) acc[6] = 1.0;
        }
    }
    __shared__ double sh[7][256];
#pragma unroll
    for (int k = 0; k < 7; k++) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < 6; k++) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
            sh[6][threadIdx.x] = fmax(sh[6][threadIdx.x], sh[6][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 7) red[blockIdx.x * 8 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_stats_final(double* __restrict__ red, int nblocks) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double t[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int b = 0; b < nblocks; b++) {
        for (int k = 0; k < 6; k++) t[k] += red[b * 8 + k];
        t[6] = fmax(t[6], red[b * 8 + 6]);
    }
    for (int k = 0; k < 7; k++) red[nblocks * 8 + k] = t[k];
}

// Remove the fluid on nodes covered at particle placement; removed mass is
// added to counters[0].
template <class P>
__global__ __launch_bounds__(256) void k_remove_covered(Box bx, typename P::S* __restrict__ f,
                                                        const uint32_t* __restrict__ owner,
                                                        double* __restrict__ counters) {
    using R = typename P::R;
    const int64_t N = bx.N;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N || owner[n] == OWN_FLUID) return;
    double m = 0.0;
#pragma unroll
    for (int c = 0; c < 2; c++) {
        const R ref = R(bx.rref[c]);
#pragma unroll
        for (int i = 0; i < Q; i++) {
            typename P::S* p = f + (size_t)(c * Q + i) * N + n;
            m += (double)P::ld(p, R(wq(i)) * ref);
            P::st(p, R(0), R(wq(i)) * ref);
        }
    }
    if (m != 0.0) unsafeAtomicAdd(counters, m);
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}
__global__ void k_fill_f64(double* __restrict__ p, double v, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

// ---------------------------------------------------------------- launchers

static inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

#define LBE_DISPATCH(prec, CALL)                  \
    switch (prec) {                               \
        case LB_FP64: { using P = PolF64; CALL; } break;  \
        case LB_FP32: { using P = PolF32; CALL; } break;  \
        case LB_FP16_DEV: { using P = PolF16; CALL; } break; \
        default: { using P = PolBF16; CALL; } break;      \
    }

hipError_t launch_init(lb_handle* h, const double* ra, const double* rb, const double* u) {
    LBE_DISPATCH(h->prm.precision,
                 hipLaunchKernelGGL(k_init<P>, dim3(nblk(h->box.N)), dim3(256), 0, h->stream, h->box,
                                    (typename P::S*)h->b.f[h->cur], ra, rb, u, h->b.owner[h->ocur]));
    return hipGetLastError();
}

hipError_t launch_density(lb_handle* h) {
    if (h->has_solid) {
        LBE_DISPATCH(h->prm.precision,
                     hipLaunchKernelGGL((k_density<P, true>), dim3(nblk(h->box.N)), dim3(256), 0, h->stream, h->box,
                                        (const typename P::S*)h->b.f[h->cur], (typename P::R*)h->b.rho,
                                        h->b.owner[h->ocur], h->b.health));
    } else {
        LBE_DISPATCH(h->prm.precision,
                     hipLaunchKernelGGL((k_density<P, false>), dim3(nblk(h->box.N)), dim3(256), 0, h->stream, h->box,
                                        (const typename P::S*)h->b.f[h->cur], (typename P::R*)h->b.rho,
                                        h->b.owner[h->ocur], h->b.health));
    }
    return hipGetLastError();
}

hipError_t launch_shell(lb_handle* h) {
    if (h->prm.precision == LB_FP64)
        hipLaunchKernelGGL(k_shell<double>, dim3(nblk(h->box.N)), dim3(256), 0, h->stream, h->box,
                           (double*)h->b.rho, h->b.owner[h->ocur], h->b.part, h->cap);
    else
        hipLaunchKernelGGL(k_shell<float>, dim3(nblk(h->box.N)), dim3(256), 0, h->stream, h->box,
                           (float*)h->b.rho, h->b.owner[h->ocur], h->b.part, h->cap);
    return hipGetLastError();
}

hipError_t launch_fused(lb_handle* h) {
    const int BX = h->box.nx >= 64 ? 64 : 32;
    const int BY = 256 / BX;
    const int tiles_x = (h->box.nx + BX - 1) / BX;
    const int tiles_y = (h->box.ny + BY - 1) / BY;
    const unsigned grid = (unsigned)(tiles_x * tiles_y * h->box.nz);
    const int o = h->cur, d = 1 - h->cur;
    if (h->has_solid) {
        LBE_DISPATCH(h->prm.precision,
                     hipLaunchKernelGGL((k_fused<P, true>), dim3(grid), dim3(256), 0, h->stream, h->box,
                                        (const typename P::S*)h->b.f[o], (typename P::S*)h->b.f[d],
                                        (const typename P::R*)h->b.rho, h->b.owner[h->ocur], h->b.part, h->cap, BX, BY,
                                        tiles_x, tiles_y));
    } else {
        LBE_DISPATCH(h->prm.precision,
                     hipLaunchKernelGGL((k_fused<P, false>), dim3(grid), dim3(256), 0, h->stream, h->box,
                                        (const typename P::S*)h->b.f[o], (typename P::S*)h->b.f[d],
                                        (const typename P::R*)h->b.rho, h->b.owner[h->ocur], h->b.part, h->cap, BX, BY,
                                        tiles_x, tiles_y));
    }
    return hipGetLastError();
}

hipError_t launch_fields(lb_handle* h, double* out) {
    LBE_DISPATCH(h->prm.precision,
                 hipLaunchKernelGGL(k_fields<P>, dim3(nblk(h->box.N)), dim3(256), 0, h->stream, h->box,
                                    (const typename P::S*)h->b.f[h->cur], h->b.owner[h->ocur], out));
    return hipGetLastError();
}

hipError_t launch_stats(lb_handle* h) {
    LBE_DISPATCH(h->prm.precision,
                 hipLaunchKernelGGL(k_stats_partial<P>, dim3(kRedBlocks), dim3(256), 0, h->stream, h->box,
                                    (const typename P::S*)h->b.f[h->cur], h->b.owner[h->ocur], h->b.red));
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, h->stream, h->b.red, kRedBlocks);
    return hipGetLastError();
}

hipError_t launch_remove_covered(lb_handle* h) {
    LBE_DISPATCH(h->prm.precision,
                 hipLaunchKernelGGL(k_remove_covered<P>, dim3(nblk(h->box.N)), dim3(256), 0, h->stream, h->box,
                                    (typename P::S*)h->b.f[h->cur], h->b.owner[h->ocur], h->b.counters));
    return hipGetLastError();
}

hipError_t launch_fill_u32(lb_handle* h, uint32_t* p, uint32_t v, int64_t n) {
    unsigned g = nblk(n);
    if (g > 65536) g = 65536;
    if (g == 0) g = 1;
    hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(256), 0, h->stream, p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_f64(lb_handle* h, double* p, double v, int64_t n) {
    unsigned g = nblk(n);
    if (g > 65536) g = 65536;
    if (g == 0) g = 1;
    hipLaunchKernelGGL(k_fill_f64, dim3(g), dim3(256), 0, h->stream, p, v, n);
    return hipGetLastError();
}

size_t elem_bytes(int precision) {
    switch (precision) {
        case LB_FP64: return 8;
        case LB_FP32: return 4;
        default: return 2;
    }
}
size_t rho_elem_bytes(int precision) { return precision == LB_FP64 ? 8 : 4; }

}  // namespace lbe
