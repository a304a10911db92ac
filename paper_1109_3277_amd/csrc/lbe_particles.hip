// Particle kernels of liblbe (gfx950): rigid-body update, rasterisation of the
// ellipsoids onto the owner map, and kill / fill of nodes that change side.
// Particle state is FP64 in every precision form.
#include "lbe_internal.h"

namespace lbe {

// Rotation matrix (body -> space) of a unit quaternion (w, x, y, z).
__device__ inline void qrot(double w, double x, double y, double z, double R[3][3]) {
#pragma clang fp contract(off)
    R[0][0] = 1.0 - 2.0 * (y * y + z * z);
    R[0][1] = 2.0 * (x * y - w * z);
    R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z);
    R[1][1] = 1.0 - 2.0 * (x * x + z * z);
    R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y);
    R[2][1] = 2.0 * (y * z + w * x);
    R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

// Closed inside test: body-frame offset b = R^T d of the minimum-image offset
// d, inside when (b_x^2 + b_y^2)/R_perp^2 + b_z^2/R_par^2 <= 1. Evaluated in a
// fixed order with FMA contraction off so the owner map is a function of the
// inputs alone.
__device__ inline bool inside_test(const double R[3][3], double dx, double dy, double dz, double rpar, double rperp) {
#pragma clang fp contract(off)
    const double bx = R[0][0] * dx + R[1][0] * dy + R[2][0] * dz;
    const double by = R[0][1] * dx + R[1][1] * dy + R[2][1] * dz;
    const double bz = R[0][2] * dx + R[1][2] * dy + R[2][2] * dz;
    const double q = (bx * bx + by * by) / (rperp * rperp) + (bz * bz) / (rpar * rpar);
    return q <= 1.0;
}

// Newton-Euler update, dt = 1: F = F_links + J, T = T_links + H; V += F/M,
// X = wrap(X + V); L += T; W = R I^-1 R^T L with the old orientation;
// q <- normalise(exp(W/2) (x) q). Link accumulators and impulses are cleared.
__global__ void k_bodies(Box bx, double* __restrict__ part, int cap, int np) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    double* P = part;
#define F_(k) P[(k) * cap + p]
    double F[3], T[3];
    F[0] = F_(FX) + F_(JX);
    F[1] = F_(FY) + F_(JY);
    F[2] = F_(FZ) + F_(JZ);
    T[0] = F_(TX) + F_(HX);
    T[1] = F_(TY) + F_(HY);
    T[2] = F_(TZ) + F_(HZ);
    F_(FX) = F_(FY) = F_(FZ) = 0.0;
    F_(TX) = F_(TY) = F_(TZ) = 0.0;
    F_(JX) = F_(JY) = F_(JZ) = 0.0;
    F_(HX) = F_(HY) = F_(HZ) = 0.0;
    F_(LFX) = F[0];
    F_(LFY) = F[1];
    F_(LFZ) = F[2];
    F_(LTX) = T[0];
    F_(LTY) = T[1];
    F_(LTZ) = T[2];
    const double M = F_(MASS);
    const int Ls[3] = {bx.nx, bx.ny, bx.nz};
    const int vk[3] = {VX, VY, VZ}, xk[3] = {PX, PY, PZ}, ok[3] = {OX, OY, OZ}, lk[3] = {LX, LY, LZ};
    for (int d = 0; d < 3; d++) {
        F_(ok[d]) = F_(xk[d]);
        const double v = F_(vk[d]) + F[d] / M;
        F_(vk[d]) = v;
        double xx = F_(xk[d]) + v;
        const double L = (double)Ls[d];
        if (xx >= L) xx -= L;
        if (xx < 0.0) xx += L;
        F_(xk[d]) = xx;
        F_(lk[d]) = F_(lk[d]) + T[d];
    }
    const double qw = F_(QW), qx = F_(QX), qy = F_(QY), qz = F_(QZ);
    double R[3][3];
    qrot(qw, qx, qy, qz, R);
    const double Lv[3] = {F_(LX), F_(LY), F_(LZ)};
    double Lb[3], Wb[3], W[3];
    for (int a = 0; a < 3; a++) Lb[a] = R[0][a] * Lv[0] + R[1][a] * Lv[1] + R[2][a] * Lv[2];
    Wb[0] = Lb[0] / F_(IPERP);
    Wb[1] = Lb[1] / F_(IPERP);
    Wb[2] = Lb[2] / F_(IPAR);
    for (int a = 0; a < 3; a++) W[a] = R[a][0] * Wb[0] + R[a][1] * Wb[1] + R[a][2] * Wb[2];
    F_(WX) = W[0];
    F_(WY) = W[1];
    F_(WZ) = W[2];
    const double th = sqrt(W[0] * W[0] + W[1] * W[1] + W[2] * W[2]);
    double dw, dx, dy, dz;
    if (th < 1e-12) {
        dw = 1.0;
        dx = 0.5 * W[0];
        dy = 0.5 * W[1];
        dz = 0.5 * W[2];
    } else {
        const double sh = sin(0.5 * th) / th;
        dw = cos(0.5 * th);
        dx = sh * W[0];
        dy = sh * W[1];
        dz = sh * W[2];
    }
    // Hamilton product dq (x) q
    double nw = dw * qw - dx * qx - dy * qy - dz * qz;
    double nxq = dw * qx + dx * qw + dy * qz - dz * qy;
    double nyq = dw * qy - dx * qz + dy * qw + dz * qx;
    double nzq = dw * qz + dx * qy - dy * qx + dz * qw;
    const double nn = sqrt(nw * nw + nxq * nxq + nyq * nyq + nzq * nzq);
    F_(QW) = nw / nn;
    F_(QX) = nxq / nn;
    F_(QY) = nyq / nn;
    F_(QZ) = nzq / nn;
#undef F_
}

// Rasterise particles [first, first + gridDim.x) into owner with atomicMin
// (smallest index wins). One block per particle, threads over its bounding box.
__global__ __launch_bounds__(256) void k_raster(Box bx, const double* __restrict__ part, int cap,
                                                uint32_t* __restrict__ owner, int first) {
    const int p = first + blockIdx.x;
    const double X[3] = {part[PX * cap + p], part[PY * cap + p], part[PZ * cap + p]};
    const double rpar = part[RPAR * cap + p], rperp = part[RPERP * cap + p];
    double R[3][3];
    qrot(part[QW * cap + p], part[QX * cap + p], part[QY * cap + p], part[QZ * cap + p], R);
    const double rb = rpar > rperp ? rpar : rperp;
    const int Ls[3] = {bx.nx, bx.ny, bx.nz};
    int lo[3], sz[3];
    for (int d = 0; d < 3; d++) {
        if (!isfinite(X[d]) || !(rb < 0.5 * Ls[d])) return;  // invalid state: touch nothing
        lo[d] = (int)ceil(X[d] - rb);
        sz[d] = (int)floor(X[d] + rb) - lo[d] + 1;
        sz[d] = max(0, min(sz[d], Ls[d]));
    }
    const int total = sz[0] * sz[1] * sz[2];
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        const int ix = t % sz[0];
        const int iy = (t / sz[0]) % sz[1];
        const int iz = t / (sz[0] * sz[1]);
        int c[3] = {lo[0] + ix, lo[1] + iy, lo[2] + iz};
        for (int d = 0; d < 3; d++) {
            c[d] %= Ls[d];
            if (c[d] < 0) c[d] += Ls[d];
        }
        const double dx = minimg((double)c[0] - X[0], Ls[0]);
        const double dy = minimg((double)c[1] - X[1], Ls[1]);
        const double dz = minimg((double)c[2] - X[2], Ls[2]);
        if (!inside_test(R, dx, dy, dz, rpar, rperp)) continue;
        const int64_t n = c[0] + (int64_t)Ls[0] * (c[1] + (int64_t)Ls[1] * c[2]);
        if (owner[n] == OWN_WALL) continue;
        atomicMin(owner + n, (uint32_t)p);
    }
}

template <class R>
__device__ inline R feq_p(int i, R rho, R ux, R uy, R uz) {
    const R uu = ux * ux + uy * uy + uz * uz;
    const R cu = R(cx(i)) * ux + R(cy(i)) * uy + R(cz(i)) * uz;
    return R(wq(i)) * rho * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
}

// Kill / fill over the union of the particle's bounding boxes before and after
// the move. Node n with old owner o and new owner o2:
//   o fluid, o2 == p : kill  -> J_p += sum_c j^c(n), H_p += r x that, f(n) = 0
//   o == p, o2 fluid : fill  -> rho_new^c = mean rho^c of neighbours fluid
//                      before and after (initial mean if none), u = V + W x r,
//                      f = f^eq(rho_new^c, u), J_p -= sum_c rho_new^c u, H_p -= r x that.
// Each changing node is handled by exactly one block (its owner).
template <class P>
__global__ __launch_bounds__(256) void k_killfill(Box bx, typename P::S* __restrict__ f,
                                                  const uint32_t* __restrict__ own_old,
                                                  const uint32_t* __restrict__ own_new, double* __restrict__ part,
                                                  int cap, double* __restrict__ counters) {
    using R = typename P::R;
    const int64_t N = bx.N;
    const int p = blockIdx.x;
    const int Ls[3] = {bx.nx, bx.ny, bx.nz};
    const double Xn[3] = {part[PX * cap + p], part[PY * cap + p], part[PZ * cap + p]};
    const double Xo[3] = {part[OX * cap + p], part[OY * cap + p], part[OZ * cap + p]};
    const double rpar = part[RPAR * cap + p], rperp = part[RPERP * cap + p];
    const double rb = rpar > rperp ? rpar : rperp;
    int lo[3], sz[3];
    for (int d = 0; d < 3; d++) {
        if (!isfinite(Xn[d]) || !isfinite(Xo[d]) || !(rb < 0.5 * Ls[d])) return;  // invalid state
        const double xn = Xo[d] + minimg(Xn[d] - Xo[d], Ls[d]);  // unwrapped new centre
        const int a = min((int)ceil(Xo[d] - rb), (int)ceil(xn - rb));
        const int b = max((int)floor(Xo[d] + rb), (int)floor(xn + rb));
        lo[d] = a;
        sz[d] = max(0, min(b - a + 1, Ls[d]));
    }
    const double V[3] = {part[VX * cap + p], part[VY * cap + p], part[VZ * cap + p]};
    const double W[3] = {part[WX * cap + p], part[WY * cap + p], part[WZ * cap + p]};
    const int total = sz[0] * sz[1] * sz[2];
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        int c[3] = {lo[0] + t % sz[0], lo[1] + (t / sz[0]) % sz[1], lo[2] + t / (sz[0] * sz[1])};
        for (int d = 0; d < 3; d++) {
            c[d] %= Ls[d];
            if (c[d] < 0) c[d] += Ls[d];
        }
        const int64_t n = c[0] + (int64_t)Ls[0] * (c[1] + (int64_t)Ls[1] * c[2]);
        const uint32_t o = own_old[n], o2 = own_new[n];
        const bool kill = (o == OWN_FLUID && o2 == (uint32_t)p);
        const bool fill = (o == (uint32_t)p && o2 == OWN_FLUID);
        if (!kill && !fill) continue;
        const double r[3] = {minimg((double)c[0] - Xn[0], Ls[0]), minimg((double)c[1] - Xn[1], Ls[1]),
                             minimg((double)c[2] - Xn[2], Ls[2])};
        if (kill) {
            double j[3] = {0.0, 0.0, 0.0}, m = 0.0;
            for (int cc = 0; cc < 2; cc++) {
                const R ref = R(bx.rref[cc]);
#pragma unroll
                for (int i = 0; i < Q; i++) {
                    typename P::S* ptr = f + (size_t)(cc * Q + i) * N + n;
                    const double v = (double)P::ld(ptr, R(wq(i)) * ref);
                    m += v;
                    j[0] += v * cx(i);
                    j[1] += v * cy(i);
                    j[2] += v * cz(i);
                    P::st(ptr, R(0), R(wq(i)) * ref);
                }
            }
            unsafeAtomicAdd(part + JX * cap + p, j[0]);
            unsafeAtomicAdd(part + JY * cap + p, j[1]);
            unsafeAtomicAdd(part + JZ * cap + p, j[2]);
            unsafeAtomicAdd(part + HX * cap + p, r[1] * j[2] - r[2] * j[1]);
            unsafeAtomicAdd(part + HY * cap + p, r[2] * j[0] - r[0] * j[2]);
            unsafeAtomicAdd(part + HZ * cap + p, r[0] * j[1] - r[1] * j[0]);
            unsafeAtomicAdd(counters + 0, m);
            unsafeAtomicAdd(counters + 1, m);
        } else {
            double rn[2] = {0.0, 0.0};
            int cnt = 0;
#pragma unroll
            for (int i = 1; i < Q; i++) {
                const int64_t m = wrapc(c[0] + cx(i), Ls[0]) +
                                  (int64_t)Ls[0] * (wrapc(c[1] + cy(i), Ls[1]) + (int64_t)Ls[1] * wrapc(c[2] + cz(i), Ls[2]));
                if (own_old[m] != OWN_FLUID || own_new[m] != OWN_FLUID) continue;
                for (int cc = 0; cc < 2; cc++) {
                    const R ref = R(bx.rref[cc]);
                    double s = 0.0;
                    for (int q = 0; q < Q; q++) s += (double)P::ld(f + (size_t)(cc * Q + q) * N + m, R(wq(q)) * ref);
                    rn[cc] += s;
                }
                cnt++;
            }
            for (int cc = 0; cc < 2; cc++) rn[cc] = cnt > 0 ? rn[cc] / (double)cnt : bx.rmean0[cc];
            const double ub[3] = {V[0] + (W[1] * r[2] - W[2] * r[1]), V[1] + (W[2] * r[0] - W[0] * r[2]),
                                  V[2] + (W[0] * r[1] - W[1] * r[0])};
            double jm[3] = {0.0, 0.0, 0.0};
            for (int cc = 0; cc < 2; cc++) {
                const R ref = R(bx.rref[cc]);
#pragma unroll
                for (int i = 0; i < Q; i++)
                    P::st(f + (size_t)(cc * Q + i) * N + n, R(feq_p<double>(i, rn[cc], ub[0], ub[1], ub[2])),
                          R(wq(i)) * ref);
                for (int d = 0; d < 3; d++) jm[d] += rn[cc] * ub[d];
            }
            unsafeAtomicAdd(part + JX * cap + p, -jm[0]);
            unsafeAtomicAdd(part + JY * cap + p, -jm[1]);
            unsafeAtomicAdd(part + JZ * cap + p, -jm[2]);
            unsafeAtomicAdd(part + HX * cap + p, -(r[1] * jm[2] - r[2] * jm[1]));
            unsafeAtomicAdd(part + HY * cap + p, -(r[2] * jm[0] - r[0] * jm[2]));
            unsafeAtomicAdd(part + HZ * cap + p, -(r[0] * jm[1] - r[1] * jm[0]));
            unsafeAtomicAdd(counters + 0, -(rn[0] + rn[1]));
            unsafeAtomicAdd(counters + 2, rn[0] + rn[1]);
        }
    }
}

hipError_t launch_bodies(lb_handle* h) {
    if (h->np <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bodies, dim3((h->np + 63) / 64), dim3(64), 0, h->stream, h->box, h->b.part, h->cap, h->np);
    return hipGetLastError();
}

hipError_t launch_clear_owner(lb_handle* h, uint32_t* owner) { return launch_fill_u32(h, owner, OWN_FLUID, h->box.N); }

hipError_t launch_raster(lb_handle* h, uint32_t* owner, int first, int count) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster, dim3(count), dim3(256), 0, h->stream, h->box, h->b.part, h->cap, owner, first);
    return hipGetLastError();
}

hipError_t launch_killfill(lb_handle* h) {
    if (h->np <= 0) return hipSuccess;
    uint32_t* oo = h->b.owner[h->ocur];
    uint32_t* on = h->b.owner[1 - h->ocur];
    void* fn = h->b.f[1 - h->cur];
    switch (h->prm.precision) {
        case LB_FP64:
            hipLaunchKernelGGL(k_killfill<PolF64>, dim3(h->np), dim3(256), 0, h->stream, h->box, (double*)fn, oo, on,
                               h->b.part, h->cap, h->b.counters);
            break;
        case LB_FP32:
            hipLaunchKernelGGL(k_killfill<PolF32>, dim3(h->np), dim3(256), 0, h->stream, h->box, (float*)fn, oo, on,
                               h->b.part, h->cap, h->b.counters);
            break;
        case LB_FP16_DEV:
            hipLaunchKernelGGL(k_killfill<PolF16>, dim3(h->np), dim3(256), 0, h->stream, h->box, (__half*)fn, oo, on,
                               h->b.part, h->cap, h->b.counters);
            break;
        default:
            hipLaunchKernelGGL(k_killfill<PolBF16>, dim3(h->np), dim3(256), 0, h->stream, h->box,
                               (__hip_bfloat16*)fn, oo, on, h->b.part, h->cap, h->b.counters);
            break;
    }
    return hipGetLastError();
}

}  // namespace lbe
