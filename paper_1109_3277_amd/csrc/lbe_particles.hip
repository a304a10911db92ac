// Particle kernels of liblbe (gfx950): shell fill, the bounce-back force and
// torque of each particle, rigid-body update, rasterisation of the ellipsoids onto
// the owner map, and kill / fill of nodes that change side.
//
// The per-node particle kernels run one block per particle that loops over the
// nodes of the particle's box (several nodes' loads in flight per thread).
// Forces, torques and kill/fill impulses are summed in fixed orders (per-block
// partial slots, added in slot order): particle state is reproducible bit for
// bit.
// Particle state is FP64 in every precision form.
#include <math.h>

#include <algorithm>

#include "lbe_internal.h"

namespace lbe {

#define LBE_PDISPATCH(prec, CALL)                            \
    switch (prec) {                                          \
        case LB_FP64: { using P = PolF64; CALL; } break;     \
        case LB_FP32: { using P = PolF32; CALL; } break;     \
        case LB_FP16_DEV: { using P = PolF16; CALL; } break; \
        default: { using P = PolBF16; CALL; } break;         \
    }

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

// Half extents of the axis-aligned box of an ellipsoid with semi-axes R_par
// (body axis) and R_perp, orientation R (body -> space), scaled by sc: along
// axis k, sc sqrt(R_perp^2 (1 - o_k^2) + R_par^2 o_k^2), o the body axis (the
// support of the ellipsoid in direction k), grown by a relative 1e-9 plus 1e-9
// nodes, far beyond the rounding of the inside tests, and capped at cap_r.
__device__ inline void ellipsoid_extent(const double R[3][3], double rpar, double rperp, double sc, double cap_r,
                                        double e[3]) {
    for (int d = 0; d < 3; d++) {
        const double o = R[d][2];
        const double e2 = rperp * rperp * fmax(0.0, 1.0 - o * o) + rpar * rpar * (o * o);
        e[d] = fmin(sc * sqrt(e2) * (1.0 + 1e-9) + 1e-9, cap_r);
    }
}

// Axis-aligned box of particle p's ellipsoid (extents above, capped at the
// bounding radius). It holds every node the inside test accepts, and for an
// elongated body it is much smaller than the bounding cube. False if the state
// is not usable.
__device__ inline bool ellipsoid_box(const Box& bx, const double* part, int cap, int p, int lo[3], int sz[3]) {
    const int Ls[3] = {bx.nx, bx.ny, bx.nz};
    const double X[3] = {part[PX * cap + p], part[PY * cap + p], part[PZ * cap + p]};
    const double rpar = part[RPAR * cap + p], rperp = part[RPERP * cap + p];
    const double rb = rpar > rperp ? rpar : rperp;
    double R[3][3], e[3];
    qrot(part[QW * cap + p], part[QX * cap + p], part[QY * cap + p], part[QZ * cap + p], R);
    ellipsoid_extent(R, rpar, rperp, 1.0, rb, e);
    for (int d = 0; d < 3; d++) {
        if (!isfinite(X[d]) || !(rb < 0.5 * Ls[d])) return false;
        lo[d] = (int)ceil(X[d] - e[d]);
        sz[d] = max(0, min((int)floor(X[d] + e[d]) - lo[d] + 1, Ls[d]));
    }
    return true;
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

// The same quadratic form with the reciprocal squared semi-axes ia2 =
// 1 / R_perp^2 and ic2 = 1 / R_par^2 (no divisions). It differs from the one
// inside_test compares with 1 by a few ulp.
__device__ inline double q_fast(const double R[3][3], double dx, double dy, double dz, double ia2, double ic2) {
#pragma clang fp contract(off)
    const double bx = R[0][0] * dx + R[1][0] * dy + R[2][0] * dz;
    const double by = R[0][1] * dx + R[1][1] * dy + R[2][1] * dz;
    const double bz = R[0][2] * dx + R[1][2] * dy + R[2][2] * dz;
    return (bx * bx + by * by) * ia2 + (bz * bz) * ic2;
}

__device__ inline int64_t node_index(const Box& bx, int x, int y, int z) {
    return x + (int64_t)bx.nx * (y + (int64_t)bx.ny * z);
}

// ---------------------------------------------------------------- raster
// Rasterise particle p into owner with atomicMin (the smallest index owns a
// node covered by several particles): one block loops over p's ellipsoid box.
__device__ inline void raster_body(const Box& bx, const double* __restrict__ part, int cap,
                                   uint32_t* __restrict__ owner, int p) {
    int lo[3], sz[3];
    if (!ellipsoid_box(bx, part, cap, p, lo, sz)) return;  // invalid state: touch nothing
    const double X[3] = {part[PX * cap + p], part[PY * cap + p], part[PZ * cap + p]};
    double R[3][3];
    qrot(part[QW * cap + p], part[QX * cap + p], part[QY * cap + p], part[QZ * cap + p], R);
    const double rpar = part[RPAR * cap + p], rperp = part[RPERP * cap + p];
    const double ia2 = 1.0 / (rperp * rperp), ic2 = 1.0 / (rpar * rpar);
    const int total = sz[0] * sz[1] * sz[2];
    const int Ls[3] = {bx.nx, bx.ny, bx.nz};
    BoxWalk w(lo, sz, Ls, threadIdx.x, kPB);
    for (int t = threadIdx.x; t < total; t += kPB, w.next()) {
        const int x = w.x(), y = w.y(), z = w.z();
        const double dx = minimg((double)x - X[0], bx.nx);
        const double dy = minimg((double)y - X[1], bx.ny);
        const double dz = minimg((double)z - X[2], bx.nz);
        // the division-free form decides unless it lies within 1e-9 of the
        // surface, where the exact test (the one the owner map is defined by)
        // does; the two differ by a few ulp
        const double q = q_fast(R, dx, dy, dz, ia2, ic2);
        if (q > 1.0 + 1e-9) continue;
        if (q >= 1.0 - 1e-9 && !inside_test(R, dx, dy, dz, rpar, rperp)) continue;
        const int64_t n = node_index(bx, x, y, z);
        if (bx.walls && owner[n] == OWN_WALL) continue;  // walls keep their code
        atomicMin(owner + n, (uint32_t)p);
    }
}
__global__ __launch_bounds__(kPB) void k_raster(Box bx, const double* __restrict__ part, int cap,
                                                uint32_t* __restrict__ owner, int first) {
    raster_body(bx, part, cap, owner, first + blockIdx.x);
}
// Batched: item = (system, particle), into the owner copy `o` of every system.
__global__ __launch_bounds__(kPB) void k_raster_batch(const SysDev* __restrict__ sd,
                                                      const WorkItem* __restrict__ items, int o) {
    const WorkItem w = items[blockIdx.x];
    const SysDev& d = sd[w.sys];
    raster_body(d.box, d.part, d.cap, d.owner[o], w.local);
}

// ---------------------------------------------------------------- S2
// Eq. (10): a node of particle p with fluid neighbours (over the 18 links)
// takes their mean density; the particle colour is added to A if positive,
// its magnitude to B if negative. Densities are recovered from the stored
// Psi and the result is stored as Psi.
// One block per particle; only nodes of p change. The block takes p's box in
// segments of kShellSeg nodes: it loads the owner codes of a whole segment
// (kShellPT per thread, all in flight), lists p's nodes in LDS, then gives
// each listed node to one thread for its 18 neighbour gathers. A node's
// result depends on its neighbours only, so the list order does not matter.
constexpr int kShellPT = 20;
constexpr int kShellSeg = kShellPT * kPB;
template <class R>
__device__ inline void shell_body(const Box& bx, R* __restrict__ psi, const R* __restrict__ rho,
                                  const uint32_t* __restrict__ owner, const double* __restrict__ part, int cap,
                                  int p) {
    const int nx = bx.nx, ny = bx.ny, nz = bx.nz;
    const int64_t N = bx.N;
    int lo[3] = {0, 0, 0}, sz[3] = {0, 0, 0};
    const int total = ellipsoid_box(bx, part, cap, p, lo, sz) ? sz[0] * sz[1] * sz[2] : 0;
    // densities of fluid nodes: the stored rho (Psi itself when Psi = rho)
    const R* dens = bx.psi_kind == 0 ? psi : rho;
    const double dr = part[DRHO * cap + p];
    const int Ls[3] = {nx, ny, nz};
    __shared__ uint32_t s_list[kShellSeg];
    __shared__ int s_cnt;
    for (int base = 0; base < total; base += kShellSeg) {
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        {
            BoxWalk w(lo, sz, Ls, base + (int)threadIdx.x, kPB);
            uint32_t ow[kShellPT];
#pragma unroll
            for (int k = 0; k < kShellPT; k++) {
                ow[k] = OWN_FLUID;
                if (base + (int)threadIdx.x + k * kPB < total) ow[k] = owner[node_index(bx, w.x(), w.y(), w.z())];
                w.next();
            }
#pragma unroll
            for (int k = 0; k < kShellPT; k++)
                if (ow[k] == (uint32_t)p) s_list[atomicAdd(&s_cnt, 1)] = (uint32_t)(base + (int)threadIdx.x + k * kPB);
        }
        __syncthreads();
        const int listed = s_cnt;
        for (int j = threadIdx.x; j < listed; j += kPB) {
            const BoxWalk w(lo, sz, Ls, (int)s_list[j], 1);
            const int x = w.x(), y = w.y(), z = w.z();
            const int64_t n = node_index(bx, x, y, z);
            // owner codes first; densities only of the fluid neighbours (the
            // gathers, not their latency, bound this loop)
            uint32_t on[Q];
            int64_t mm[Q];
            R d0[Q], d1[Q];
#pragma unroll
            for (int i = 1; i < Q; i++) {
                mm[i] = node_index(bx, wrapc(x + cx(i), nx), wrapc(y + cy(i), ny), wrapc(z + cz(i), nz));
                on[i] = owner[mm[i]];
            }
#pragma unroll
            for (int i = 1; i < Q; i++) {
                d0[i] = d1[i] = R(0);
                if (on[i] == OWN_FLUID) {
                    d0[i] = dens[mm[i]];
                    d1[i] = dens[N + mm[i]];
                }
            }
            R s0 = R(0), s1 = R(0);
            int k = 0;
#pragma unroll
            for (int i = 1; i < Q; i++) {
                if (on[i] != OWN_FLUID) continue;
                s0 += d0[i];
                s1 += d1[i];
                k++;
            }
            if (k == 0) {
                psi[n] = R(0);
                psi[N + n] = R(0);
            } else {
                R a = s0 / R(k), b = s1 / R(k);
                if (dr > 0.0) a += R(dr);
                else if (dr < 0.0) b += R(-dr);
                psi[n] = psi_kept(a, bx.psi_kind, R(bx.eref[0]));
                psi[N + n] = psi_kept(b, bx.psi_kind, R(bx.eref[1]));
            }
        }
        __syncthreads();  // the list is read before the next segment resets it
    }
}
template <class R>
__global__ __launch_bounds__(kPB) void k_shell(Box bx, R* __restrict__ psi, const R* __restrict__ rho,
                                               const uint32_t* __restrict__ owner, const double* __restrict__ part,
                                               int cap) {
    shell_body<R>(bx, psi, rho, owner, part, cap, blockIdx.x);
}
template <class R>
__global__ __launch_bounds__(kPB) void k_shell_batch(const SysDev* __restrict__ sd, const WorkItem* __restrict__ items,
                                                     int o) {
    const WorkItem w = items[blockIdx.x];
    const SysDev& d = sd[w.sys];
    shell_body<R>(d.box, (R*)d.psi, (const R*)d.rho, d.owner[o], d.part, d.cap, w.local);
}

// ---------------------------------------------------------------- S6 forces
// Bounce-back force and torque of particle p (Eq. (5)). The fused kernel left,
// for every fluid node n linked to p, the node's force F_n = sum over its
// links into p of (2 f*_i + C) c_i (both components) in p's record cell of n.
// The force is the sum of the F_n and the torque the sum of r_n x F_n. One
// block per particle walks the record cells that can hold a link: cell t of
// the walk goes to thread t mod kPB, each thread's cells in increasing order,
// then a fixed block sum, so the result is reproducible bit for bit. Records
// read are cleared for the next step. A linked fluid node lies within sqrt(2)
// of a node of p. In coordinates scaled by the semi-axes that is a step of at
// most sqrt(2) / min(R_par, R_perp), so the node lies inside p's ellipsoid
// scaled about its centre by 1 + 1.5 / min(R_par, R_perp): the walk covers the
// record cells inside that ellipsoid's axis-aligned box (on an axis where the
// record box spans the whole lattice, all of them), and loads only the cells
// inside the scaled ellipsoid itself; other cells are never written.
__device__ inline void linkforce_body(const Box& bx, double* __restrict__ rec, int rstride,
                                      double* __restrict__ part, int cap, int p) {
    const int Ls[3] = {bx.nx, bx.ny, bx.nz};
    const double X[3] = {part[PX * cap + p], part[PY * cap + p], part[PZ * cap + p]};
    int lo[3] = {0, 0, 0}, sz[3] = {0, 0, 0}, esz[3];
    const bool ok = particle_box(bx, part, cap, p, lo, sz);
    for (int d = 0; d < 3; d++) esz[d] = min(sz[d] + 2, Ls[d]);
    double Rm[3][3];
    qrot(part[QW * cap + p], part[QX * cap + p], part[QY * cap + p], part[QZ * cap + p], Rm);
    const double rpar = part[RPAR * cap + p], rperp = part[RPERP * cap + p];
    const double sc = 1.0 + 1.5 / (rpar < rperp ? rpar : rperp);
    const double ga = sc * rperp, gc = sc * rpar;
    // a filter only: linked nodes lie strictly inside the scaled ellipsoid,
    // by far more than rounding, so the division-free form serves
    const double ia2 = 1.0 / (ga * ga), ic2 = 1.0 / (gc * gc);
    // the walked box [slo, slo + ssz) inside the record box, whose cells are
    // numbered from its corner lo - 1 (the numbering the fused kernel writes)
    double es[3];
    ellipsoid_extent(Rm, rpar, rperp, sc, (double)(Ls[0] + Ls[1] + Ls[2]), es);
    int slo[3], ssz[3], off[3];
    for (int d = 0; d < 3; d++) {
        const int elo = lo[d] - 1;
        if (!ok || esz[d] >= Ls[d]) {
            slo[d] = elo;
            ssz[d] = esz[d];
        } else {
            const int a = max((int)ceil(X[d] - es[d]), elo);
            const int b = min((int)floor(X[d] + es[d]), elo + esz[d] - 1);
            slo[d] = a;
            ssz[d] = max(0, b - a + 1);
        }
        off[d] = slo[d] - elo;
    }
    const int cells = ok ? ssz[0] * ssz[1] * ssz[2] : 0;
    double* rp = rec + (size_t)p * rstride * kRec;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    constexpr int U = 4;  // cells per thread in flight
    BoxWalk w(slo, ssz, Ls, threadIdx.x, kPB);
    for (int base = 0; base < cells; base += U * kPB) {
        double F[U][3], r[U][3];
        int cell[U];
#pragma unroll
        for (int k = 0; k < U; k++, w.next()) {
            const int t = base + k * kPB + (int)threadIdx.x;
            F[k][0] = F[k][1] = F[k][2] = 0.0;
            r[k][0] = r[k][1] = r[k][2] = 0.0;
            cell[k] = ((off[2] + w.iz) * esz[1] + off[1] + w.iy) * esz[0] + off[0] + w.ix;
            if (t < cells) {
                r[k][0] = minimg((double)w.x() - X[0], Ls[0]);
                r[k][1] = minimg((double)w.y() - X[1], Ls[1]);
                r[k][2] = minimg((double)w.z() - X[2], Ls[2]);
                if (q_fast(Rm, r[k][0], r[k][1], r[k][2], ia2, ic2) <= 1.0) {
                    const int c = cell[k];
                    F[k][0] = rp[(size_t)c * kRec];
                    F[k][1] = rp[(size_t)c * kRec + 1];
                    F[k][2] = rp[(size_t)c * kRec + 2];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < U; k++) {
            if (F[k][0] == 0.0 && F[k][1] == 0.0 && F[k][2] == 0.0) continue;
            const int c = cell[k];
            rp[(size_t)c * kRec] = 0.0;
            rp[(size_t)c * kRec + 1] = 0.0;
            rp[(size_t)c * kRec + 2] = 0.0;
            const double rx = r[k][0], ry = r[k][1], rz = r[k][2];
            acc[0] += F[k][0];
            acc[1] += F[k][1];
            acc[2] += F[k][2];
            acc[3] += ry * F[k][2] - rz * F[k][1];
            acc[4] += rz * F[k][0] - rx * F[k][2];
            acc[5] += rx * F[k][1] - ry * F[k][0];
        }
    }
    double tot[6];
    block_sum<6>(acc, tot);
    if (threadIdx.x == 0) {
        const int fld[6] = {FX, FY, FZ, TX, TY, TZ};
        for (int k = 0; k < 6; k++) part[fld[k] * cap + p] = tot[k];
    }
}
__global__ __launch_bounds__(kPB, 4) void k_linkforce(Box bx, double* __restrict__ rec, int rstride,
                                                   double* __restrict__ part, int cap) {
    linkforce_body(bx, rec, rstride, part, cap, blockIdx.x);
}
// Batched: item = (system, particle).
__global__ __launch_bounds__(kPB, 4) void k_linkforce_batch(const SysDev* __restrict__ sd,
                                                         const WorkItem* __restrict__ items) {
    const WorkItem w = items[blockIdx.x];
    const SysDev& d = sd[w.sys];
    linkforce_body(d.box, d.rec, d.kext * d.kext * d.kext, d.part, d.cap, w.local);
}

// ---------------------------------------------------------------- S7
// Newton-Euler update, dt = 1: F = F_links + J + F_pairs, T = T_links + H +
// T_pairs (the pair terms are zero unless particle-particle interactions are
// on); V += F/M,
// X = wrap(X + V); L += T; W = R I^-1 R^T L with the old orientation;
// q <- normalise(exp(W/2) (x) q). F_links / T_links come from k_linkforce;
// J / H are the stored impulses plus the kill/fill slots. One wave per
// particle: lane l sums slots l, l + 64, ... in order, then a fixed shuffle
// tree; lane 0 updates the body.
__device__ inline void bodies_body(const Box& bx, double* __restrict__ part, int cap,
                                   const double* __restrict__ kpart, int nk, double* __restrict__ pfast, int p) {
    const int lane = threadIdx.x;
    double Jk[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = lane; s < nk; s += 64)
        for (int k = 0; k < 8; k++) Jk[k] += kpart[((size_t)p * nk + s) * 8 + k];
#pragma unroll
    for (int k = 0; k < 8; k++)
        for (int off = 32; off > 0; off >>= 1) Jk[k] += __shfl_down(Jk[k], off, 64);
    if (lane != 0) return;
    double* P = part;
#define F_(k) P[(k) * cap + p]
    F_(KMASS) += Jk[6];
    F_(FMASS) += Jk[7];
    const double Fl[6] = {F_(FX), F_(FY), F_(FZ), F_(TX), F_(TY), F_(TZ)};
    const double J[3] = {F_(JX) + Jk[0], F_(JY) + Jk[1], F_(JZ) + Jk[2]};
    const double H[3] = {F_(HX) + Jk[3], F_(HY) + Jk[4], F_(HZ) + Jk[5]};
    double F[3], T[3];
    for (int d = 0; d < 3; d++) {
        F[d] = Fl[d] + J[d] + F_(PFX + d);
        T[d] = Fl[3 + d] + H[d] + F_(PTX + d);
    }
    F_(FX) = Fl[0];
    F_(FY) = Fl[1];
    F_(FZ) = Fl[2];
    F_(TX) = Fl[3];
    F_(TY) = Fl[4];
    F_(TZ) = Fl[5];
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
    F_(OQW) = qw;
    F_(OQX) = qx;
    F_(OQY) = qy;
    F_(OQZ) = qz;
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
    const double nw = dw * qw - dx * qx - dy * qy - dz * qz;
    const double nxq = dw * qx + dx * qw + dy * qz - dz * qy;
    const double nyq = dw * qy - dx * qz + dy * qw + dz * qx;
    const double nzq = dw * qz + dx * qy - dy * qx + dz * qw;
    const double nn = sqrt(nw * nw + nxq * nxq + nyq * nyq + nzq * nzq);
    F_(QW) = nw / nn;
    F_(QX) = nxq / nn;
    F_(QY) = nyq / nn;
    F_(QZ) = nzq / nn;
#undef F_
    pack_fast(part, cap, p, pfast);
}
__global__ __launch_bounds__(64) void k_bodies(Box bx, double* __restrict__ part, int cap,
                                               const double* __restrict__ kpart, int nk,
                                               double* __restrict__ pfast) {
    bodies_body(bx, part, cap, kpart, nk, pfast, blockIdx.x);
}
__global__ __launch_bounds__(64) void k_bodies_batch(const SysDev* __restrict__ sd,
                                                     const WorkItem* __restrict__ items) {
    const WorkItem w = items[blockIdx.x];
    const SysDev& d = sd[w.sys];
    bodies_body(d.box, d.part, d.cap, d.kpart, 1, d.pfast, w.local);
}

// Packed particle table of particles [0, np) from the particle table.
__global__ void k_pack_fast(const double* __restrict__ part, int cap, int np, double* __restrict__ pfast) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < np) pack_fast(part, cap, p, pfast);
}

// Pending kill/fill impulses: add the partial slots into the particle's J, H
// and clear the slots (before the slot layout changes or the state is saved).
__global__ void k_fold_impulses(double* __restrict__ part, int cap, int np, double* __restrict__ kpart, int nk) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    double J[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = 0; s < nk; s++)
        for (int k = 0; k < 8; k++) {
            J[k] += kpart[((size_t)p * nk + s) * 8 + k];
            kpart[((size_t)p * nk + s) * 8 + k] = 0.0;
        }
    const int fld[8] = {JX, JY, JZ, HX, HY, HZ, KMASS, FMASS};
    for (int k = 0; k < 8; k++) part[fld[k] * cap + p] += J[k];
}

// ---------------------------------------------------------------- S8
template <class R>
__device__ inline R feq_p(int i, R rho, R ux, R uy, R uz) {
    const R uu = ux * ux + uy * uy + uz * uz;
    const R cu = R(cx(i)) * ux + R(cy(i)) * uy + R(cz(i)) * uz;
    return R(wq(i)) * rho * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
}

// Kill / fill over the smallest box holding the particle's axis-aligned
// ellipsoid boxes before and after the move (the boxes the raster walked, so
// every node it gave to p in either owner map); runs after the density pass of the next step (populations after
// streaming, nodes fluid in both owner maps). Node n with old owner o and new
// owner o2:
//   o fluid, o2 == p : kill  -> J_p += sum_c j^c(n), H_p += r x that (the node's
//                      populations are dropped: a solid node's slots are not read)
//   o == p, o2 fluid : fill  -> rho_new^c = mean rho^c of neighbours fluid
//                      before and after (initial mean if none), u = V + W x r,
//                      f = f^eq(rho_new^c, u), J_p -= sum_c rho_new^c u, H_p -= r x that;
//                      the node's Psi (and rho) follow from the stored f.
// Each changing node is handled by exactly one thread (of its owner's block).
// One block loops over that box, eight nodes per thread in flight; the
// block's fixed-order sum is the particle's impulse (and killed / filled
// mass) of this step. A box wider than kext (a move of more than two
// spacings) raises health bit 2.
template <class P>
__device__ inline void killfill_node(const Box& bx, typename P::S* __restrict__ f,
                                     const uint32_t* __restrict__ own_old, const uint32_t* __restrict__ own_new,
                                     uint32_t* __restrict__ bmask, typename P::R* __restrict__ psi,
                                     typename P::R* __restrict__ rho, const double* __restrict__ part, int cap, int p,
                                     bool kill, int x, int y, int z, int64_t n, const double (&Xn)[3],
                                     double (&acc)[8]) {
    using R = typename P::R;
    const int64_t N = bx.N;
    const int Ls[3] = {bx.nx, bx.ny, bx.nz};
    const double r[3] = {minimg((double)x - Xn[0], Ls[0]), minimg((double)y - Xn[1], Ls[1]),
                         minimg((double)z - Xn[2], Ls[2])};
    double d[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // impulse, torque, killed, filled mass
    if (kill) {
        // the node's populations after streaming, where its bounce mask puts them
        const uint32_t bm = bmask[n];
        double j[3] = {0.0, 0.0, 0.0}, m = 0.0;
#pragma unroll
        for (int cc = 0; cc < 2; cc++) {
            typename P::S v[Q];  // a component's loads all issued before its in-order sums
#pragma unroll
            for (int i = 0; i < Q; i++) {
                const bool u = (bm >> i) & 1u;
                const int64_t src = u ? (int64_t)upstream(Ls[0], Ls[1], Ls[2], x, y, z, i) : n;
                v[i] = f[(size_t)(cc * Q + (u ? opp(i) : i)) * N + src];
            }
#pragma unroll
            for (int i = 0; i < Q; i++) {
                const double w = pop64<P>(v[i], wq(i) * bx.rref[cc]);
                m += w;
                j[0] += w * cx(i);
                j[1] += w * cy(i);
                j[2] += w * cz(i);
            }
        }
        d[0] = j[0];
        d[1] = j[1];
        d[2] = j[2];
        d[3] = r[1] * j[2] - r[2] * j[1];
        d[4] = r[2] * j[0] - r[0] * j[2];
        d[5] = r[0] * j[1] - r[1] * j[0];
        d[6] = m;
    } else {
        const double V[3] = {part[VX * cap + p], part[VY * cap + p], part[VZ * cap + p]};
        const double W[3] = {part[WX * cap + p], part[WY * cap + p], part[WZ * cap + p]};
        // neighbour densities after streaming: the density pass that precedes
        // kill / fill has stored them for every node fluid before and after
        const R* dens = bx.psi_kind == 0 ? psi : rho;
        double rn[2] = {0.0, 0.0};
        int cnt = 0;
        uint32_t oo[Q], on[Q];
        uint32_t up[Q];
        R d0[Q], d1[Q];
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const int64_t m = node_index(bx, wrapc(x + cx(i), Ls[0]), wrapc(y + cy(i), Ls[1]), wrapc(z + cz(i), Ls[2]));
            oo[i] = own_old[m];
            on[i] = own_new[m];
            d0[i] = dens[m];
            d1[i] = dens[N + m];
            up[i] = upstream(Ls[0], Ls[1], Ls[2], x, y, z, i);
        }
#pragma unroll
        for (int i = 1; i < Q; i++) {
            if (oo[i] != OWN_FLUID || on[i] != OWN_FLUID) continue;
            rn[0] += (double)d0[i];
            rn[1] += (double)d1[i];
            cnt++;
        }
#pragma unroll
        for (int cc = 0; cc < 2; cc++)
            rn[cc] = cnt > 0 ? rho_full<R>(R(0), bx.rref[cc]) + rn[cc] / (double)cnt : bx.rmean0[cc];
        const double ub[3] = {V[0] + (W[1] * r[2] - W[2] * r[1]), V[1] + (W[2] * r[0] - W[0] * r[2]),
                              V[2] + (W[0] * r[1] - W[1] * r[0])};
        // Population i of the node goes to its own slot (i, n), unless the
        // upstream neighbour n - c_i was fluid at the push: that neighbour's
        // bounced population sits in (i, n), and the slot (ibar, n - c_i),
        // which this node filled with a zero, takes the value instead (bit i
        // of the node's bounce mask).
        uint32_t bm = 0u;
#pragma unroll
        for (int i = 1; i < Q; i++)
            if (oo[opp(i)] == OWN_FLUID) bm |= 1u << i;  // n + c_ibar = n - c_i
        double jm[3] = {0.0, 0.0, 0.0};
        R rs[2];
#pragma unroll
        for (int cc = 0; cc < 2; cc++) {
            R r = R(0);
#pragma unroll
            for (int i = 0; i < Q; i++) {
                const bool u = (bm >> i) & 1u;
                typename P::S* dst = f + (size_t)(cc * Q + (u ? opp(i) : i)) * N + (u ? (int64_t)up[i] : n);
                const typename P::S e = enc64<P>(feq_p<double>(i, rn[cc], ub[0], ub[1], ub[2]), wq(i) * bx.rref[cc]);
                *dst = e;
                // the node's density as the density pass forms it from the stored values
                r += P::raw(e);
            }
            for (int d = 0; d < 3; d++) jm[d] += rn[cc] * ub[d];
            rs[cc] = r;  // the kept density (the deviation in the float forms)
        }
        bmask[n] = bm;
        psi[n] = psi_kept(rs[0], bx.psi_kind, R(bx.eref[0]));
        psi[N + n] = psi_kept(rs[1], bx.psi_kind, R(bx.eref[1]));
        if (bx.psi_kind != 0) {
            rho[n] = rs[0];
            rho[N + n] = rs[1];
        }
        d[0] = -jm[0];
        d[1] = -jm[1];
        d[2] = -jm[2];
        d[3] = -(r[1] * jm[2] - r[2] * jm[1]);
        d[4] = -(r[2] * jm[0] - r[0] * jm[2]);
        d[5] = -(r[0] * jm[1] - r[1] * jm[0]);
        d[7] = rn[0] + rn[1];
    }
    // every slot takes a term (zero where this kind has none), so the
    // accumulator stays in registers
#pragma unroll
    for (int k = 0; k < 8; k++) acc[k] += d[k];
}

template <class P>
__device__ inline void killfill_body(const Box& bx, typename P::S* __restrict__ f,
                                     const uint32_t* __restrict__ own_old, const uint32_t* __restrict__ own_new,
                                     uint32_t* __restrict__ bmask, typename P::R* __restrict__ psi,
                                     typename P::R* __restrict__ rho,
                                     const double* __restrict__ part, int cap, int kext, double* __restrict__ kpart,
                                     int* __restrict__ health, int p) {
    const int Ls[3] = {bx.nx, bx.ny, bx.nz};
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // J, H, killed mass, filled mass
    int lo[3] = {0, 0, 0}, sz[3] = {0, 0, 0};
    bool ok = true;
    const double Xn[3] = {part[PX * cap + p], part[PY * cap + p], part[PZ * cap + p]};
    const double Xo[3] = {part[OX * cap + p], part[OY * cap + p], part[OZ * cap + p]};
    const double rpar = part[RPAR * cap + p], rperp = part[RPERP * cap + p];
    const double rb = rpar > rperp ? rpar : rperp;
    // the boxes the raster walked before and after the move (same extents,
    // from the same centres and orientations), the new one lifted next to the
    // old centre
    double Ro[3][3], Rn[3][3], eo[3], en[3];
    qrot(part[OQW * cap + p], part[OQX * cap + p], part[OQY * cap + p], part[OQZ * cap + p], Ro);
    qrot(part[QW * cap + p], part[QX * cap + p], part[QY * cap + p], part[QZ * cap + p], Rn);
    ellipsoid_extent(Ro, rpar, rperp, 1.0, rb, eo);
    ellipsoid_extent(Rn, rpar, rperp, 1.0, rb, en);
    for (int d = 0; d < 3; d++) {
        if (!isfinite(Xn[d]) || !isfinite(Xo[d]) || !(rb < 0.5 * Ls[d])) {
            ok = false;
            break;
        }
        const double xn = Xo[d] + minimg(Xn[d] - Xo[d], Ls[d]);  // unwrapped new centre
        const int a = min((int)ceil(Xo[d] - eo[d]), (int)ceil(xn - en[d]));
        const int b = max((int)floor(Xo[d] + eo[d]), (int)floor(xn + en[d]));
        lo[d] = a;
        sz[d] = max(0, min(b - a + 1, Ls[d]));
        if (sz[d] > kext && threadIdx.x == 0) atomicOr(health, 2);
    }
    const int total = ok ? sz[0] * sz[1] * sz[2] : 0;
    constexpr int U = 8;  // nodes per thread with owner loads in flight (4: +6 %, 12: +3 % time)
    for (int base = 0; base < total; base += U * kPB) {
        uint32_t oo[U], on[U];  // every owner load of this thread issued before any is used
#pragma unroll
        for (int k = 0; k < U; k++) {
            const int t = base + k * kPB + threadIdx.x;
            oo[k] = on[k] = OWN_FLUID;
            if (t < total) {
                int ix, iy, iz;
                box_node(t, sz, ix, iy, iz);
                const int64_t n = node_index(bx, wrapc_any(lo[0] + ix, Ls[0]), wrapc_any(lo[1] + iy, Ls[1]),
                                             wrapc_any(lo[2] + iz, Ls[2]));
                oo[k] = own_old[n];
                on[k] = own_new[n];
            }
        }
        // one call site for the (rare) changing nodes: bit 2k marks a kill,
        // bit 2k + 1 a fill of node k, whose coordinates are formed again
        uint32_t todo = 0u;
#pragma unroll
        for (int k = 0; k < U; k++) {
            if (oo[k] == OWN_FLUID && on[k] == (uint32_t)p) todo |= 1u << (2 * k);
            if (oo[k] == (uint32_t)p && on[k] == OWN_FLUID) todo |= 2u << (2 * k);
        }
#pragma unroll 1
        for (int k = 0; k < U; k++) {
            const uint32_t b = (todo >> (2 * k)) & 3u;
            if (b == 0u) continue;
            int ix, iy, iz;
            box_node(base + k * kPB + threadIdx.x, sz, ix, iy, iz);
            const int x = wrapc_any(lo[0] + ix, Ls[0]), y = wrapc_any(lo[1] + iy, Ls[1]),
                      z = wrapc_any(lo[2] + iz, Ls[2]);
            killfill_node<P>(bx, f, own_old, own_new, bmask, psi, rho, part, cap, p, b == 1u, x, y, z,
                             node_index(bx, x, y, z), Xn, acc);
        }
    }
    double tot[8];
    block_sum<8>(acc, tot);
    if (threadIdx.x == 0)
        for (int k = 0; k < 8; k++) kpart[(size_t)p * 8 + k] = tot[k];
}
template <class P>
__global__ __launch_bounds__(kPB, 3) void k_killfill(Box bx, typename P::S* __restrict__ f,
                                                  const uint32_t* __restrict__ own_old,
                                                  const uint32_t* __restrict__ own_new, uint32_t* __restrict__ bmask,
                                                  typename P::R* __restrict__ psi, typename P::R* __restrict__ rho,
                                                  const double* __restrict__ part, int cap, int kext,
                                                  double* __restrict__ kpart, int* __restrict__ health) {
    killfill_body<P>(bx, f, own_old, own_new, bmask, psi, rho, part, cap, kext, kpart, health, blockIdx.x);
}
// Batched: item = (system, particle); owner copy `oo` is the old map, 1 - oo
// the new one; populations copy `fd`.
template <class P>
__global__ __launch_bounds__(kPB, 3) void k_killfill_batch(const SysDev* __restrict__ sd,
                                                        const WorkItem* __restrict__ items, int oo, int fd) {
    const WorkItem w = items[blockIdx.x];
    const SysDev& d = sd[w.sys];
    killfill_body<P>(d.box, (typename P::S*)d.f[fd], d.owner[oo], d.owner[1 - oo], d.bmask[fd], (typename P::R*)d.psi,
                     (typename P::R*)d.rho, d.part, d.cap, d.kext, d.kpart, d.health, w.local);
}

// ---------------------------------------------------------------- launchers

// Largest extent of a raster box for bounding radius rb: floor(2 rb) + 1, at
// most the longest side; the kill/fill box of a move below two spacings has
// at most two more nodes (this also sizes the record boxes).
int raster_extent(int nx, int ny, int nz, double rb) {
    const int L = std::max(nx, std::max(ny, nz));
    return std::min((int)floor(2.0 * rb) + 1, L);
}
int killfill_extent(int nx, int ny, int nz, double rb) {
    const int L = std::max(nx, std::max(ny, nz));
    return std::min(raster_extent(nx, ny, nz, rb) + 2, L);
}
int kill_ext(const lb_handle* h) { return killfill_extent(h->box.nx, h->box.ny, h->box.nz, h->rmax); }

hipError_t launch_shell(lb_handle* h) {
    if (h->np <= 0) return hipSuccess;
    if (h->prm.precision == LB_FP64)
        hipLaunchKernelGGL(k_shell<double>, dim3(h->np), dim3(kPB), 0, h->stream, h->box, (double*)h->b.psi,
                           (const double*)h->b.rho, h->b.owner[h->ocur], h->b.part, h->cap);
    else
        hipLaunchKernelGGL(k_shell<float>, dim3(h->np), dim3(kPB), 0, h->stream, h->box, (float*)h->b.psi,
                           (const float*)h->b.rho, h->b.owner[h->ocur], h->b.part, h->cap);
    return hipGetLastError();
}

hipError_t launch_forces(lb_handle* h) {
    if (h->np <= 0) return hipSuccess;
    const int ke = kill_ext(h);
    hipLaunchKernelGGL(k_linkforce, dim3(h->np), dim3(kPB), 0, h->stream, h->box, h->b.rec, ke * ke * ke, h->b.part,
                       h->cap);
    return hipGetLastError();
}
hipError_t launch_bodies(lb_handle* h) {
    if (h->np <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bodies, dim3(h->np), dim3(64), 0, h->stream, h->box, h->b.part, h->cap, h->b.kpart, 1,
                       h->b.pfast);
    return hipGetLastError();
}
hipError_t launch_pack_fast(lb_handle* h) {
    if (h->np <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_fast, dim3((h->np + 255) / 256), dim3(256), 0, h->stream, h->b.part, h->cap, h->np,
                       h->b.pfast);
    return hipGetLastError();
}

hipError_t launch_fold_impulses(lb_handle* h) {
    if (h->np <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fold_impulses, dim3((h->np + 63) / 64), dim3(64), 0, h->stream, h->b.part, h->cap, h->np,
                       h->b.kpart, 1);
    return hipGetLastError();
}

hipError_t launch_clear_owner(lb_handle* h, uint32_t* owner) { return launch_fill_u32(h, owner, OWN_FLUID, h->box.N); }

hipError_t launch_raster(lb_handle* h, uint32_t* owner, int first, int count) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster, dim3(count), dim3(kPB), 0, h->stream, h->box, h->b.part, h->cap, owner, first);
    return hipGetLastError();
}

hipError_t launch_killfill(lb_handle* h) {
    if (h->np <= 0) return hipSuccess;
    uint32_t* oo = h->b.owner[h->ocur];
    uint32_t* on = h->b.owner[1 - h->ocur];
    void* fn = h->b.f[1 - h->cur];
    const int kext = kill_ext(h);
    LBE_PDISPATCH(h->prm.precision,
                  hipLaunchKernelGGL(k_killfill<P>, dim3(h->np), dim3(kPB), 0, h->stream, h->box,
                                     (typename P::S*)fn, oo, on, h->b.bmask[1 - h->cur], (typename P::R*)h->b.psi,
                                     (typename P::R*)h->b.rho,
                                     h->b.part, h->cap, kext, h->b.kpart, h->b.health));
    return hipGetLastError();
}

// ---------------------------------------------------------------- batched launchers

hipError_t launch_batch_shell(const BatchLaunch& bl, int precision, hipStream_t st, int o) {
    if (bl.n[BI_PART] == 0) return hipSuccess;
    if (precision == LB_FP64)
        hipLaunchKernelGGL(k_shell_batch<double>, dim3(bl.n[BI_PART]), dim3(kPB), 0, st, bl.sys, bl.items[BI_PART], o);
    else
        hipLaunchKernelGGL(k_shell_batch<float>, dim3(bl.n[BI_PART]), dim3(kPB), 0, st, bl.sys, bl.items[BI_PART], o);
    return hipGetLastError();
}

hipError_t launch_batch_forces(const BatchLaunch& bl, hipStream_t st) {
    if (bl.n[BI_PART] == 0) return hipSuccess;
    hipLaunchKernelGGL(k_linkforce_batch, dim3(bl.n[BI_PART]), dim3(kPB), 0, st, bl.sys, bl.items[BI_PART]);
    return hipGetLastError();
}

hipError_t launch_batch_bodies(const BatchLaunch& bl, hipStream_t st) {
    if (bl.n[BI_PART] == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bodies_batch, dim3(bl.n[BI_PART]), dim3(64), 0, st, bl.sys, bl.items[BI_PART]);
    return hipGetLastError();
}

hipError_t launch_batch_raster(const BatchLaunch& bl, hipStream_t st, int o) {
    if (bl.n[BI_PART] == 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster_batch, dim3(bl.n[BI_PART]), dim3(kPB), 0, st, bl.sys, bl.items[BI_PART], o);
    return hipGetLastError();
}

hipError_t launch_batch_killfill(const BatchLaunch& bl, int precision, hipStream_t st, int oo, int fd) {
    if (bl.n[BI_PART] == 0) return hipSuccess;
    LBE_PDISPATCH(precision, hipLaunchKernelGGL(k_killfill_batch<P>, dim3(bl.n[BI_PART]), dim3(kPB), 0, st, bl.sys,
                                                bl.items[BI_PART], oo, fd));
    return hipGetLastError();
}

}  // namespace lbe
