// Fluid kernels of liblbe (gfx950): densities, the fused force + collision +
// streaming step, initialisation, field readout and deterministic FP64
// reductions.
//
// Layout in HBM: populations f[c][i][n] (structure of arrays, x fastest, one
// plane of N values per (component, velocity)), two copies (current / next);
// effective masses Psi[c][n]; owner map uint32 per node. One thread per node, tiles
// of 64x4 (or 32x8) nodes of one xy-plane per 256-thread block, tiles of
// neighbouring z on the same XCD.
#include <algorithm>
#include <type_traits>

#include "lbe_internal.h"

namespace lbe {

// Workgroups are dispatched round-robin over the 8 XCDs. Remap the block index
// so each XCD walks a contiguous range of tiles: the rows a tile reads from
// its neighbours then sit in the same L2.
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

// ---------------------------------------------------------------- S1
// rho^c(n) = sum_i f_i^c(n) on fluid nodes (rho_ref^c + sum_i h_i^c in the
// deviation forms), stored as the effective mass
// Psi^c(n) of Eq. (3) (what the force stencil reads) and, when the shell fill
// needs it, as rho^c(n); health flag on NaN / rho < 0.
// With owner_old given (the pass that follows the re-rasterisation), nodes that
// were not fluid before are skipped: kill / fill sets a filled node's values.
template <class P, bool SOLID>
__device__ inline void density_body(const Box& bx, const typename P::S* __restrict__ f,
                                    typename P::R* __restrict__ psi, typename P::R* __restrict__ rho,
                                    const uint32_t* __restrict__ owner, const uint32_t* __restrict__ owner_old,
                                    const uint32_t* __restrict__ bmask, int* __restrict__ health, int blk) {
    using R = typename P::R;
    const uint32_t N = (uint32_t)bx.N;
    const uint32_t n = (uint32_t)blk * 256u + threadIdx.x;
    if (n >= N) return;
    // densities of fluid nodes (not just filled); the other lanes store zero
    // so that every line of Psi is written whole (the shell and fill passes
    // write those nodes before anything reads them)
    const bool live = (!SOLID || owner[n] == OWN_FLUID) && (!owner_old || owner_old[n] == OWN_FLUID);
    const R ref0 = R(bx.rref[0]), ref1 = R(bx.rref[1]);
    R r0 = R(0), r1 = R(0);
    const uint32_t bm = (SOLID && live) ? bmask[n] : 0u;
    if (!SOLID || __ballot(bm != 0u) == 0ull) {
        // no lane of the wave reads a bounced population: plane bases are
        // wave-uniform, offsets 32-bit
        const uint32_t nb = n * (uint32_t)sizeof(typename P::S);
        if (live) {
#pragma unroll
            for (int i = 0; i < Q; i++) {
                r0 += P::raw(*at(f + (size_t)i * N, nb));
                r1 += P::raw(*at(f + (size_t)(Q + i) * N, nb));
            }
        }
    } else if (live) {
        // population i from its own slot, or from plane ibar at n - c_i when
        // bit i of the bounce mask is set
        uint32_t up[Q];
#pragma unroll
        for (int i = 0; i < Q; i++) up[i] = n;
        if (bm != 0u) {
            const int nx = bx.nx, ny = bx.ny, nz = bx.nz;
            const uint32_t pl = (uint32_t)nx * (uint32_t)ny;
            const int z = (int)(n / pl);
            const uint32_t rem = n - (uint32_t)z * pl;
            const int y = (int)(rem / (uint32_t)nx), x = (int)(rem - (uint32_t)y * (uint32_t)nx);
            const uint32_t xs[3] = {(uint32_t)x, (uint32_t)(x + 1 == nx ? 0 : x + 1),
                                    (uint32_t)(x == 0 ? nx - 1 : x - 1)};
            const uint32_t ys[3] = {(uint32_t)(y * nx), (uint32_t)((y + 1 == ny ? 0 : y + 1) * nx),
                                    (uint32_t)((y == 0 ? ny - 1 : y - 1) * nx)};
            const uint32_t zs[3] = {(uint32_t)z * pl, (uint32_t)(z + 1 == nz ? 0 : z + 1) * pl,
                                    (uint32_t)(z == 0 ? nz - 1 : z - 1) * pl};
#define LBE_SEL(c) ((c) == 0 ? 0 : ((c) > 0 ? 1 : 2))
#pragma unroll
            for (int i = 1; i < Q; i++)
                if ((bm >> i) & 1u) up[i] = xs[LBE_SEL(-cx(i))] + ys[LBE_SEL(-cy(i))] + zs[LBE_SEL(-cz(i))];
#undef LBE_SEL
        }
        // every load issued before the in-order sums
        R v0[Q], v1[Q];
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const bool u = (bm >> i) & 1u;
            const uint32_t ob = up[i] * (uint32_t)sizeof(typename P::S);
            v0[i] = P::raw(*at(u ? f + (size_t)opp(i) * N : f + (size_t)i * N, ob));
            v1[i] = P::raw(*at(u ? f + (size_t)(Q + opp(i)) * N : f + (size_t)(Q + i) * N, ob));
        }
#pragma unroll
        for (int i = 0; i < Q; i++) {
            r0 += v0[i];
            r1 += v1[i];
        }
    }
    // r0, r1 are the kept densities (deviations rho - rho_ref in the float
    // forms, where the population sums are sums of deviations)
    psi[n] = live ? psi_kept<R>(r0, bx.psi_kind, R(bx.eref[0])) : R(0);
    psi[N + n] = live ? psi_kept<R>(r1, bx.psi_kind, R(bx.eref[1])) : R(0);
    if (rho) {  // densities, for the shell fill (exponential Psi only)
        rho[n] = r0;
        rho[N + n] = r1;
    }
    if (P::dev) {  // rho^c = rho_ref^c + sum of the deviations
        r0 += ref0;
        r1 += ref1;
    }
    if (live && (!(r0 >= R(0)) || !(r1 >= R(0)))) atomicOr(health, 1);
}
template <class P, bool SOLID>
__global__ __launch_bounds__(256) void k_density(Box bx, const typename P::S* __restrict__ f,
                                                 typename P::R* __restrict__ psi, typename P::R* __restrict__ rho,
                                                 const uint32_t* __restrict__ owner,
                                                 const uint32_t* __restrict__ owner_old,
                                                 const uint32_t* __restrict__ bmask, int* __restrict__ health) {
    density_body<P, SOLID>(bx, f, psi, rho, owner, owner_old, bmask, health, blockIdx.x);
}
// The densities rho^c of a batched system are kept (written by the density
// pass, read by the shell fills) exactly when a lone handle keeps them: the
// system has solid nodes (particles or walls), Psi is not rho itself, and the
// workspace holds the buffer.
__device__ inline void* sys_rho(const SysDev& d) {
    return (d.rho && (d.np > 0 || d.box.walls != 0) && d.box.psi_kind != 0) ? d.rho : nullptr;
}
// Batched: item = (system, block of 256 nodes); populations copy `c`, owner
// copy `o` (and, if oo >= 0, old owner copy `oo`); rho is written where the
// system keeps it (sys_rho).
template <class P>
__global__ __launch_bounds__(256) void k_density_batch(const SysDev* __restrict__ sd,
                                                       const WorkItem* __restrict__ items, int c, int o, int oo) {
    const WorkItem w = items[blockIdx.x];
    const SysDev& d = sd[w.sys];
    typename P::R* rho = (typename P::R*)sys_rho(d);
    density_body<P, true>(d.box, (const typename P::S*)d.f[c], (typename P::R*)d.psi, rho, d.owner[o],
                          oo >= 0 ? d.owner[oo] : nullptr, d.bmask[c], d.health, w.local);
}

// ---------------------------------------------------------------- S3-S6
// Per fluid node: Shan-Chen force (Eq. (3)) from neighbour Psi, BGK collision
// (Eq. (2)) with the common-velocity shift u^eq_c = u' + tau F^c/rho^c, then
// push streaming (Eq. (1)). With solids present, a link i into a solid node
// is replaced by moving bounce-back (Eq. (4)): the value f*_i(n) + C,
// C = 6 w_i rho^c(n) (u_b . c_ibar), becomes f'_ibar(n); it is pushed into
// the solid node's slot (i, n + c_i) like any other population, and the
// node's bounce mask tells the readers of f'_ibar(n) where it is. For a rigid
// body the surface velocity at the link midpoint, V + W x (r_n + c_i/2), has
// the same projection on c_i as U_n = V + W x r_n at the node (W x c_i is
// normal to c_i), so C needs one U_n per node and particle. The particle's
// share (2 f*_i + C) c_i of Eq. (5) is summed per node and particle and
// written into node n's record of that particle; k_linkforce sums the
// records (force, and torque r_n x force).

// Neighbour sums S^c = sum_i Psi^c(n + c_i) c_i over the 18 links, in link
// order; ps0(i) / ps1(i) give Psi^A / Psi^B of neighbour i. Formed straight
// from the staged tile so that the 36 neighbour values are never all live.
template <class R, class F0, class F1>
__device__ inline void psi_sums(F0 ps0, F1 ps1, R (&s0)[3], R (&s1)[3]) {
    R s0x = R(0), s0y = R(0), s0z = R(0), s1x = R(0), s1y = R(0), s1z = R(0);
#pragma unroll
    for (int i = 1; i < Q; i++) {
        const R p0 = ps0(i), p1 = ps1(i);
        if (cx(i) > 0) { s0x += p0; s1x += p1; }
        if (cx(i) < 0) { s0x -= p0; s1x -= p1; }
        if (cy(i) > 0) { s0y += p0; s1y += p1; }
        if (cy(i) < 0) { s0y -= p0; s1y -= p1; }
        if (cz(i) > 0) { s0z += p0; s1z += p1; }
        if (cz(i) < 0) { s0z -= p0; s1z -= p1; }
    }
    s0[0] = s0x; s0[1] = s0y; s0[2] = s0z;
    s1[0] = s1x; s1[1] = s1y; s1[2] = s1z;
}

// Moments, Shan-Chen velocity shift and BGK relaxation of one node, in place
// on f0 / f1 (component A / B): the populations themselves (FP64) or their
// deviations h_i = f_i - w_i rho_ref^c (the other forms; then
// f^eq_i - w_i rho_ref = w_i [(rho - rho_ref) + rho (3 c.u + 4.5 (c.u)^2 -
// 1.5 u.u)] and rho - rho_ref = sum_i h_i). S0, S1: the neighbour sums of
// Psi^A, Psi^B. r0, r1 return the densities.
template <class P>
__device__ inline void collide_node(const Box& bx, typename P::R (&f0)[Q], typename P::R (&f1)[Q],
                                    const typename P::R (&S0)[3], const typename P::R (&S1)[3],
                                    typename P::R& r0, typename P::R& r1) {
    using R = typename P::R;
    R jx = R(0), jy = R(0), jz = R(0);
    R d0 = R(0), d1 = R(0);  // sums of the stored numbers
#pragma unroll
    for (int i = 0; i < Q; i++) {
        d0 += f0[i];
        d1 += f1[i];
        const R s = f0[i] + f1[i];
        if (cx(i) > 0) jx += s;
        if (cx(i) < 0) jx -= s;
        if (cy(i) > 0) jy += s;
        if (cy(i) < 0) jy -= s;
        if (cz(i) > 0) jz += s;
        if (cz(i) < 0) jz -= s;
    }
    r0 = P::dev ? R(bx.rref[0]) + d0 : d0;
    r1 = P::dev ? R(bx.rref[1]) + d1 : d1;
    const R s0x = S0[0], s0y = S0[1], s0z = S0[2], s1x = S1[0], s1y = S1[1], s1z = S1[2];
    const int kind = bx.psi_kind;
    const R tau = R(bx.tau);
    const R irt = R(1) / (r0 + r1);
    const R ux = jx * irt, uy = jy * irt, uz = jz * irt;
    const R k0 = -R(bx.g) * psi_ratio(r0, kind);
    const R k1 = -R(bx.g) * psi_ratio(r1, kind);
    const R ax = R(bx.ax), ay = R(bx.ay), az = R(bx.az);
    const R u0x = ux + tau * (k0 * s1x + ax), u0y = uy + tau * (k0 * s1y + ay), u0z = uz + tau * (k0 * s1z + az);
    const R u1x = ux + tau * (k1 * s0x + ax), u1y = uy + tau * (k1 * s0y + ay), u1z = uz + tau * (k1 * s0z + az);
    const R uu0 = u0x * u0x + u0y * u0y + u0z * u0z;
    const R uu1 = u1x * u1x + u1y * u1y + u1z * u1z;
    const R om = R(bx.omega);
#pragma unroll
    for (int i = 0; i < Q; i++) {
        R e0, e1;
        if (P::dev) {
            const R c0 = R(cx(i)) * u0x + R(cy(i)) * u0y + R(cz(i)) * u0z;
            const R c1 = R(cx(i)) * u1x + R(cy(i)) * u1y + R(cz(i)) * u1z;
            e0 = R(wq(i)) * (d0 + r0 * (R(3) * c0 + R(4.5) * c0 * c0 - R(1.5) * uu0));
            e1 = R(wq(i)) * (d1 + r1 * (R(3) * c1 + R(4.5) * c1 * c1 - R(1.5) * uu1));
        } else {
            e0 = feq_i(i, r0, u0x, u0y, u0z, uu0);
            e1 = feq_i(i, r1, u1x, u1y, u1z, uu1);
        }
        f0[i] = f0[i] - om * (f0[i] - e0);
        f1[i] = f1[i] - om * (f1[i] - e1);
    }
}

// Tile kernel (any box): BX x BY nodes of one xy-plane per 256-thread block,
// Psi and owner codes of the tile and its one-node halo staged in LDS.
template <class P, bool SOLID, int BX, int BY>
__device__ inline void fused_body(const Box& bx, const typename P::S* __restrict__ fs, typename P::S* __restrict__ fd,
                                  const typename P::R* __restrict__ psi, const uint32_t* __restrict__ owner,
                                  const uint32_t* __restrict__ bm_in, uint32_t* __restrict__ bm_out,
                                  const double* __restrict__ pfast,
                                  double* __restrict__ rec, int rstride, int tiles_x, int tiles_y, int tile,
                                  bool zrun) {
    using R = typename P::R;
    using S = typename P::S;
    static_assert(BX * BY == 256, "one node per thread");
    constexpr int TX = BX + 2, TY = BY + 2, TP = TX * TY;  // tile plane with a one-node halo
    __shared__ R s_psi[2][3 * TP];
    __shared__ uint32_t s_own[SOLID ? 3 * TP : 1];

    const int nx = bx.nx, ny = bx.ny, nz = bx.nz;
    const uint32_t N = (uint32_t)bx.N;
    // tile order: x fastest, then y, then z; or, with zrun, x, then z, then y,
    // so a tile's z-neighbours are a few tiles away in dispatch order and
    // their rows (halo Psi and owners, redirected loads) are still in L2
    int tx, ty, z;
    if (zrun) {
        const int tq = tile / tiles_x;
        tx = tile - tq * tiles_x;
        ty = tq / nz;
        z = tq - ty * nz;
    } else {
        const int txy = tiles_x * tiles_y;
        z = tile / txy;
        const int rem = tile - z * txy;
        ty = rem / tiles_x;
        tx = rem - ty * tiles_x;
    }
    const int lx = threadIdx.x % BX, ly = threadIdx.x / BX;
    const int x0 = tx * BX, y0 = ty * BY;
    const int x = x0 + lx, y = y0 + ly;
    const bool active = (x < nx) && (y < ny);
    const uint32_t n = active ? (uint32_t)(x + nx * (y + ny * z)) : 0u;
    // owner code and bounce mask, both loaded before either is waited for
    const uint32_t own_n = (SOLID && active) ? owner[n] : OWN_FLUID;
    const uint32_t bm = (SOLID && active) ? bm_in[n] : 0u;
    const bool fluid = active && own_n == OWN_FLUID;
    const uint32_t nb = n * (uint32_t)sizeof(S);  // byte offset of the node within a plane
    const R ref0 = R(bx.rref[0]), ref1 = R(bx.rref[1]);
    // offsets of the neighbour rows / planes (periodic)
    const int xs[3] = {x, x + 1 == nx ? 0 : x + 1, x == 0 ? nx - 1 : x - 1};
    const uint32_t ys[3] = {(uint32_t)(y * nx), (uint32_t)((y + 1 == ny ? 0 : y + 1) * nx),
                            (uint32_t)((y == 0 ? ny - 1 : y - 1) * nx)};
    const uint32_t pl = (uint32_t)(nx * ny);
    const uint32_t zs[3] = {(uint32_t)z * pl, (uint32_t)(z + 1 == nz ? 0 : z + 1) * pl,
                            (uint32_t)(z == 0 ? nz - 1 : z - 1) * pl};
#define LBE_SEL(c) ((c) == 0 ? 0 : ((c) > 0 ? 1 : 2))
#define LBE_NB(i) ((uint32_t)xs[LBE_SEL(cx(i))] + ys[LBE_SEL(cy(i))] + zs[LBE_SEL(cz(i))])

    // this node's 2 x 19 populations after streaming (in flight while the
    // tile loads); with solids, a set bit i of the bounce mask takes
    // population i from plane ibar at n - c_i
    R f0[Q], f1[Q];
    if (fluid) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const bool up = SOLID && ((bm >> i) & 1u);
            const int pi = up ? opp(i) : i;
            const uint32_t ob = up ? LBE_NB(opp(i)) * (uint32_t)sizeof(S) : nb;
            f0[i] = P::raw(*at(fs + (size_t)pi * N, ob));
            f1[i] = P::raw(*at(fs + (size_t)(Q + pi) * N, ob));
        }
    } else {
#pragma unroll
        for (int i = 0; i < Q; i++) f0[i] = f1[i] = R(0);
    }
    // halo tile: every load of this thread issued before any is waited for
    constexpr int NE = (3 * TP + 255) / 256;
    R t0[NE], t1[NE];
    uint32_t to[NE];
#pragma unroll
    for (int k = 0; k < NE; k++) {
        const int e = threadIdx.x + 256 * k;
        if (e < 3 * TP) {
            const int lz = e / TP, r = e - lz * TP, yy = r / TX, xx = r - yy * TX;
            // periodic wrap; positions past a ragged edge (only read by
            // inactive threads) are clamped into the box
            int gx = x0 - 1 + xx, gy = y0 - 1 + yy;
            gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
            gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
            gx = gx < nx ? gx : 0;
            gy = gy < ny ? gy : 0;
            const int gz = wrapc(z - 1 + lz, nz);
            const uint32_t m = (uint32_t)(gx + nx * (gy + ny * gz));
            t0[k] = psi[m];
            t1[k] = psi[N + m];
            if (SOLID) to[k] = owner[m];
        }
    }
#pragma unroll
    for (int k = 0; k < NE; k++) {
        const int e = threadIdx.x + 256 * k;
        if (e < 3 * TP) {
            s_psi[0][e] = t0[k];
            s_psi[1][e] = t1[k];
            if (SOLID) s_own[e] = to[k];
        }
    }
    __syncthreads();
    // with solids, the lanes of solid nodes take part in the pushes (zeros),
    // so that every slot of every plane is written exactly once
    if (!(SOLID ? active : fluid)) return;

#define LBE_LS(i) ((1 + cz(i)) * TP + (ly + 1 + cy(i)) * TX + (lx + 1 + cx(i)))
    R S0[3], S1[3];
    psi_sums<R>([&](int i) { return s_psi[0][LBE_LS(i)]; }, [&](int i) { return s_psi[1][LBE_LS(i)]; }, S0, S1);
    R r0 = R(0), r1 = R(0);
    if (fluid) collide_node<P>(bx, f0, f1, S0, S1, r0, r1);
    *atw(fd, nb) = P::mk(fluid ? f0[0] : empty_raw<P>(R(wq(0)) * ref0));
    *atw(fd + (size_t)Q * N, nb) = P::mk(fluid ? f1[0] : empty_raw<P>(R(wq(0)) * ref1));
    if constexpr (!SOLID) {
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const uint32_t mb = LBE_NB(i) * (uint32_t)sizeof(S);
            *atw(fd + (size_t)i * N, mb) = P::mk(f0[i]);
            *atw(fd + (size_t)(Q + i) * N, mb) = P::mk(f1[i]);
        }
    } else {
        // U_n of the first two particles each fluid lane links to: the wave
        // visits the distinct particles among them one at a time, reading
        // each one's centre and velocities with wave-uniform loads. Walls do
        // not move unless the box says so. Links to further particles of the
        // same node (rare) read them per lane in the 4- and 8-byte forms. The
        // 2-byte forms defer them until after the pushes (see below) and do
        // the link arithmetic in float (their stored deviations carry 8 to 11
        // bits): this keeps them within 128 VGPRs, four waves per SIMD.
        constexpr bool kDefer = sizeof(S) == 2;
        using L = typename std::conditional<kDefer, float, double>::type;
        uint32_t on[Q];  // owner codes of the links, held in registers unless deferring
        auto own = [&](int i) -> uint32_t {
            if constexpr (kDefer)
                return s_own[LBE_LS(i)];
            else
                return on[i];
        };
        uint32_t p1 = OWN_FLUID;
        uint32_t mask = 0u;  // the node's bounce mask in the written copy
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const uint32_t o = s_own[LBE_LS(i)];
            if constexpr (!kDefer) on[i] = o;
            p1 = (fluid && p1 == OWN_FLUID && o < OWN_WALL) ? o : p1;
            mask |= (o != OWN_FLUID ? 1u : 0u) << opp(i);
        }
        bm_out[n] = fluid ? mask : 0u;
        uint32_t p2 = OWN_FLUID;
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const uint32_t o = own(i);
            p2 = (fluid && p2 == OWN_FLUID && o < OWN_WALL && o != p1) ? o : p2;
        }
        // per particle slot: surface velocity U_n at this node and the
        // node's cell in the particle's link records
        L Ux2 = L(0), Uy2 = L(0), Uz2 = L(0);
        int cb2 = -1;
        bool need2 = p2 < OWN_WALL;
        L Ux1 = L(0), Uy1 = L(0), Uz1 = L(0);
        int cb1 = -1;
        bool need = p1 < OWN_WALL;
        const int Ls[3] = {nx, ny, nz};
        const int xyz[3] = {x, y, z};
        while (true) {
            const unsigned long long m = __ballot(need || need2);
            if (m == 0ull) break;
            const int lead = __ffsll(m) - 1;
            const uint32_t q = __builtin_amdgcn_readfirstlane(__shfl(need ? p1 : p2, lead, 64));
            const double* pq = pfast + (size_t)q * kPF;
            const double qX[3] = {pq[PF_X], pq[PF_X + 1], pq[PF_X + 2]};
            const double qVx = pq[PF_V], qVy = pq[PF_V + 1], qVz = pq[PF_V + 2];
            const double qWx = pq[PF_W], qWy = pq[PF_W + 1], qWz = pq[PF_W + 2];
            const double rx = minimg((double)x - qX[0], nx), ry = minimg((double)y - qX[1], ny),
                         rz = minimg((double)z - qX[2], nz);
            const L ux = L(qVx + (qWy * rz - qWz * ry));
            const L uy = L(qVy + (qWz * rx - qWx * rz));
            const L uz = L(qVz + (qWx * ry - qWy * rx));
            int lo[3], sz[3];
            const int cb = box_of(bx, qX, pq[PF_RB], lo, sz) ? rec_cell(xyz, lo, sz, Ls) : -1;
            if (need && p1 == q) {
                Ux1 = ux;
                Uy1 = uy;
                Uz1 = uz;
                cb1 = cb;
                need = false;
            }
            if (need2 && p2 == q) {
                Ux2 = ux;
                Uy2 = uy;
                Uz2 = uz;
                cb2 = cb;
                need2 = false;
            }
        }
        // one store per direction, to (i, n + c_i) on every lane: f*_i for a
        // fluid target, the bounced f*_i + C for a solid one, zero from a
        // solid lane. A particle link adds its momentum exchange
        // (2 f*_i + C) c_i to the node's force on that particle: in registers
        // for the first two particles, in the record itself for others (or,
        // deferring, not yet: the link is stored without C and marked).
        L F1[3] = {L(0), L(0), L(0)}, F2[3] = {L(0), L(0), L(0)};
        uint32_t rare = 0u;  // deferred links
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const uint32_t o = own(i);
            R C0 = R(0), C1 = R(0);
            if (fluid && o < OWN_WALL) {
                if (kDefer && o != p1 && o != p2) {
                    rare |= 1u << i;
                } else {
                    L Ux = o == p1 ? Ux1 : Ux2, Uy = o == p1 ? Uy1 : Uy2, Uz = o == p1 ? Uz1 : Uz2;
                    int cb = o == p1 ? cb1 : cb2;
                    if (!kDefer && o != p1 && o != p2) {
                        const double* po = pfast + (size_t)o * kPF;
                        const double X[3] = {po[PF_X], po[PF_X + 1], po[PF_X + 2]};
                        const double rx = minimg((double)x - X[0], nx);
                        const double ry = minimg((double)y - X[1], ny);
                        const double rz = minimg((double)z - X[2], nz);
                        const double wx = po[PF_W], wy = po[PF_W + 1], wz = po[PF_W + 2];
                        Ux = L(po[PF_V] + (wy * rz - wz * ry));
                        Uy = L(po[PF_V + 1] + (wz * rx - wx * rz));
                        Uz = L(po[PF_V + 2] + (wx * ry - wy * rx));
                        int lo[3], sz[3];
                        cb = box_of(bx, X, po[PF_RB], lo, sz) ? rec_cell(xyz, lo, sz, Ls) : -1;
                    }
                    const L cu = Ux * L(cx(i)) + Uy * L(cy(i)) + Uz * L(cz(i));
                    C0 = R(L(-6.0 * wq(i)) * cu) * r0;
                    C1 = R(L(-6.0 * wq(i)) * cu) * r1;
                    // (2 f*_i + C) over both components (f = h + w rho_ref in the deviation forms)
                    const L fsum = L(f0[i]) + L(f1[i]) + L(P::dev ? wq(i) * (bx.rref[0] + bx.rref[1]) : 0.0);
                    const L mag = L(2) * fsum + (L(C0) + L(C1));
                    if (o == p1) {
                        F1[0] += mag * L(cx(i));
                        F1[1] += mag * L(cy(i));
                        F1[2] += mag * L(cz(i));
                    } else if (o == p2) {
                        F2[0] += mag * L(cx(i));
                        F2[1] += mag * L(cy(i));
                        F2[2] += mag * L(cz(i));
                    } else if (cb >= 0) {  // a third particle (rare): this lane alone updates the record
                        double* r = rec + ((size_t)o * rstride + cb) * kRec;
                        r[0] += (double)mag * cx(i);
                        r[1] += (double)mag * cy(i);
                        r[2] += (double)mag * cz(i);
                    }
                }
            } else if (bx.walls == 2 && fluid && o == OWN_WALL) {
                // a moving wall: the same term with the wall velocity
                const double cu = bx.uw[0] * cx(i) + bx.uw[1] * cy(i) + bx.uw[2] * cz(i);
                C0 = R(-6.0 * wq(i) * cu) * r0;
                C1 = R(-6.0 * wq(i) * cu) * r1;
            }
            const uint32_t mb = LBE_NB(i) * (uint32_t)sizeof(S);
            *atw(fd + (size_t)i * N, mb) = P::mk(fluid ? f0[i] + C0 : empty_raw<P>(R(wq(i)) * ref0));
            *atw(fd + (size_t)(Q + i) * N, mb) = P::mk(fluid ? f1[i] + C1 : empty_raw<P>(R(wq(i)) * ref1));
        }
        if (fluid && p1 < OWN_WALL && cb1 >= 0) {
            double* r = rec + ((size_t)p1 * rstride + cb1) * kRec;
            r[0] = F1[0];
            r[1] = F1[1];
            r[2] = F1[2];
        }
        if (fluid && p2 < OWN_WALL && cb2 >= 0) {
            double* r = rec + ((size_t)p2 * rstride + cb2) * kRec;
            r[0] = F2[0];
            r[1] = F2[1];
            r[2] = F2[2];
        }
        if constexpr (kDefer) {
            // deferred links into further particles: the wave visits those
            // particles one at a time; a linked lane reads back the value it
            // has just stored for each such link, adds C, stores it again and
            // writes its cell of that particle's records. The force then uses
            // the stored (rounded) f*_i.
            uint32_t mine = OWN_FLUID;
#pragma unroll
            for (int i = 1; i < Q; i++)
                mine = (((rare >> i) & 1u) && mine == OWN_FLUID) ? s_own[LBE_LS(i)] : mine;
            while (true) {
                const unsigned long long m = __ballot(rare != 0u);
                if (m == 0ull) break;
                const int lead = __ffsll(m) - 1;
                const uint32_t q = __builtin_amdgcn_readfirstlane(__shfl(mine, lead, 64));
                uint32_t sel = 0u, nxt = OWN_FLUID;
#pragma unroll
                for (int i = 1; i < Q; i++) {
                    if ((rare >> i) & 1u) {
                        const uint32_t o = s_own[LBE_LS(i)];
                        if (o == q)
                            sel |= 1u << i;
                        else if (nxt == OWN_FLUID)
                            nxt = o;
                    }
                }
                if (!sel) continue;
                rare &= ~sel;
                mine = nxt;
                const double* po = pfast + (size_t)q * kPF;
                const double X[3] = {po[PF_X], po[PF_X + 1], po[PF_X + 2]};
                const double rx = minimg((double)x - X[0], nx);
                const double ry = minimg((double)y - X[1], ny);
                const double rz = minimg((double)z - X[2], nz);
                const double wx = po[PF_W], wy = po[PF_W + 1], wz = po[PF_W + 2];
                const L Ux = L(po[PF_V] + (wy * rz - wz * ry));
                const L Uy = L(po[PF_V + 1] + (wz * rx - wx * rz));
                const L Uz = L(po[PF_V + 2] + (wx * ry - wy * rx));
                L F[3] = {L(0), L(0), L(0)};
#pragma unroll
                for (int i = 1; i < Q; i++) {
                    if ((sel >> i) & 1u) {
                        const L cu = Ux * L(cx(i)) + Uy * L(cy(i)) + Uz * L(cz(i));
                        const R C0 = R(L(-6.0 * wq(i)) * cu) * r0;
                        const R C1 = R(L(-6.0 * wq(i)) * cu) * r1;
                        const uint32_t mb = LBE_NB(i) * (uint32_t)sizeof(S);
                        S* a0 = atw(fd + (size_t)i * N, mb);
                        S* a1 = atw(fd + (size_t)(Q + i) * N, mb);
                        const R v0 = P::raw(*a0), v1 = P::raw(*a1);
                        *a0 = P::mk(v0 + C0);
                        *a1 = P::mk(v1 + C1);
                        const L fsum = L(v0) + L(v1) + L(P::dev ? wq(i) * (bx.rref[0] + bx.rref[1]) : 0.0);
                        const L mag = L(2) * fsum + (L(C0) + L(C1));
                        F[0] += mag * L(cx(i));
                        F[1] += mag * L(cy(i));
                        F[2] += mag * L(cz(i));
                    }
                }
                int lo[3], sz[3];
                const int cb = box_of(bx, X, po[PF_RB], lo, sz) ? rec_cell(xyz, lo, sz, Ls) : -1;
                if (cb >= 0) {
                    double* r = rec + ((size_t)q * rstride + cb) * kRec;
                    r[0] = F[0];
                    r[1] = F[1];
                    r[2] = F[2];
                }
            }
        }
    }
#undef LBE_NB
#undef LBE_SEL
#undef LBE_LS
}
template <class P, bool SOLID, int BX, int BY>
__global__ __launch_bounds__(256, sizeof(typename P::R) == 8 ? 2 : (sizeof(typename P::S) == 2 ? 4 : 3)) void k_fused(
    Box bx, const typename P::S* __restrict__ fs, typename P::S* __restrict__ fd, const typename P::R* __restrict__ psi,
    const uint32_t* __restrict__ owner, const uint32_t* __restrict__ bm_in, uint32_t* __restrict__ bm_out,
    const double* __restrict__ pfast, double* __restrict__ rec, int rstride, int tiles_x, int tiles_y, int zrun) {
    fused_body<P, SOLID, BX, BY>(bx, fs, fd, psi, owner, bm_in, bm_out, pfast, rec, rstride, tiles_x, tiles_y,
                                 xcd_remap(blockIdx.x, gridDim.x), zrun != 0);
}
// Batched: item = (system, tile); SOLID for the systems with particles.
// Items of one system are contiguous, so the XCD remap keeps neighbouring
// tiles together.
template <class P, bool SOLID, int BX, int BY>
__global__ __launch_bounds__(256, sizeof(typename P::R) == 8 ? 2 : (sizeof(typename P::S) == 2 ? 4 : 3)) void k_fused_batch(
    const SysDev* __restrict__ sd, const WorkItem* __restrict__ items, int c, int o) {
    const WorkItem w = items[xcd_remap(blockIdx.x, gridDim.x)];
    const SysDev& d = sd[w.sys];
    fused_body<P, SOLID, BX, BY>(d.box, (const typename P::S*)d.f[c], (typename P::S*)d.f[1 - c],
                                 (const typename P::R*)d.psi, d.owner[o], d.bmask[c], d.bmask[1 - c], d.pfast, d.rec,
                                 d.kext * d.kext * d.kext, d.tiles_x, d.tiles_y, w.local, false);
}

// Row kernel for boxes without solids (nx a multiple of 64): a block holds
// ROWS whole x-rows of one z-plane (NXT = nx nodes each). Because a block owns
// complete rows, every push can be written aligned: the value a lane stores at
// x comes from the source node x - c_ix, one lane over (wave shuffle; the wave
// edges through LDS, rows wrapping periodically inside the block). Psi of the
// rows y-1 .. y+ROWS in planes z-1..z+1 is staged in LDS.
template <class P, int NXT, int ROWS>
__global__ __launch_bounds__(NXT * ROWS, NXT * ROWS == 256 ? (sizeof(typename P::R) == 8 ? 3 : 4) : 1) void k_fused_rows(
    Box bx, const typename P::S* __restrict__ fs, typename P::S* __restrict__ fd,
    const typename P::R* __restrict__ psi) {
    using R = typename P::R;
    using S = typename P::S;
    constexpr int NT = NXT * ROWS;      // threads per block
    constexpr int NW = NT / 64;         // waves per block
    constexpr int WPR = NXT / 64;       // waves per row
    constexpr int LR = (ROWS + 2) * 3;  // staged rows
    static_assert(NXT % 64 == 0 && NT >= 256 && NT <= 1024, "row kernel shape");
    __shared__ R s_psi[2][LR * NXT];
    // wave-edge values of the 10 directions with c_ix != 0: [wave][slot][comp]
    __shared__ R s_edge[NW][10][2];

    const int ny = bx.ny, nz = bx.nz;
    constexpr int nx = NXT;
    const uint32_t N = (uint32_t)bx.N;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int t = threadIdx.x;
    const int r = t / NXT, x = t - r * NXT;
    const int w = t >> 6, lane = t & 63, wr = (t - r * NXT) >> 6;
    const int row0 = blk * ROWS;
    const int y0 = row0 % ny, z = row0 / ny;
    const int y = y0 + r;
    const uint32_t n = (uint32_t)(x + nx * (y + ny * z));
    const uint32_t nb = n * (uint32_t)sizeof(S);

    R f0[Q], f1[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) {
        f0[i] = P::raw(*at(fs + (size_t)i * N, nb));
        f1[i] = P::raw(*at(fs + (size_t)(Q + i) * N, nb));
    }
    // halo rows: every load of this thread issued before any is waited for
    constexpr int NE = (LR * NXT + NT - 1) / NT;
    R t0[NE], t1[NE];
#pragma unroll
    for (int k = 0; k < NE; k++) {
        const int e = t + NT * k;
        if (e < LR * NXT) {
            const int lrow = e / NXT, xx = e - lrow * NXT;
            const int dz = lrow / (ROWS + 2) - 1, ry = lrow % (ROWS + 2) - 1;
            const int gy = wrapc(y0 + ry, ny), gz = wrapc(z + dz, nz);
            const uint32_t m = (uint32_t)(xx + nx * (gy + ny * gz));
            t0[k] = psi[m];
            t1[k] = psi[N + m];
        }
    }
#pragma unroll
    for (int k = 0; k < NE; k++) {
        const int e = t + NT * k;
        if (e < LR * NXT) {
            s_psi[0][e] = t0[k];
            s_psi[1][e] = t1[k];
        }
    }
    __syncthreads();

    const int xp = x + 1 == nx ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
#define LBE_LS(i) (((1 + cz(i)) * (ROWS + 2) + (r + 1 + cy(i))) * NXT + (cx(i) == 0 ? x : (cx(i) > 0 ? xp : xm)))
    R r0, r1;
    {
        R S0[3], S1[3];
        psi_sums<R>([&](int i) { return s_psi[0][LBE_LS(i)]; }, [&](int i) { return s_psi[1][LBE_LS(i)]; }, S0, S1);
        collide_node<P>(bx, f0, f1, S0, S1, r0, r1);
    }
#undef LBE_LS
    // publish the wave-edge values: lane 63 for c_ix = +1, lane 0 for c_ix = -1
    {
        int sl = 0;
#pragma unroll
        for (int i = 1; i < Q; i++) {
            if (cx(i) == 0) continue;
            const bool mine = (cx(i) > 0) ? (lane == 63) : (lane == 0);
            if (mine) {
                s_edge[w][sl][0] = f0[i];
                s_edge[w][sl][1] = f1[i];
            }
            sl++;
        }
    }
    __syncthreads();
    const int wprev = r * WPR + (wr == 0 ? WPR - 1 : wr - 1);  // wave holding x0 - 1 (periodic)
    const int wnext = r * WPR + (wr == WPR - 1 ? 0 : wr + 1);  // wave holding x0 + 64

    // rest population
    *atw(fd, nb) = P::mk(f0[0]);
    *atw(fd + (size_t)Q * N, nb) = P::mk(f1[0]);
    // aligned row stores: plane i, destination row (y + c_iy, z + c_iz), this x
    const uint32_t pl = (uint32_t)(nx * ny);
    const uint32_t yrow[3] = {(uint32_t)(y * nx), (uint32_t)((y + 1 == ny ? 0 : y + 1) * nx),
                              (uint32_t)((y == 0 ? ny - 1 : y - 1) * nx)};
    const uint32_t zpl[3] = {(uint32_t)z * pl, (uint32_t)(z + 1 == nz ? 0 : z + 1) * pl,
                             (uint32_t)(z == 0 ? nz - 1 : z - 1) * pl};
    int sl = 0;
#pragma unroll
    for (int i = 1; i < Q; i++) {
        R v0 = f0[i], v1 = f1[i];
        if (cx(i) > 0) {
            const R u0 = __shfl_up(v0, 1, 64), u1 = __shfl_up(v1, 1, 64);
            v0 = lane == 0 ? s_edge[wprev][sl][0] : u0;
            v1 = lane == 0 ? s_edge[wprev][sl][1] : u1;
            sl++;
        } else if (cx(i) < 0) {
            const R u0 = __shfl_down(v0, 1, 64), u1 = __shfl_down(v1, 1, 64);
            v0 = lane == 63 ? s_edge[wnext][sl][0] : u0;
            v1 = lane == 63 ? s_edge[wnext][sl][1] : u1;
            sl++;
        }
        const uint32_t mb =
            ((uint32_t)x + yrow[cy(i) == 0 ? 0 : (cy(i) > 0 ? 1 : 2)] + zpl[cz(i) == 0 ? 0 : (cz(i) > 0 ? 1 : 2)]) *
            (uint32_t)sizeof(S);
        *atw(fd + (size_t)i * N, mb) = P::mk(v0);
        *atw(fd + (size_t)(Q + i) * N, mb) = P::mk(v1);
    }
}

// ---------------------------------------------------------------- init
template <class P>
__global__ __launch_bounds__(256) void k_init(Box bx, typename P::S* __restrict__ f, const double* __restrict__ ra,
                                              const double* __restrict__ rb, const double* __restrict__ u,
                                              const uint32_t* __restrict__ owner) {
    const int64_t N = bx.N;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const bool fluid = owner[n] == OWN_FLUID;
    const double ux = u ? u[3 * n] : 0.0, uy = u ? u[3 * n + 1] : 0.0, uz = u ? u[3 * n + 2] : 0.0;
    const double uu = ux * ux + uy * uy + uz * uz;
    const double rr[2] = {ra[n], rb[n]};
#pragma unroll
    for (int c = 0; c < 2; c++) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const double v = fluid ? feq_i<double>(i, rr[c], ux, uy, uz, uu) : 0.0;
            f[(size_t)(c * Q + i) * N + n] = enc64<P>(v, wq(i) * bx.rref[c]);
        }
    }
}

// ---------------------------------------------------------------- readout
template <class P>
__global__ __launch_bounds__(256) void k_fields(Box bx, const typename P::S* __restrict__ f,
                                                const uint32_t* __restrict__ owner,
                                                const uint32_t* __restrict__ bmask, double* __restrict__ out) {
    using R = typename P::R;
    const int64_t N = bx.N;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double r[2] = {0.0, 0.0}, j[3] = {0.0, 0.0, 0.0};
    const bool fluid = owner[n] == OWN_FLUID;
    if (fluid) {
        const uint32_t bm = bmask[n];
        int x, y, z;
        node_xyz(bx, (uint32_t)n, x, y, z);
#pragma unroll
        for (int c = 0; c < 2; c++) {
#pragma unroll
            for (int i = 0; i < Q; i++) {
                int pi;
                uint32_t m;
                pop_src(bx, (uint32_t)n, x, y, z, bm, i, pi, m);
                const double v = pop64<P>(f[(size_t)(c * Q + pi) * N + m], wq(i) * bx.rref[c]);
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

// Owner codes as the ABI reports them: -1 fluid, -2 wall, else the particle index.
__global__ void k_owner_codes(const uint32_t* __restrict__ owner, int32_t* __restrict__ out, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t o = owner[k];
        out[k] = o == OWN_FLUID ? -1 : (o == OWN_WALL ? -2 : (int32_t)o);
    }
}
hipError_t launch_owner_codes(lb_handle* h, int32_t* dev_out) {
    unsigned g = (unsigned)std::min<int64_t>((h->box.N + 255) / 256, 65536);
    hipLaunchKernelGGL(k_owner_codes, dim3(g), dim3(256), 0, h->stream, h->b.owner[h->ocur], dev_out, h->box.N);
    return hipGetLastError();
}

// Deterministic reduction: fixed grid, per-block LDS tree, then one ordered pass.
template <class P>
__global__ __launch_bounds__(256) void k_stats_partial(Box bx, const typename P::S* __restrict__ f,
                                                       const uint32_t* __restrict__ owner,
                                                       const uint32_t* __restrict__ bmask, double* __restrict__ red) {
    using R = typename P::R;
    const int64_t N = bx.N;
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        if (owner[n] != OWN_FLUID) continue;
        acc[5] += 1.0;
        const uint32_t bm = bmask[n];
        int x, y, z;
        node_xyz(bx, (uint32_t)n, x, y, z);
#pragma unroll
        for (int c = 0; c < 2; c++) {
            double r = 0.0;
#pragma unroll
            for (int i = 0; i < Q; i++) {
                int pi;
                uint32_t m;
                pop_src(bx, (uint32_t)n, x, y, z, bm, i, pi, m);
                const double v = pop64<P>(f[(size_t)(c * Q + pi) * N + m], wq(i) * bx.rref[c]);
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

// Remove the fluid on nodes covered at particle placement (the removed mass is
// measured by fixed-order reductions before and after).
template <class P>
__global__ __launch_bounds__(256) void k_remove_covered(Box bx, typename P::S* __restrict__ f,
                                                        const uint32_t* __restrict__ owner) {
    const int64_t N = bx.N;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N || owner[n] == OWN_FLUID) return;
#pragma unroll
    for (int c = 0; c < 2; c++) {
#pragma unroll
        for (int i = 0; i < Q; i++) f[(size_t)(c * Q + i) * N + n] = enc64<P>(0.0, wq(i) * bx.rref[c]);
    }
}

// Plain form: the populations of every fluid node, read where its bounce
// mask puts them, copied into its own slots of the other population copy
// (zeros on solid nodes); the masks are then all zero. Stored values are
// copied bit for bit (w_ibar = w_i).
template <class P>
__global__ __launch_bounds__(256) void k_canonical(Box bx, const typename P::S* __restrict__ fs,
                                                   typename P::S* __restrict__ fd, const uint32_t* __restrict__ owner,
                                                   uint32_t* __restrict__ bmask) {
    using S = typename P::S;
    const int64_t N = bx.N;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const bool fluid = owner[n] == OWN_FLUID;
    const uint32_t bm = fluid ? bmask[n] : 0u;
    int x, y, z;
    node_xyz(bx, (uint32_t)n, x, y, z);
    for (int c = 0; c < 2; c++) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
            int pi;
            uint32_t m;
            pop_src(bx, (uint32_t)n, x, y, z, bm, i, pi, m);
            const S v = fluid ? fs[(size_t)(c * Q + pi) * N + m] : enc64<P>(0.0, wq(i) * bx.rref[c]);
            fd[(size_t)(c * Q + i) * N + n] = v;
        }
    }
    bmask[n] = 0u;
}

__global__ void k_copy16(const uint4* __restrict__ a, uint4* __restrict__ b, size_t n) {
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        b[k] = a[k];
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
    const size_t n = bytes / 16;
    unsigned g = (unsigned)std::min<size_t>((n + 255) / 256, 1u << 20);
    if (g == 0) g = 1;
    hipLaunchKernelGGL(k_copy16, dim3(g), dim3(256), 0, st, (const uint4*)src, (uint4*)dst, n);
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}
// Batched clear of owner copy `o`: item = (system, block of 256 nodes).
__global__ __launch_bounds__(256) void k_clear_owner_batch(const SysDev* __restrict__ sd,
                                                           const WorkItem* __restrict__ items, int o) {
    const WorkItem w = items[blockIdx.x];
    const SysDev& d = sd[w.sys];
    const int64_t n = (int64_t)w.local * 256 + threadIdx.x;
    if (n < d.box.N) d.owner[o][n] = (d.box.walls && d.owner[1 - o][n] == OWN_WALL) ? OWN_WALL : OWN_FLUID;
}
// Eq. (10) for wall nodes (colour 0): a wall node with fluid neighbours
// (over the 18 links) takes their mean density, stored as Psi; 0 without
// fluid neighbours. Densities of fluid nodes: the stored rho where kept, else
// Psi itself (Psi = rho) or recovered from it (all as kept values).
template <class R>
__device__ inline void wall_shell_node(const Box& bx, R* __restrict__ psi, const R* __restrict__ rho,
                                       const uint32_t* __restrict__ owner, int64_t n) {
    if (owner[n] != OWN_WALL) return;
    const int64_t N = bx.N;
    int x, y, z;
    node_xyz(bx, (uint32_t)n, x, y, z);
    R s0 = R(0), s1 = R(0);
    int k = 0;
    for (int i = 1; i < Q; i++) {
        const uint32_t m = upstream(bx.nx, bx.ny, bx.nz, x, y, z, opp(i));  // n + c_i
        if (owner[m] != OWN_FLUID) continue;
        R d0, d1;
        if (bx.psi_kind == 0) {
            d0 = psi[m];
            d1 = psi[N + m];
        } else if (rho) {
            d0 = rho[m];
            d1 = rho[N + m];
        } else {
            d0 = rho_kept_of_psi(psi[m], 1, R(bx.eref[0]));
            d1 = rho_kept_of_psi(psi[N + m], 1, R(bx.eref[1]));
        }
        s0 += d0;
        s1 += d1;
        k++;
    }
    psi[n] = k == 0 ? R(0) : psi_kept(s0 / R(k), bx.psi_kind, R(bx.eref[0]));
    psi[N + n] = k == 0 ? R(0) : psi_kept(s1 / R(k), bx.psi_kind, R(bx.eref[1]));
}
template <class R>
__global__ __launch_bounds__(256) void k_wall_shell(Box bx, R* __restrict__ psi, const R* __restrict__ rho,
                                                    const uint32_t* __restrict__ owner) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < bx.N) wall_shell_node<R>(bx, psi, rho, owner, n);
}
template <class R>
__global__ __launch_bounds__(256) void k_wall_shell_batch(const SysDev* __restrict__ sd,
                                                          const WorkItem* __restrict__ items, int o) {
    const WorkItem w = items[blockIdx.x];
    const SysDev& d = sd[w.sys];
    if (d.box.walls == 0) return;
    const int64_t n = (int64_t)w.local * 256 + threadIdx.x;
    if (n < d.box.N) wall_shell_node<R>(d.box, (R*)d.psi, (const R*)sys_rho(d), d.owner[o], n);
}
// Owner copy cleared for re-rasterisation, wall nodes kept (from the current copy).
__global__ void k_clear_keep_walls(uint32_t* __restrict__ dst, const uint32_t* __restrict__ cur, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        dst[k] = cur[k] == OWN_WALL ? OWN_WALL : OWN_FLUID;
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
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_fill_u32(h, h->b.bmask[h->cur], 0u, h->box.N);  // populations in plain form
}

// Densities of populations copy `c` on the nodes fluid in owner copy `o`
// (and, when oo >= 0, also fluid in owner copy `oo`).
hipError_t launch_density(lb_handle* h, int c, int o, int oo) {
    void* rho_out = (h->has_solid && h->prm.psi_kind != 0) ? h->b.rho : nullptr;
    const uint32_t* own_old = oo >= 0 ? h->b.owner[oo] : nullptr;
    if (h->has_solid) {
        LBE_DISPATCH(h->prm.precision,
                     hipLaunchKernelGGL((k_density<P, true>), dim3(nblk(h->box.N)), dim3(256), 0, h->stream, h->box,
                                        (const typename P::S*)h->b.f[c], (typename P::R*)h->b.psi,
                                        (typename P::R*)rho_out, h->b.owner[o], own_old, h->b.bmask[c],
                                        h->b.health));
    } else {
        LBE_DISPATCH(h->prm.precision,
                     hipLaunchKernelGGL((k_density<P, false>), dim3(nblk(h->box.N)), dim3(256), 0, h->stream, h->box,
                                        (const typename P::S*)h->b.f[c], (typename P::R*)h->b.psi,
                                        (typename P::R*)nullptr, h->b.owner[o], nullptr, nullptr, h->b.health));
    }
    return hipGetLastError();
}

Tiles fused_tiles(int nx, int ny, bool solids, int precision) {
    Tiles t;
    // Boxes without solids whose rows fill whole blocks use the row kernel
    // (aligned stores) for 4- and 2-byte populations, and for FP64 on rows of
    // up to 128 nodes (three waves per SIMD; 128^3: 0.236 against 0.245 ms).
    // Wider FP64 rows and boxes with solids use the tile kernel (256^3 FP64:
    // 2.09 against 2.17 ms for the row kernel).
    if (!solids && (precision != LB_FP64 || nx <= 128) &&
        ((nx == 64 && ny % 4 == 0) || (nx == 128 && ny % 2 == 0) || nx == 256 || nx == 512)) {
        // row kernel: whole x-rows per block
        t.BX = nx;
        t.BY = nx >= 256 ? 1 : 256 / nx;
        t.tiles_x = 1;
        t.tiles_y = ny / t.BY;
        return t;
    }
    t.BX = nx >= 64 ? 64 : 32;
    t.BY = 256 / t.BX;
    t.tiles_x = (nx + t.BX - 1) / t.BX;
    t.tiles_y = (ny + t.BY - 1) / t.BY;
    // z-runs pay for 8- and 4-byte populations on planes of many tiles
    // (256^3 bijel: fused kernel -9 % FP64, -4 % FP32). On a plane of few
    // tiles (128^3: 64) the z-neighbours are in flight together anyway and
    // z-runs only move the y-neighbours away (FP64 +40 %); 2-byte planes are
    // small enough that the plane-by-plane order finds them in L2.
    t.zrun = (precision == LB_FP64 || precision == LB_FP32) && t.tiles_x * t.tiles_y >= 256;
    return t;
}

template <class P, bool SOLID>
static void launch_fused_t(lb_handle* h, const Tiles& tl, unsigned grid) {
    const int o = h->cur, d = 1 - h->cur;
    auto fs = (const typename P::S*)h->b.f[o];
    auto fd = (typename P::S*)h->b.f[d];
    auto ps = (const typename P::R*)h->b.psi;
    const uint32_t* ow = h->b.owner[h->ocur];
    if (!SOLID && tl.tiles_x == 1 && tl.BX >= 64 && tl.BX == h->box.nx) {
        const dim3 blk(tl.BX * tl.BY);
        switch (tl.BX) {
            case 64:
                hipLaunchKernelGGL((k_fused_rows<P, 64, 4>), dim3(grid), blk, 0, h->stream, h->box, fs, fd, ps);
                break;
            case 128:
                hipLaunchKernelGGL((k_fused_rows<P, 128, 2>), dim3(grid), blk, 0, h->stream, h->box, fs, fd, ps);
                break;
            case 256:
                hipLaunchKernelGGL((k_fused_rows<P, 256, 1>), dim3(grid), blk, 0, h->stream, h->box, fs, fd, ps);
                break;
            default:
                hipLaunchKernelGGL((k_fused_rows<P, 512, 1>), dim3(grid), blk, 0, h->stream, h->box, fs, fd, ps);
                break;
        }
        return;
    }
    const int ke = h->np > 0 ? kill_ext(h) : 0;
    const int rstride = ke * ke * ke;
    if (tl.BX == 64)
        hipLaunchKernelGGL((k_fused<P, SOLID, 64, 4>), dim3(grid), dim3(256), 0, h->stream, h->box, fs, fd, ps, ow,
                           h->b.bmask[h->cur], h->b.bmask[1 - h->cur], h->b.pfast, h->b.rec, rstride, tl.tiles_x,
                           tl.tiles_y, tl.zrun ? 1 : 0);
    else
        hipLaunchKernelGGL((k_fused<P, SOLID, 32, 8>), dim3(grid), dim3(256), 0, h->stream, h->box, fs, fd, ps, ow,
                           h->b.bmask[h->cur], h->b.bmask[1 - h->cur], h->b.pfast, h->b.rec, rstride, tl.tiles_x,
                           tl.tiles_y, tl.zrun ? 1 : 0);
}

hipError_t launch_fused(lb_handle* h) {
    const Tiles tl = fused_tiles(h->box.nx, h->box.ny, h->has_solid, h->prm.precision);
    const unsigned grid = (unsigned)(tl.tiles_x * tl.tiles_y * h->box.nz);
    if (h->has_solid) {
        LBE_DISPATCH(h->prm.precision, (launch_fused_t<P, true>(h, tl, grid)));
    } else {
        LBE_DISPATCH(h->prm.precision, (launch_fused_t<P, false>(h, tl, grid)));
    }
    return hipGetLastError();
}

hipError_t launch_fields(lb_handle* h, double* out) {
    LBE_DISPATCH(h->prm.precision,
                 hipLaunchKernelGGL(k_fields<P>, dim3(nblk(h->box.N)), dim3(256), 0, h->stream, h->box,
                                    (const typename P::S*)h->b.f[h->cur], h->b.owner[h->ocur], h->b.bmask[h->cur],
                                    out));
    return hipGetLastError();
}

hipError_t launch_stats(lb_handle* h) {
    LBE_DISPATCH(h->prm.precision,
                 hipLaunchKernelGGL(k_stats_partial<P>, dim3(kRedBlocks), dim3(256), 0, h->stream, h->box,
                                    (const typename P::S*)h->b.f[h->cur], h->b.owner[h->ocur], h->b.bmask[h->cur],
                                    h->b.red));
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, h->stream, h->b.red, kRedBlocks);
    return hipGetLastError();
}

hipError_t launch_canonical(lb_handle* h) {
    if (!h->has_solid) return hipSuccess;  // no solids: every mask is zero
    LBE_DISPATCH(h->prm.precision,
                 hipLaunchKernelGGL(k_canonical<P>, dim3(nblk(h->box.N)), dim3(256), 0, h->stream, h->box,
                                    (const typename P::S*)h->b.f[h->cur], (typename P::S*)h->b.f[1 - h->cur],
                                    h->b.owner[h->ocur], h->b.bmask[h->cur]));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // back into the current copy: the copy index stays as it was (a batch's
    // systems share one parity)
    // (the copies are padded to 256 bytes, so the length rounds up to 16)
    const size_t bytes = (2 * Q * (size_t)h->box.N * elem_bytes(h->prm.precision) + 15) / 16 * 16;
    return launch_copy(h->b.f[h->cur], h->b.f[1 - h->cur], bytes, h->stream);
}

hipError_t launch_remove_covered(lb_handle* h) {
    LBE_DISPATCH(h->prm.precision,
                 hipLaunchKernelGGL(k_remove_covered<P>, dim3(nblk(h->box.N)), dim3(256), 0, h->stream, h->box,
                                    (typename P::S*)h->b.f[h->cur], h->b.owner[h->ocur]));
    return hipGetLastError();
}

hipError_t launch_fill_u32(lb_handle* h, uint32_t* p, uint32_t v, int64_t n) {
    unsigned g = nblk(n);
    if (g > 65536) g = 65536;
    if (g == 0) g = 1;
    hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(256), 0, h->stream, p, v, n);
    return hipGetLastError();
}
hipError_t launch_wall_shell(lb_handle* h) {
    if (!h->box.walls) return hipSuccess;
    const void* rho = (h->has_solid && h->prm.psi_kind != 0) ? h->b.rho : nullptr;
    if (h->prm.precision == LB_FP64)
        hipLaunchKernelGGL(k_wall_shell<double>, dim3(nblk(h->box.N)), dim3(256), 0, h->stream, h->box,
                           (double*)h->b.psi, (const double*)rho, h->b.owner[h->ocur]);
    else
        hipLaunchKernelGGL(k_wall_shell<float>, dim3(nblk(h->box.N)), dim3(256), 0, h->stream, h->box,
                           (float*)h->b.psi, (const float*)rho, h->b.owner[h->ocur]);
    return hipGetLastError();
}
hipError_t launch_batch_wall_shell(const BatchLaunch& bl, int precision, hipStream_t st, int o) {
    if (precision == LB_FP64)
        hipLaunchKernelGGL(k_wall_shell_batch<double>, dim3(bl.n[BI_NODE]), dim3(256), 0, st, bl.sys,
                           bl.items[BI_NODE], o);
    else
        hipLaunchKernelGGL(k_wall_shell_batch<float>, dim3(bl.n[BI_NODE]), dim3(256), 0, st, bl.sys,
                           bl.items[BI_NODE], o);
    return hipGetLastError();
}
hipError_t launch_clear_keep_walls(lb_handle* h, uint32_t* dst, const uint32_t* cur) {
    unsigned g = nblk(h->box.N);
    if (g > 65536) g = 65536;
    if (g == 0) g = 1;
    hipLaunchKernelGGL(k_clear_keep_walls, dim3(g), dim3(256), 0, h->stream, dst, cur, h->box.N);
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

// ---------------------------------------------------------------- batched launchers

hipError_t launch_batch_density(const BatchLaunch& bl, int precision, hipStream_t st, int c, int o, int oo) {
    if (bl.n[BI_NODE] == 0) return hipSuccess;
    LBE_DISPATCH(precision, hipLaunchKernelGGL(k_density_batch<P>, dim3(bl.n[BI_NODE]), dim3(256), 0, st, bl.sys,
                                               bl.items[BI_NODE], c, o, oo));
    return hipGetLastError();
}

template <class P, bool SOLID>
static void launch_batch_fused_t(const BatchLaunch& bl, hipStream_t st, int c, int o) {
    const int k = SOLID ? BI_TILE : BI_TILE_PLAIN;
    if (bl.n[k] == 0) return;
    if (bl.bx == 64)
        hipLaunchKernelGGL((k_fused_batch<P, SOLID, 64, 4>), dim3(bl.n[k]), dim3(256), 0, st, bl.sys, bl.items[k], c,
                           o);
    else if (bl.bx == 32)
        hipLaunchKernelGGL((k_fused_batch<P, SOLID, 32, 8>), dim3(bl.n[k]), dim3(256), 0, st, bl.sys, bl.items[k], c,
                           o);
    else
        hipLaunchKernelGGL((k_fused_batch<P, SOLID, 16, 16>), dim3(bl.n[k]), dim3(256), 0, st, bl.sys, bl.items[k],
                           c, o);
}

hipError_t launch_batch_fused(const BatchLaunch& bl, int precision, hipStream_t st, int c, int o) {
    LBE_DISPATCH(precision, (launch_batch_fused_t<P, true>(bl, st, c, o)));
    LBE_DISPATCH(precision, (launch_batch_fused_t<P, false>(bl, st, c, o)));
    return hipGetLastError();
}

hipError_t launch_batch_clear_owner(const BatchLaunch& bl, hipStream_t st, int o) {
    if (bl.n[BI_NODE] == 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_owner_batch, dim3(bl.n[BI_NODE]), dim3(256), 0, st, bl.sys, bl.items[BI_NODE], o);
    return hipGetLastError();
}

}  // namespace lbe
