// Device-side definitions shared by the HIP kernels of liblbe (gfx950, wave64).
//
// Lattice: D3Q19 (the paper's Sec. 2 uses D3Q19, i = 1..19). This library orders
// the 19 velocities as: 0 rest, 1..9 one member of each opposite pair, and
// 10..18 their opposites, so opp(i) = i + 9 for 1 <= i <= 9 and i - 9 above.
// Weights w_i = 1/3, 1/18 (axis), 1/36 (face diagonal); c_s^2 = 1/3.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace lbe {

constexpr int Q = 19;
constexpr uint32_t OWN_FLUID = 0xFFFFFFFFu;  // owner code of a fluid node
constexpr uint32_t OWN_WALL = 0xFFFFFFFEu;   // static wall node (no particle)

__host__ __device__ constexpr int cx(int i) {
    constexpr int t[Q] = {0, 1, 0, 0, 1, 1, 1, 1, 0, 0, -1, 0, 0, -1, -1, -1, -1, 0, 0};
    return t[i];
}
__host__ __device__ constexpr int cy(int i) {
    constexpr int t[Q] = {0, 0, 1, 0, 1, -1, 0, 0, 1, 1, 0, -1, 0, -1, 1, 0, 0, -1, -1};
    return t[i];
}
__host__ __device__ constexpr int cz(int i) {
    constexpr int t[Q] = {0, 0, 0, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 0, 0, -1, 1, -1, 1};
    return t[i];
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i <= 9 ? i + 9 : i - 9); }
__host__ __device__ constexpr double wq(int i) {
    return i == 0 ? 1.0 / 3.0 : ((cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i)) == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// Particle table: structure of arrays of doubles, field k of particle p at
// part[k * cap + p].
enum PField : int {
    PX = 0, PY, PZ,            // centre
    QW, QX, QY, QZ,            // orientation quaternion
    VX, VY, VZ,                // velocity
    WX, WY, WZ,                // angular velocity (space frame)
    LX, LY, LZ,                // angular momentum (space frame)
    RPAR, RPERP, DRHO, MASS, IPERP, IPAR,
    FX, FY, FZ, TX, TY, TZ,    // bounce-back force / torque of the current step
    JX, JY, JZ, HX, HY, HZ,    // pending kill/fill impulses
    LFX, LFY, LFZ, LTX, LTY, LTZ,  // totals applied in the last body update
    OX, OY, OZ,                // centre before the last body update
    OQW, OQX, OQY, OQZ,        // orientation before the last body update
    KMASS, FMASS,              // fluid mass killed / filled by this particle (cumulative)
    PFX, PFY, PFZ, PTX, PTY, PTZ,  // particle-particle force / torque of the current step
    NPFIELD
};

// Population storage policies. S is the stored type, R the arithmetic type.
// FP64 stores the population f_i itself. The other forms store the deviation
// h_i = f_i - w_i rho_ref^c from the rest state of the component's initial
// mean density, and the collision works on the h_i directly (the moments
// follow from rho^c = rho_ref^c + sum_i h_i and j^c = sum_i h_i c_i, since the
// w_i sum to one and sum_i w_i c_i = 0), so storage and arithmetic rounding
// scale with the deviations, not with the populations.
// raw(s) is the stored number as an R; mk(v) stores an R number.
struct PolF64 {
    using S = double;
    using R = double;
    static constexpr bool dev = false;
    __device__ static R raw(S s) { return s; }
    __device__ static S mk(R v) { return v; }
};
struct PolF32 {
    using S = float;
    using R = float;
    static constexpr bool dev = true;
    __device__ static R raw(S s) { return s; }
    __device__ static S mk(R v) { return v; }
};
struct PolF16 {
    using S = __half;
    using R = float;
    static constexpr bool dev = true;
    __device__ static R raw(S s) { return __half2float(s); }
    __device__ static S mk(R v) { return __float2half_rn(v); }
};
struct PolBF16 {
    using S = __hip_bfloat16;
    using R = float;
    static constexpr bool dev = true;
    __device__ static R raw(S s) { return __bfloat162float(s); }
    __device__ static S mk(R v) { return __float2bfloat16(v); }
};
// Population f_i in double from a stored number (wref = w_i rho_ref^c).
template <class P>
__device__ inline double pop64(typename P::S s, double wref) {
    return P::dev ? (double)P::raw(s) + wref : (double)P::raw(s);
}
// Stored number of population f_i given in double (the deviation is formed in
// double, then rounded once).
template <class P>
__device__ inline typename P::S enc64(double f, double wref) {
    return P::mk(typename P::R(P::dev ? f - wref : f));
}
// Stored number of an empty slot (f_i = 0), in the arithmetic type.
template <class P>
__device__ inline typename P::R empty_raw(typename P::R wref) {
    return P::dev ? -wref : typename P::R(0);
}

// Everything a kernel needs to know about one periodic box.
struct Box {
    int nx, ny, nz;
    int64_t N;       // nx*ny*nz
    double tau;
    double omega;    // 1 / tau
    double g;        // g_br
    int psi_kind;    // 0: Psi = rho, 1: Psi = 1 - exp(-rho)
    double ax, ay, az;  // body acceleration
    double rref[2];  // deviation reference density per component
    double eref[2];  // exp(-rref): Psi(rref) = 1 - eref for the exponential form
    double rmean0[2];  // initial global mean density per component
    double uw[3];    // velocity of the static-solid (wall) nodes
    int walls;       // 0: no wall nodes, 1: resting walls, 2: moving walls
    int pairs;       // particle-particle interactions on (Eqs. (6)-(9))
    double K_H;      // Hertz constant
    double delta_c;  // lubrication cut-off
};

// Element at a 32-bit byte offset from a uniform base (lets the compiler use a
// scalar base plus one 32-bit vector offset per access).
template <class T>
__device__ inline const T* at(const T* base, uint32_t byte_off) {
    return (const T*)((const char*)base + byte_off);
}
template <class T>
__device__ inline T* atw(T* base, uint32_t byte_off) {
    return (T*)((char*)base + byte_off);
}

__device__ inline int wrapc(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }
// Streaming with solids: every node pushes all of its populations to
// (i, n + c_i); a population sent into a solid node is stored there already
// bounced back (Eq. (4)). The bounce mask of a fluid node has bit i set when
// its neighbour n - c_i was solid at that push: population i after streaming
// then sits in plane ibar at n - c_i (where the node sent its population ibar)
// instead of in plane i at n. Node index of n - c_i:
__device__ inline uint32_t upstream(int nx, int ny, int nz, int x, int y, int z, int i) {
    return (uint32_t)(wrapc(x - cx(i), nx) + nx * (wrapc(y - cy(i), ny) + ny * wrapc(z - cz(i), nz)));
}
// Plane and node holding population i of fluid node n (coordinates x, y, z)
// after streaming, given its bounce mask bm.
__device__ inline void pop_src(const Box& bx, uint32_t n, int x, int y, int z, uint32_t bm, int i, int& plane,
                               uint32_t& node) {
    if ((bm >> i) & 1u) {
        plane = opp(i);
        node = upstream(bx.nx, bx.ny, bx.nz, x, y, z, i);
    } else {
        plane = i;
        node = n;
    }
}
__device__ inline void node_xyz(const Box& bx, uint32_t n, int& x, int& y, int& z) {
    const uint32_t pl = (uint32_t)bx.nx * (uint32_t)bx.ny;
    z = (int)(n / pl);
    const uint32_t r = n - (uint32_t)z * pl;
    y = (int)(r / (uint32_t)bx.nx);
    x = (int)(r - (uint32_t)y * (uint32_t)bx.nx);
}
// periodic wrap of any integer coordinate
__device__ inline int wrapc_any(int a, int n) {
    a %= n;
    return a < 0 ? a + n : a;
}

// Minimum-image difference along one periodic axis of length L.
__device__ inline double minimg(double d, int L) {
    double h = 0.5 * (double)L;
    if (d > h) return d - (double)L;
    if (d < -h) return d + (double)L;
    return d;
}

template <class R>
__device__ inline R psi_of(R r, int kind) {
    if (kind == 0) return r;
    return -expm1(-r);
}
// Inverse of psi_of: rho = -log(1 - Psi) for the exponential form.
template <class R>
__device__ inline R rho_of_psi(R p, int kind) {
    return kind == 0 ? p : -log1p(-p);
}
// Psi(rho)/rho, equal to 1 at rho = 0 for both kinds.
template <class R>
__device__ inline R psi_ratio(R r, int kind) {
    if (kind == 0) return R(1);
    if (r == R(0)) return R(1);
    return -expm1(-r) / r;
}

// Densities rho^c and effective masses Psi^c of Eq. (3) kept per node (the
// density pass, the shell fills and kill / fill write them; the force stencil
// and the shell fills read them). FP64 keeps the values themselves. The float
// forms keep their deviations from the reference state, rho - rho_ref^c and
// Psi(rho) - Psi(rho_ref^c): the force needs only differences of Psi between
// neighbours (sum_i c_i = 0), which then carry no rounding of the large common
// part. A kept density d is the deviation in the float forms; eref =
// exp(-rho_ref^c).
template <class R>
__device__ inline constexpr bool kept_dev() {
    return sizeof(R) != sizeof(double);
}
template <class R>
__device__ inline R psi_kept(R d, int kind, R eref) {
    if (!kept_dev<R>()) return psi_of(d, kind);
    return kind == 0 ? d : -eref * expm1(-d);  // e^-ref - e^-(ref + d)
}
// Kept density from a kept Psi value (the inverse of psi_kept).
template <class R>
__device__ inline R rho_kept_of_psi(R p, int kind, R eref) {
    if (!kept_dev<R>()) return rho_of_psi(p, kind);
    return kind == 0 ? p : -log1p(-p / eref);
}
// The density itself from a kept density.
template <class R>
__device__ inline double rho_full(R d, double ref) {
    return kept_dev<R>() ? (double)d + ref : (double)d;
}

// Bounding box of a particle with centre X and bounding radius rb: first
// node lo[d] and extent sz[d] per axis; false if the state is not usable
// (then nothing is touched).
__device__ inline bool box_of(const Box& bx, const double X[3], double rb, int lo[3], int sz[3]) {
    const int Ls[3] = {bx.nx, bx.ny, bx.nz};
    for (int d = 0; d < 3; d++) {
        if (!isfinite(X[d]) || !(rb < 0.5 * Ls[d])) return false;
        lo[d] = (int)ceil(X[d] - rb);
        sz[d] = max(0, min((int)floor(X[d] + rb) - lo[d] + 1, Ls[d]));
    }
    return true;
}
__device__ inline double bound_radius(const double* part, int cap, int p) {
    const double rpar = part[RPAR * cap + p], rperp = part[RPERP * cap + p];
    return rpar > rperp ? rpar : rperp;
}
__device__ inline bool particle_box(const Box& bx, const double* part, int cap, int p, int lo[3], int sz[3]) {
    const double X[3] = {part[PX * cap + p], part[PY * cap + p], part[PZ * cap + p]};
    return box_of(bx, X, bound_radius(part, cap, p), lo, sz);
}

// Packed copy of what the fused kernel reads of a particle: kPF doubles per
// particle (one 128-byte line), centre, velocity, angular velocity and
// bounding radius, so that a wave reads a particle with one scalar load.
// Rewritten whenever the particle table changes (body update, placement,
// state load).
constexpr int kPF = 16;
enum PFastField : int { PF_X = 0, PF_V = 3, PF_W = 6, PF_RB = 9 };
__device__ inline void pack_fast(const double* part, int cap, int p, double* __restrict__ pfast) {
    double* o = pfast + (size_t)p * kPF;
    const int src[9] = {PX, PY, PZ, VX, VY, VZ, WX, WY, WZ};
    for (int k = 0; k < 9; k++) o[k] = part[src[k] * cap + p];
    o[PF_RB] = bound_radius(part, cap, p);
    for (int k = PF_RB + 1; k < kPF; k++) o[k] = 0.0;
}

// Tiles of the fused kernel: BX x BY nodes of one xy-plane per 256-thread
// block (or, for the row kernel, BY whole x-rows of BX = nx nodes).
struct Tiles {
    int BX, BY, tiles_x, tiles_y;
    bool zrun = false;  // tile kernel: walk z before y (see fused_body)
};

// Per-particle kernels run one block of kPB threads per particle, looping
// over the nodes of the particle's box in chunks of kPB nodes.
constexpr int kPB = 256;

// Link records of a particle: one record of kRec doubles per node of its
// record box (its bounding box grown by one node on every side, each edge at
// most the lattice edge; x fastest). The record of fluid node n holds the
// node's momentum-exchange force on the particle, the sum over its links
// n -> n + c_i into the particle of (2 f*_i + C) c_i over both components.
// Records are zero between steps: the fused kernel writes those of its links,
// the force pass reads and clears them.
constexpr int kRec = 3;

// Record cell of node xyz for a particle whose bounding box is (lo, sz), or
// -1 when the node lies outside the record box.
__device__ inline int rec_cell(const int xyz[3], const int lo[3], const int sz[3], const int Ls[3]) {
    int off[3], esz[3];
    bool in = true;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        int v = xyz[d] - (lo[d] - 1);  // in (-L, 2L) for a centre in [0, L) and rb < L / 2
        v = v < 0 ? v + Ls[d] : (v >= Ls[d] ? v - Ls[d] : v);
        esz[d] = min(sz[d] + 2, Ls[d]);
        off[d] = v;
        in = in && (unsigned)v < (unsigned)esz[d];
    }
    return in ? (off[2] * esz[1] + off[1]) * esz[0] + off[0] : -1;
}

// Node (ix, iy, iz) of box index t in a box of sz[0] x sz[1] x sz[2].
__device__ inline void box_node(int t, const int sz[3], int& ix, int& iy, int& iz) {
    ix = t % sz[0];
    const int r = t / sz[0];
    iy = r % sz[1];
    iz = r / sz[1];
}

// Walk over a box of nodes (sz nodes from node lo, x fastest, periodic):
// box index t = t0, t0 + step, ... without a division per node. The step is
// split once into mixed-radix digits and added with carries; coordinates wrap
// with one compare (the origin is wrapped once).
struct BoxWalk {
    int s0, s1, a0, a1, a2;  // box extents along x and y, digits of the step
    int ix, iy, iz;          // offsets of the current node in the box
    int b[3], L[3];          // wrapped origin, lattice extents
    __device__ BoxWalk(const int lo[3], const int sz[3], const int Ls[3], int t0, int step) {
        s0 = max(sz[0], 1);
        s1 = max(sz[1], 1);
        a0 = step % s0;
        const int q = step / s0;
        a1 = q % s1;
        a2 = q / s1;
        ix = t0 % s0;
        const int r = t0 / s0;
        iy = r % s1;
        iz = r / s1;
        for (int d = 0; d < 3; d++) {
            b[d] = wrapc_any(lo[d], Ls[d]);
            L[d] = Ls[d];
        }
    }
    __device__ void next() {
        ix += a0;
        int c = ix >= s0 ? 1 : 0;
        ix -= c * s0;
        iy += a1 + c;
        c = iy >= s1 ? 1 : 0;
        iy -= c * s1;
        iz += a2 + c;
    }
    // coordinates of the current node (offsets below the lattice extents)
    __device__ int x() const { return b[0] + ix >= L[0] ? b[0] + ix - L[0] : b[0] + ix; }
    __device__ int y() const { return b[1] + iy >= L[1] ? b[1] + iy - L[1] : b[1] + iy; }
    __device__ int z() const { return b[2] + iz >= L[2] ? b[2] + iz - L[2] : b[2] + iz; }
};

// One system as the batched kernels see it: its box, its buffers (both
// population and owner copies; the launch names the current ones), its
// particle table and its launch geometry.
struct SysDev {
    Box box;
    void* f[2];
    void* psi;
    void* rho;
    uint32_t* owner[2];
    uint32_t* bmask[2];  // bounce masks of population copy 0 / 1
    double* part;
    double* rec;
    double* pfast;
    double* kpart;
    int* health;
    double* counters;  // [0] fluid mass removed at particle placement
    int cap, np;
    int tiles_x, tiles_y;
    int kext;  // largest kill/fill box edge of a normal step
};

// A batched launch: block b works on item items[b] = (system, local block).
struct WorkItem {
    int sys;
    int local;
};

// Deterministic block sum of K doubles (every thread of the block calls it;
// blockDim.x is a multiple of 64). The result is valid in thread 0.
template <int K>
__device__ inline void block_sum(double (&v)[K], double (&out)[K]) {
    __shared__ double sh[16][K];
#pragma unroll
    for (int k = 0; k < K; k++)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    if (lane == 0)
        for (int k = 0; k < K; k++) sh[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < K; k++) {
            double s = 0.0;
            for (int j = 0; j < nw; j++) s += sh[j][k];
            out[k] = s;
        }
}

}  // namespace lbe
