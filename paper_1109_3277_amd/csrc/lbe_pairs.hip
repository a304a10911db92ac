// Particle-particle interactions of liblbe (gfx950): Hertz repulsion extended
// to ellipsoids after Berne and Pechukas, and the lubrication correction
// (Sec. 2, Eqs. (6)-(9)), with a device cell list.
//
// Each step, before the rigid-body update: the particle centres are binned
// into cells of edge >= the interaction range (count, scan, fill, then each
// cell's list sorted by particle index so that every sum below runs in a
// fixed order), and one thread per particle sums, over the particles of the
// 27 neighbouring cells (fewer when the box holds fewer than three cells
// along an axis), the force and torque every pair exerts on it. The results
// go to the particle table's pair fields, which the body update adds.
//
// Pair (i, j), r = minimum image of X_i - X_j, u = r / |r|, o the body axes:
//   Hertz (Eq. (6)) eps phi~(|r| / sigma), phi~(x) = (1 - x)^{5/2} for x < 1,
//   eps = eps_bar / sqrt(1 - chi^2 (o_i.o_j)^2), sigma = sigma_bar /
//   sqrt(1 - chi/2 G), G = (a + b)^2 / (1 + chi c) + (a - b)^2 / (1 - chi c),
//   a = u.o_i, b = u.o_j, c = o_i.o_j (Eqs. (7)-(8)), sigma_bar = 2 R_o,
//   eps_bar = K_H sigma_bar^{5/2}, chi = (R_p^2 - R_o^2) / (R_p^2 + R_o^2), with
//   R_p and R_o the means of the pair's; force on i = -d phi / d X_i, torque
//   on i = -o_i x d phi / d o_i.
//   Lubrication (Eq. (9)) for a gap h = |r| - sigma < Delta_c: force on i
//   -(3 pi mu R^2 / 2) u (u.(V_i - V_j)) (1/h - 1/Delta_c), R = sigma / 2,
//   h no smaller than Delta_c / 4, mu = (rho_A + rho_B)(tau - 1/2) / 3 from
//   the initial mean densities.
#include <math.h>

#include <algorithm>

#include "lbe_internal.h"

namespace lbe {

__device__ inline void body_axis(const double* part, int cap, int p, double o[3]) {
    const double w = part[QW * cap + p], x = part[QX * cap + p], y = part[QY * cap + p], z = part[QZ * cap + p];
    o[0] = 2.0 * (x * z + w * y);
    o[1] = 2.0 * (y * z - w * x);
    o[2] = 1.0 - 2.0 * (x * x + y * y);
}

// Force on i and torque on i of pair (i, j); r = X_i - X_j (minimum image).
__device__ inline void pair_on_i(const Box& bx, const double* part, int cap, int i, int j, const double r[3],
                                 double F[3], double T[3]) {
    const double rp = 0.5 * (part[RPAR * cap + i] + part[RPAR * cap + j]);
    const double ro = 0.5 * (part[RPERP * cap + i] + part[RPERP * cap + j]);
    const double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rn < 2.0 * fmax(rp, ro) + bx.delta_c) || rn == 0.0) return;
    const double chi = (rp * rp - ro * ro) / (rp * rp + ro * ro);
    const double sbar = 2.0 * ro;
    const double u[3] = {r[0] / rn, r[1] / rn, r[2] / rn};
    double oi[3], oj[3];
    body_axis(part, cap, i, oi);
    body_axis(part, cap, j, oj);
    const double a = u[0] * oi[0] + u[1] * oi[1] + u[2] * oi[2];
    const double b = u[0] * oj[0] + u[1] * oj[1] + u[2] * oj[2];
    const double c = oi[0] * oj[0] + oi[1] * oj[1] + oi[2] * oj[2];
    const double cp = 1.0 + chi * c, cm = 1.0 - chi * c;
    const double G = (a + b) * (a + b) / cp + (a - b) * (a - b) / cm;
    const double sig = sbar / sqrt(1.0 - 0.5 * chi * G);
    const double x = rn / sig;
    if (x < 1.0) {  // Hertz / Berne-Pechukas
        const double ebar = bx.K_H * pow(sbar, 2.5);
        const double den = 1.0 - chi * chi * c * c;
        const double eps = ebar / sqrt(den);
        const double ph = pow(1.0 - x, 2.5);
        const double dph = -2.5 * eps * pow(1.0 - x, 1.5);          // d phi / d x
        const double sG = 0.25 * chi * sig * sig * sig / (sbar * sbar);  // d sigma / d G
        const double Ga = 2.0 * (a + b) / cp + 2.0 * (a - b) / cm;
        const double Gb = 2.0 * (a + b) / cp - 2.0 * (a - b) / cm;
        const double Gc = -chi * (a + b) * (a + b) / (cp * cp) + chi * (a - b) * (a - b) / (cm * cm);
        const double ec = ebar * chi * chi * c / pow(den, 1.5);       // d eps / d c
        for (int d = 0; d < 3; d++)
            F[d] -= dph * (u[d] / sig - (sG / (sig * sig)) * (Ga * (oi[d] - a * u[d]) + Gb * (oj[d] - b * u[d])));
        const double k = dph * (-rn / (sig * sig)) * sG;  // d phi / d G
        double g[3];
        for (int d = 0; d < 3; d++) g[d] = (ec * ph + k * Gc) * oj[d] + k * Ga * u[d];  // d phi / d o_i
        T[0] -= oi[1] * g[2] - oi[2] * g[1];
        T[1] -= oi[2] * g[0] - oi[0] * g[2];
        T[2] -= oi[0] * g[1] - oi[1] * g[0];
    }
    double h = rn - sig;
    if (h < bx.delta_c) {  // lubrication
        if (h < 0.25 * bx.delta_c) h = 0.25 * bx.delta_c;
        const double mu = (bx.rmean0[0] + bx.rmean0[1]) * (bx.tau - 0.5) / 3.0;
        const double R = 0.5 * sig;
        double un = 0.0;
        for (int d = 0; d < 3; d++) un += u[d] * (part[(VX + d) * cap + i] - part[(VX + d) * cap + j]);
        const double mag = -1.5 * M_PI * mu * R * R * un * (1.0 / h - 1.0 / bx.delta_c);
        for (int d = 0; d < 3; d++) F[d] += mag * u[d];
    }
}

__device__ inline int cell_axis(double x, int L, int nc) {
    int c = (int)floor(x * (double)nc / (double)L);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ void k_cell_count(Box bx, const double* __restrict__ part, int cap, int np, CellGrid cg,
                             int* __restrict__ count, int* __restrict__ pcell) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int c = (cell_axis(part[PZ * cap + p], bx.nz, cg.nc[2]) * cg.nc[1] +
                   cell_axis(part[PY * cap + p], bx.ny, cg.nc[1])) * cg.nc[0] +
                  cell_axis(part[PX * cap + p], bx.nx, cg.nc[0]);
    pcell[p] = c;
    atomicAdd(count + c, 1);
}

// Exclusive prefix sum of the counts into start[0..ncells] (one block of
// kScanT threads, each over a contiguous chunk, then a scan of the chunk
// totals); the counts are cleared for use as fill cursors.
constexpr int kScanT = 1024;
__global__ __launch_bounds__(kScanT) void k_cell_scan(int* __restrict__ count, int* __restrict__ start, int ncells) {
    __shared__ int tot[kScanT];
    const int t = threadIdx.x;
    const int per = (ncells + kScanT - 1) / kScanT;
    const int a = min(t * per, ncells), b = min(a + per, ncells);
    int s = 0;
    for (int c = a; c < b; c++) s += count[c];
    tot[t] = s;
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int k = 0; k < kScanT; k++) {
            const int v = tot[k];
            tot[k] = run;
            run += v;
        }
        start[ncells] = run;
    }
    __syncthreads();
    int run = tot[t];
    for (int c = a; c < b; c++) {
        start[c] = run;
        run += count[c];
        count[c] = 0;
    }
}

__global__ void k_cell_fill(int np, const int* __restrict__ pcell, const int* __restrict__ start,
                            int* __restrict__ cursor, int* __restrict__ list) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int c = pcell[p];
    list[start[c] + atomicAdd(cursor + c, 1)] = p;
}

// Each cell's particles in increasing index (insertion sort; cells hold few).
__global__ void k_cell_sort(const int* __restrict__ start, int* __restrict__ list, int ncells) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const int a = start[c], b = start[c + 1];
    for (int k = a + 1; k < b; k++) {
        const int v = list[k];
        int m = k - 1;
        while (m >= a && list[m] > v) {
            list[m + 1] = list[m];
            m--;
        }
        list[m + 1] = v;
    }
}

__global__ void k_pairs(Box bx, double* __restrict__ part, int cap, int np, CellGrid cg,
                        const int* __restrict__ start, const int* __restrict__ list, const int* __restrict__ pcell) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const int Ls[3] = {bx.nx, bx.ny, bx.nz};
    const double Xi[3] = {part[PX * cap + i], part[PY * cap + i], part[PZ * cap + i]};
    const int ci = pcell[i];
    const int cc[3] = {ci % cg.nc[0], (ci / cg.nc[0]) % cg.nc[1], ci / (cg.nc[0] * cg.nc[1])};
    double F[3] = {0.0, 0.0, 0.0}, T[3] = {0.0, 0.0, 0.0};
    // neighbour cell offsets per axis: -1, 0, 1 (or 0, 1 / 0 with fewer cells)
    int lo[3], hi[3];
    for (int d = 0; d < 3; d++) {
        lo[d] = cg.nc[d] >= 3 ? -1 : 0;
        hi[d] = cg.nc[d] >= 2 ? 1 : 0;
    }
    for (int dz = lo[2]; dz <= hi[2]; dz++)
        for (int dy = lo[1]; dy <= hi[1]; dy++)
            for (int dx = lo[0]; dx <= hi[0]; dx++) {
                const int c = (wrapc(cc[2] + dz, cg.nc[2]) * cg.nc[1] + wrapc(cc[1] + dy, cg.nc[1])) * cg.nc[0] +
                              wrapc(cc[0] + dx, cg.nc[0]);
                for (int k = start[c]; k < start[c + 1]; k++) {
                    const int j = list[k];
                    if (j == i) continue;
                    const double r[3] = {minimg(Xi[0] - part[PX * cap + j], Ls[0]),
                                         minimg(Xi[1] - part[PY * cap + j], Ls[1]),
                                         minimg(Xi[2] - part[PZ * cap + j], Ls[2])};
                    pair_on_i(bx, part, cap, i, j, r, F, T);
                }
            }
    for (int d = 0; d < 3; d++) {
        part[(PFX + d) * cap + i] = F[d];
        part[(PTX + d) * cap + i] = T[d];
    }
}

// Cells per axis for interaction range `range`: the largest count whose edge
// is at least the range, at most kMaxCellsPerAxis and at most the box side
// (the workspace holds that many).
CellGrid cell_grid(int nx, int ny, int nz, double range) {
    CellGrid g;
    const int Ls[3] = {nx, ny, nz};
    for (int d = 0; d < 3; d++) {
        const double n = range > 0.0 ? floor((double)Ls[d] / range) : (double)kMaxCellsPerAxis;
        g.nc[d] = (int)std::max(1.0, std::min(n, (double)std::min(Ls[d], kMaxCellsPerAxis)));
    }
    return g;
}

hipError_t launch_pairs(lb_handle* h) {
    if (!h->box.pairs || h->np < 2) return hipSuccess;
    const CellGrid cg = cell_grid(h->box.nx, h->box.ny, h->box.nz, 2.0 * h->rmax + h->box.delta_c);
    const int ncells = cg.nc[0] * cg.nc[1] * cg.nc[2];
    int* count = h->b.cells;
    int* start = count + ncells;
    int* pcell = start + ncells + 1;
    int* list = pcell + h->cap;
    const int pb = (h->np + 255) / 256;
    hipError_t e = launch_fill_u32(h, (uint32_t*)count, 0u, ncells);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cell_count, dim3(pb), dim3(256), 0, h->stream, h->box, h->b.part, h->cap, h->np, cg, count,
                       pcell);
    hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(kScanT), 0, h->stream, count, start, ncells);
    hipLaunchKernelGGL(k_cell_fill, dim3(pb), dim3(256), 0, h->stream, h->np, pcell, start, count, list);
    hipLaunchKernelGGL(k_cell_sort, dim3((ncells + 255) / 256), dim3(256), 0, h->stream, start, list, ncells);
    hipLaunchKernelGGL(k_pairs, dim3(pb), dim3(256), 0, h->stream, h->box, h->b.part, h->cap, h->np, cg, start, list,
                       pcell);
    return hipGetLastError();
}

}  // namespace lbe
