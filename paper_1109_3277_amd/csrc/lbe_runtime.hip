// Host runtime and C ABI of liblbe: parameter checks, workspace carving,
// host <-> device transfers, the per-step kernel sequence and error state.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lbe_internal.h"

using namespace lbe;

namespace {
thread_local std::string g_create_err;
}  // namespace

namespace lbe {

int fail(lb_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    else g_create_err = msg;
    return code;
}

#define LBE_HIP(h, call) LBE_HIP_OR_FAIL(h, call)

bool params_ok(const lb_params* p, std::string* why) {
    if (!p) { *why = "params is NULL"; return false; }
    if (p->nx < 3 || p->ny < 3 || p->nz < 3) { *why = "each dimension must be >= 3"; return false; }
    // in double: exact near the bound, and no overflow for any int32 extents
    if ((double)p->nx * (double)p->ny * (double)p->nz * 8.0 >= 4294967296.0) {
        *why = "too many nodes (one population plane must stay below 4 GiB: N < 2^29)";
        return false;
    }
    if (!(p->tau > 0.5) || !isfinite(p->tau)) { *why = "tau must be finite and > 1/2"; return false; }
    if (!isfinite(p->g_br)) { *why = "g_br must be finite"; return false; }
    if (p->psi_kind != 0 && p->psi_kind != 1) { *why = "psi_kind must be 0 or 1"; return false; }
    if (p->precision < LB_FP64 || p->precision > LB_BF16_DEV) { *why = "unknown precision"; return false; }
    if (p->max_particles < 0) { *why = "max_particles must be >= 0"; return false; }
    if (p->max_particles > 0) {
        const double minL = (double)std::min(p->nx, std::min(p->ny, p->nz));
        if (!(p->max_radius > 0.0) || !(p->max_radius < 0.5 * minL)) {
            *why = "max_radius must be > 0 and < min(nx, ny, nz)/2 when particles are allowed";
            return false;
        }
    }
    return true;
}

Layout layout_of(const lb_params* p) {
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    const size_t cap = (size_t)std::max(p->max_particles, 1);
    Layout L;
    L.f = align_up(2 * Q * N * elem_bytes(p->precision));
    L.psi = align_up(2 * N * rho_elem_bytes(p->precision));
    L.rho = p->max_particles > 0 ? align_up(2 * N * rho_elem_bytes(p->precision)) : 0;
    L.owner = align_up(N * sizeof(uint32_t));
    L.bmask = align_up(N * sizeof(uint32_t));
    L.part = align_up(NPFIELD * cap * sizeof(double));
    L.pfast = align_up(kPF * cap * sizeof(double));
    const double rmax = p->max_particles > 0 ? p->max_radius : 0.5;
    const size_t kext = (size_t)killfill_extent(p->nx, p->ny, p->nz, rmax);
    L.rec = p->max_particles > 0 ? align_up(cap * kext * kext * kext * kRec * sizeof(double)) : 0;
    L.kpart = align_up(cap * 8 * sizeof(double));
    L.red = align_up((kRedBlocks + 1) * 8 * sizeof(double));
    L.counters = align_up(8 * sizeof(double));
    L.health = align_up(sizeof(int));
    // pair cell list: counts and starts of at most kMaxCellsPerAxis^3 cells
    // (one cell per node at most), the cell of each particle and the list
    size_t ncell = 1;
    for (int d : {p->nx, p->ny, p->nz}) ncell *= (size_t)std::min(d, kMaxCellsPerAxis);
    L.cells = p->max_particles > 1 ? align_up((2 * ncell + 1 + 2 * cap) * sizeof(int)) : 0;
    L.total = 2 * L.f + L.psi + L.rho + 2 * L.owner + 2 * L.bmask + L.part + L.pfast + L.rec + L.kpart + L.red +
              L.counters + L.health + L.cells;
    return L;
}

int setup_handle(lb_handle* h, const lb_params* prm, char* ws, size_t ws_bytes, hipStream_t stream) {
    const Layout L = layout_of(prm);
    h->prm = *prm;
    h->stream = stream;
    (void)hipGetDevice(&h->device);
    h->ws = ws;
    h->ws_bytes = ws_bytes;
    h->cap = std::max(prm->max_particles, 1);
    Box& b = h->box;
    b.nx = prm->nx;
    b.ny = prm->ny;
    b.nz = prm->nz;
    b.N = (int64_t)prm->nx * prm->ny * prm->nz;
    b.tau = prm->tau;
    b.omega = 1.0 / prm->tau;
    b.g = prm->g_br;
    b.psi_kind = prm->psi_kind;
    b.ax = b.ay = b.az = 0.0;
    b.rref[0] = b.rref[1] = 0.0;
    b.eref[0] = b.eref[1] = 1.0;
    b.rmean0[0] = b.rmean0[1] = 0.0;
    b.uw[0] = b.uw[1] = b.uw[2] = 0.0;
    b.walls = 0;
    b.pairs = 0;
    b.K_H = 100.0;
    b.delta_c = 2.0 / 3.0;
    char* p = h->ws;
    h->b.f[0] = p; p += L.f;
    h->b.f[1] = p; p += L.f;
    h->b.psi = p; p += L.psi;
    h->b.rho = L.rho ? p : nullptr; p += L.rho;
    h->b.owner[0] = (uint32_t*)p; p += L.owner;
    h->b.owner[1] = (uint32_t*)p; p += L.owner;
    h->b.bmask[0] = (uint32_t*)p; p += L.bmask;
    h->b.bmask[1] = (uint32_t*)p; p += L.bmask;
    h->b.part = (double*)p; p += L.part;
    h->b.pfast = (double*)p; p += L.pfast;
    h->b.rec = L.rec ? (double*)p : nullptr; p += L.rec;
    h->b.kpart = (double*)p; p += L.kpart;
    h->b.red = (double*)p; p += L.red;
    h->b.counters = (double*)p; p += L.counters;
    h->b.health = (int*)p; p += L.health;
    h->b.cells = L.cells ? (int*)p : nullptr; p += L.cells;
    int rc = LB_OK;
    auto chk = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == LB_OK) rc = fail(nullptr, LB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    };
    chk(launch_fill_u32(h, h->b.owner[0], OWN_FLUID, b.N), "clear owner");
    chk(launch_fill_u32(h, h->b.owner[1], OWN_FLUID, b.N), "clear owner");
    chk(launch_fill_u32(h, h->b.bmask[0], 0u, b.N), "clear bounce masks");
    chk(launch_fill_u32(h, h->b.bmask[1], 0u, b.N), "clear bounce masks");
    chk(launch_fill_f64(h, h->b.part, 0.0, (int64_t)NPFIELD * h->cap), "clear particles");
    chk(launch_fill_f64(h, h->b.kpart, 0.0, (int64_t)(L.kpart / sizeof(double))), "clear impulse slots");
    if (L.rec) chk(launch_fill_f64(h, h->b.rec, 0.0, (int64_t)(L.rec / sizeof(double))), "clear link records");
    h->kpart_len = (int64_t)(L.kpart / sizeof(double));
    chk(launch_fill_f64(h, h->b.counters, 0.0, 8), "clear counters");
    chk(launch_fill_u32(h, (uint32_t*)h->b.health, 0u, 1), "clear health");
    chk(hipStreamSynchronize(h->stream), "synchronize");
    return rc;
}

}  // namespace lbe

namespace {

// Staging for host transfers: the population copy that is not current (its
// contents are dead between steps). Large enough for 5N doubles in every form.
void* staging(lb_handle* h) { return h->b.f[1 - h->cur]; }

// Phase timing: a start / end event pair around each launch when enabled.
hipError_t mark(lb_handle* h, int phase, bool start) {
    if (!h->prof_on) return hipSuccess;
    if (start) {
        while (h->ev_pool.size() < h->ev_used + 2) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            h->ev_pool.push_back(e);
        }
        h->ev_marks.emplace_back(phase, (int)h->ev_used);
        h->ev_used += 2;
        return hipEventRecord(h->ev_pool[h->ev_used - 2], h->stream);
    }
    return hipEventRecord(h->ev_pool[h->ev_used - 1], h->stream);
}

// Per-system calls on a batch handle are refused (they go to lb_batch_system).
#define LBE_NOT_BATCH(h) \
    if ((h)->batch) return fail((h), LB_ESTATE, "per-system call on a batch handle: use lb_batch_system")

#define LBE_PHASE(h, ph, call)                  \
    do {                                        \
        LBE_HIP(h, mark(h, ph, true));          \
        LBE_HIP(h, call);                       \
        LBE_HIP(h, mark(h, ph, false));         \
    } while (0)

// One time step. With particles, the densities of the next step are formed
// right after the re-rasterisation (on nodes fluid before and after), so that
// kill / fill reads its neighbours' densities instead of summing their
// populations; the next step then starts from them.
int enqueue_step(lb_handle* h) {
    if (!h->dens_ready) LBE_PHASE(h, 0, launch_density(h, h->cur, h->ocur, -1));
    h->dens_ready = false;
    if (h->np > 0) LBE_PHASE(h, 1, launch_shell(h));
    if (h->box.walls) LBE_PHASE(h, 1, launch_wall_shell(h));
    LBE_PHASE(h, 2, launch_fused(h));
    if (h->np > 0) {
        LBE_PHASE(h, 3, launch_forces(h));
        if (h->box.pairs) LBE_PHASE(h, 3, launch_pairs(h));
        LBE_PHASE(h, 4, launch_bodies(h));
        uint32_t* on = h->b.owner[1 - h->ocur];
        LBE_HIP(h, mark(h, 5, true));
        if (h->box.walls)
            LBE_HIP(h, launch_clear_keep_walls(h, on, h->b.owner[h->ocur]));
        else
            LBE_HIP(h, launch_clear_owner(h, on));
        LBE_HIP(h, launch_raster(h, on, 0, h->np));
        LBE_HIP(h, mark(h, 5, false));
        LBE_PHASE(h, 0, launch_density(h, 1 - h->cur, 1 - h->ocur, h->ocur));
        LBE_PHASE(h, 6, launch_killfill(h));
        h->ocur = 1 - h->ocur;
        h->dens_ready = true;
    }
    h->cur = 1 - h->cur;
    return LB_OK;
}

}  // namespace

extern "C" {

size_t lb_workspace_bytes(const lb_params* prm) {
    std::string why;
    if (!params_ok(prm, &why)) return 0;
    return layout_of(prm).total;
}

int lb_create(const lb_params* prm, void* dev_ws, size_t ws_bytes, void* hip_stream, lb_handle** out) {
    if (!out) return fail(nullptr, LB_EINVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    if (!params_ok(prm, &why)) return fail(nullptr, LB_EINVAL, why);
    if (!dev_ws) return fail(nullptr, LB_EINVAL, "workspace is NULL");
    const Layout L = layout_of(prm);
    if (ws_bytes < L.total)
        return fail(nullptr, LB_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
    if (((uintptr_t)dev_ws) % kAlign != 0) return fail(nullptr, LB_EINVAL, "workspace must be 256-byte aligned");
    lb_handle* h = new lb_handle();
    const int rc = setup_handle(h, prm, (char*)dev_ws, ws_bytes, (hipStream_t)hip_stream);
    if (rc != LB_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return LB_OK;
}

void lb_destroy(lb_handle* h) {
    if (!h || h->parent) return;  // a batch's system handles go with the batch
    if (h->batch) batch_destroy(h);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    delete h;
}

int lb_profile_enable(lb_handle* h, int on) {
    if (!h) return LB_EINVAL;
    LBE_NOT_BATCH(h);
    if (on) {
        h->ev_marks.clear();
        h->ev_used = 0;
    }
    h->prof_on = on != 0;
    return LB_OK;
}

int lb_profile_read(lb_handle* h, double* ms, int64_t* launches) {
    if (!h || !ms || !launches) return LB_EINVAL;
    for (int k = 0; k < LB_NPHASES; k++) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    if (h->ev_used) LBE_HIP(h, hipEventSynchronize(h->ev_pool[h->ev_used - 1]));
    for (const auto& m : h->ev_marks) {
        float t = 0.0f;
        LBE_HIP(h, hipEventElapsedTime(&t, h->ev_pool[m.second], h->ev_pool[m.second + 1]));
        ms[m.first] += (double)t;
        launches[m.first] += 1;
    }
    return LB_OK;
}

int lb_init_fields(lb_handle* h, const double* rho_a, const double* rho_b, const double* u) {
    if (!h) return LB_EINVAL;
    if (h->batch) return fail(h, LB_ESTATE, "initialise each system of a batch through lb_batch_system");
    if (!rho_a || !rho_b) return fail(h, LB_EINVAL, "rho_a and rho_b are required");
    const int64_t N = h->box.N;
    double s[2] = {0.0, 0.0};
    for (int64_t n = 0; n < N; n++) s[0] += rho_a[n];
    for (int64_t n = 0; n < N; n++) s[1] += rho_b[n];
    for (int c = 0; c < 2; c++) {
        h->box.rmean0[c] = s[c] / (double)N;
        h->box.rref[c] = h->box.rmean0[c];
        h->box.eref[c] = exp(-h->box.rref[c]);
    }
    double* st = (double*)staging(h);
    double* d_ra = st;
    double* d_rb = st + N;
    double* d_u = u ? st + 2 * N : nullptr;
    LBE_HIP(h, hipMemcpyAsync(d_ra, rho_a, N * sizeof(double), hipMemcpyHostToDevice, h->stream));
    LBE_HIP(h, hipMemcpyAsync(d_rb, rho_b, N * sizeof(double), hipMemcpyHostToDevice, h->stream));
    if (u) LBE_HIP(h, hipMemcpyAsync(d_u, u, 3 * N * sizeof(double), hipMemcpyHostToDevice, h->stream));
    LBE_HIP(h, launch_init(h, d_ra, d_rb, d_u));
    LBE_HIP(h, hipStreamSynchronize(h->stream));
    h->inited = true;
    h->dens_ready = false;
    batch_touch(h);
    return LB_OK;
}

int lb_add_ellipsoids(lb_handle* h, int32_t n, const double* radii, const double* pos, const double* quat,
                      const double* delta_rho, const double* density) {
    if (!h) return LB_EINVAL;
    if (h->batch) return fail(h, LB_ESTATE, "add particles to each system of a batch through lb_batch_system");
    if (!h->inited) return fail(h, LB_ESTATE, "lb_init_fields must come before lb_add_ellipsoids");
    if (n < 0) return fail(h, LB_EINVAL, "n must be >= 0");
    if (n == 0) return LB_OK;
    if (!radii || !pos || !quat) return fail(h, LB_EINVAL, "radii, pos and quat are required");
    if (h->np + n > h->prm.max_particles) return fail(h, LB_ENOMEM, "particle capacity exceeded");
    const int Ls[3] = {h->box.nx, h->box.ny, h->box.nz};
    const double minL = (double)std::min(Ls[0], std::min(Ls[1], Ls[2]));
    for (int k = 0; k < n; k++) {
        const double a = radii[2 * k], b = radii[2 * k + 1];
        if (!(a > 0.0) || !(b > 0.0) || !isfinite(a) || !isfinite(b))
            return fail(h, LB_EGEOM, "particle " + std::to_string(k) + ": radii must be finite and > 0");
        if (!(std::max(a, b) < 0.5 * minL))
            return fail(h, LB_EGEOM, "particle " + std::to_string(k) + ": bounding radius must be < min(L)/2");
        if (!(std::max(a, b) <= h->prm.max_radius))
            return fail(h, LB_EGEOM, "particle " + std::to_string(k) + ": bounding radius exceeds max_radius");
        for (int d = 0; d < 3; d++)
            if (!isfinite(pos[3 * k + d])) return fail(h, LB_EINVAL, "non-finite particle position");
        const double* q = quat + 4 * k;
        const double qn = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
        if (!(qn > 0.0) || !isfinite(qn)) return fail(h, LB_EINVAL, "quaternion must be finite and nonzero");
        if (delta_rho && !isfinite(delta_rho[k])) return fail(h, LB_EINVAL, "non-finite delta_rho");
        if (density && !(density[k] > 0.0 && isfinite(density[k]))) return fail(h, LB_EINVAL, "density must be > 0");
    }
    // pending kill/fill impulses move into the particle table before the
    // partial-slot layout (set by the largest radius) can change
    LBE_HIP(h, launch_fold_impulses(h));
    // plain form first: the removal below clears every solid node's slots,
    // where bounced populations of fluid neighbours may sit
    LBE_HIP(h, launch_canonical(h));
    std::vector<double> t((size_t)NPFIELD * n, 0.0);
    auto F = [&](int field, int k) -> double& { return t[(size_t)field * n + k]; };
    for (int k = 0; k < n; k++) {
        for (int d = 0; d < 3; d++) {
            const double L = (double)Ls[d];
            double v = fmod(pos[3 * k + d], L);
            if (v < 0.0) v += L;
            if (v >= L) v -= L;
            F(PX + d, k) = v;
            F(OX + d, k) = v;
        }
        const double* q = quat + 4 * k;
        {
#pragma clang fp contract(off)
            const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
            F(QW, k) = q[0] / qn;
            F(QX, k) = q[1] / qn;
            F(QY, k) = q[2] / qn;
            F(QZ, k) = q[3] / qn;
            for (int d = 0; d < 4; d++) F(OQW + d, k) = F(QW + d, k);
        }
        const double rpar = radii[2 * k], rperp = radii[2 * k + 1];
        const double dens = density ? density[k] : 1.0;
        F(RPAR, k) = rpar;
        F(RPERP, k) = rperp;
        F(DRHO, k) = delta_rho ? delta_rho[k] : 0.0;
        const double M = dens * (4.0 / 3.0) * M_PI * rpar * rperp * rperp;
        F(MASS, k) = M;
        F(IPERP, k) = M * (rperp * rperp + rpar * rpar) / 5.0;
        F(IPAR, k) = M * (2.0 * rperp * rperp) / 5.0;
        h->rmax = std::max(h->rmax, std::max(rpar, rperp));
    }
    const int first = h->np;
    for (int fld = 0; fld < NPFIELD; fld++)
        LBE_HIP(h, hipMemcpyAsync(h->b.part + (size_t)fld * h->cap + first, &t[(size_t)fld * n], n * sizeof(double),
                                  hipMemcpyHostToDevice, h->stream));
    // fluid mass removed under the new particles: fixed-order totals before
    // and after the removal
    double before[7], after[7], removed = 0.0;
    LBE_HIP(h, launch_stats(h));
    LBE_HIP(h, hipMemcpyAsync(before, h->b.red + kRedBlocks * 8, 7 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    h->np += n;
    h->has_solid = true;
    LBE_HIP(h, launch_pack_fast(h));
    LBE_HIP(h, launch_raster(h, h->b.owner[h->ocur], first, n));
    LBE_HIP(h, launch_remove_covered(h));
    LBE_HIP(h, launch_stats(h));
    LBE_HIP(h, hipMemcpyAsync(after, h->b.red + kRedBlocks * 8, 7 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    LBE_HIP(h, hipMemcpyAsync(&removed, h->b.counters, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    LBE_HIP(h, hipStreamSynchronize(h->stream));
    removed += (before[0] + before[1]) - (after[0] + after[1]);
    LBE_HIP(h, hipMemcpyAsync(h->b.counters, &removed, sizeof(double), hipMemcpyHostToDevice, h->stream));
    LBE_HIP(h, hipStreamSynchronize(h->stream));
    h->dens_ready = false;
    batch_touch(h);
    return LB_OK;
}

int lb_step_async(lb_handle* h, int32_t nsteps) {
    if (!h) return LB_EINVAL;
    if (nsteps < 0) return fail(h, LB_EINVAL, "nsteps must be >= 0");
    if (h->parent) return fail(h, LB_ESTATE, "a system of a batch advances only with its batch (step the batch handle)");
    if (h->batch) return batch_step_async(h, nsteps);
    if (!h->inited) return fail(h, LB_ESTATE, "lb_init_fields must come before lb_step");
    for (int s = 0; s < nsteps; s++) {
        int rc = enqueue_step(h);
        if (rc != LB_OK) return rc;
    }
    return LB_OK;
}

int lb_step(lb_handle* h, int32_t nsteps) {
    int rc = lb_step_async(h, nsteps);
    if (rc != LB_OK) return rc;
    if (h->batch) return batch_health(h);
    int bad = 0;
    LBE_HIP(h, hipMemcpyAsync(&bad, h->b.health, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    LBE_HIP(h, hipStreamSynchronize(h->stream));
    if (bad & 2) return fail(h, LB_EUNSTABLE, "a particle moved more than two lattice spacings in one step");
    if (bad) return fail(h, LB_EUNSTABLE, "NaN or negative density detected");
    return LB_OK;
}

int lb_read_fields(lb_handle* h, double* rho_a, double* rho_b, double* u, int32_t* owner) {
    if (!h) return LB_EINVAL;
    LBE_NOT_BATCH(h);
    if (!h->inited) return fail(h, LB_ESTATE, "fields not initialised");
    const int64_t N = h->box.N;
    double* st = (double*)staging(h);
    if (rho_a || rho_b || u) {
        LBE_HIP(h, launch_fields(h, st));
        if (rho_a) LBE_HIP(h, hipMemcpyAsync(rho_a, st, N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        if (rho_b) LBE_HIP(h, hipMemcpyAsync(rho_b, st + N, N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        if (u) LBE_HIP(h, hipMemcpyAsync(u, st + 2 * N, 3 * N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    }
    if (owner) {
        LBE_HIP(h, hipMemcpyAsync(owner, h->b.owner[h->ocur], N * sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
    }
    LBE_HIP(h, hipStreamSynchronize(h->stream));
    if (owner) {
        for (int64_t n = 0; n < N; n++) {
            const uint32_t o = (uint32_t)owner[n];
            owner[n] = o == OWN_FLUID ? -1 : (o == OWN_WALL ? -2 : (int32_t)o);
        }
    }
    return LB_OK;
}

int lb_read_fields_dev(lb_handle* h, double* dev_rho_a, double* dev_rho_b, double* dev_u, int32_t* dev_owner) {
    if (!h) return LB_EINVAL;
    LBE_NOT_BATCH(h);
    if (!h->inited) return fail(h, LB_ESTATE, "fields not initialised");
    const int64_t N = h->box.N;
    double* st = (double*)staging(h);
    if (dev_rho_a || dev_rho_b || dev_u) {
        LBE_HIP(h, launch_fields(h, st));
        if (dev_rho_a)
            LBE_HIP(h, hipMemcpyAsync(dev_rho_a, st, N * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
        if (dev_rho_b)
            LBE_HIP(h, hipMemcpyAsync(dev_rho_b, st + N, N * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
        if (dev_u)
            LBE_HIP(h, hipMemcpyAsync(dev_u, st + 2 * N, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    }
    if (dev_owner) LBE_HIP(h, launch_owner_codes(h, dev_owner));
    return LB_OK;
}

int lb_num_particles(const lb_handle* h) { return h ? h->np : LB_EINVAL; }

int lb_set_particle_motion(lb_handle* h, int32_t k, const double* vel, const double* omega, const double* angmom) {
    if (!h) return LB_EINVAL;
    LBE_NOT_BATCH(h);
    if (k < 0 || k >= h->np) return fail(h, LB_EINVAL, "particle index out of range");
    const double* src[3] = {vel, omega, angmom};
    const int fld[3] = {VX, WX, LX};
    double v[9];
    for (int a = 0; a < 3; a++)
        for (int d = 0; d < 3; d++) {
            if (src[a] && !isfinite(src[a][d])) return fail(h, LB_EINVAL, "non-finite particle motion");
            v[3 * a + d] = src[a] ? src[a][d] : 0.0;
        }
    for (int a = 0; a < 3; a++)
        if (src[a])
            for (int d = 0; d < 3; d++)
                LBE_HIP(h, hipMemcpyAsync(h->b.part + (size_t)(fld[a] + d) * h->cap + k, &v[3 * a + d], sizeof(double),
                                          hipMemcpyHostToDevice, h->stream));
    LBE_HIP(h, launch_pack_fast(h));
    LBE_HIP(h, hipStreamSynchronize(h->stream));
    return LB_OK;
}

int lb_read_particles(lb_handle* h, double* pos, double* quat, double* vel, double* omega, double* force,
                      double* torque) {
    if (!h) return LB_EINVAL;
    LBE_NOT_BATCH(h);
    const int np = h->np;
    if (np == 0) return LB_OK;
    std::vector<double> t((size_t)NPFIELD * h->cap);
    LBE_HIP(h, hipMemcpyAsync(t.data(), h->b.part, t.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    LBE_HIP(h, hipStreamSynchronize(h->stream));
    auto F = [&](int field, int k) { return t[(size_t)field * h->cap + k]; };
    for (int k = 0; k < np; k++) {
        for (int d = 0; d < 3; d++) {
            if (pos) pos[3 * k + d] = F(PX + d, k);
            if (vel) vel[3 * k + d] = F(VX + d, k);
            if (omega) omega[3 * k + d] = F(WX + d, k);
            if (force) force[3 * k + d] = F(LFX + d, k);
            if (torque) torque[3 * k + d] = F(LTX + d, k);
        }
        if (quat)
            for (int d = 0; d < 4; d++) quat[4 * k + d] = F(QW + d, k);
    }
    return LB_OK;
}

int lb_stats(lb_handle* h, double out[8]) {
    if (!h || !out) return LB_EINVAL;
    LBE_NOT_BATCH(h);
    if (!h->inited) return fail(h, LB_ESTATE, "fields not initialised");
    LBE_HIP(h, launch_stats(h));
    double t[7], c0 = 0.0;
    std::vector<double> km((size_t)h->np), fm((size_t)h->np), kp((size_t)h->np * 8);
    LBE_HIP(h, hipMemcpyAsync(t, h->b.red + kRedBlocks * 8, 7 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    LBE_HIP(h, hipMemcpyAsync(&c0, h->b.counters, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    if (h->np > 0) {
        LBE_HIP(h, hipMemcpyAsync(km.data(), h->b.part + (size_t)KMASS * h->cap, h->np * sizeof(double),
                                  hipMemcpyDeviceToHost, h->stream));
        LBE_HIP(h, hipMemcpyAsync(fm.data(), h->b.part + (size_t)FMASS * h->cap, h->np * sizeof(double),
                                  hipMemcpyDeviceToHost, h->stream));
        LBE_HIP(h, hipMemcpyAsync(kp.data(), h->b.kpart, kp.size() * sizeof(double), hipMemcpyDeviceToHost,
                                  h->stream));
    }
    LBE_HIP(h, hipStreamSynchronize(h->stream));
    // removed at placement, plus killed minus filled by each particle (the
    // last step's amounts still wait in its kill/fill slot), in order
    double removed = c0;
    for (int k = 0; k < h->np; k++) removed += (km[k] + kp[8 * k + 6]) - (fm[k] + kp[8 * k + 7]);
    out[0] = t[0];
    out[1] = t[1];
    out[2] = t[2];
    out[3] = t[3];
    out[4] = t[4];
    out[5] = removed;
    out[6] = t[5];
    out[7] = t[6];
    return LB_OK;
}

int lb_set_body_accel(lb_handle* h, const double a[3]) {
    if (!h || !a) return LB_EINVAL;
    LBE_NOT_BATCH(h);
    for (int d = 0; d < 3; d++)
        if (!isfinite(a[d])) return fail(h, LB_EINVAL, "non-finite acceleration");
    h->box.ax = a[0];
    h->box.ay = a[1];
    h->box.az = a[2];
    batch_touch(h);
    return LB_OK;
}

int lb_set_pair_interactions(lb_handle* h, int on, double K_H, double delta_c) {
    if (!h) return LB_EINVAL;
    LBE_NOT_BATCH(h);
    if (h->parent) return fail(h, LB_ESTATE, "particle-particle interactions are not available on batch systems");
    if (on) {
        if (!(K_H >= 0.0) || !isfinite(K_H)) return fail(h, LB_EINVAL, "K_H must be finite and >= 0");
        if (!(delta_c > 0.0) || !isfinite(delta_c)) return fail(h, LB_EINVAL, "delta_c must be finite and > 0");
        if (h->prm.max_particles < 2) return fail(h, LB_ESTATE, "the workspace holds fewer than two particles");
        h->box.K_H = K_H;
        h->box.delta_c = delta_c;
    } else {
        // clear the pair terms the next body update would otherwise add
        LBE_HIP(h, launch_fill_f64(h, h->b.part + (size_t)PFX * h->cap, 0.0, (int64_t)6 * h->cap));
    }
    h->box.pairs = on ? 1 : 0;
    return LB_OK;
}

int lb_set_static_solid(lb_handle* h, const uint8_t* mask, const double* wall_u) {
    if (!h || !mask) return LB_EINVAL;
    LBE_NOT_BATCH(h);
    if (h->inited) return fail(h, LB_ESTATE, "lb_set_static_solid must come before lb_init_fields");
    double u[3] = {0.0, 0.0, 0.0};
    if (wall_u)
        for (int d = 0; d < 3; d++) {
            if (!isfinite(wall_u[d])) return fail(h, LB_EINVAL, "non-finite wall velocity");
            u[d] = wall_u[d];
        }
    const size_t N = (size_t)h->box.N;
    std::vector<uint32_t> ow(N);
    bool any = false;
    for (size_t n = 0; n < N; n++) {
        ow[n] = mask[n] ? OWN_WALL : OWN_FLUID;
        any = any || mask[n];
    }
    for (int k = 0; k < 2; k++)
        LBE_HIP(h, hipMemcpyAsync(h->b.owner[k], ow.data(), N * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream));
    LBE_HIP(h, hipStreamSynchronize(h->stream));
    for (int d = 0; d < 3; d++) h->box.uw[d] = u[d];
    h->box.walls = !any ? 0 : ((u[0] != 0.0 || u[1] != 0.0 || u[2] != 0.0) ? 2 : 1);
    h->has_solid = h->np > 0 || any;
    batch_touch(h);
    return LB_OK;
}

// State image: [header 8 doubles][populations][owner][particle table][counters 8].
size_t lb_state_bytes(const lb_handle* h) {
    if (!h) return 0;
    const size_t N = (size_t)h->box.N;
    return 8 * sizeof(double) + 2 * Q * N * elem_bytes(h->prm.precision) + N * sizeof(uint32_t) +
           (size_t)NPFIELD * h->cap * sizeof(double) + 8 * sizeof(double);
}

int lb_save_state(lb_handle* h, void* host_buf, size_t bytes) {
    if (!h || !host_buf) return LB_EINVAL;
    LBE_NOT_BATCH(h);
    if (!h->inited) return fail(h, LB_ESTATE, "fields not initialised");
    if (bytes < lb_state_bytes(h)) return fail(h, LB_EINVAL, "buffer too small");
    LBE_HIP(h, launch_fold_impulses(h));
    LBE_HIP(h, launch_canonical(h));  // the state is stored in plain form
    const size_t N = (size_t)h->box.N;
    char* p = (char*)host_buf;
    double hdr[8] = {(double)h->np, h->box.rmean0[0], h->box.rmean0[1], h->box.rref[0], h->box.rref[1], h->rmax,
                     (double)h->prm.precision, (double)N};
    memcpy(p, hdr, sizeof hdr);
    p += sizeof hdr;
    const size_t fb = 2 * Q * N * elem_bytes(h->prm.precision);
    LBE_HIP(h, hipMemcpyAsync(p, h->b.f[h->cur], fb, hipMemcpyDeviceToHost, h->stream));
    p += fb;
    LBE_HIP(h, hipMemcpyAsync(p, h->b.owner[h->ocur], N * sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
    p += N * sizeof(uint32_t);
    const size_t pb = (size_t)NPFIELD * h->cap * sizeof(double);
    LBE_HIP(h, hipMemcpyAsync(p, h->b.part, pb, hipMemcpyDeviceToHost, h->stream));
    p += pb;
    LBE_HIP(h, hipMemcpyAsync(p, h->b.counters, 8 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    LBE_HIP(h, hipStreamSynchronize(h->stream));
    return LB_OK;
}

int lb_load_state(lb_handle* h, const void* host_buf, size_t bytes) {
    if (!h || !host_buf) return LB_EINVAL;
    LBE_NOT_BATCH(h);
    if (bytes < lb_state_bytes(h)) return fail(h, LB_EINVAL, "buffer too small");
    const size_t N = (size_t)h->box.N;
    const char* p = (const char*)host_buf;
    bool any_wall = false;
    double hdr[8];
    memcpy(hdr, p, sizeof hdr);
    p += sizeof hdr;
    if ((int)hdr[6] != h->prm.precision || (size_t)hdr[7] != N || (int)hdr[0] > h->prm.max_particles ||
        (hdr[0] > 0 && !(hdr[5] <= h->prm.max_radius)))
        return fail(h, LB_EINVAL, "state does not match this handle's parameters");
    const size_t fb = 2 * Q * N * elem_bytes(h->prm.precision);
    {
        // owner codes must be fluid, wall, or an index below the particle count
        const uint32_t* ow = (const uint32_t*)(p + fb);
        const uint32_t np = (uint32_t)hdr[0];
        for (size_t n = 0; n < N; n++) {
            if (ow[n] != OWN_FLUID && ow[n] != OWN_WALL && ow[n] >= np)
                return fail(h, LB_EINVAL, "state holds an invalid owner code");
            any_wall = any_wall || ow[n] == OWN_WALL;
        }
    }
    LBE_HIP(h, hipMemcpyAsync(h->b.f[h->cur], p, fb, hipMemcpyHostToDevice, h->stream));
    p += fb;
    LBE_HIP(h, hipMemcpyAsync(h->b.owner[h->ocur], p, N * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream));
    p += N * sizeof(uint32_t);
    const size_t pb = (size_t)NPFIELD * h->cap * sizeof(double);
    LBE_HIP(h, hipMemcpyAsync(h->b.part, p, pb, hipMemcpyHostToDevice, h->stream));
    p += pb;
    LBE_HIP(h, hipMemcpyAsync(h->b.counters, p, 8 * sizeof(double), hipMemcpyHostToDevice, h->stream));
    LBE_HIP(h, launch_fill_u32(h, (uint32_t*)h->b.health, 0u, 1));
    LBE_HIP(h, launch_fill_u32(h, h->b.bmask[h->cur], 0u, (int64_t)N));  // stored in plain form
    LBE_HIP(h, launch_fill_f64(h, h->b.kpart, 0.0, h->kpart_len));
    LBE_HIP(h, hipStreamSynchronize(h->stream));
    h->np = (int)hdr[0];
    h->box.rmean0[0] = hdr[1];
    h->box.rmean0[1] = hdr[2];
    h->box.rref[0] = hdr[3];
    h->box.rref[1] = hdr[4];
    h->box.eref[0] = exp(-hdr[3]);
    h->box.eref[1] = exp(-hdr[4]);
    h->rmax = hdr[5];
    // wall nodes come with the owner map; their velocity is the handle's own
    const bool moving = h->box.uw[0] != 0.0 || h->box.uw[1] != 0.0 || h->box.uw[2] != 0.0;
    h->box.walls = !any_wall ? 0 : (moving ? 2 : 1);
    h->has_solid = h->np > 0 || any_wall;
    LBE_HIP(h, launch_pack_fast(h));
    h->inited = true;
    h->dens_ready = false;
    batch_touch(h);
    return LB_OK;
}

const char* lb_last_error(const lb_handle* h) { return h ? h->err.c_str() : g_create_err.c_str(); }

}  // extern "C"
