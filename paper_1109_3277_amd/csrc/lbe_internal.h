// Host-side internals of liblbe: the handle and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lbe.h"
#include "lbe_device.h"

namespace lbe {

// Device buffers of one system, carved from the caller's workspace.
struct Buffers {
    void* f[2] = {nullptr, nullptr};   // populations [2][19][N] in the storage type
    void* psi = nullptr;               // Psi^c per node [2][N] (double for FP64, float otherwise)
    void* rho = nullptr;               // rho^c per node [2][N], for the shell fill (exponential Psi)
    uint32_t* owner[2] = {nullptr, nullptr};
    double* part = nullptr;            // particle table, NPFIELD x cap
    uint2* slist = nullptr;            // surface list segments, cap x nslab(raster) x 64 (node, link mask)
    int* scount = nullptr;             // entries per surface list segment, cap x nslab(raster)
    double* kpart = nullptr;           // kill/fill impulse partial slots, cap x nslab x 6
    double* red = nullptr;             // reduction partials, kRedBlocks x 8, then totals
    double* counters = nullptr;        // [0] mass removed (cumulative), [1] kill mass, [2] fill mass
    int* health = nullptr;             // nonzero once a NaN / negative density was seen
};

constexpr int kRedBlocks = 1024;       // fixed grid of the deterministic reductions

}  // namespace lbe

struct lb_handle {
    lb_params prm;
    lbe::Box box;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    lbe::Buffers b;
    int cur = 0;         // index of the current population buffer
    int ocur = 0;        // index of the current owner map
    int np = 0, cap = 0;
    double rmax = 0.0;   // largest bounding radius of any particle
    int64_t kpart_len = 0;  // doubles in the kill/fill slot buffer
    bool inited = false;
    bool has_solid = false;
    std::string err;
    // phase timing (lb_profile_*)
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;      // created lazily, reused
    std::vector<std::pair<int, int>> ev_marks;  // (phase, index of start event); end = start + 1
    size_t ev_used = 0;
};

namespace lbe {

size_t elem_bytes(int precision);
size_t rho_elem_bytes(int precision);

// Launchers (all enqueue on h->stream; return hipSuccess or the launch error).
hipError_t launch_init(lb_handle* h, const double* d_rho_a, const double* d_rho_b, const double* d_u);
hipError_t launch_density(lb_handle* h);
hipError_t launch_shell(lb_handle* h);
hipError_t launch_fused(lb_handle* h);
hipError_t launch_forces(lb_handle* h);
Tiles fused_tiles(int nx, int ny, bool solids, int precision);
hipError_t launch_fields(lb_handle* h, double* d_out);       // rho_a, rho_b, u (5 x N doubles)
hipError_t launch_stats(lb_handle* h);                       // totals into b.red[kRedBlocks*8 ...]
hipError_t launch_remove_covered(lb_handle* h);
hipError_t launch_bodies(lb_handle* h);
hipError_t launch_raster(lb_handle* h, uint32_t* owner, int first, int count);
hipError_t launch_clear_owner(lb_handle* h, uint32_t* owner);
hipError_t launch_killfill(lb_handle* h);
hipError_t launch_fold_impulses(lb_handle* h);
Slab make_slab(int ext);
int raster_extent(int nx, int ny, int nz, double rb);
int killfill_extent(int nx, int ny, int nz, double rb);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
hipError_t launch_fill_u32(lb_handle* h, uint32_t* p, uint32_t v, int64_t n);
hipError_t launch_fill_f64(lb_handle* h, double* p, double v, int64_t n);

}  // namespace lbe
