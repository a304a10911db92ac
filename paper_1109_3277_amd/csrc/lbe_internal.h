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
    uint32_t* bmask[2] = {nullptr, nullptr};  // bounce masks of population copy 0 / 1 (per node)
    double* part = nullptr;            // particle table, NPFIELD x cap
    double* rec = nullptr;             // link records, cap x kext^3 cells x kRec
    double* pfast = nullptr;           // packed particle copy read by the fused kernel, cap x kPF
    double* kpart = nullptr;           // kill/fill impulse and masses of the last step, cap x 8
    double* red = nullptr;             // reduction partials, kRedBlocks x 8, then totals
    double* counters = nullptr;        // [0] fluid mass removed at particle placement (cumulative)
    int* health = nullptr;             // nonzero once a NaN / negative density was seen
    int* cells = nullptr;              // pair cell list: counts, starts, cell of each particle, list
};

// Cell grid of the particle-particle cell list (cells per axis).
struct CellGrid {
    int nc[3];
};
constexpr int kMaxCellsPerAxis = 64;

constexpr int kRedBlocks = 1024;       // fixed grid of the deterministic reductions

struct BatchState;

// Work-item lists of a batched launch, one per kind of block.
// BI_TILE: tiles of systems with particles; BI_TILE_PLAIN: tiles of systems
// without (they run the kernel a lone handle would run).
enum BatchItems { BI_NODE = 0, BI_TILE, BI_TILE_PLAIN, BI_PART, BI_COUNT };
struct BatchLaunch {
    const SysDev* sys = nullptr;
    const WorkItem* items[BI_COUNT] = {};
    int n[BI_COUNT] = {};
    int bx = 64;  // fused tile width: 64 (64x4) or 32 (32x8)
};

}  // namespace lbe

struct lb_handle {
    lb_params prm;
    lbe::Box box;
    hipStream_t stream = nullptr;
    int device = 0;      // the GPU current at creation
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
    bool dens_ready = false;  // Psi (and rho) of the current populations already computed (end of the last step)
    std::string err;
    // phase timing (lb_profile_*)
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;      // created lazily, reused
    std::vector<std::pair<int, int>> ev_marks;  // (phase, index of start event); end = start + 1
    size_t ev_used = 0;
    // batches: a batch handle owns its systems' handles; a system handle
    // points back at its batch
    lb_handle* parent = nullptr;
    lbe::BatchState* batch = nullptr;
};

namespace lbe {

// Return LB_EHIP from the calling API function when a HIP call fails.
#define LBE_HIP_OR_FAIL(h, call)                                                                           \
    do {                                                                                                   \
        hipError_t e_ = (call);                                                                            \
        if (e_ != hipSuccess)                                                                              \
            return ::lbe::fail((h), LB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));           \
    } while (0)

// Shared host helpers (lbe_runtime.hip).
constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
struct Layout {
    size_t f, psi, rho, owner, bmask, part, pfast, rec, kpart, red, counters, health, cells, total;
};
bool params_ok(const lb_params* p, std::string* why);
Layout layout_of(const lb_params* p);
int fail(lb_handle* h, int code, const std::string& msg);
// Carve one system's buffers from ws and clear them (synchronizes stream).
int setup_handle(lb_handle* h, const lb_params* prm, char* ws, size_t ws_bytes, hipStream_t stream);

// Descriptor of one system as the batched kernels see it (lbe_batch.hip).
SysDev sys_dev(const lb_handle* q);
// Device descriptors and systems of a batch. Stale tables are uploaded again
// (host work, a copy and a stream synchronisation) unless refresh_ok is false;
// then a stale batch is refused with LB_ESTATE.
int batch_sys(lb_handle* h, const SysDev** d_sys, int* nsys, int* parity, bool refresh_ok = true);

// Batches (lbe_batch.hip).
int batch_step_async(lb_handle* h, int nsteps);
int batch_health(lb_handle* h);
void batch_destroy(lb_handle* h);
void batch_touch(lb_handle* sub);  // a system changed: its batch refreshes its tables before stepping

// Batched launchers (one launch per phase over every system).
hipError_t launch_batch_density(const BatchLaunch& bl, int precision, hipStream_t st, int c, int o, int oo);
hipError_t launch_batch_fused(const BatchLaunch& bl, int precision, hipStream_t st, int c, int o);
hipError_t launch_batch_clear_owner(const BatchLaunch& bl, hipStream_t st, int o);
hipError_t launch_batch_wall_shell(const BatchLaunch& bl, int precision, hipStream_t st, int o);
hipError_t launch_batch_shell(const BatchLaunch& bl, int precision, hipStream_t st, int o);
hipError_t launch_batch_forces(const BatchLaunch& bl, hipStream_t st);
hipError_t launch_batch_bodies(const BatchLaunch& bl, hipStream_t st);
hipError_t launch_batch_raster(const BatchLaunch& bl, hipStream_t st, int o);
hipError_t launch_batch_killfill(const BatchLaunch& bl, int precision, hipStream_t st, int oo, int fd);
int kill_ext(const lb_handle* h);     // kill/fill box edge bound at the current largest radius

size_t elem_bytes(int precision);
size_t rho_elem_bytes(int precision);

// Launchers (all enqueue on h->stream; return hipSuccess or the launch error).
hipError_t launch_init(lb_handle* h, const double* d_rho_a, const double* d_rho_b, const double* d_u);
hipError_t launch_density(lb_handle* h, int c, int o, int oo);
hipError_t launch_shell(lb_handle* h);
hipError_t launch_fused(lb_handle* h);
hipError_t launch_forces(lb_handle* h);
Tiles fused_tiles(int nx, int ny, bool solids, int precision);
hipError_t launch_fields(lb_handle* h, double* d_out);       // rho_a, rho_b, u (5 x N doubles)
hipError_t launch_owner_codes(lb_handle* h, int32_t* dev_out);  // ABI owner codes, N int32
hipError_t launch_stats(lb_handle* h);                       // totals into b.red[kRedBlocks*8 ...]
hipError_t launch_remove_covered(lb_handle* h);
// Populations into plain form (every value in its node's own slot, masks
// zero), through the other population copy and back.
hipError_t launch_canonical(lb_handle* h);
hipError_t launch_bodies(lb_handle* h);
hipError_t launch_pack_fast(lb_handle* h);  // packed particle copy from the particle table
hipError_t launch_raster(lb_handle* h, uint32_t* owner, int first, int count);
hipError_t launch_clear_owner(lb_handle* h, uint32_t* owner);
hipError_t launch_clear_keep_walls(lb_handle* h, uint32_t* dst, const uint32_t* cur);  // walls copied from cur
hipError_t launch_wall_shell(lb_handle* h);  // Psi of wall nodes next to fluid
hipError_t launch_killfill(lb_handle* h);
hipError_t launch_fold_impulses(lb_handle* h);
// Particle-particle forces and torques into the particle table (lbe_pairs.hip).
hipError_t launch_pairs(lb_handle* h);
CellGrid cell_grid(int nx, int ny, int nz, double range);
int raster_extent(int nx, int ny, int nz, double rb);
int killfill_extent(int nx, int ny, int nz, double rb);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
hipError_t launch_fill_u32(lb_handle* h, uint32_t* p, uint32_t v, int64_t n);
hipError_t launch_fill_f64(lb_handle* h, double* p, double v, int64_t n);

}  // namespace lbe
