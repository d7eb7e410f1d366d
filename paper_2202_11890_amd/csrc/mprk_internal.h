// mprk_internal.h -- launch parameters shared by the host layer and the HIP
// kernels of the MPRK library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mprk {

constexpr int NV = 4;          // 2D: (rho, rho u, rho w, rho E)
constexpr int NV3 = 5;         // 3D: (rho, rho u, rho v, rho w, rho E)

// Stage tile shapes: TX columns x TZ rows of cells per workgroup of TX*TZ
// threads, one cell per thread.  The conserved state is staged with a 2-cell
// halo (reconstruction stencil), primitives with a 1-cell halo.  Every kernel
// is instantiated for each shape; the host picks one per context (32 x 16
// with FP64 fluxes, 32 x 8 with FP32 fluxes, or the autotuner's choice).
enum TileShape : int32_t {
    TILE_32x16 = 0,
    TILE_16x32 = 1,
    TILE_64x8 = 2,
    TILE_32x8 = 3,
    TILE_SHAPES = 4,
};

struct TileDims {
    int tx, tz, nt;
};

struct TileDims3 {
    int tx, ty, tz, nt;
};

constexpr TileDims tile_dims(int shape)
{
    switch (shape) {
    case TILE_16x32: return {16, 32, 512};
    case TILE_64x8: return {64, 8, 512};
    case TILE_32x8: return {32, 8, 256};
    default: return {32, 16, 512};
    }
}

// What a stage launch writes for a cell.
enum Mode : int32_t {
    MODE_RHS = 0,        // out = R
    MODE_STAGE = 1,      // out = U + inc, inc = beta (Qin - U) + beta h R
                         // (= alpha U + beta (Qin + h R), alpha + beta = 1)
    MODE_ACC_FIRST = 2,  // acc = inc
    MODE_ACC_ADD = 3,    // acc += inc
    MODE_ACC_FINAL = 4,  // out = U + (acc + inc) / m
};

struct Combine {
    double alpha;   // weight of the substep base U
    double beta;    // weight of the stage input Qin (1 - alpha)
    double bh;      // beta * step
    int32_t mode;
    int32_t pad;
};

// Rows of DomainArgs::vk.
enum : int { VK_NN = 0, VK_N = 1, VK_Q = 2, VK_TT = 3, VK_TN = 4 };

// Domain arrays are [nv][nz][ny][nx] (ny = 1 in 2D); a "row" is a z-plane.
struct DomainArgs {
    const double* qin;     // stage value read by the stencil [nv][nz][ny][nx]
    const double* base;    // substep base U (pointwise)
    double* out;           // destination of MODE_RHS / STAGE / ACC_FINAL
    double* acc;           // buffer accumulator [NV][b_hi-b_lo][nx]
    const double* ret_in;  // retained slow rows [NV][2][nx], read for rows outside
                           // [b_lo, b_hi) when use_ret is set
    double* ret_out;       // if set: save Qin rows [ret_lo, ret_lo+2) here
    int32_t nz;
    int32_t row_lo, row_hi;  // rows computed by this launch (fixed tiles meeting
                             // this range; each computes its rows inside it)
    int32_t b_lo, b_hi;      // buffer rows (empty range: none)
    int32_t ret_lo;          // first of the two retained slow rows next to B
    int32_t use_ret;
    int32_t gamma_top;       // 1: the interface is above the top row
    int32_t gamma_bot;       // 1: the interface is below row 0
    int32_t tiles_x, tiles_z, ntiles;
    int32_t tiles_y;         // 3D only (1 in 2D)
    double dz, inv_dz;
    double hinv_dz;          // inv_dz / 2: the face routines return twice the flux
    double mu, kappa;
    float inv_dz_f, mu_f, kappa_f, pad_f;   // FP32 copies (round to nearest) for FP32 fluxes
    // Viscous coefficients of the face routines, per direction d (0 x, 1 y,
    // 2 z; 2D uses x and z), applied to raw differences of the staged
    // primitives: [VK_NN] 4/3 mu / h_d and [VK_N] mu / h_d (normal
    // derivatives), [VK_Q] 2 kappa / h_d (heat flux of the doubled flux),
    // [VK_TT] -2/3 mu / (4 h_d) and [VK_TN] mu / (4 h_d) (tangential
    // derivatives, averaged over the two cells of the face).
    double vk[5][3];
    float vk_f[5][3];
    float pad_vk;
    Combine main;            // rows outside [b_lo, b_hi)
    Combine buf;             // rows inside  [b_lo, b_hi)
};

struct StageArgs {
    DomainArgs d[2];         // 0 = lower, 1 = upper
    int32_t nx;
    int32_t ny;              // 1 in 2D
    double dy, inv_dy;       // 3D only
    int32_t nblocks;         // d[0].ntiles + d[1].ntiles
    int32_t first;           // domain whose tiles take the first blocks
    int32_t flux32;          // 1: face fluxes in FP32 (state, stage sums, interface flux FP64)
    int32_t dev_stores;      // 1: stage results stored with device coherence (see st_dev)
    double dx, inv_dx;
    double hinv_dx, hinv_dy;  // inv_dx / 2, inv_dy / 2 (divergence of the doubled fluxes)
    double gamma, gm1, gravity;
    float inv_dx_f, inv_dy_f, gamma_f, gm1_f;   // FP32 copies (round to nearest) for FP32 fluxes
    double bu, bT;           // bulk coefficients of the interface flux
    double half_dz1_mu1;     // dz_lower / (2 mu_lower): wall velocity u_w1 = u1 + sigma * this
    double inv_m;
};

// Reductions: per-domain fields.
constexpr int RED_BLOCKS = 256;   // partial blocks per domain
constexpr int RED_THREADS = 256;
constexpr int RED_FIELDS = 14;    // sum[5], comp[5], lambda, courant, visc, bad

struct ReduceArgs {
    const double* q[2];
    int32_t nz[2];
    int32_t nx, ny;          // ny = 1 in 2D
    int32_t nv;              // 4 (2D) or 5 (3D)
    int32_t pad;
    double inv_dx, inv_dy, inv_dz[2];
    double visc_coef[2];     // max(4/3, gamma/Pr) * mu_d * sum over directions of 1/h^2
    double gamma, gm1;
    double* partial;         // [2][RED_BLOCKS][RED_FIELDS]
    double* final_;          // [2][RED_FIELDS]
};

// Persistent (dataflow) execution: one launch runs many stages of one or
// more members.  Each fixed tile of each domain has a progress counter (the
// last stage it finished); a tile starts stage g once its eight neighbours
// and, next to the interface, the tile across it have finished g - 1.
struct TileRef {
    int32_t member;
    int32_t dom;       // 0 lower, 1 upper
    int32_t tx, tz;    // fixed-tile coordinates (tiles of the launch's shape, z aligned
                       // at multiples of the tile height)
};

// Stage g = 1, 2, ... of a persistent launch is slot (g-1) % nslots of slow
// step (g-1) / nslots; a member computes its stage record slot_stage[slot]
// there (slot itself when slot_stage is null; nothing when it is -1).
struct MemberRun {
    const StageArgs* stages;   // m*s records of one slow step, index (k-1)*s + (j-1)
    const int32_t* slot_stage; // per slot: record index or -1; null: record = slot
    int32_t nslots;            // slots per slow step
    int32_t nsteps;            // slow steps in this launch
    int32_t done_base[2];      // progress-counter index of tile (0, 0) per domain
    int32_t tiles_x;
    int32_t tiles_z[2];
    int32_t pad;
};

struct PersistArgs {
    const TileRef* tiles;      // every fixed tile of every member
    const MemberRun* members;
    int32_t* done;             // progress counters, zero before the launch
    int32_t* abort_flag;       // set (never cleared by the kernel) if the launch timed out
    int32_t ntiles;
    int32_t gmax;              // stages of the launch: nslots * nsteps
    int64_t run_ticks;         // longest the launch may run, in wall-clock ticks: a tile
                               // still waiting for a neighbour after that aborts it
};

// Batched launches: the blocks of one launch are split into consecutive
// ranges, one per member with a stage in the launch; each block finds its
// range in a per-block map whose entry names the stage record (of some
// member) that its range computes.
struct BatchEntry {
    int32_t arg;       // index into the stage-record table
    int32_t begin;     // first block of this block's range
};

// Kernel of a launch, for building graphs: function, block size and the
// argument block.
struct KernelRef {
    const void* func;
    int block;
};

hipError_t launch_stage(const StageArgs& a, int shape, hipStream_t s);
KernelRef stage_kernel_ref(bool flux32, int shape);
hipError_t launch_batch(const StageArgs* tab, const BatchEntry* bmap, int nblocks, bool flux32,
                        int shape, hipStream_t s);
KernelRef batch_kernel_ref(bool flux32, int shape);
hipError_t launch_persistent(const PersistArgs& a, int grid, bool flux32, int shape, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t value, int n, hipStream_t s);
int persistent_blocks_per_cu(bool flux32, int shape);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s);

// Doubles of the file-scope device scratch of the allocation-free
// diagnostics (partials, then finals); the need does not depend on the
// problem size (the reduction is grid-stride over a fixed block count).
constexpr size_t STATIC_SCRATCH_DOUBLES = (size_t)2 * RED_BLOCKS * RED_FIELDS + (size_t)2 * RED_FIELDS;
hipError_t static_scratch_address(double** out);
// 3D stage kernel (one tile shape per flux type).
hipError_t launch_stage3(const StageArgs& a, hipStream_t s);
KernelRef stage3_kernel_ref(bool flux32);
TileDims3 tile3_dims(bool flux32);
hipError_t launch_reduce_batch(const ReduceArgs* tab, int n, hipStream_t s);

}  // namespace mprk
