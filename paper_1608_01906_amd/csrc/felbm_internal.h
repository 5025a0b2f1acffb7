// Private layout shared by the host side (felbm_host.cpp) and the kernels
// (felbm_kernels.hip, felbm_solver.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "../../include/felbm.h"

namespace fel {

// Rows are processed in tiles of TILE rows (one block per tile); every
// instance starts on a tile boundary so a tile never mixes instances and a
// block's reduction partials belong to one instance.
constexpr int TILE = 256;

// Per-instance physics and layout, resident on the device.
struct InstParams {
    double rho_l, rho_v, tau_l, tau_v, dt;
    double grav[3];
    double beta, kappa;
    double scale;          // deviation scale s (FP32 modes): psi_a = w_a (ref + s d_a)
    int row_begin, row_end;  // valid rows of the instance [row_begin, row_end)
    int tile_begin, tile_count;
    int fb_begin, fb_count;  // fused-reduction blocks of the instance (see fblocks)
};

// Device pointers of one context (all sub-allocated in the bound workspace).
// R = total padded rows, W = ELL width, NB = stream basis matrices
// (2-D: Gx Gy Kxx Kyy Kxy; 3-D: Gx Gy Gz Kxx Kyy Kzz Kxy Kxz Kyz, where
// K_rs here is K_rs + K_sr for r != s).
struct DevLayout {
    int64_t R;
    int W, NB, Q, dim, ninst, ntiles;
    int precision;         // 0 fp64, 1 fp32, 2 fp32 with fp16 deviations
    // pattern and operators, ELL slot-major: value[k * R + row]
    const int32_t* col;
    const void* Mval;      // T [W][R]
    const void* basis;     // T [NB][W][R]
    const void* minv;      // T [R]   1/m (1 on padding rows)
    const double* mlump;   // double [R] lumped mass (0 on padding rows)
    const uint32_t* wmask; // [R] bit a set: population a takes its opposite after streaming
    // LDS staging of a tile: its halo (columns outside the tile, ascending)
    // and the slot columns as tile-local indices (< TILE: own row,
    // TILE + h: halo entry h); stage rows are `sw` values apart
    const uint16_t* lcol;       // [W][R]
    const int32_t* halo_ptr;    // [ntiles + 1]
    const int32_t* halo_col;    // [halo_ptr[ntiles]]
    int sw;                     // TILE + largest halo, rounded up to 64
    // LDS staging per wavefront (staging form 3; null where the layout has
    // none): each 64-row wavefront of a tile stages its own rows and its
    // own halo (columns outside those 64 rows, ascending, at most
    // kWaveHaloRounds * 64); slot columns < TILE are the row's tile-local
    // index (a row of the same wavefront), TILE + w kWaveHaloRounds 64 + h
    // is halo entry h of wavefront w of the tile
    const uint16_t* wlcol;      // [W][R]
    const int32_t* whalo_ptr;   // [4 ntiles + 1]
    const int32_t* whalo_col;   // [whalo_ptr[4 ntiles]]
    const int32_t* tile_inst;   // [ntiles]
    const InstParams* params;   // [ninst]
    // populations
    void* psi;             // FP64: double [2Q][R];  FP32 modes: deviations float/half [2Q][R]
    float* ref;            // FP32 modes: [2][R] reference of f (rho) and g (p / cs^2)
    // CG work vectors over the 2(Q-1) moving populations, T [2(Q-1)][R]
    void* X;
    void* Rv;
    void* Pa;              // Chebyshev: an iterate; CG recurrence form: q = M p
    void* Pb;              // right-hand side of the solve
    // CG search directions of every iteration, T [K][2(Q-1)][R]: x is
    // formed once after the last iteration as x_0 + sum_k alpha_k p_k
    void* Ph;
    int K;                 // CG iterations per solve
    // nodal fields, T
    void* rho;             // [R]
    void* grad;            // [dim][R]
    void* mu;              // [R]
    void* S;               // [dim][R]
    void* u;               // [dim][R]
    void* p;               // [R]
    // reductions
    double* partial;       // [2(Q-1)][ntiles] tile partials (also reused for the conserved sums)
    double* rz;            // [ninst][2(Q-1)]
    double* rz0;           // [ninst][2(Q-1)]
    double* alpha;         // [K][ninst][2(Q-1)] (one slice per CG iteration)
    double* beta;          // [ninst][2(Q-1)]
    double* sums;          // [ninst][8]
    uint32_t* status;      // [1] bit 0 non-finite, bit 1 CG residual above tolerance
    // fused reductions (2-D): blocks of up to 4 tiles; entry b of fblocks =
    // (first tile, tiles, instance, block index within the instance), in
    // dispatch order; block partials [NP][nfb] alternate between fpart0
    // (r.z) and fpart1 (p.q); srz [2][ninst][NP] holds r.z by iteration parity
    const int4* fblocks;
    int nfb;
    double* fpart0;
    double* fpart1;
    double* srz;
    double cg_tol2;        // squared relative residual tolerance of the CG check
    int lap_mode;          // 0 nested recovery, 1 weak form
};

enum KernelClass {
    KC_STREAM = 0,
    KC_CG_INIT,
    KC_CG_A,
    KC_CG_B,
    KC_LUMPED,
    KC_MOMENTS,
    KC_GRAD,
    KC_DIV,
    KC_COLLIDE,
    KC_INIT,
    KC_SUMS,
    KC_FINALIZE,
    KC_CHEB,
    KC_CG_X,
    KC_COUNT
};

const char* kernel_class_name(int k);

// Events the next launch records around the kernel's own execution (profiling).
struct LaunchEvents {
    hipEvent_t a = nullptr, b = nullptr;
};
extern thread_local LaunchEvents g_launch_events;

// Launchers (felbm_kernels.hip, felbm_solver.hip).  tile_begin/ntiles
// select the tile range; every launcher returns the hipError_t of the launch.
// staged: the LDS-staged form (2-D, ELL width 7, deviation storage only)
hipError_t launch_stream(const DevLayout& L, int tile_begin, int ntiles, bool staged, hipStream_t s);
// The solver launchers take the population batch (1, 2 or 4) of their
// pipeline or LDS pass and the staging form: 1 direct gathers, 2 a stage
// per tile, 3 a stage per wavefront (ELL width 7 layouts with wavefront
// halos, wlcol set).
hipError_t launch_cg_init(const DevLayout& L, int tile_begin, int ntiles, int batch, int stage, hipStream_t s);
// it = CG iteration: p_it is written to (cg_a) and read from (cg_b) slice
// it of Ph, alpha_it to slice it of alpha.
hipError_t launch_cg_a(const DevLayout& L, int tile_begin, int ntiles, bool first, int it, int batch, int stage,
                       hipStream_t s);
hipError_t launch_cg_b(const DevLayout& L, int tile_begin, int ntiles, int it, int batch, int stage,
                       hipStream_t s);
// x = rhs / m + sum over the K iterations of alpha_k p_k, in iteration
// order, from the stored directions (x is written, never read); with check
// set it also runs the fused CG's final residual check
hipError_t launch_cg_x(const DevLayout& L, int tile_begin, int ntiles, bool check, hipStream_t s);
// op: 0 CG init, 1 alpha, 2 beta, 3 final residual check, 4 conserved sums;
// nvals values per tile (partials stored population-major)
hipError_t launch_finalize(const DevLayout& L, int inst_begin, int ninst, int op, int nvals, hipStream_t s,
                           int it = 0);
hipError_t launch_lumped(const DevLayout& L, int tile_begin, int ntiles, hipStream_t s);
// Fused-reduction CG (2-D, no finalize launches): every block sums the
// previous launch's block partials of its instance itself.  it = iteration.
hipError_t launch_cg_init_fused(const DevLayout& L, int batch, hipStream_t s);
hipError_t launch_cg_a_fused(const DevLayout& L, int it, int batch, hipStream_t s);
hipError_t launch_cg_b_fused(const DevLayout& L, int it, int batch, hipStream_t s);
// Largest population batch built for a fused kernel class (KC_CG_INIT,
// KC_CG_A, KC_CG_B) at a precision: the larger ones would spill registers.
int fused_max_batch(int cls, int precision);
// ELL widths from which the CG carries q = M p by its own recurrence (the
// 3-D layouts, where neighbour gathers dominate): the second CG kernel then
// reads own rows only and has no staged form.
constexpr int kQRecurrenceWidth = 15;
// Largest population batch of the direct solver kernels: in FP64 at ELL
// width 12 and up the double-buffered gathers of a batch of 4 would spill
// registers, so those layouts stop at 2 (a fixed batch of 4 runs, and
// reads back from fel_tuning, as 2).
constexpr int direct_max_batch(int W, int elem_bytes) { return elem_bytes == 8 && W >= 12 ? 2 : 4; }
constexpr int kHaloRounds = 4;       // LDS staging: halo entries per thread at most (halo <= 4 TILE)
// LDS staging per wavefront: halo entries per lane at most (a wavefront's
// halo <= 192), and the stage row: the tile's rows, then 3 x 64 halo slots
// for each of its 4 wavefronts
constexpr int kWaveHaloRounds = 3;
constexpr int kWaveStageWidth = TILE + (TILE / 64) * kWaveHaloRounds * 64;
// The staged solver kernels address a [2(Q-1)][R] vector through one buffer
// resource with 32-bit byte offsets: its size must stay below 2 GiB (larger
// layouts run the direct kernels).
inline bool staged_vectors_fit(int np, int64_t R, int precision) {
    return (int64_t)np * R * (precision == 0 ? 8 : 4) < ((int64_t)1 << 31);
}
constexpr int kStageBytes = 60 * 1024;  // LDS staging: dynamic LDS per block at most (2 batches of sw rows)
constexpr int kFusedTiles = 4;       // tiles per fused-reduction block
constexpr int kFusedMaxBlocks = 256; // per instance (a lane of a fused block loads at most 4 of its partials)
// Chebyshev solve: first launch writes x_0 to buffer out0 and x_1 to the
// other (0 = X, 1 = Pa); each later launch reads x_k from buffer cur.
hipError_t launch_cheb_first(const DevLayout& L, int tile_begin, int ntiles, int out0, double gamma, int batch,
                             int stage, hipStream_t s);
hipError_t launch_cheb(const DevLayout& L, int tile_begin, int ntiles, int cur, double omega, double gamma, int batch,
                       int stage, hipStream_t s);
hipError_t launch_moments(const DevLayout& L, int tile_begin, int ntiles, hipStream_t s);
hipError_t launch_grad(const DevLayout& L, int tile_begin, int ntiles, hipStream_t s);
hipError_t launch_div(const DevLayout& L, int tile_begin, int ntiles, hipStream_t s);
hipError_t launch_collide(const DevLayout& L, int tile_begin, int ntiles, hipStream_t s);
hipError_t launch_init(const DevLayout& L, int tile_begin, int ntiles, hipStream_t s);
hipError_t launch_sums(const DevLayout& L, int tile_begin, int ntiles, hipStream_t s);

// The static workspace (fel_bind_static): one file-scope device array of
// kStaticWorkspaceBytes per device, looked up once per device in
// felbm_static.hip; devices 0..kMaxDevices-1.
constexpr size_t kStaticWorkspaceBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

}  // namespace fel

// Host-side helpers of the static binding (felbm_host.cpp).
struct fel_ctx;
namespace fel {
// Binds ctx to `bytes` bytes of device memory at ptr that the library owns
// (the static array of `device`): fixes schedules left to timing, runs steps
// without a graph of its own, and marks ctx as the array's user, which makes
// every earlier context bound to it report FEL_ESTATE.
fel_status bind_static_workspace(fel_ctx* c, void* ptr, size_t bytes, void* hip_stream, int device);
// Records an error message on ctx and returns st.
fel_status set_error(fel_ctx* c, fel_status st, const char* msg);
}  // namespace fel
