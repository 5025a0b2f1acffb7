/*
 * felbm.h - C ABI of the MI355X finite-element lattice Boltzmann library for
 * binary fluids (Lee-Lin free-energy model with characteristic-Galerkin
 * streaming and local collision/forcing; Matin et al., arXiv 1608.01906).
 *
 * One context advances one or more independent meshes ("instances") on one
 * GPU.  Per time step (Section 2.2, pre-streaming / streaming /
 * post-streaming split) the library runs, for every instance and every
 * population of both distributions (f: order parameter = density,
 * g: pressure-momentum):
 *   1. streaming right-hand side  -(dt C_a + dt^2 D_a) psi_a   (Section 2.2.1)
 *   2. the mass-matrix solve M Delta_a = rhs_a by lumped-preconditioned
 *      conjugate gradients with a fixed iteration count (or the lumped-mass
 *      approximation of Section 2.2.1)
 *   3. walls (nodal bounce-back) and the density moment (Section 2.2)
 *   4. nodal derivatives by volume-weighted recovery (Section 2.3)
 *   5. one fused post-streaming + pre-streaming collision with the
 *      potential-form force F, stress-form force G and exact-difference
 *      body force (Sections 2.1, 2.2)
 *
 * Conventions for every call:
 *  - All arrays passed in or out are HOST arrays in the caller's node order;
 *    the library copies them.  Vector fields are [n_nodes][dim], row-major.
 *    Populations are [2Q][n_nodes]: f_0..f_{Q-1} then g_0..g_{Q-1}, in the
 *    velocity order documented under FEL_LATTICE_*.
 *  - Device memory is one caller-owned buffer handed over by fel_bind (e.g.
 *    a PyTorch uint8 tensor); the library sub-allocates it and never frees
 *    it.  The library never calls hipMalloc for state.  The caller's stream
 *    orders all device work.
 *  - Every function returns a fel_status; on failure fel_last_error gives a
 *    message.  No exception or abort crosses the ABI.  fel_step is
 *    asynchronous: device-side conditions (non-finite values, CG residual
 *    above tolerance) surface at the next fel_sync / read call.
 *  - A context is not thread-safe.
 */
#ifndef FELBM_H
#define FELBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FEL_API __attribute__((visibility("default")))

typedef struct fel_ctx fel_ctx;

typedef enum {
    FEL_OK = 0,
    FEL_EINVAL = -1,      /* bad argument, bad mesh (inverted element, index out of range) */
    FEL_ENOMEM = -2,      /* host allocation failed or bound workspace too small */
    FEL_EDEVICE = -3,     /* a HIP runtime call failed */
    FEL_ESTATE = -4,      /* call out of order (e.g. step before bind / init) */
    FEL_ENOTCONV = -5,    /* a CG solve ended above the residual tolerance (state still advanced) */
    FEL_ENONFINITE = -6   /* a non-finite population or field was produced */
} fel_status;

/* Lattices (Section 2.1 uses D3Q19; 2-D meshes use D2Q9).
 * D2Q9 order:  0 (0,0); 1 (1,0); 2 (0,1); 3 (-1,0); 4 (0,-1); 5 (1,1); 6 (-1,1); 7 (-1,-1); 8 (1,-1).
 * D3Q19 order: 0 rest; 1..6 (+-x, +-y, +-z as +x,-x,+y,-y,+z,-z);
 *              7..10 (1,1,0),(-1,-1,0),(1,-1,0),(-1,1,0); 11..14 (1,0,1),(-1,0,-1),(1,0,-1),(-1,0,1);
 *              15..18 (0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1).  Weights are the standard ones. */
#define FEL_LATTICE_D2Q9 9
#define FEL_LATTICE_D3Q19 19

#define FEL_PREC_FP64 0        /* everything in FP64 */
#define FEL_PREC_FP32 1        /* FP32 operators, vectors and collision; populations stored as FP32
                                  scaled deviations from w_a * a node reference; FP64 CG dots and sums */
#define FEL_PREC_FP32_FP16 2   /* as FP32 but the stored deviations are FP16 */

#define FEL_MASS_CONSISTENT 0  /* solve with the consistent mass matrix (conjugate gradients) */
#define FEL_MASS_LUMPED 1      /* lumped-mass approximation (end of Section 2.2.1) */
#define FEL_MASS_CHEBYSHEV 2   /* consistent mass, Chebyshev semi-iteration preconditioned by the lumped
                                  mass with the a-priori spectrum bounds [1/(d+2), 1] of m^-1 M: the
                                  same solution as CG to the same contraction per iteration, no inner
                                  products (cg_iters iterations; cg_tol unused) */

#define FEL_ORDER_CALLER 0     /* device rows follow the caller's node order */
#define FEL_ORDER_ZCURVE 1     /* device rows follow a Z-order (Morton) curve of the node positions */

#define FEL_LAP_NESTED 0       /* Laplacian = recovered divergence of the recovered gradient */
#define FEL_LAP_WEAK 1         /* Laplacian = -m^-1 (sum_r K_rr) rho (Galerkin, lumped mass) */

typedef struct {
    int lattice;          /* FEL_LATTICE_D2Q9 or FEL_LATTICE_D3Q19 */
    int precision;        /* FEL_PREC_* */
    int mass_mode;        /* FEL_MASS_* */
    int cg_iters;         /* CG (or Chebyshev) iterations per solve; 0 = default (2-D: 30 FP64 / 15 FP32;
                             3-D: 34 / 17).  The CG keeps every iteration's search direction (x is
                             formed once after the last), so its workspace holds cg_iters vectors of
                             2(Q-1) values per node row */
    double cg_tol;        /* after the last iteration, sqrt(r.z / r0.z0) above this flags FEL_ENOTCONV;
                             0 = default (1e-11 FP64, 1e-5 FP32) */
    int laplacian_mode;   /* FEL_LAP_* */
    int max_instances;    /* number of independent meshes this context may hold (>= 1) */
    int node_order;       /* FEL_ORDER_*: the row order of the device layout.  Row-major grids are
                             already coalesced (each neighbour slot of 64 consecutive rows is one
                             contiguous run); unstructured meshes in arbitrary order need the curve.
                             Fields always cross the ABI in the caller's order. */
    int solver_batch;     /* populations a mass-solve kernel works on together: with direct gathers
                             the populations whose neighbour loads it issues ahead of use (its
                             software-pipeline depth), with LDS staging the populations staged per
                             pass; 1, 2 or 4 for every solver kernel, or 0 = chosen per kernel by
                             timing on the bound layout before the first step.  FP64 layouts of ELL
                             width 12 and up run the direct kernels at batch 2 at most (4 would spill
                             registers): a fixed 4 with direct gathers runs and reads back as 2 */
    int lds_staging;      /* mass-solve kernels read neighbour values 1 = by direct gathers from
                             memory, 2 = from a per-tile stage in LDS (the tile's rows and its halo
                             loaded once per population, coalesced; a block barrier per pass),
                             3 = from a per-wavefront stage (each 64-row wavefront stages its rows
                             and its own halo, no barriers; ELL width 7 layouts whose wavefront
                             halos hold at most 192 columns), 0 = chosen per kernel by timing.
                             On 3-D layouts (ELL width 15 and up) the CG carries M p by its own
                             recurrence: its second kernel reads no neighbour values and runs direct.
                             Staging needs tile halos of at most 1024 rows, two stages of the
                             population batch within 60 KB of LDS and CG vectors below 2 GiB; a
                             forced 2 or 3 that does not fit makes the first fel_step return
                             FEL_EINVAL (0 then keeps direct gathers).
                             The option also covers the streaming kernel, whose staged form (one
                             lattice direction per pass, per tile: 3 selects it as 2 does) exists
                             for D2Q9 layouts of ELL width 7 in FP32 or FP16 storage; elsewhere
                             binding settles it to 1.
                             Every schedule computes the same sums in the same order; results agree
                             to rounding (the staged and direct forms may contract multiply-adds
                             differently) */
    int fused_reductions; /* consistent-mass CG: 1 = a finalize launch forms each CG scalar from the
                             tile partials (two per iteration); 2 = fused: 1024-thread blocks leave
                             at most 256 partials per instance and every block of the next launch
                             sums them itself (D2Q9 layouts of ELL width 7 with instances of at most
                             1024 tiles, else fel_bind returns FEL_EINVAL); 0 = chosen by timing both solves on
                             the bound layout before the first step (1 where fused is unavailable).
                             Same results to rounding (the partial sums group rows differently).
                             The fused kernels' 1024-thread blocks leave 128 registers per thread,
                             so their population batch is at most 1 for the first kernel of an
                             iteration, 4 (FP32) / 1 (FP64) for the second and 4 / 2 for the
                             initial residual; solver_batch above that runs the largest built.
                             The lumped and Chebyshev mass modes reduce nothing: there the option is
                             ignored and fel_tuning reads 1 after the first step */
} fel_options;

/* Physical parameters of one instance (Section 2.1).  rho_l is the heavy
 * (liquid) bulk density, rho_v the light (vapour) one, rho_l > rho_v > 0.
 * tau_* are the dimensionless bulk relaxation times (kinematic viscosity
 * cs^2 tau dt), combined by the composition-weighted harmonic mean.  sigma
 * and xi give beta = 12 sigma / (xi (rho_l - rho_v)^4) and
 * kappa = 3 xi sigma / (2 (rho_l - rho_v)^2).  grav is the body
 * acceleration (components beyond dim are ignored). */
typedef struct {
    double rho_l, rho_v, tau_l, tau_v, sigma, xi, dt, grav[3];
} fel_phys;

/* Creates a context.  Validates the options; allocates host memory only. */
FEL_API fel_status fel_create(const fel_options* opt, fel_ctx** out);

/* Uploads the P1 simplex mesh of instance `inst` (0 <= inst < max_instances)
 * and assembles its operators on the host (Section 2.2.1, finite-element
 * matrices; Section 2.3, recovery).  Must precede fel_workspace_size/bind.
 *   dim         2 (triangles, D2Q9) or 3 (tetrahedra, D3Q19)
 *   xyz         [n_nodes][dim] node coordinates
 *   conn        [n_elems][dim+1] vertex indices (0-based), positively oriented
 *   shift       [n_elems][dim+1][dim] periodic image of each vertex (unwrapped
 *               position = xyz + shift * box), or NULL for none
 *   box         [dim] period per axis (0 = not periodic), may be NULL if shift is NULL
 *   wall        [n_nodes] 1 on no-slip wall nodes, or NULL
 *   wall_normal [n_nodes][dim] unit normal into the fluid at wall nodes, or NULL
 * Errors: FEL_EINVAL on a bad index, a non-positive element volume, a
 * dimension that does not match the lattice, or a re-upload after fel_bind. */
FEL_API fel_status fel_upload_mesh(fel_ctx* ctx, int inst, int dim, int64_t n_nodes, const double* xyz,
                                   int64_t n_elems, const int32_t* conn, const int8_t* shift,
                                   const double* box, const uint8_t* wall, const double* wall_normal);

/* Device bytes needed for every uploaded instance (call after all uploads). */
FEL_API fel_status fel_workspace_size(fel_ctx* ctx, size_t* bytes);

/* Binds a caller-owned device buffer of at least fel_workspace_size bytes
 * (256-byte aligned) and the HIP stream (hipStream_t, NULL = default
 * stream) all work is ordered on; copies the operators to the device. */
FEL_API fel_status fel_bind(fel_ctx* ctx, void* dev_ptr, size_t bytes, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): fel_bind
 * without a caller buffer.  The context is bound to the library's own
 * static device array of FEL_STATIC_WORKSPACE_BYTES per GPU (the current
 * device's; each GPU holds its copy until the process ends), found once per
 * device by symbol lookup; the call allocates no device memory.
 *  - The uploaded meshes must fit: fel_workspace_size <= FEL_STATIC_WORKSPACE_BYTES,
 *    else FEL_ENOMEM and the context stays unbound.
 *  - Schedules the options leave to timing take fixed defaults instead
 *    (population batch 2, direct gathers, finalize-launch reductions), and
 *    fel_step launches its kernels directly, with no graph of the library's
 *    own (so the caller may capture fel_step after its first call).
 *  - One array per GPU serves every context bound this way on that GPU: it
 *    keeps the last user's contents (the bind clears the state and scratch
 *    regions it lays out), binding another context takes it over and every
 *    earlier context bound to it then returns FEL_ESTATE, and calls that
 *    overlap on one GPU (several streams, several threads) race.
 * Otherwise as fel_bind: FEL_ESTATE if already bound, operators copied on
 * the given stream (hipStream_t, NULL = default stream). */
#define FEL_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
FEL_API fel_status fel_bind_static(fel_ctx* ctx, void* hip_stream);

/* Sets the physics of `inst` and initialises its populations to the
 * equilibrium of the given nodal density rho [n], velocity u [n][dim] and
 * pressure p [n] (the equilibria f_eq = rho Gamma(u) and
 * g_eq = w p / cs^2 + rho (Gamma(u) - Gamma(0)) of Section 2.1), plus the
 * forcing of a pre-streaming collision (Section 2.2; its BGK part vanishes
 * at equilibrium).  The recovered derivatives the forcing needs are those
 * of Section 2.3.  u or p may be NULL for zero.  May be called again on a
 * stepped context to restart the instance.  Errors: FEL_EINVAL on a
 * non-positive or non-finite rho, rho_l <= rho_v, a non-positive tau, dt or
 * xi, a negative sigma, or an instance out of range; FEL_ESTATE before
 * fel_bind.  Synchronises the stream. */
FEL_API fel_status fel_init_fields(fel_ctx* ctx, int inst, const fel_phys* phys, const double* rho,
                                   const double* u, const double* p);

/* Advances every instance by n_steps time steps; asynchronous on the bound
 * stream.  The first call also settles whatever schedule the options left
 * to timing (fel_options.solver_batch, lds_staging, fused_reductions): it
 * launches the candidate kernels, then graphs of the whole mass solve, on
 * the solve's scratch buffers and synchronizes the stream, so it must not
 * be made while the caller captures that stream into a graph.  The library captures the step into a graph of its own on
 * the first call and replays it afterwards (on a non-default stream and
 * while not profiling). */
FEL_API fel_status fel_step(fel_ctx* ctx, int n_steps);

/* Waits for the stream and reports device conditions raised since the last
 * sync: FEL_ENONFINITE, then FEL_ENOTCONV; clears them. */
FEL_API fel_status fel_sync(fel_ctx* ctx);

/* Fields of the last step of `inst` (or of its initial state), the
 * moments of the streamed populations (Section 2.2): density rho = sum f,
 * velocity [n][dim] from rho u = sum e g + dt/2 (S + rho grav), pressure
 * p = cs^2 sum g + dt/2 cs^2 u . grad rho, and the composition
 * C = (rho - rho_v)/(rho_l - rho_v) that sets the relaxation time
 * (Section 2.1).  Any pointer may be NULL; arrays are caller-owned, in the
 * caller's node order.  Errors: FEL_EINVAL for an instance out of range,
 * FEL_ESTATE before fel_bind.  Synchronises the stream. */
FEL_API fel_status fel_read_fields(fel_ctx* ctx, int inst, double* rho, double* u, double* p, double* C);

/* Per-instance FP64 sums over nodes with the lumped mass m as weight
 * (the integrals of the P1 fields, Section 2.2.1): out[0] = sum m rho,
 * out[1] = sum m C, out[2] = sum m (1 - C) (mass of each phase, conserved by
 * the streaming and collision of Section 2.2 on periodic meshes),
 * out[3..5] = sum m sum_a e_a gbar_a (momentum; zero beyond dim), from the
 * stored pre-streaming populations.  out is caller-owned.  Errors:
 * FEL_EINVAL for an instance out of range, FEL_ESTATE before fel_bind.
 * Synchronises the stream. */
FEL_API fel_status fel_conserved_sums(fel_ctx* ctx, int inst, double out[6]);

/* Checkpoint / restart: the stored pre-streaming populations of `inst` as
 * [2Q][n_nodes] FP64 (FP32 modes convert).  fel_set_state needs the
 * physics set by a prior fel_init_fields. */
FEL_API fel_status fel_get_state(fel_ctx* ctx, int inst, double* psibar);
FEL_API fel_status fel_set_state(fel_ctx* ctx, int inst, const double* psibar);

/* Diagnostics of the last step of `inst`, in FP64, caller node order:
 * FEL_AUX_GRADRHO [n][dim] recovered density gradient; FEL_AUX_MU [n]
 * chemical potential mu_phi - kappa lap rho; FEL_AUX_S [n][dim] stress
 * vector kappa [d_i |grad rho|^2 - d_j (d_i rho d_j rho)]; FEL_AUX_DELTA
 * [2Q][n] streaming increments (rest direction zero). */
#define FEL_AUX_GRADRHO 0
#define FEL_AUX_MU 1
#define FEL_AUX_S 2
#define FEL_AUX_DELTA 3
FEL_API fel_status fel_read_aux(fel_ctx* ctx, int inst, int which, double* out);

/* Kernel timing with HIP events on the bound stream, for roofline
 * measurement.  fel_profile(ctx, 1) starts recording an event pair around
 * every kernel launch of fel_step (graph replay is disabled meanwhile);
 * fel_profile_read returns, per kernel class k < n_classes, the launch count
 * and the summed duration in ms, and the class names; fel_profile(ctx, 0)
 * stops and clears. */
FEL_API fel_status fel_profile(fel_ctx* ctx, int enable);
FEL_API fel_status fel_profile_read(fel_ctx* ctx, int max_classes, int* n_classes, int64_t* counts,
                                    double* total_ms, const char** names);

/* Sizes of the device layout (for traffic accounting): total padded rows,
 * ELL width, number of stored populations, CG iterations per step, and the
 * largest and mean per-tile halo (columns referenced outside a 256-row
 * tile).  Any pointer may be NULL. */
FEL_API fel_status fel_layout_info(fel_ctx* ctx, int64_t* rows, int* ell_width, int* pops, int* cg_iters,
                                   int* halo_max, double* halo_mean);

/* The LDS staging tables of the layout, before fel_bind (they are freed
 * there): form 2 = per tile, 3 = per 64-row wavefront of a tile (built for
 * ELL width 7 layouts whose wavefront halos hold at most 192 columns and
 * whose schedule may use the form: lds_staging 0 or 3, a mass mode with a
 * solve).  A list per tile (form 2) or per wavefront (form 3, 4 per tile):
 * the columns its rows reference outside it, ascending, as device rows.
 * lcol [ell_width][rows] (row-major by slot, as the device holds it): the
 * LDS slot each ELL slot reads, < 256 the row's tile-local index, else
 * 256 + h (form 2) or 256 + 192 w + h (form 3, w the wavefront within the
 * tile) for entry h of the list.  The device row order is the caller's
 * unless node_order asks for the curve.  n_lists and n_cols (the length of
 * list_col) are always written; lcol, list_ptr [n_lists + 1] and list_col
 * may be NULL.  FEL_ESTATE after binding, FEL_EINVAL for a form the layout
 * does not have. */
FEL_API fel_status fel_stage_tables(fel_ctx* ctx, int form, int64_t* n_lists, int64_t* n_cols, uint16_t* lcol,
                                    int32_t* list_ptr, int32_t* list_col);

/* Schedule in use for each kernel class k < max_classes (same classes and
 * order as fel_profile_read): population batch and staging (1 direct,
 * 2 LDS-staged per tile, 3 per wavefront; the streaming kernel's batch is
 * always 1); kernels without
 * a tunable schedule read 1; and the CG reduction form (fused_reductions:
 * 1 or 2).  Values left to the tuner (option 0) read 0 until the first
 * fel_step.  batch, staging and fused may be NULL. */
FEL_API fel_status fel_tuning(fel_ctx* ctx, int max_classes, int* n_classes, int* batch, int* staging,
                              int* fused);

FEL_API fel_status fel_destroy(fel_ctx* ctx);
FEL_API const char* fel_last_error(const fel_ctx* ctx);
FEL_API const char* fel_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FELBM_H */
