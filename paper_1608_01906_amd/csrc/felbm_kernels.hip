// HIP kernels of the FE lattice Boltzmann step for gfx950 (MI355X).
//
// Every kernel is row-parallel over the concatenated, tile-padded node rows
// of all instances: one block of TILE threads per tile, one row per thread.
// Sparse operators are stored as ELL, slot-major (value[k * R + row]), so a
// wavefront's loads of one slot are contiguous and its gathers hit the few
// grid rows around the tile.  Blocks are mapped to tiles XCD-aware: the 8
// XCDs receive contiguous tile ranges, so the halo rows a tile gathers were
// fetched by the same XCD's L2.
//
// Reductions (CG dot products, conserved sums) are FP64: per-tile partials
// in a fixed order (wavefront shuffles, then LDS), then one small finalize
// launch per instance sums the partials in a fixed order, so results are
// bitwise reproducible.
#include "felbm_internal.h"

#include <hip/hip_ext.h>

namespace fel {

thread_local LaunchEvents g_launch_events;

// With a pair of events armed, the launch goes through
// hipExtLaunchKernelGGL, whose events are stamped by the kernel's own
// dispatch: the elapsed time is the kernel's execution, without host gaps.
#define FEL_LAUNCH(K, G, B, SH, S, ...)                                                                    \
    do {                                                                                                  \
        if (g_launch_events.a)                                                                            \
            hipExtLaunchKernelGGL(K, G, B, SH, S, g_launch_events.a, g_launch_events.b, 0, __VA_ARGS__); \
        else                                                                                              \
            hipLaunchKernelGGL(K, G, B, SH, S, __VA_ARGS__);                                              \
    } while (0)

// ---------------------------------------------------------------------------
// lattices (standard D2Q9 / D3Q19, cs^2 = 1/3)
template <int Q> struct Lat;
template <> struct Lat<9> {
    static constexpr int D = 2;
    static constexpr int NB = 5;
    __host__ __device__ static constexpr int e(int a, int r) {
        constexpr int E[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                                 {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
        return E[a][r];
    }
    __host__ __device__ static constexpr double w(int a) {
        return a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    __host__ __device__ static constexpr int opp(int a) {
        constexpr int O[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
        return O[a];
    }
};
template <> struct Lat<19> {
    static constexpr int D = 3;
    static constexpr int NB = 9;
    __host__ __device__ static constexpr int e(int a, int r) {
        constexpr int E[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                                  {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                  {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                  {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
        return E[a][r];
    }
    __host__ __device__ static constexpr double w(int a) {
        return a == 0 ? 1.0 / 3.0 : (a < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    __host__ __device__ static constexpr int opp(int a) {
        constexpr int O[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
        return O[a];
    }
};

const char* kernel_class_name(int k) {
    static const char* names[KC_COUNT] = {"stream", "cg_init", "cg_a", "cg_b", "lumped", "moments",
                                          "grad", "div", "collide", "init", "sums", "finalize", "cheb"};
    return (k >= 0 && k < KC_COUNT) ? names[k] : "?";
}

// ---------------------------------------------------------------------------
// helpers

// Block -> tile, XCD-aware: block b runs on XCD b % 8; give each XCD a
// contiguous range of tiles.
__device__ __forceinline__ int tile_of_block(int b, int nblocks) {
    constexpr int NX = 8;
    const int xcd = b % NX, idx = b / NX;
    const int base = nblocks / NX, extra = nblocks % NX;
    return xcd * base + min(xcd, extra) + idx;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the wavefront of N values per lane (N a power of two <= 64) in
// log2(N) + log2(64 / N) exchange steps instead of N * 6: at each of the
// first log2(N) steps a lane pair splits its values in halves, each lane
// keeps one half and adds the partner's copy of it; plain xor steps finish.
// Afterwards v[0] of lane l holds the total of value l / (64 / N).  Every
// step is a commutative pairwise add, so all lanes of a group agree bitwise.
template <int N, int M>
struct Butterfly {
    static __device__ __forceinline__ void run(double* v, int lane) {
        constexpr int H = N / 2;
        const bool up = (lane & M) != 0;
#pragma unroll
        for (int i = 0; i < H; i++) {
            const double send = up ? v[i] : v[i + H];
            const double keep = up ? v[i + H] : v[i];
            v[i] = keep + __shfl_xor(send, M, 64);
        }
        Butterfly<H, M / 2>::run(v, lane);
    }
};
template <int M>
struct Butterfly<1, M> {
    static __device__ __forceinline__ void run(double* v, int) {
#pragma unroll
        for (int m = M; m >= 1; m >>= 1) v[0] += __shfl_xor(v[0], m, 64);
    }
};

template <typename T> __device__ __forceinline__ T ld(const void* p, int64_t i) {
    return reinterpret_cast<const T*>(p)[i];
}
template <typename T> __device__ __forceinline__ void st(void* p, int64_t i, T v) {
    reinterpret_cast<T*>(p)[i] = v;
}

// Deterministic FP64 reduction of NP values per tile: add(j, v) reduces
// v over the wavefront (shuffles) into LDS; finish() sums the waves in a
// fixed order and stores the tile's partials with plain stores.  The
// instance totals are formed by k_finalize in the next launch, so no
// kernel needs a device-scope fence (on multi-XCD parts such a fence writes
// back and invalidates the XCD's L2, which would discard the neighbour
// reuse the gathers depend on).
template <int NP>
struct TileReducer {
    static_assert(NP <= TILE, "too many reduction values");
    double (*lds)[NP];
    __device__ __forceinline__ explicit TileReducer(double (*buf)[NP]) : lds(buf) {}
    __device__ __forceinline__ void add(int j, double v) {
        v = wave_sum(v);
        if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6][j] = v;
    }
    // values j0 .. j0 + G - 1 at once (G a power of two)
    template <int G>
    __device__ __forceinline__ void add_group(int j0, double (&v)[G]) {
        const int lane = threadIdx.x & 63;
        Butterfly<G, 32>::run(v, lane);
        constexpr int S = 64 / G;
        if ((lane & (S - 1)) == 0) lds[threadIdx.x >> 6][j0 + lane / S] = v[0];
    }
    __device__ __forceinline__ void finish(const DevLayout& L, int tile) {
        __syncthreads();
        for (int j = threadIdx.x; j < NP; j += TILE) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < TILE / 64; w++) s += lds[w][j];
            L.partial[(int64_t)tile * NP + j] = s;
        }
    }
};

// What a finalize launch does with the instance totals.
enum FinOp { FIN_CG_INIT = 0, FIN_CG_A, FIN_CG_B, FIN_CG_LAST, FIN_SUMS };

// One block per (instance, value j): sums the instance's tile partials of
// value j in a fixed order (strided per thread, then wavefront shuffles and
// the waves in order) and derives the CG scalar (or stores the conserved sum).
constexpr int FIN_THREADS = 256;

template <int NP>
__global__ __launch_bounds__(FIN_THREADS) void k_finalize(DevLayout L, int inst_begin, int op) {
    __shared__ double fin[FIN_THREADS / 64];
    const int inst = inst_begin + blockIdx.x;
    const int j = blockIdx.y;
    const int tb = L.params[inst].tile_begin, nt = L.params[inst].tile_count;
    const double* src = L.partial + (int64_t)tb * NP + j;
    double s = 0.0;
#pragma unroll 4
    for (int t = threadIdx.x; t < nt; t += FIN_THREADS) s += src[(int64_t)t * NP];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) fin[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < FIN_THREADS / 64; w++) tot += fin[w];
    const int i = inst * NP + j;
    switch (op) {
    case FIN_CG_INIT:
        L.rz[i] = tot;
        L.rz0[i] = tot;
        L.beta[i] = 0.0;
        break;
    case FIN_CG_A:
        L.alpha[i] = (tot != 0.0) ? L.rz[i] / tot : 0.0;
        break;
    case FIN_CG_B: {
        const double rz = L.rz[i];
        L.beta[i] = (rz != 0.0) ? tot / rz : 0.0;
        L.rz[i] = tot;
        break;
    }
    case FIN_CG_LAST: {
        const double r0 = L.rz0[i];
        if (r0 > 0.0 && !(tot <= L.cg_tol2 * r0)) atomicOr(L.status, 2u);
        break;
    }
    case FIN_SUMS:
        L.sums[inst * 8 + j] = tot;
        break;
    }
}

#define FEL_REDUCER(NAME, NP)                         \
    __shared__ double NAME##_buf[TILE / 64][NP];      \
    TileReducer<NP> NAME(NAME##_buf)

// gathers through a uniform base and a 32-bit byte offset
template <typename T>
__device__ __forceinline__ T gat(const T* base, int idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)idx * (uint32_t)sizeof(T));
}

// ---------------------------------------------------------------------------
// streaming right-hand side, FP64 populations:
// rhs_a = -(dt sum_r c_ar G_r + dt^2/2 sum_rs c_ar c_as K_rs) psi_a  for a != 0
template <int Q, int W>
__global__ __launch_bounds__(TILE) void k_stream_plain(DevLayout L, int tile_begin) {
    using LT = Lat<Q>;
    constexpr int D = LT::D, NB = LT::NB, NP = 2 * (Q - 1);
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int64_t R = L.R;
    const int64_t row = (int64_t)tile * TILE + threadIdx.x;
    const InstParams& P = L.params[L.tile_inst[tile]];
    const double dt = P.dt, h2 = 0.5 * dt * dt;
    const double* psi = reinterpret_cast<const double*>(L.psi);
    const double* B = reinterpret_cast<const double*>(L.basis);
    double acc[NP];
#pragma unroll
    for (int j = 0; j < NP; j++) acc[j] = 0.0;
#pragma unroll
    for (int k = 0; k < W; k++) {
        const int64_t c = L.col[k * R + row];
        double b[NB];
#pragma unroll
        for (int n = 0; n < NB; n++) b[n] = B[((int64_t)n * W + k) * R + row];
#pragma unroll
        for (int a = 1; a < Q; a++) {
            const double ex = LT::e(a, 0), ey = LT::e(a, 1), ez = LT::e(a, 2);
            double coef;
            if constexpr (D == 2) {
                coef = dt * (ex * b[0] + ey * b[1]) + h2 * (ex * ex * b[2] + ey * ey * b[3] + ex * ey * b[4]);
            } else {
                coef = dt * (ex * b[0] + ey * b[1] + ez * b[2]) +
                       h2 * (ex * ex * b[3] + ey * ey * b[4] + ez * ez * b[5] + ex * ey * b[6] +
                             ex * ez * b[7] + ey * ez * b[8]);
            }
            acc[a - 1] += coef * psi[(int64_t)a * R + c];
            acc[Q - 1 + a - 1] += coef * psi[(int64_t)(Q + a) * R + c];
        }
    }
    double* rhs = reinterpret_cast<double*>(L.Pb);
#pragma unroll
    for (int j = 0; j < NP; j++) rhs[(int64_t)j * R + row] = -acc[j];
}

// ---------------------------------------------------------------------------
// conjugate gradients on M (batched over populations and instances),
// lumped preconditioner z = r / m, start x0 = rhs / m.

// Thread layout of the solver kernels: one thread per row, a block covers
// one tile of TILE rows, so every wavefront load is 64 consecutive rows of
// one population.  Each kernel walks the NP populations of its row as a
// two-stage software pipeline (run_rows): the loads of the next batch of CH
// populations (neighbour gathers and own-row values) are issued before the
// current batch is used, so a wave has up to 2 CH populations' loads in
// flight.  CH (1, 2 or 4) is chosen per kernel by the autotuner.  A batch
// only writes its own populations' rows and only reads populations or
// buffers that the launch does not write, so the early loads are safe.
// The FP64 dot products are reduced RG populations at a time.
constexpr int RG = 4;

template <int NP, int CH, class Body>
__device__ __forceinline__ void run_rows(Body& body, TileReducer<NP>* red) {
    static_assert(NP % CH == 0 && NP % RG == 0, "population batches must tile NP");
    typename Body::Regs buf[2][CH];
#pragma unroll
    for (int u = 0; u < CH; u++) body.load(u, buf[0][u]);
    double dots[RG];
#pragma unroll
    for (int j0 = 0; j0 < NP; j0 += CH) {
        const int cur = (j0 / CH) & 1;
        if (j0 + CH < NP) {
#pragma unroll
            for (int u = 0; u < CH; u++) body.load(j0 + CH + u, buf[cur ^ 1][u]);
        }
#pragma unroll
        for (int u = 0; u < CH; u++) {
            const int j = j0 + u;
            const double d = body.use(j, buf[cur][u]);
            if constexpr (Body::kDots) {
                dots[j % RG] = d;
                if (j % RG == RG - 1) red->add_group(j - (RG - 1), dots);
            }
        }
    }
}

#define FEL_ROW_LAYOUT()                                                 \
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x); \
    const int64_t R = L.R;                                               \
    const int row = tile * TILE + threadIdx.x

// Row operands shared by the solver bodies: ELL columns and mass values of
// the row, and (MI) the inverse lumped mass at the columns.
template <typename T, int W, bool MI>
struct RowOps {
    int c[W];
    T mv[W], mi[MI ? W : 1];
    T mrow;
    __device__ __forceinline__ void load(const DevLayout& L, int64_t R, int row) {
        const T* minv = reinterpret_cast<const T*>(L.minv);
#pragma unroll
        for (int k = 0; k < W; k++) {
            c[k] = L.col[k * R + row];
            mv[k] = ld<T>(L.Mval, k * R + row);
            if constexpr (MI) mi[k] = gat(minv, c[k]);
        }
        mrow = minv[row];
    }
};

// cg_init: X = rhs / m, r = rhs - M X, reduces r.z
template <typename T, int W, int NP>
struct CgInitRows {
    static constexpr bool kDots = true;
    struct Regs { T g[W]; T own; };
    RowOps<T, W, true> o;
    const T* rhs;
    T *X, *Rv;
    int64_t R;
    int row;
    __device__ __forceinline__ void load(int j, Regs& r) const {
        const T* b = rhs + (int64_t)j * R;
#pragma unroll
        for (int k = 0; k < W; k++) r.g[k] = gat(b, o.c[k]);
        r.own = b[row];
    }
    __device__ __forceinline__ double use(int j, const Regs& r) const {
        T acc = 0;
#pragma unroll
        for (int k = 0; k < W; k++) acc += o.mv[k] * (r.g[k] * o.mi[k]);
        const T res = r.own - acc;
        const int64_t i = (int64_t)j * R + row;
        X[i] = r.own * o.mrow;
        Rv[i] = res;
        return (double)res * (double)res * (double)o.mrow;
    }
};

// cg_a: p_new = r / m + beta p_old (p_old unread on the first iteration),
// q = M p_new recomputed from neighbour values; reduces p.q -> alpha.
template <typename T, int W, int NP, bool FIRST>
struct CgARows {
    static constexpr bool kDots = true;
    struct Regs { T g[W]; T h[FIRST ? 1 : W]; T own, ownp; };
    RowOps<T, W, true> o;
    const T *Rv, *Pold;
    T* Pnew;
    const double* beta;
    int64_t R;
    int row;
    __device__ __forceinline__ void load(int j, Regs& r) const {
        const T* rv = Rv + (int64_t)j * R;
#pragma unroll
        for (int k = 0; k < W; k++) r.g[k] = gat(rv, o.c[k]);
        r.own = rv[row];
        if constexpr (!FIRST) {
            const T* po = Pold + (int64_t)j * R;
#pragma unroll
            for (int k = 0; k < W; k++) r.h[k] = gat(po, o.c[k]);
            r.ownp = po[row];
        }
    }
    __device__ __forceinline__ double use(int j, const Regs& r) const {
        T acc = 0, pown;
        if constexpr (FIRST) {
#pragma unroll
            for (int k = 0; k < W; k++) acc += o.mv[k] * (r.g[k] * o.mi[k]);
            pown = r.own * o.mrow;
        } else {
            const T bet = (T)beta[j];
#pragma unroll
            for (int k = 0; k < W; k++) acc += o.mv[k] * (r.g[k] * o.mi[k] + bet * r.h[k]);
            pown = r.own * o.mrow + bet * r.ownp;
        }
        Pnew[(int64_t)j * R + row] = pown;
        return (double)pown * (double)acc;
    }
};

// cg_b: x += alpha p, r -= alpha M p (M p recomputed), reduces r.z -> beta
template <typename T, int W, int NP>
struct CgBRows {
    static constexpr bool kDots = true;
    struct Regs { T g[W]; T own, x, r; };
    RowOps<T, W, false> o;
    const T* Pn;
    T *X, *Rv;
    const double* alpha;
    int64_t R;
    int row;
    __device__ __forceinline__ void load(int j, Regs& r) const {
        const T* p = Pn + (int64_t)j * R;
#pragma unroll
        for (int k = 0; k < W; k++) r.g[k] = gat(p, o.c[k]);
        r.own = p[row];
        const int64_t i = (int64_t)j * R + row;
        r.x = X[i];
        r.r = Rv[i];
    }
    __device__ __forceinline__ double use(int j, const Regs& r) const {
        T qq = 0;
#pragma unroll
        for (int k = 0; k < W; k++) qq += o.mv[k] * r.g[k];
        const T al = (T)alpha[j];
        const int64_t i = (int64_t)j * R + row;
        const T res = r.r - al * qq;
        X[i] = r.x + al * r.own;
        Rv[i] = res;
        return (double)res * (double)res * (double)o.mrow;
    }
};

template <typename T, int W, int NP, int CH>
__global__ __launch_bounds__(TILE) void k_cg_init(DevLayout L, int tile_begin) {
    FEL_ROW_LAYOUT();
    CgInitRows<T, W, NP> b;
    b.o.load(L, R, row);
    b.rhs = reinterpret_cast<const T*>(L.Pb);
    b.X = reinterpret_cast<T*>(L.X);
    b.Rv = reinterpret_cast<T*>(L.Rv);
    b.R = R;
    b.row = row;
    FEL_REDUCER(red, NP);
    run_rows<NP, CH>(b, &red);
    red.finish(L, tile);
}

template <typename T, int W, int NP, int CH>
__global__ __launch_bounds__(TILE) void k_cg_a(DevLayout L, int tile_begin, int first, int flip) {
    FEL_ROW_LAYOUT();
    const int inst = L.tile_inst[tile];
    const T* Rv = reinterpret_cast<const T*>(L.Rv);
    const T* Pold = reinterpret_cast<const T*>(flip ? L.Pa : L.Pb);
    T* Pnew = reinterpret_cast<T*>(flip ? L.Pb : L.Pa);
    FEL_REDUCER(red, NP);
    if (first) {
        CgARows<T, W, NP, true> b;
        b.o.load(L, R, row);
        b.Rv = Rv, b.Pold = Pold, b.Pnew = Pnew, b.beta = L.beta + inst * NP, b.R = R, b.row = row;
        run_rows<NP, CH>(b, &red);
    } else {
        CgARows<T, W, NP, false> b;
        b.o.load(L, R, row);
        b.Rv = Rv, b.Pold = Pold, b.Pnew = Pnew, b.beta = L.beta + inst * NP, b.R = R, b.row = row;
        run_rows<NP, CH>(b, &red);
    }
    red.finish(L, tile);
}

template <typename T, int W, int NP, int CH>
__global__ __launch_bounds__(TILE) void k_cg_b(DevLayout L, int tile_begin, int flip) {
    FEL_ROW_LAYOUT();
    const int inst = L.tile_inst[tile];
    CgBRows<T, W, NP> b;
    b.o.load(L, R, row);
    b.Pn = reinterpret_cast<const T*>(flip ? L.Pb : L.Pa);
    b.X = reinterpret_cast<T*>(L.X);
    b.Rv = reinterpret_cast<T*>(L.Rv);
    b.alpha = L.alpha + inst * NP;
    b.R = R;
    b.row = row;
    FEL_REDUCER(red, NP);
    run_rows<NP, CH>(b, &red);
    red.finish(L, tile);
}

// Chebyshev semi-iteration on M Delta = rhs, preconditioned by the lumped
// mass, with the a-priori spectrum bounds of m^-1 M ([1/(d+2), 1] for P1
// simplices, element by element):
//   x_0 = rhs / m,   x_1 = x_0 + gamma z_0,
//   x_{k+1} = omega_{k+1} (gamma z_k + x_k - x_{k-1}) + x_{k-1},
//   z_k = m^-1 (rhs - M x_k).
// No inner products, so no reductions; sum m x is conserved at every iterate
// (sum m z_k = 0).  The two iterates live in buf 0 = X and buf 1 = Pa; a
// launch reads x_k (gathered) and x_{k-1} (own row) and overwrites x_{k-1}.
template <typename T>
__device__ __forceinline__ T* cheb_buf(const DevLayout& L, int b) {
    return reinterpret_cast<T*>(b ? L.Pa : L.X);
}

template <typename T, int W, int NP>
struct ChebFirstRows {
    static constexpr bool kDots = false;
    struct Regs { T g[W]; T own; };
    RowOps<T, W, true> o;
    const T* rhs;
    T *x0, *x1;
    T gamma;
    int64_t R;
    int row;
    __device__ __forceinline__ void load(int j, Regs& r) const {
        const T* b = rhs + (int64_t)j * R;
#pragma unroll
        for (int k = 0; k < W; k++) r.g[k] = gat(b, o.c[k]);
        r.own = b[row];
    }
    __device__ __forceinline__ double use(int j, const Regs& r) const {
        T acc = 0;
#pragma unroll
        for (int k = 0; k < W; k++) acc += o.mv[k] * (r.g[k] * o.mi[k]);
        const T xa = r.own * o.mrow;
        const int64_t i = (int64_t)j * R + row;
        x0[i] = xa;
        x1[i] = xa + gamma * ((r.own - acc) * o.mrow);
        return 0.0;
    }
};

template <typename T, int W, int NP>
struct ChebRows {
    static constexpr bool kDots = false;
    struct Regs { T g[W]; T own, b, xp; };
    RowOps<T, W, false> o;
    const T *rhs, *xk;
    T* xp;
    T omega, gamma;
    int64_t R;
    int row;
    __device__ __forceinline__ void load(int j, Regs& r) const {
        const T* x = xk + (int64_t)j * R;
#pragma unroll
        for (int k = 0; k < W; k++) r.g[k] = gat(x, o.c[k]);
        r.own = x[row];
        const int64_t i = (int64_t)j * R + row;
        r.b = rhs[i];
        r.xp = xp[i];
    }
    __device__ __forceinline__ double use(int j, const Regs& r) const {
        T acc = 0;
#pragma unroll
        for (int k = 0; k < W; k++) acc += o.mv[k] * r.g[k];
        const T z = (r.b - acc) * o.mrow;
        xp[(int64_t)j * R + row] = omega * (gamma * z + r.own - r.xp) + r.xp;
        return 0.0;
    }
};

template <typename T, int W, int NP, int CH>
__global__ __launch_bounds__(TILE) void k_cheb_first(DevLayout L, int tile_begin, int out0, double gamma_d) {
    FEL_ROW_LAYOUT();
    ChebFirstRows<T, W, NP> b;
    b.o.load(L, R, row);
    b.rhs = reinterpret_cast<const T*>(L.Pb);
    b.x0 = cheb_buf<T>(L, out0);
    b.x1 = cheb_buf<T>(L, 1 - out0);
    b.gamma = (T)gamma_d;
    b.R = R;
    b.row = row;
    run_rows<NP, CH>(b, (TileReducer<NP>*)nullptr);
}

template <typename T, int W, int NP, int CH>
__global__ __launch_bounds__(TILE) void k_cheb(DevLayout L, int tile_begin, int cur, double omega_d,
                                               double gamma_d) {
    FEL_ROW_LAYOUT();
    ChebRows<T, W, NP> b;
    b.o.load(L, R, row);
    b.rhs = reinterpret_cast<const T*>(L.Pb);
    b.xk = cheb_buf<T>(L, cur);
    b.xp = cheb_buf<T>(L, 1 - cur);
    b.omega = (T)omega_d;
    b.gamma = (T)gamma_d;
    b.R = R;
    b.row = row;
    run_rows<NP, CH>(b, (TileReducer<NP>*)nullptr);
}

// lumped-mass approximation: Delta = rhs / m
template <typename T, int NP>
__global__ __launch_bounds__(TILE) void k_lumped(DevLayout L, int tile_begin) {
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int64_t R = L.R;
    const int64_t row = (int64_t)tile * TILE + threadIdx.x;
    const T mrow = ld<T>(L.minv, row);
#pragma unroll 4
    for (int j = 0; j < NP; j++) st<T>(L.X, (int64_t)j * R + row, ld<T>(L.Pb, (int64_t)j * R + row) * mrow);
}

// ---------------------------------------------------------------------------
// walls + density moment, FP64 populations
template <int Q>
__device__ __forceinline__ void streamed_plain(const DevLayout& L, int64_t row, int base, double (&v)[Q]) {
    // base = 0 for f, Q for g; X holds Delta for populations 1..Q-1 of each
    const int64_t R = L.R;
    const double* psi = reinterpret_cast<const double*>(L.psi);
    const double* X = reinterpret_cast<const double*>(L.X);
    const int xb = base ? (Q - 1) : 0;
    v[0] = psi[(int64_t)base * R + row];
#pragma unroll
    for (int a = 1; a < Q; a++) v[a] = psi[(int64_t)(base + a) * R + row] + X[(int64_t)(xb + a - 1) * R + row];
}

template <int Q, typename T>
__device__ __forceinline__ void bounce(uint32_t mask, T (&v)[Q]) {
    if (!mask) return;
    T t[Q];
#pragma unroll
    for (int a = 0; a < Q; a++) t[a] = v[a];
#pragma unroll
    for (int a = 0; a < Q; a++)
        if (mask & (1u << a)) v[a] = t[Lat<Q>::opp(a)];
}

template <int Q>
__global__ __launch_bounds__(TILE) void k_moments_plain(DevLayout L, int tile_begin) {
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int64_t row = (int64_t)tile * TILE + threadIdx.x;
    double f[Q];
    streamed_plain<Q>(L, row, 0, f);
    bounce<Q>(L.wmask[row], f);
    double rho = 0.0;
#pragma unroll
    for (int a = 0; a < Q; a++) rho += f[a];
    st<double>(L.rho, row, rho);
}

// ---------------------------------------------------------------------------
// nodal recovery (volume-weighted averaging == m^-1 G)
template <typename T, int W, int D>
__global__ __launch_bounds__(TILE) void k_grad(DevLayout L, int tile_begin) {
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int64_t R = L.R;
    const int64_t row = (int64_t)tile * TILE + threadIdx.x;
    const T* rho = reinterpret_cast<const T*>(L.rho);
    const T* B = reinterpret_cast<const T*>(L.basis);
    T g[D];
#pragma unroll
    for (int r = 0; r < D; r++) g[r] = 0;
#pragma unroll
    for (int k = 0; k < W; k++) {
        const T v = rho[L.col[k * R + row]];
#pragma unroll
        for (int r = 0; r < D; r++) g[r] += B[((int64_t)r * W + k) * R + row] * v;
    }
    const T mi = ld<T>(L.minv, row);
#pragma unroll
    for (int r = 0; r < D; r++) st<T>(L.grad, (int64_t)r * R + row, g[r] * mi);
}

// Laplacian, stress vector S and chemical potential mu at each node
template <typename T, int W, int D>
__global__ __launch_bounds__(TILE) void k_div(DevLayout L, int tile_begin) {
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int64_t R = L.R;
    const int64_t row = (int64_t)tile * TILE + threadIdx.x;
    const InstParams& P = L.params[L.tile_inst[tile]];
    const T* grad = reinterpret_cast<const T*>(L.grad);
    const T* rhoA = reinterpret_cast<const T*>(L.rho);
    const T* B = reinterpret_cast<const T*>(L.basis);
    T lap = 0, S[D];
#pragma unroll
    for (int r = 0; r < D; r++) S[r] = 0;
#pragma unroll
    for (int k = 0; k < W; k++) {
        const int64_t c = L.col[k * R + row];
        T gk[D], Gk[D];
        T E = 0;
#pragma unroll
        for (int r = 0; r < D; r++) {
            gk[r] = grad[(int64_t)r * R + c];
            Gk[r] = B[((int64_t)r * W + k) * R + row];
            E += gk[r] * gk[r];
        }
        T gG = 0;
#pragma unroll
        for (int r = 0; r < D; r++) gG += Gk[r] * gk[r];
        if (L.lap_mode == 0) lap += gG;
#pragma unroll
        for (int i = 0; i < D; i++) S[i] += Gk[i] * E - gk[i] * gG;
        if (L.lap_mode == 1) {
            T ksum = 0;
#pragma unroll
            for (int r = 0; r < D; r++) ksum += B[((int64_t)(D + r) * W + k) * R + row];
            lap -= ksum * rhoA[c];
        }
    }
    const T mi = ld<T>(L.minv, row);
    const T kappa = (T)P.kappa, beta = (T)P.beta;
    const T rl = (T)P.rho_l, rv = (T)P.rho_v;
    const T rho = rhoA[row];
    const T muphi = (T)4 * beta * (rho - rv) * (rho - rl) * (rho - (T)0.5 * (rv + rl));
    st<T>(L.mu, row, muphi - kappa * lap * mi);
#pragma unroll
    for (int i = 0; i < D; i++) st<T>(L.S, (int64_t)i * R + row, kappa * S[i] * mi);
}

// ---------------------------------------------------------------------------
// local physics: equilibria and forcing at one node (Sections 2.1, 2.2)
struct NodeState {
    double rho, p, u[3], gr[3], S[3], gm[3], g[3], dt;
};

// calls fn(a, feq, geq, F, G + Gbody) for every direction
template <int Q, typename Fn>
__device__ __forceinline__ void node_terms(const NodeState& n, Fn fn) {
    using LT = Lat<Q>;
    constexpr int D = LT::D;
    double uu = 0.0, u2[3], uu2 = 0.0;
#pragma unroll
    for (int r = 0; r < 3; r++) {
        uu += n.u[r] * n.u[r];
        u2[r] = n.u[r] + n.g[r] * n.dt;
        uu2 += u2[r] * u2[r];
    }
    const double hdt = 0.5 * n.dt;
#pragma unroll
    for (int a = 0; a < Q; a++) {
        const double w = LT::w(a);
        double eu = 0.0, eu2 = 0.0, ef = 0.0, eg = 0.0, eS = 0.0;
#pragma unroll
        for (int r = 0; r < D; r++) {
            const double e = LT::e(a, r);
            const double em = e - n.u[r];
            eu += e * n.u[r];
            eu2 += e * u2[r];
            ef += em * (n.gr[r] * (1.0 / 3.0) - n.rho * n.gm[r]);
            eg += em * n.gr[r];
            eS += em * n.S[r];
        }
        const double gam = w * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        const double gam2 = w * (1.0 + 3.0 * eu2 + 4.5 * eu2 * eu2 - 1.5 * uu2);
        const double feq = n.rho * gam;
        const double geq = w * 3.0 * n.p + n.rho * (gam - w);
        const double F = hdt * 3.0 * ef * gam;
        const double G = hdt * eg * (gam - w) + hdt * 3.0 * eS * gam;
        const double Gb = 0.5 * n.rho * (gam2 - gam);
        fn(a, feq, geq, F, G + Gb);
    }
}

template <int W, int D>
__device__ __forceinline__ void gather_gradmu(const DevLayout& L, int64_t row, double (&gm)[3]) {
    const int64_t R = L.R;
    const double* mu = reinterpret_cast<const double*>(L.mu);
    const double* B = reinterpret_cast<const double*>(L.basis);
#pragma unroll
    for (int r = 0; r < 3; r++) gm[r] = 0.0;
#pragma unroll
    for (int k = 0; k < W; k++) {
        const double v = mu[L.col[k * R + row]];
#pragma unroll
        for (int r = 0; r < D; r++) gm[r] += B[((int64_t)r * W + k) * R + row] * v;
    }
    const double mi = ld<double>(L.minv, row);
#pragma unroll
    for (int r = 0; r < D; r++) gm[r] *= mi;
}

__device__ __forceinline__ double tau_of(const InstParams& P, double rho) {
    double C = (rho - P.rho_v) / (P.rho_l - P.rho_v);
    C = fmin(fmax(C, 0.0), 1.0);
    return 1.0 / (C / P.tau_l + (1.0 - C) / P.tau_v);
}

// fused post-streaming + pre-streaming collision, FP64 populations
template <int Q, int W>
__global__ __launch_bounds__(TILE) void k_collide_plain(DevLayout L, int tile_begin) {
    using LT = Lat<Q>;
    constexpr int D = LT::D;
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int64_t R = L.R;
    const int64_t row = (int64_t)tile * TILE + threadIdx.x;
    const InstParams& P = L.params[L.tile_inst[tile]];
    if (row >= P.row_end) return;
    double f[Q], g[Q];
    streamed_plain<Q>(L, row, 0, f);
    streamed_plain<Q>(L, row, Q, g);
    const uint32_t mask = L.wmask[row];
    bounce<Q>(mask, f);
    bounce<Q>(mask, g);
    NodeState n;
    n.dt = P.dt;
    n.rho = ld<double>(L.rho, row);
    double sg = 0.0, mom[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < Q; a++) {
        sg += g[a];
#pragma unroll
        for (int r = 0; r < D; r++) mom[r] += LT::e(a, r) * g[a];
    }
    double ugr = 0.0;
#pragma unroll
    for (int r = 0; r < 3; r++) {
        n.g[r] = (r < D) ? P.grav[r] : 0.0;
        n.gr[r] = (r < D) ? ld<double>(L.grad, (int64_t)r * R + row) : 0.0;
        n.S[r] = (r < D) ? ld<double>(L.S, (int64_t)r * R + row) : 0.0;
        n.u[r] = (r < D) ? (mom[r] + 0.5 * n.dt * n.S[r] + 0.5 * n.dt * n.rho * n.g[r]) / n.rho : 0.0;
        ugr += n.u[r] * n.gr[r];
    }
    n.p = sg * (1.0 / 3.0) + 0.5 * n.dt * ugr * (1.0 / 3.0);
    gather_gradmu<W, D>(L, row, n.gm);
    const double tau = tau_of(P, n.rho);
    const double om = 2.0 / (2.0 * tau + 1.0), ph = 4.0 * tau / (2.0 * tau + 1.0);
    double* psi = reinterpret_cast<double*>(L.psi);
    bool bad = false;
    node_terms<Q>(n, [&](int a, double feq, double geq, double F, double Gt) {
        const double fn = f[a] - om * (f[a] - feq) + ph * F;
        const double gn = g[a] - om * (g[a] - geq) + ph * Gt;
        bad |= !isfinite(fn) || !isfinite(gn);
        psi[(int64_t)a * R + row] = fn;
        psi[(int64_t)(Q + a) * R + row] = gn;
    });
#pragma unroll
    for (int r = 0; r < D; r++) st<double>(L.u, (int64_t)r * R + row, n.u[r]);
    st<double>(L.p, row, n.p);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(L.status, 1u);
}

// initial populations: equilibrium of (rho, u, p) plus the pre-streaming forcing
template <int Q, int W>
__global__ __launch_bounds__(TILE) void k_init_plain(DevLayout L, int tile_begin) {
    using LT = Lat<Q>;
    constexpr int D = LT::D;
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int64_t R = L.R;
    const int64_t row = (int64_t)tile * TILE + threadIdx.x;
    const InstParams& P = L.params[L.tile_inst[tile]];
    double* psi = reinterpret_cast<double*>(L.psi);
    if (row >= P.row_end) {
#pragma unroll
        for (int a = 0; a < 2 * Q; a++) psi[(int64_t)a * R + row] = 0.0;
        return;
    }
    NodeState n;
    n.dt = P.dt;
    n.rho = ld<double>(L.rho, row);
    n.p = ld<double>(L.p, row);
#pragma unroll
    for (int r = 0; r < 3; r++) {
        n.g[r] = (r < D) ? P.grav[r] : 0.0;
        n.gr[r] = (r < D) ? ld<double>(L.grad, (int64_t)r * R + row) : 0.0;
        n.S[r] = (r < D) ? ld<double>(L.S, (int64_t)r * R + row) : 0.0;
        n.u[r] = (r < D) ? ld<double>(L.u, (int64_t)r * R + row) : 0.0;
    }
    gather_gradmu<W, D>(L, row, n.gm);
    node_terms<Q>(n, [&](int a, double feq, double geq, double F, double Gt) {
        psi[(int64_t)a * R + row] = feq + F;
        psi[(int64_t)(Q + a) * R + row] = geq + Gt;
    });
}

// conserved sums (FP64), FP64 populations:
// m rho, m C, m (1 - C), m sum_a e_a gbar_a
template <int Q>
__global__ __launch_bounds__(TILE) void k_sums_plain(DevLayout L, int tile_begin) {
    using LT = Lat<Q>;
    constexpr int D = LT::D;
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int inst = L.tile_inst[tile];
    const int64_t R = L.R;
    const int64_t row = (int64_t)tile * TILE + threadIdx.x;
    const InstParams& P = L.params[inst];
    const double* psi = reinterpret_cast<const double*>(L.psi);
    const double m = L.mlump[row];
    double part[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    bool bad = false;
    if (row < P.row_end) {
        double rho = 0.0, mom[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < Q; a++) {
            const double fa = psi[(int64_t)a * R + row], ga = psi[(int64_t)(Q + a) * R + row];
            bad |= !isfinite(fa) || !isfinite(ga);
            rho += fa;
#pragma unroll
            for (int r = 0; r < D; r++) mom[r] += LT::e(a, r) * ga;
        }
        const double C = (rho - P.rho_v) / (P.rho_l - P.rho_v);
        part[0] = m * rho;
        part[1] = m * C;
        part[2] = m * (1.0 - C);
#pragma unroll
        for (int r = 0; r < D; r++) part[3 + r] = m * mom[r];
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(L.status, 1u);
    FEL_REDUCER(red, 8);
#pragma unroll
    for (int j = 0; j < 8; j++) red.add(j, part[j]);
    red.finish(L, tile);
}

// ---------------------------------------------------------------------------
// FP32 path: populations stored as scaled deviations from a node reference,
//   f_a = w_a (ref_f + s d_a),   g_a = w_a (ref_g + s d_{Q+a}),
// with ref_f the density and ref_g = p / cs^2 of the last collision and s
// a per-instance power of two.  Every FP32 operation below acts on small
// quantities: the streaming operator on differences to the row's own value
// (each row of dt C + dt^2 D sums to zero), the collision on deviations from
// the new reference.

template <typename S> __device__ __forceinline__ float ldS(const void* p, int64_t i) {
    return (float)reinterpret_cast<const S*>(p)[i];
}
template <typename S> __device__ __forceinline__ void stS(void* p, int64_t i, float v) {
    reinterpret_cast<S*>(p)[i] = (S)v;
}

template <int Q, int W, typename S>
__global__ __launch_bounds__(TILE) void k_stream_dev(DevLayout L, int tile_begin) {
    using LT = Lat<Q>;
    constexpr int D = LT::D, NB = LT::NB, NP = 2 * (Q - 1);
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int64_t R = L.R;
    const int row = tile * TILE + threadIdx.x;
    const InstParams& P = L.params[L.tile_inst[tile]];
    const float dt = (float)P.dt, h2 = 0.5f * dt * dt, sc = (float)P.scale;
    const float* B = reinterpret_cast<const float*>(L.basis);
    const float* reff = L.ref;
    const float* refg = L.ref + R;
    const float rf0 = reff[row], rg0 = refg[row];
    float d0[NP];
#pragma unroll
    for (int a = 1; a < Q; a++) {
        d0[a - 1] = ldS<S>(L.psi, (int64_t)a * R + row);
        d0[Q - 1 + a - 1] = ldS<S>(L.psi, (int64_t)(Q + a) * R + row);
    }
    float acc[NP];
#pragma unroll
    for (int j = 0; j < NP; j++) acc[j] = 0.0f;
#pragma unroll
    for (int k = 0; k < W; k++) {
        const int c = L.col[k * R + row];
        float b[NB];
#pragma unroll
        for (int n = 0; n < NB; n++) b[n] = B[((int64_t)n * W + k) * R + row];
        const float drf = gat(reff, c) - rf0, drg = gat(refg, c) - rg0;
#pragma unroll
        for (int a = 1; a < Q; a++) {
            const float ex = LT::e(a, 0), ey = LT::e(a, 1), ez = LT::e(a, 2);
            float coef;
            if constexpr (D == 2) {
                coef = dt * (ex * b[0] + ey * b[1]) + h2 * (ex * ex * b[2] + ey * ey * b[3] + ex * ey * b[4]);
            } else {
                coef = dt * (ex * b[0] + ey * b[1] + ez * b[2]) +
                       h2 * (ex * ex * b[3] + ey * ey * b[4] + ez * ez * b[5] + ex * ey * b[6] +
                             ex * ez * b[7] + ey * ez * b[8]);
            }
            const float df = ldS<S>(L.psi, (int64_t)a * R + c) - d0[a - 1];
            const float dg = ldS<S>(L.psi, (int64_t)(Q + a) * R + c) - d0[Q - 1 + a - 1];
            acc[a - 1] += coef * (drf + sc * df);
            acc[Q - 1 + a - 1] += coef * (drg + sc * dg);
        }
    }
    float* rhs = reinterpret_cast<float*>(L.Pb);
#pragma unroll
    for (int a = 1; a < Q; a++) {
        const float w = (float)LT::w(a);
        rhs[(int64_t)(a - 1) * R + row] = -w * acc[a - 1];
        rhs[(int64_t)(Q - 1 + a - 1) * R + row] = -w * acc[Q - 1 + a - 1];
    }
}

// streamed deviations e_a = s d_a + Delta_a / w_a of one distribution
// (base 0: f, base Q: g), walls applied: psi_s,a = w_a (ref + e_a)
template <int Q, typename S>
__device__ __forceinline__ void streamed_dev(const DevLayout& L, int row, int base, float sc, float (&e)[Q]) {
    using LT = Lat<Q>;
    const int64_t R = L.R;
    const float* X = reinterpret_cast<const float*>(L.X);
    const int xb = base ? (Q - 1) : 0;
    e[0] = sc * ldS<S>(L.psi, (int64_t)base * R + row);
#pragma unroll
    for (int a = 1; a < Q; a++)
        e[a] = sc * ldS<S>(L.psi, (int64_t)(base + a) * R + row) +
               X[(int64_t)(xb + a - 1) * R + row] * (float)(1.0 / LT::w(a));
}

template <int Q, typename S>
__global__ __launch_bounds__(TILE) void k_moments_dev(DevLayout L, int tile_begin) {
    using LT = Lat<Q>;
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int row = tile * TILE + threadIdx.x;
    const InstParams& P = L.params[L.tile_inst[tile]];
    float e[Q];
    streamed_dev<Q, S>(L, row, 0, (float)P.scale, e);
    bounce<Q>(L.wmask[row], e);
    float drho = 0.0f;
#pragma unroll
    for (int a = 0; a < Q; a++) drho += (float)LT::w(a) * e[a];
    st<float>(L.rho, row, L.ref[row] + drho);
}

template <int W, int D, typename T>
__device__ __forceinline__ void gather_grad_of(const DevLayout& L, const void* field, int row, T (&gm)[3]) {
    const int64_t R = L.R;
    const T* f = reinterpret_cast<const T*>(field);
    const T* B = reinterpret_cast<const T*>(L.basis);
#pragma unroll
    for (int r = 0; r < 3; r++) gm[r] = 0;
#pragma unroll
    for (int k = 0; k < W; k++) {
        const T v = gat(f, L.col[k * R + row]);
#pragma unroll
        for (int r = 0; r < D; r++) gm[r] += B[((int64_t)r * W + k) * R + row] * v;
    }
    const T mi = ld<T>(L.minv, row);
#pragma unroll
    for (int r = 0; r < D; r++) gm[r] *= mi;
}

// Per-direction deviation terms at one node, all divided by w_a:
//   gh   = Gamma_a(u) / w_a - 1
//   F    = F_a / w_a,  G = (G_a + body force) / w_a
struct NodeF {
    float rho, P, u[3], gr[3], S[3], gm[3], g[3], dt;
};

template <int Q, typename Fn>
__device__ __forceinline__ void node_terms_dev(const NodeF& n, Fn fn) {
    using LT = Lat<Q>;
    constexpr int D = LT::D;
    float uu = 0.0f, u2[3], uu2 = 0.0f;
#pragma unroll
    for (int r = 0; r < 3; r++) {
        uu += n.u[r] * n.u[r];
        u2[r] = n.u[r] + n.g[r] * n.dt;
        uu2 += u2[r] * u2[r];
    }
    const float hdt = 0.5f * n.dt;
#pragma unroll
    for (int a = 0; a < Q; a++) {
        float eu = 0.0f, eu2 = 0.0f, ef = 0.0f, eg = 0.0f, eS = 0.0f;
#pragma unroll
        for (int r = 0; r < D; r++) {
            const float e = (float)LT::e(a, r);
            const float em = e - n.u[r];
            eu += e * n.u[r];
            eu2 += e * u2[r];
            ef += em * (n.gr[r] * (1.0f / 3.0f) - n.rho * n.gm[r]);
            eg += em * n.gr[r];
            eS += em * n.S[r];
        }
        const float gh = 3.0f * eu + 4.5f * eu * eu - 1.5f * uu;
        const float gh2 = 3.0f * eu2 + 4.5f * eu2 * eu2 - 1.5f * uu2;
        const float F = hdt * 3.0f * ef * (1.0f + gh);
        const float G = hdt * eg * gh + hdt * 3.0f * eS * (1.0f + gh) + 0.5f * n.rho * (gh2 - gh);
        fn(a, gh, F, G);
    }
}

__device__ __forceinline__ float tau_of_f(const InstParams& P, float rho) {
    float C = (rho - (float)P.rho_v) / (float)(P.rho_l - P.rho_v);
    C = fminf(fmaxf(C, 0.0f), 1.0f);
    return 1.0f / (C / (float)P.tau_l + (1.0f - C) / (float)P.tau_v);
}

template <int Q, int W, typename S>
__global__ __launch_bounds__(TILE) void k_collide_dev(DevLayout L, int tile_begin) {
    using LT = Lat<Q>;
    constexpr int D = LT::D;
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int64_t R = L.R;
    const int row = tile * TILE + threadIdx.x;
    const InstParams& P = L.params[L.tile_inst[tile]];
    if (row >= P.row_end) return;
    const float sc = (float)P.scale, isc = 1.0f / sc;
    float ef[Q], eg[Q];
    streamed_dev<Q, S>(L, row, 0, sc, ef);
    streamed_dev<Q, S>(L, row, Q, sc, eg);
    const uint32_t mask = L.wmask[row];
    bounce<Q>(mask, ef);
    bounce<Q>(mask, eg);
    NodeF n;
    n.dt = (float)P.dt;
    const float reff = L.ref[row], refg = L.ref[R + row];
    n.rho = ld<float>(L.rho, row);            // = reff + sum_a w_a ef_a
    float dg = 0.0f, mom[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int a = 0; a < Q; a++) {
        const float we = (float)LT::w(a) * eg[a];
        dg += we;
#pragma unroll
        for (int r = 0; r < D; r++) mom[r] += (float)LT::e(a, r) * we;
    }
    float ugr = 0.0f;
#pragma unroll
    for (int r = 0; r < 3; r++) {
        n.g[r] = (r < D) ? (float)P.grav[r] : 0.0f;
        n.gr[r] = (r < D) ? ld<float>(L.grad, (int64_t)r * R + row) : 0.0f;
        n.S[r] = (r < D) ? ld<float>(L.S, (int64_t)r * R + row) : 0.0f;
        n.u[r] = (r < D) ? (mom[r] + 0.5f * n.dt * n.S[r] + 0.5f * n.dt * n.rho * n.g[r]) / n.rho : 0.0f;
        ugr += n.u[r] * n.gr[r];
    }
    n.P = refg + (dg + 0.5f * n.dt * ugr);    // p / cs^2
    gather_grad_of<W, D, float>(L, L.mu, row, n.gm);
    const float tau = tau_of_f(P, n.rho);
    const float om = 2.0f / (2.0f * tau + 1.0f), ph = 4.0f * tau / (2.0f * tau + 1.0f);
    const float d_rf = reff - n.rho, d_rg = refg - n.P;   // old minus new reference (exact)
    bool bad = false;
    node_terms_dev<Q>(n, [&](int a, float gh, float F, float G) {
        const float eqd = n.rho * gh;                    // f_eq / w - rho  and  g_eq / w - p / cs^2
        const float Ef = d_rf + ef[a], Eg = d_rg + eg[a];
        const float fn = Ef - om * (Ef - eqd) + ph * F;
        const float gn = Eg - om * (Eg - eqd) + ph * G;
        bad |= !isfinite(fn) || !isfinite(gn);
        stS<S>(L.psi, (int64_t)a * R + row, fn * isc);
        stS<S>(L.psi, (int64_t)(Q + a) * R + row, gn * isc);
    });
    L.ref[row] = n.rho;
    L.ref[R + row] = n.P;
#pragma unroll
    for (int r = 0; r < D; r++) st<float>(L.u, (int64_t)r * R + row, n.u[r]);
    st<float>(L.p, row, n.P * (1.0f / 3.0f));
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(L.status, 1u);
}

template <int Q, int W, typename S>
__global__ __launch_bounds__(TILE) void k_init_dev(DevLayout L, int tile_begin) {
    using LT = Lat<Q>;
    constexpr int D = LT::D;
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int64_t R = L.R;
    const int row = tile * TILE + threadIdx.x;
    const InstParams& P = L.params[L.tile_inst[tile]];
    if (row >= P.row_end) {
#pragma unroll
        for (int a = 0; a < 2 * Q; a++) stS<S>(L.psi, (int64_t)a * R + row, 0.0f);
        L.ref[row] = 0.0f;
        L.ref[R + row] = 0.0f;
        return;
    }
    NodeF n;
    n.dt = (float)P.dt;
    n.rho = ld<float>(L.rho, row);
    n.P = 3.0f * ld<float>(L.p, row);
#pragma unroll
    for (int r = 0; r < 3; r++) {
        n.g[r] = (r < D) ? (float)P.grav[r] : 0.0f;
        n.gr[r] = (r < D) ? ld<float>(L.grad, (int64_t)r * R + row) : 0.0f;
        n.S[r] = (r < D) ? ld<float>(L.S, (int64_t)r * R + row) : 0.0f;
        n.u[r] = (r < D) ? ld<float>(L.u, (int64_t)r * R + row) : 0.0f;
    }
    gather_grad_of<W, D, float>(L, L.mu, row, n.gm);
    const float isc = 1.0f / (float)P.scale;
    node_terms_dev<Q>(n, [&](int a, float gh, float F, float G) {
        stS<S>(L.psi, (int64_t)a * R + row, (n.rho * gh + F) * isc);
        stS<S>(L.psi, (int64_t)(Q + a) * R + row, (n.rho * gh + G) * isc);
    });
    L.ref[row] = n.rho;
    L.ref[R + row] = n.P;
}

template <int Q, typename S>
__global__ __launch_bounds__(TILE) void k_sums_dev(DevLayout L, int tile_begin) {
    using LT = Lat<Q>;
    constexpr int D = LT::D;
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int inst = L.tile_inst[tile];
    const int64_t R = L.R;
    const int row = tile * TILE + threadIdx.x;
    const InstParams& P = L.params[inst];
    const double m = L.mlump[row];
    double part[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    bool bad = false;
    if (row < P.row_end) {
        const double sc = P.scale;
        double drho = 0.0, mom[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < Q; a++) {
            const double fa = ldS<S>(L.psi, (int64_t)a * R + row), ga = ldS<S>(L.psi, (int64_t)(Q + a) * R + row);
            bad |= !isfinite(fa) || !isfinite(ga);
            drho += LT::w(a) * sc * fa;
#pragma unroll
            for (int r = 0; r < D; r++) mom[r] += LT::e(a, r) * LT::w(a) * sc * ga;
        }
        const double rho = (double)L.ref[row] + drho;
        const double C = (rho - P.rho_v) / (P.rho_l - P.rho_v);
        part[0] = m * rho;
        part[1] = m * C;
        part[2] = m * (1.0 - C);
#pragma unroll
        for (int r = 0; r < D; r++) part[3 + r] = m * mom[r];
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(L.status, 1u);
    FEL_REDUCER(red, 8);
#pragma unroll
    for (int j = 0; j < 8; j++) red.add(j, part[j]);
    red.finish(L, tile);
}

// ---------------------------------------------------------------------------
// dispatch

#define FEL_CHECK_LAUNCH() return hipGetLastError()

// run body<Q, W>() for the context's lattice and ELL width
template <template <int, int> class Body, typename... A>
static hipError_t dispatch_qw(const DevLayout& L, A... args) {
    (void)hipGetLastError();  // the launch status is read with hipGetLastError: start clean
    if (L.Q == 9) {
        if (L.W == 7) return Body<9, 7>::run(L, args...);
        if (L.W == 12) return Body<9, 12>::run(L, args...);
    } else if (L.Q == 19) {
        if (L.W == 15) return Body<19, 15>::run(L, args...);
        if (L.W == 24) return Body<19, 24>::run(L, args...);
    }
    return hipErrorInvalidValue;
}

template <int Q, int W> struct StreamBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        if (L.precision == 0)
            FEL_LAUNCH((k_stream_plain<Q, W>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else if (L.precision == 1)
            FEL_LAUNCH((k_stream_dev<Q, W, float>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else
            FEL_LAUNCH((k_stream_dev<Q, W, __half>), dim3(nt), dim3(TILE), 0, s, L, tb);
        FEL_CHECK_LAUNCH();
    }
};
// launches kernel K<T, W, NP, CH> for the context's value type and the
// requested population batch (1, 2 or 4)
#define FEL_SOLVER_LAUNCH(K, ch, s, nt, ...)                                                     \
    do {                                                                                        \
        const bool f64_ = L.precision == 0;                                                     \
        switch (ch) {                                                                           \
        case 4:                                                                                 \
            if (f64_) FEL_LAUNCH((K<double, W, NP, 4>), dim3(nt), dim3(TILE), 0, s, __VA_ARGS__); \
            else FEL_LAUNCH((K<float, W, NP, 4>), dim3(nt), dim3(TILE), 0, s, __VA_ARGS__);       \
            break;                                                                              \
        case 2:                                                                                 \
            if (f64_) FEL_LAUNCH((K<double, W, NP, 2>), dim3(nt), dim3(TILE), 0, s, __VA_ARGS__); \
            else FEL_LAUNCH((K<float, W, NP, 2>), dim3(nt), dim3(TILE), 0, s, __VA_ARGS__);       \
            break;                                                                              \
        default:                                                                                \
            if (f64_) FEL_LAUNCH((K<double, W, NP, 1>), dim3(nt), dim3(TILE), 0, s, __VA_ARGS__); \
            else FEL_LAUNCH((K<float, W, NP, 1>), dim3(nt), dim3(TILE), 0, s, __VA_ARGS__);       \
        }                                                                                       \
    } while (0)

template <int Q, int W> struct CgInitBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, int ch, hipStream_t s) {
        constexpr int NP = 2 * (Q - 1);
        FEL_SOLVER_LAUNCH(k_cg_init, ch, s, nt, L, tb);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct CgABody {
    static hipError_t run(const DevLayout& L, int tb, int nt, bool first, bool flip, int ch, hipStream_t s) {
        constexpr int NP = 2 * (Q - 1);
        FEL_SOLVER_LAUNCH(k_cg_a, ch, s, nt, L, tb, (int)first, (int)flip);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct CgBBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, bool flip, int ch, hipStream_t s) {
        constexpr int NP = 2 * (Q - 1);
        FEL_SOLVER_LAUNCH(k_cg_b, ch, s, nt, L, tb, (int)flip);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct LumpedBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        constexpr int NP = 2 * (Q - 1);
        if (L.precision == 0)
            FEL_LAUNCH((k_lumped<double, NP>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else
            FEL_LAUNCH((k_lumped<float, NP>), dim3(nt), dim3(TILE), 0, s, L, tb);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct MomentsBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        if (L.precision == 0)
            FEL_LAUNCH((k_moments_plain<Q>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else if (L.precision == 1)
            FEL_LAUNCH((k_moments_dev<Q, float>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else
            FEL_LAUNCH((k_moments_dev<Q, __half>), dim3(nt), dim3(TILE), 0, s, L, tb);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct GradBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        constexpr int D = Lat<Q>::D;
        if (L.precision == 0)
            FEL_LAUNCH((k_grad<double, W, D>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else
            FEL_LAUNCH((k_grad<float, W, D>), dim3(nt), dim3(TILE), 0, s, L, tb);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct DivBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        constexpr int D = Lat<Q>::D;
        if (L.precision == 0)
            FEL_LAUNCH((k_div<double, W, D>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else
            FEL_LAUNCH((k_div<float, W, D>), dim3(nt), dim3(TILE), 0, s, L, tb);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct CollideBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        if (L.precision == 0)
            FEL_LAUNCH((k_collide_plain<Q, W>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else if (L.precision == 1)
            FEL_LAUNCH((k_collide_dev<Q, W, float>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else
            FEL_LAUNCH((k_collide_dev<Q, W, __half>), dim3(nt), dim3(TILE), 0, s, L, tb);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct InitBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        if (L.precision == 0)
            FEL_LAUNCH((k_init_plain<Q, W>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else if (L.precision == 1)
            FEL_LAUNCH((k_init_dev<Q, W, float>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else
            FEL_LAUNCH((k_init_dev<Q, W, __half>), dim3(nt), dim3(TILE), 0, s, L, tb);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct SumsBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        if (L.precision == 0)
            FEL_LAUNCH((k_sums_plain<Q>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else if (L.precision == 1)
            FEL_LAUNCH((k_sums_dev<Q, float>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else
            FEL_LAUNCH((k_sums_dev<Q, __half>), dim3(nt), dim3(TILE), 0, s, L, tb);
        FEL_CHECK_LAUNCH();
    }
};

hipError_t launch_stream(const DevLayout& L, int tb, int nt, hipStream_t s) {
    return dispatch_qw<StreamBody>(L, tb, nt, s);
}
hipError_t launch_cg_init(const DevLayout& L, int tb, int nt, int ch, hipStream_t s) {
    return dispatch_qw<CgInitBody>(L, tb, nt, ch, s);
}
hipError_t launch_cg_a(const DevLayout& L, int tb, int nt, bool first, bool flip, int ch, hipStream_t s) {
    return dispatch_qw<CgABody>(L, tb, nt, first, flip, ch, s);
}
hipError_t launch_cg_b(const DevLayout& L, int tb, int nt, bool flip, int ch, hipStream_t s) {
    return dispatch_qw<CgBBody>(L, tb, nt, flip, ch, s);
}
hipError_t launch_finalize(const DevLayout& L, int inst_begin, int ninst, int op, int np, hipStream_t s) {
    (void)hipGetLastError();
    if (np == 16)
        FEL_LAUNCH((k_finalize<16>), dim3(ninst, 16), dim3(FIN_THREADS), 0, s, L, inst_begin, op);
    else if (np == 36)
        FEL_LAUNCH((k_finalize<36>), dim3(ninst, 36), dim3(FIN_THREADS), 0, s, L, inst_begin, op);
    else if (np == 8)
        FEL_LAUNCH((k_finalize<8>), dim3(ninst, 8), dim3(FIN_THREADS), 0, s, L, inst_begin, op);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}
template <int Q, int W> struct ChebFirstBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, int out0, double gamma, int ch, hipStream_t s) {
        constexpr int NP = 2 * (Q - 1);
        FEL_SOLVER_LAUNCH(k_cheb_first, ch, s, nt, L, tb, out0, gamma);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct ChebBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, int cur, double omega, double gamma, int ch,
                          hipStream_t s) {
        constexpr int NP = 2 * (Q - 1);
        FEL_SOLVER_LAUNCH(k_cheb, ch, s, nt, L, tb, cur, omega, gamma);
        FEL_CHECK_LAUNCH();
    }
};
hipError_t launch_cheb_first(const DevLayout& L, int tb, int nt, int out0, double gamma, int ch, hipStream_t s) {
    return dispatch_qw<ChebFirstBody>(L, tb, nt, out0, gamma, ch, s);
}
hipError_t launch_cheb(const DevLayout& L, int tb, int nt, int cur, double omega, double gamma, int ch,
                       hipStream_t s) {
    return dispatch_qw<ChebBody>(L, tb, nt, cur, omega, gamma, ch, s);
}

hipError_t launch_lumped(const DevLayout& L, int tb, int nt, hipStream_t s) {
    return dispatch_qw<LumpedBody>(L, tb, nt, s);
}
hipError_t launch_moments(const DevLayout& L, int tb, int nt, hipStream_t s) {
    return dispatch_qw<MomentsBody>(L, tb, nt, s);
}
hipError_t launch_grad(const DevLayout& L, int tb, int nt, hipStream_t s) {
    return dispatch_qw<GradBody>(L, tb, nt, s);
}
hipError_t launch_div(const DevLayout& L, int tb, int nt, hipStream_t s) {
    return dispatch_qw<DivBody>(L, tb, nt, s);
}
hipError_t launch_collide(const DevLayout& L, int tb, int nt, hipStream_t s) {
    return dispatch_qw<CollideBody>(L, tb, nt, s);
}
hipError_t launch_init(const DevLayout& L, int tb, int nt, hipStream_t s) {
    return dispatch_qw<InitBody>(L, tb, nt, s);
}
hipError_t launch_sums(const DevLayout& L, int tb, int nt, hipStream_t s) {
    return dispatch_qw<SumsBody>(L, tb, nt, s);
}

}  // namespace fel
