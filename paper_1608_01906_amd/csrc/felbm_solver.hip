// Mass-matrix solve of the streaming step (Section 2.2.1): M Delta = rhs for
// every moving population of every instance, on gfx950.
//
//   k_cg_init / k_cg_a / k_cg_b   batched conjugate gradients, lumped
//                                 preconditioner z = r / m, x0 = rhs / m
//   k_cg_x                        x = x0 + sum_k alpha_k p_k from the rhs and
//                                 the stored directions, once after the last
//                                 iteration (x0 itself is never stored)
//   k_finalize                    per-instance totals of the tile partials
//                                 -> CG scalars (fixed summation order)
//   k_cg_*_fused                  the same CG with the scalars formed by
//                                 every block of the next launch (2-D; the
//                                 final residual check then runs in k_cg_x)
//   k_cheb_first / k_cheb         Chebyshev semi-iteration, no reductions
//   *_lds                         LDS-staged forms of the above (neighbour
//                                 values read from a per-tile stage)
//   k_lumped                      lumped-mass shortcut Delta = rhs / m
//
// Every launch covers the NP = 2(Q - 1) moving populations of all
// instances.  Vectors are population-major [NP][R]; the per-tile partials
// are population-major too ([NP][ntiles], so a finalize block reads one
// contiguous run); the CG scalars are [instance][NP].
#include "felbm_device.h"

namespace fel {

// What a finalize launch does with the instance totals.
enum FinOp { FIN_CG_INIT = 0, FIN_CG_A, FIN_CG_B, FIN_CG_LAST, FIN_SUMS };

// One block per (instance, value j = blockIdx.y): sums the instance's tile
// partials of value j in a fixed order (strided per thread, then wavefront
// shuffles and the waves in order) and derives the CG scalar (or stores the
// conserved sum); NP is the stride of the scalar arrays.  The partials of
// one value are contiguous, so the block's loads are coalesced, and the
// unrolled strided loop covers instances of up to 8 K tiles (2 M rows) in
// one round of loads.
constexpr int FIN_THREADS = 1024;

template <int NP>
__global__ __launch_bounds__(FIN_THREADS) void k_finalize(DevLayout L, int inst_begin, int op, int it) {
    __shared__ double fin[FIN_THREADS / 64];
    const int inst = inst_begin + blockIdx.x;
    const int j = blockIdx.y;
    const int tb = L.params[inst].tile_begin, nt = L.params[inst].tile_count;
    const double* src = L.partial + (int64_t)j * L.ntiles + tb;
    double s = 0.0;
#pragma unroll 8
    for (int t = threadIdx.x; t < nt; t += FIN_THREADS) s += src[t];
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
        L.alpha[(int64_t)it * L.ninst * NP + i] = (tot != 0.0) ? L.rz[i] / tot : 0.0;
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

// ---------------------------------------------------------------------------
// Thread layout of the solver kernels: one thread per row, a block covers
// one tile of TILE rows, so every wavefront load is 64 consecutive rows of
// one population.  Each kernel walks the NP populations as a two-stage
// software pipeline (run_rows): the loads of the next batch of CH
// populations (neighbour gathers and own-row values) are issued before the
// current batch is used, so a wave has up to 2 CH populations' loads in
// flight.  CH (1, 2 or 4) is chosen per kernel by the autotuner.  A batch
// only writes its own populations' rows and only reads populations or
// buffers that the launch does not write, so the early loads are safe.
// The FP64 dot products are reduced RG populations at a time.
constexpr int RG = 4;

struct NoHook {
    __device__ __forceinline__ void operator()() const {}
};

// `before_use` runs once the loads of the first two batches are issued,
// before any population is used (the fused kernels form their CG scalars
// there, so that latency overlaps the loads).  PIPE = false loads each
// batch only after the previous one is used (one register set instead of
// two, for kernels that would spill otherwise).
template <int NP, int CH, bool PIPE = true, class Body, class Red, class Hook = NoHook>
__device__ __forceinline__ void run_rows(Body& body, Red* red, Hook before_use = Hook()) {
    static_assert(NP % CH == 0 && NP % RG == 0, "population batches must tile NP");
    typename Body::Regs buf[PIPE ? 2 : 1][CH];
#pragma unroll
    for (int u = 0; u < CH; u++) body.load(u, buf[0][u]);
    double dots[RG];
#pragma unroll
    for (int j0 = 0; j0 < NP; j0 += CH) {
        const int cur = PIPE ? (j0 / CH) & 1 : 0;
        if (PIPE && j0 + CH < NP) {
#pragma unroll
            for (int u = 0; u < CH; u++) body.load(j0 + CH + u, buf[cur ^ 1][u]);
        }
        if (j0 == 0) before_use();
#pragma unroll
        for (int u = 0; u < CH; u++) {
            const int j = j0 + u;
            const double d = body.use(j, buf[cur][u]);
            if constexpr (Body::kDots) {
                dots[j % RG] = d;
                if (j % RG == RG - 1) red->add_group(j - (RG - 1), dots);
            }
        }
        if (!PIPE && j0 + CH < NP) {
#pragma unroll
            for (int u = 0; u < CH; u++) body.load(j0 + CH + u, buf[0][u]);
        }
    }
}

#define FEL_ROW_LAYOUT()                                                 \
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x); \
    const int64_t R = L.R;                                               \
    const int row = tile * TILE + threadIdx.x

// Row operands shared by the solver bodies: ELL columns and mass values of
// the row, and (MI) the inverse lumped mass at the columns.  Slot 0 holds
// the diagonal (the host builds every pattern row diagonal-first, padding
// rows included), so its column is the row itself: it is not loaded, and
// the bodies take its value from the row's own load instead of a gather.
template <typename T, int W, bool MI>
struct RowOps {
    int c[W];
    T mv[W], mi[MI ? W : 1];
    T mrow;
    __device__ __forceinline__ void load(const DevLayout& L, int64_t R, int row) {
        const T* minv = reinterpret_cast<const T*>(L.minv);
        mrow = minv[row];
        c[0] = row;
        mv[0] = ld<T>(L.Mval, row);
        if constexpr (MI) mi[0] = mrow;
#pragma unroll
        for (int k = 1; k < W; k++) {
            c[k] = L.col[k * R + row];
            mv[k] = ld<T>(L.Mval, k * R + row);
            if constexpr (MI) mi[k] = gat(minv, c[k]);
        }
    }
};

// The residual vector the CG keeps between its kernels: r in the recompute
// form (2-D layouts), the preconditioned residual z = r / m in the
// recurrence form (ELL width 15 and up), whose cg_a then needs no inverse
// masses at the neighbour columns: W registers fewer per thread, which lets
// the 3-D cg_a run three waves per SIMD instead of two.  (In 2-D the same
// change made the staged cg_a slower.)
template <int W>
constexpr bool z_form() { return W >= kQRecurrenceWidth; }

// cg_init: r = rhs - M x0 with x0 = rhs / m; stores the residual in the
// layout's form (r, or z = r / m in the recurrence form) and reduces r.z
// (x0 is formed again by cg_x, from the same operands, so it is not stored
// here)
template <typename T, int W>
struct CgInitRows {
    static constexpr bool kDots = true;
    struct Regs { T g[W]; T own; };
    RowOps<T, W, true> o;
    const T* rhs;
    T* Rv;
    int64_t R;
    int row;
    bool live = true;  // false: a fused block's spare wave (loads only, no stores, zero terms)
    __device__ __forceinline__ void load(int j, Regs& r) const {
        const T* b = rhs + (int64_t)j * R;
        r.own = b[row];
        r.g[0] = r.own;
#pragma unroll
        for (int k = 1; k < W; k++) r.g[k] = gat(b, o.c[k]);
    }
    __device__ __forceinline__ double use(int j, const Regs& r) const {
        T acc = 0;
#pragma unroll
        for (int k = 0; k < W; k++) acc += o.mv[k] * (r.g[k] * o.mi[k]);
        const T res = r.own - acc;
        const int64_t i = (int64_t)j * R + row;
        if (!live) return 0.0;
        Rv[i] = z_form<W>() ? res * o.mrow : res;
        return (double)res * (double)res * (double)o.mrow;
    }
};

// cg_a: p_new = r / m + beta p_old (p_old unread on the first iteration),
// q = M p_new recomputed from neighbour values; reduces p.q -> alpha.
template <typename T, int W, bool FIRST>
struct CgARows {
    static constexpr bool kDots = true;
    struct Regs { T g[W]; T h[FIRST ? 1 : W]; T own, ownp; };
    RowOps<T, W, true> o;
    const T *Rv, *Pold;
    T* Pnew;
    const double* beta;
    int64_t R;
    int row;
    bool live = true;
    __device__ __forceinline__ void load(int j, Regs& r) const {
        const T* rv = Rv + (int64_t)j * R;
        r.own = rv[row];
        r.g[0] = r.own;
#pragma unroll
        for (int k = 1; k < W; k++) r.g[k] = gat(rv, o.c[k]);
        if constexpr (!FIRST) {
            const T* po = Pold + (int64_t)j * R;
            r.ownp = po[row];
            r.h[0] = r.ownp;
#pragma unroll
            for (int k = 1; k < W; k++) r.h[k] = gat(po, o.c[k]);
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
        if (!live) return 0.0;
        Pnew[(int64_t)j * R + row] = pown;
        return (double)pown * (double)acc;
    }
};

// cg_b: r -= alpha M p (M p recomputed), reduces r.z -> beta (x is formed
// after the last iteration from the stored directions)
template <typename T, int W>
struct CgBRows {
    static constexpr bool kDots = true;
    struct Regs { T g[W]; T own, r; };
    RowOps<T, W, false> o;
    const T* Pn;
    T* Rv;
    const double* alpha;
    int64_t R;
    int row;
    bool live = true;
    __device__ __forceinline__ void load(int j, Regs& r) const {
        const T* p = Pn + (int64_t)j * R;
        r.own = p[row];
        r.g[0] = r.own;
#pragma unroll
        for (int k = 1; k < W; k++) r.g[k] = gat(p, o.c[k]);
        r.r = Rv[(int64_t)j * R + row];
    }
    __device__ __forceinline__ double use(int j, const Regs& r) const {
        T qq = 0;
#pragma unroll
        for (int k = 0; k < W; k++) qq += o.mv[k] * r.g[k];
        const T al = (T)alpha[j];
        const int64_t i = (int64_t)j * R + row;
        const T res = r.r - al * qq;
        if (!live) return 0.0;
        Rv[i] = res;
        return (double)res * (double)res * (double)o.mrow;
    }
};

// Two forms of the CG iteration.  Both store every iteration's search
// direction p_k (slice k of Ph) and form x once after the last iteration
// (k_cg_x), so the iterations themselves never touch x.  The recompute
// form above forms M p twice from neighbour values of p: cg_a gathers r and
// p_{k-1}, cg_b gathers p_k.  On the 3-D layouts (ELL width 15 and up)
// gathers dominate, so there q = M p is kept as a vector of its own (in Pa)
// with the recurrence q = M z + beta q, which is M p in exact arithmetic:
// cg_a gathers only z (the form keeps z = r / m, see z_form), cg_b reads
// own rows only (q and z).
template <int W>
constexpr bool q_recurrence() { return W >= kQRecurrenceWidth; }
static_assert(z_form<15>() == q_recurrence<15>() && z_form<7>() == q_recurrence<7>(),
              "the recurrence bodies keep z, the recompute bodies r");

// cg_a, recurrence form: p = z + beta p, q = M z + beta q (p, q of the
// previous iteration unread on the first); reduces p.q -> alpha.
template <typename T, int W, bool FIRST>
struct CgAQRows {
    static constexpr bool kDots = true;
    struct Regs { T g[W]; T own, p, q; };
    RowOps<T, W, false> o;
    const T *Rv, *Pold;
    T *Pnew, *Qv;
    const double* beta;
    int64_t R;
    int row;
    __device__ __forceinline__ void load(int j, Regs& r) const {
        const T* rv = Rv + (int64_t)j * R;
        r.own = rv[row];
        r.g[0] = r.own;
#pragma unroll
        for (int k = 1; k < W; k++) r.g[k] = gat(rv, o.c[k]);
        if constexpr (!FIRST) {
            const int64_t i = (int64_t)j * R + row;
            r.p = Pold[i];
            r.q = Qv[i];
        }
    }
    __device__ __forceinline__ double use(int j, const Regs& r) const {
        T acc = 0;
#pragma unroll
        for (int k = 0; k < W; k++) acc += o.mv[k] * r.g[k];
        T pn = r.own, qn = acc;
        if constexpr (!FIRST) {
            const T bet = (T)beta[j];
            pn += bet * r.p;
            qn += bet * r.q;
        }
        const int64_t i = (int64_t)j * R + row;
        Pnew[i] = pn;
        Qv[i] = qn;
        return (double)pn * (double)qn;
    }
};

// cg_b, recurrence form: z -= alpha m^-1 q; reduces r.z = m z.z -> beta.
template <typename T>
struct CgBQRows {
    static constexpr bool kDots = true;
    struct Regs { T q, r; };
    const T* Qv;
    T* Rv;
    const double* alpha;
    T mrow;
    int64_t R;
    int row;
    __device__ __forceinline__ void load(int j, Regs& r) const {
        const int64_t i = (int64_t)j * R + row;
        r.q = Qv[i];
        r.r = Rv[i];
    }
    __device__ __forceinline__ double use(int j, const Regs& r) const {
        const T al = (T)alpha[j];
        const T zn = r.r - al * (r.q * mrow);
        const int64_t i = (int64_t)j * R + row;
        Rv[i] = zn;
        return (double)zn * (double)zn * (1.0 / (double)mrow);
    }
};

template <typename T>
__device__ __forceinline__ T* vec(void* base) {
    return reinterpret_cast<T*>(base);
}

// search direction of CG iteration k: slice k of Ph, [NP][R] each
template <typename T, int NP>
__device__ __forceinline__ T* ph(const DevLayout& L, int k) {
    return reinterpret_cast<T*>(L.Ph) + (int64_t)k * NP * L.R;
}
template <int NP>
__device__ __forceinline__ const double* alpha_of(const DevLayout& L, int k, int inst) {
    return L.alpha + ((int64_t)k * L.ninst + inst) * NP;
}

// x = x_0 + alpha_0 p_0 + alpha_1 p_1 + ...: the CG solution, formed once
// from the stored directions in iteration order (the same sums, in the same
// order, as updating x in every iteration).  x_0 = rhs / m is the product
// cg_init takes, rounded on its own (not contracted into the first update).
// A thread keeps its row's NP values and loads one direction slice at a
// time, NP loads in flight.  With check set (after the fused CG), the first
// wave of each block also takes the residual checks c = blockIdx.x,
// blockIdx.x + gridDim.x, ... of the ninst * NP (instance, value) pairs,
// which saves the fused path a launch of its own for them.
template <int NP>
__device__ __forceinline__ void fused_residual_check(const DevLayout& L, int inst, int j);
template <typename T, int NP>
__global__ __launch_bounds__(TILE) void k_cg_x(DevLayout L, int tile_begin, int check) {
    FEL_ROW_LAYOUT();
    const int inst = L.tile_inst[tile];
    const T* rhs = vec<T>(L.Pb);
    const T mrow = reinterpret_cast<const T*>(L.minv)[row];
    T* X = vec<T>(L.X);
    T x[NP];
    {
#pragma clang fp contract(off)
#pragma unroll
        for (int j = 0; j < NP; j++) x[j] = rhs[(int64_t)j * R + row] * mrow;
    }
    // two (D2Q9) or four (D3Q19) directions per trip: the next slices' loads
    // are issued before the current ones are summed
    constexpr int kDirUnroll = NP <= 16 ? 2 : 4;
#pragma unroll kDirUnroll
    for (int k = 0; k < L.K; k++) {
        const T* p = ph<T, NP>(L, k);
        const double* al = alpha_of<NP>(L, k, inst);
        T v[NP];
        // every direction is read here for the last time: non-temporal loads
        // keep them from displacing data the next kernels reuse
#pragma unroll
        for (int j = 0; j < NP; j++) v[j] = __builtin_nontemporal_load(&p[(int64_t)j * R + row]);
#pragma unroll
        for (int j = 0; j < NP; j++) x[j] = x[j] + (T)al[j] * v[j];
    }
#pragma unroll
    for (int j = 0; j < NP; j++) X[(int64_t)j * R + row] = x[j];
    if (check && threadIdx.x < 64)
        for (int c = blockIdx.x; c < L.ninst * NP; c += gridDim.x) fused_residual_check<NP>(L, c / NP, c % NP);
}

template <typename T, int W, int NP, int CH>
__global__ __launch_bounds__(TILE) void k_cg_init(DevLayout L, int tile_begin) {
    FEL_ROW_LAYOUT();
    CgInitRows<T, W> b;
    b.o.load(L, R, row);
    b.rhs = vec<T>(L.Pb);
    b.Rv = vec<T>(L.Rv);
    b.R = R;
    b.row = row;
    FEL_REDUCER(red, NP);
    run_rows<NP, CH>(b, &red);
    red.finish(L, tile);
}

template <typename T, int W, int NP, int CH>
__global__ __launch_bounds__(TILE) void k_cg_a(DevLayout L, int tile_begin, int first, int it) {
    FEL_ROW_LAYOUT();
    const int inst = L.tile_inst[tile];
    const T* Rv = vec<T>(L.Rv);
    const T* Pold = ph<T, NP>(L, it > 0 ? it - 1 : 0);  // unread on the first iteration
    T* Pnew = ph<T, NP>(L, it);
    const double* beta = L.beta + inst * NP;
    FEL_REDUCER(red, NP);
    if constexpr (q_recurrence<W>()) {
        auto go = [&](auto& b) {
            b.o.load(L, R, row);
            b.Rv = Rv, b.Pold = Pold, b.Pnew = Pnew, b.Qv = vec<T>(L.Pa), b.beta = beta, b.R = R, b.row = row;
            run_rows<NP, CH>(b, &red);
        };
        if (first) {
            CgAQRows<T, W, true> b;
            go(b);
        } else {
            CgAQRows<T, W, false> b;
            go(b);
        }
    } else if (first) {
        CgARows<T, W, true> b;
        b.o.load(L, R, row);
        b.Rv = Rv, b.Pold = Pold, b.Pnew = Pnew, b.beta = beta, b.R = R, b.row = row;
        run_rows<NP, CH>(b, &red);
    } else {
        CgARows<T, W, false> b;
        b.o.load(L, R, row);
        b.Rv = Rv, b.Pold = Pold, b.Pnew = Pnew, b.beta = beta, b.R = R, b.row = row;
        run_rows<NP, CH>(b, &red);
    }
    red.finish(L, tile);
}

template <typename T, int W, int NP, int CH>
__global__ __launch_bounds__(TILE) void k_cg_b(DevLayout L, int tile_begin, int it) {
    FEL_ROW_LAYOUT();
    const int inst = L.tile_inst[tile];
    FEL_REDUCER(red, NP);
    if constexpr (q_recurrence<W>()) {
        CgBQRows<T> b;
        b.Qv = vec<T>(L.Pa);
        b.Rv = vec<T>(L.Rv);
        b.alpha = alpha_of<NP>(L, it, inst);
        b.mrow = ld<T>(L.minv, row);
        b.R = R;
        b.row = row;
        run_rows<NP, CH>(b, &red);
    } else {
        CgBRows<T, W> b;
        b.o.load(L, R, row);
        b.Pn = ph<T, NP>(L, it);
        b.Rv = vec<T>(L.Rv);
        b.alpha = alpha_of<NP>(L, it, inst);
        b.R = R;
        b.row = row;
        run_rows<NP, CH>(b, &red);
    }
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

template <typename T, int W>
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
        r.own = b[row];
        r.g[0] = r.own;
#pragma unroll
        for (int k = 1; k < W; k++) r.g[k] = gat(b, o.c[k]);
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

template <typename T, int W>
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
        r.own = x[row];
        r.g[0] = r.own;
#pragma unroll
        for (int k = 1; k < W; k++) r.g[k] = gat(x, o.c[k]);
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
__global__ __launch_bounds__(TILE) void k_cheb_first(DevLayout L, int tile_begin, int out0,
                                                     double gamma_d) {
    FEL_ROW_LAYOUT();
    ChebFirstRows<T, W> b;
    b.o.load(L, R, row);
    b.rhs = vec<T>(L.Pb);
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
    ChebRows<T, W> b;
    b.o.load(L, R, row);
    b.rhs = vec<T>(L.Pb);
    b.xk = cheb_buf<T>(L, cur);
    b.xp = cheb_buf<T>(L, 1 - cur);
    b.omega = (T)omega_d;
    b.gamma = (T)gamma_d;
    b.R = R;
    b.row = row;
    run_rows<NP, CH>(b, (TileReducer<NP>*)nullptr);
}

// ---------------------------------------------------------------------------
// Fused-reduction CG (2-D instances of up to kFusedMaxBlocks blocks).  A
// block covers kFusedTiles tiles (1024 threads), so an instance has at most
// 256 block partials, and instead of a finalize launch between the two
// kernels of an iteration every block sums the partials the previous launch
// left for its instance (wave w sums values w, w + 16, ...: a few coalesced
// loads per lane), in the same fixed order in every block, so all blocks of
// an instance hold bitwise the same alpha or beta.  r.z is kept by
// iteration parity in srz (the first block of the instance writes it; the
// launch reads the other slot), so no block reads what this launch writes.
// Block partials: cg_init and cg_b write fpart0 (r.z), cg_a writes fpart1
// (p.q).  The final residual check of the finalize path is taken by
// k_cg_x (its check argument) on the last cg_b's partials, with no launch
// of its own.
constexpr int FB_THREADS = kFusedTiles * TILE;
constexpr int FB_WAVES = FB_THREADS / 64;

#define FEL_FUSED_LAYOUT()                                            \
    const int4 fb = L.fblocks[blockIdx.x];                            \
    const int64_t R = L.R;                                            \
    const int sub = threadIdx.x / TILE;                               \
    const bool active = sub < fb.y;                                   \
    const int tile = fb.x + (active ? sub : 0);                       \
    const int row = tile * TILE + (threadIdx.x & (TILE - 1));         \
    const int inst = fb.z;                                            \
    const int pidx = L.params[inst].fb_begin + fb.w

// tot[j] = sum over the instance's blocks of src[j][block], j < NP.  Wave
// w sums population w: lane l holds blocks l, l + 64, ... (at most
// kFusedMaxBlocks / 64 of them).  load() issues those loads at kernel start,
// ahead of the row loads, so they have arrived when reduce() needs them
// before the first population is used.
template <int NP>
struct FusedTotals {
    static_assert(NP <= FB_WAVES, "one population per wave");
    static constexpr int K = kFusedMaxBlocks / 64;
    double v[K];
    __device__ __forceinline__ void load(const DevLayout& L, const double* src, int inst) {
        const InstParams& P = L.params[inst];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const double* p = src + (int64_t)(wave < NP ? wave : 0) * L.nfb + P.fb_begin;
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int b = lane + 64 * k;
            v[k] = (wave < NP && b < P.fb_count) ? p[b] : 0.0;
        }
    }
    __device__ __forceinline__ void reduce(double* tot) const {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < K; k++) s += v[k];
        s = wave_sum(s);
        if (lane == 0 && wave < NP) tot[wave] = s;
        __syncthreads();
    }
};

// Every thread of a fused block runs the row pipeline (spare waves of an
// instance's last, short block on its first tile with stores masked), so
// all reach the same barriers.  The row operands and the first population
// batch are loaded before the block forms its CG scalars (the hook), so the
// two latencies overlap.
template <typename T, int W, int NP, int CH>
__global__ __launch_bounds__(FB_THREADS) void k_cg_init_fused(DevLayout L) {
    FEL_FUSED_LAYOUT();
    FEL_REDUCER_N(red, NP, FB_WAVES);
    CgInitRows<T, W> b;
    b.o.load(L, R, row);
    b.rhs = vec<T>(L.Pb);
    b.Rv = vec<T>(L.Rv);
    b.R = R;
    b.row = row;
    b.live = active;
    run_rows<NP, CH>(b, &red);
    red.finish_to(L.fpart0, L.nfb, pidx, FB_WAVES);
}

template <typename T, int W, int NP, int CH>
__global__ __launch_bounds__(FB_THREADS) void k_cg_a_fused(DevLayout L, int it) {
    FEL_FUSED_LAYOUT();
    __shared__ double tot[NP], bet[NP];
    const int cur = it & 1;
    FusedTotals<NP> rz;
    rz.load(L, L.fpart0, inst);  // r.z of the current residual
    auto scalars = [&] {
        rz.reduce(tot);
        if (threadIdx.x < NP) {
            const int j = threadIdx.x;
            if (fb.w == 0) {
                L.srz[((int64_t)cur * L.ninst + inst) * NP + j] = tot[j];
                if (it == 0) L.rz0[inst * NP + j] = tot[j];
            }
            const double old = it == 0 ? 0.0 : L.srz[((int64_t)(1 - cur) * L.ninst + inst) * NP + j];
            bet[j] = (old != 0.0) ? tot[j] / old : 0.0;
        }
        __syncthreads();
    };
    FEL_REDUCER_N(red, NP, FB_WAVES);
    const T* Rv = vec<T>(L.Rv);
    const T* Pold = ph<T, NP>(L, it > 0 ? it - 1 : 0);  // unread on the first iteration
    T* Pnew = ph<T, NP>(L, it);
    // FP64: the two population register sets of the pipeline would spill
    // under the 128 registers of a 1024-thread block
    constexpr bool pipe = sizeof(T) == 4;
    if (it == 0) {
        CgARows<T, W, true> b;
        b.o.load(L, R, row);
        b.Rv = Rv, b.Pold = Pold, b.Pnew = Pnew, b.beta = bet, b.R = R, b.row = row, b.live = active;
        run_rows<NP, CH, pipe>(b, &red, scalars);
    } else {
        CgARows<T, W, false> b;
        b.o.load(L, R, row);
        b.Rv = Rv, b.Pold = Pold, b.Pnew = Pnew, b.beta = bet, b.R = R, b.row = row, b.live = active;
        run_rows<NP, CH, pipe>(b, &red, scalars);
    }
    red.finish_to(L.fpart1, L.nfb, pidx, FB_WAVES);
}

template <typename T, int W, int NP, int CH>
__global__ __launch_bounds__(FB_THREADS) void k_cg_b_fused(DevLayout L, int it) {
    FEL_FUSED_LAYOUT();
    __shared__ double tot[NP], alp[NP];
    FusedTotals<NP> pq;
    pq.load(L, L.fpart1, inst);  // p.q
    auto scalars = [&] {
        pq.reduce(tot);
        if (threadIdx.x < NP) {
            const int j = threadIdx.x;
            const double rz = L.srz[((int64_t)(it & 1) * L.ninst + inst) * NP + j];
            alp[j] = (tot[j] != 0.0) ? rz / tot[j] : 0.0;
            // the instance's first block keeps alpha for forming x (k_cg_x)
            if (fb.w == 0) L.alpha[((int64_t)it * L.ninst + inst) * NP + j] = alp[j];
        }
        __syncthreads();
    };
    FEL_REDUCER_N(red, NP, FB_WAVES);
    CgBRows<T, W> b;
    b.o.load(L, R, row);
    b.Pn = ph<T, NP>(L, it);
    b.Rv = vec<T>(L.Rv);
    b.alpha = alp;
    b.R = R;
    b.row = row;
    b.live = active;
    run_rows<NP, CH>(b, &red, scalars);
    red.finish_to(L.fpart0, L.nfb, pidx, FB_WAVES);
}

// Final residual check of the fused CG, run by one whole wavefront: r.z
// after the last iteration (the fused blocks' partials, summed in a fixed
// order) against r0.z0 for value j of an instance.
template <int NP>
__device__ __forceinline__ void fused_residual_check(const DevLayout& L, int inst, int j) {
    const InstParams& P = L.params[inst];
    const double* p = L.fpart0 + (int64_t)j * L.nfb + P.fb_begin;
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int b = lane; b < P.fb_count; b += 64) s += p[b];
    s = wave_sum(s);
    if (lane == 0) {
        const double r0 = L.rz0[inst * NP + j];
        if (r0 > 0.0 && !(s <= L.cg_tol2 * r0)) atomicOr(L.status, 2u);
    }
}

// ---------------------------------------------------------------------------
// LDS-staged variants.  A pass stages, for CH populations, the value every
// row of the tile and every halo entry contributes to the M-product (own
// rows with coalesced loads, the halo with one load per entry, values the
// same expression the direct kernels apply to their gathers), then each
// row reads its W neighbours from LDS through the 16-bit local columns.
// A wavefront thus issues 1 + halo/TILE global loads per population and
// vector instead of W gathers.  CH populations per pass, rows sw apart.
// The stage is double-buffered: the loads of the next pass are issued
// right after the barrier that publishes the current one, so they are in
// flight while the rows read LDS, and one barrier per pass suffices (a
// buffer is rewritten two passes later, after every row has passed the
// intervening barrier).  Each thread stages at most HR halo entries, HR
// = 2 when the layout's largest halo is at most 2 TILE, else 4 (halo <=
// kHaloRounds * TILE; the host checks): the halo registers of the
// 2-round form leave room for more resident blocks.  Vectors are read and
// written through buffer resources (BufVec): a thread keeps one byte
// offset per row it stages (its own, and one per halo round), shared by
// every population and vector.  A halo round in which a wavefront has no
// entry is skipped by the whole wavefront; the idle lanes of a wavefront
// that has entries load with an out-of-range offset (0, no memory access)
// and write their LDS slot, which no row reads (sw covers the halo rounded
// up to whole wavefronts).
//
// The same driver with HR = 0 is the per-wavefront form: each wavefront
// stages its own 64 rows and its own halo (kWaveHaloRounds rounds of 64,
// rows of sibling wavefronts included) into slots only it reads, so a pass
// is published by a wavefront-level fence instead of a block barrier and
// the four wavefronts of a tile run their passes independently.  LDS
// operations of one wavefront complete in issue order; the fence keeps the
// compiler from moving a lane's stage reads above the other lanes' writes.

template <int W>
struct LocalCols {
    int lc[W];
    // lcol: the tile form's columns (L.lcol) or the wavefront form's (L.wlcol)
    __device__ __forceinline__ void load(const uint16_t* lcol, int64_t R, int row) {
        lc[0] = row % TILE;  // slot 0: the row itself
#pragma unroll
        for (int k = 1; k < W; k++) lc[k] = gat(lcol + k * R, row);
    }
};

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sum_k mv[k] * stage[lc[k]]
template <typename T, int W>
__device__ __forceinline__ T lds_row_product(const T* mv, const LocalCols<W>& l, const T* stage) {
    T acc = 0;
#pragma unroll
    for (int k = 0; k < W; k++) acc += mv[k] * stage[l.lc[k]];
    return acc;
}

// Drives the passes: body.pre(o) is a per-row value the staged values of
// the row at byte offset o need for every population (loaded once per
// tile); body.load(j, o, raw) issues the loads of population j's staged
// value at that row and body.value(j, raw, pre) forms it, when the stage
// is written (a pass later: forming it where the loads are issued would
// make the wavefront wait for them there, inside the halo branch, before
// it has used the current pass); body.keep(j, own) loads what the row
// keeps in registers for population j; body.use(j, stage_row, own)
// finishes the row and returns its dot-product term.  sh holds 2 CH stage
// rows (sw values each, or kWaveStageWidth in the wavefront form, HR = 0).
template <typename T, int NP, int CH, int HR, class Body>
__device__ __forceinline__ void run_staged(Body& body, const DevLayout& L, int tile, int row, T* sh,
                                           TileReducer<NP>* red) {
    static_assert(HR >= 0 && HR <= kHaloRounds, "halo rounds out of range");
    static_assert(NP % CH == 0 && NP % RG == 0, "population passes must tile NP");
    constexpr bool kWave = HR == 0;
    constexpr int NR = kWave ? kWaveHaloRounds : HR;  // halo rounds per thread
    constexpr int RS = kWave ? 64 : TILE;             // halo entries per round
    const int sw = kWave ? kWaveStageWidth : L.sw;
    const int lr = threadIdx.x;
    const int wb = __builtin_amdgcn_readfirstlane(lr) & ~63;  // the wavefront's first thread
    // halo list; hl: this thread's entry in round 0; hs: its LDS slot in round 0
    int hb, hn, hl, hs;
    if constexpr (kWave) {
        const int wv = tile * (TILE / 64) + wb / 64;
        hb = L.whalo_ptr[wv];
        hn = L.whalo_ptr[wv + 1] - hb;
        hl = lr - wb;
        hs = TILE + (wb / 64) * NR * 64 + hl;
    } else {
        hb = L.halo_ptr[tile];
        hn = L.halo_ptr[tile + 1] - hb;
        hl = lr;
        hs = TILE + lr;
    }
    const int32_t* hcol = kWave ? L.whalo_col : L.halo_col;
    bool act[NR];
    uint32_t ho[NR];
    T pre_h[NR];
#pragma unroll
    for (int i = 0; i < NR; i++) {
        const int h = hl + i * RS;
        act[i] = hn > i * RS + (kWave ? 0 : wb);  // uniform over the wavefront
        ho[i] = h < hn ? (uint32_t)hcol[hb + h] * (uint32_t)sizeof(T) : kIdleRow;
        pre_h[i] = act[i] ? body.pre(ho[i]) : T(0);
    }
    const T pre_own = body.pre(body.ro);
    // The tile's own rows (coalesced, most of the bytes) are loaded two
    // passes ahead, the halo (mostly L2 hits) and the kept values one.
    typename Body::Own own[2][CH];
    typename Body::Raw v[2][CH], vh[NR][CH];
    auto fetch_own = [&](int j0, typename Body::Raw* dst) {
#pragma unroll
        for (int u = 0; u < CH; u++) body.load(j0 + u, body.ro, dst[u]);
    };
    auto fetch = [&](int j0, typename Body::Own* o) {
#pragma unroll
        for (int u = 0; u < CH; u++) body.keep(j0 + u, o[u]);
#pragma unroll
        for (int i = 0; i < NR; i++) {
            if (act[i]) {
#pragma unroll
                for (int u = 0; u < CH; u++) body.load(j0 + u, ho[i], vh[i][u]);
            }
        }
    };
    fetch_own(0, v[0]);
    fetch(0, own[0]);
    if (CH < NP) fetch_own(CH, v[1]);
    double dots[RG];
#pragma unroll
    for (int j0 = 0; j0 < NP; j0 += CH) {
        const int p = (j0 / CH) & 1;
        T* buf = sh + p * CH * sw;
#pragma unroll
        for (int u = 0; u < CH; u++) buf[u * sw + lr] = body.value(j0 + u, v[p][u], pre_own);
#pragma unroll
        for (int i = 0; i < NR; i++) {
            if (act[i]) {
#pragma unroll
                for (int u = 0; u < CH; u++) buf[u * sw + hs + i * RS] = body.value(j0 + u, vh[i][u], pre_h[i]);
            }
        }
        if constexpr (kWave)
            wave_lds_sync();
        else
            __syncthreads();
        if (j0 + CH < NP) fetch(j0 + CH, own[p ^ 1]);
        if (j0 + 2 * CH < NP) fetch_own(j0 + 2 * CH, v[p]);
#pragma unroll
        for (int u = 0; u < CH; u++) {
            const int j = j0 + u;
            const double d = body.use(j, buf + u * sw, own[p][u]);
            if constexpr (Body::kDots) {
                dots[j % RG] = d;
                if (j % RG == RG - 1) red->add_group(j - (RG - 1), dots);
            }
        }
        // keep the next pass's staged values from being formed (and their
        // loads waited for) ahead of this pass's rows
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Row state of every staged body: local columns, mass values, the row's
// byte offset ro and the byte size sR of one population's slice.
template <typename T, int W>
struct StagedRow {
    LocalCols<W> l;
    T mv[W];
    uint32_t ro, sR;
    __device__ __forceinline__ uint32_t so(int j) const { return (uint32_t)j * sR; }
};

// cg_init staged: stage rhs / m
template <typename T, int W>
struct CgInitStaged : StagedRow<T, W> {
    static constexpr bool kDots = true;
    struct Own { T rhs; };
    struct Raw { T v; };
    T mrow;
    BufVec<T> rhs, minv, rv;
    __device__ __forceinline__ T pre(uint32_t o) const { return minv.load(o, 0); }
    __device__ __forceinline__ void load(int j, uint32_t o, Raw& w) const { w.v = rhs.load(o, this->so(j)); }
    __device__ __forceinline__ T value(int, const Raw& w, T mg) const { return w.v * mg; }
    __device__ __forceinline__ void keep(int j, Own& w) const { w.rhs = rhs.load(this->ro, this->so(j)); }
    __device__ __forceinline__ double use(int j, const T* st, const Own& w) const {
        const T acc = lds_row_product<T, W>(this->mv, this->l, st);
        const T res = w.rhs - acc;
        rv.store(z_form<W>() ? res * mrow : res, this->ro, this->so(j));
        return (double)res * (double)res * (double)mrow;
    }
};

// cg_a staged: stage p_new = r / m + beta p_old
template <typename T, int W, bool FIRST>
struct CgAStaged : StagedRow<T, W> {
    static constexpr bool kDots = true;
    struct Own {};
    struct Raw { T r, p; };
    BufVec<T> rv, pold, pnew, minv;
    const T* beta;  // LDS copy
    __device__ __forceinline__ T pre(uint32_t o) const { return minv.load(o, 0); }
    __device__ __forceinline__ void load(int j, uint32_t o, Raw& w) const {
        w.r = rv.load(o, this->so(j));
        if constexpr (!FIRST) w.p = pold.load(o, this->so(j));
    }
    __device__ __forceinline__ T value(int j, const Raw& w, T mg) const {
        if constexpr (FIRST)
            return w.r * mg;
        else
            return w.r * mg + beta[j] * w.p;
    }
    __device__ __forceinline__ void keep(int, Own&) const {}
    __device__ __forceinline__ double use(int j, const T* st, const Own&) const {
        const T acc = lds_row_product<T, W>(this->mv, this->l, st);
        const T pown = st[threadIdx.x];
        pnew.store(pown, this->ro, this->so(j));
        return (double)pown * (double)acc;
    }
};

// cg_a staged, recurrence form: stage z; p = z + beta p and q = M z +
// beta q in place.  (The recurrence form's cg_b reads no
// neighbour values and has no staged form.)
template <typename T, int W, bool FIRST>
struct CgAQStaged : StagedRow<T, W> {
    static constexpr bool kDots = true;
    struct Own { T p, q; };
    struct Raw { T v; };
    BufVec<T> rv, pold, pnew, qv;
    const T* beta;  // LDS copy
    __device__ __forceinline__ T pre(uint32_t) const { return T(0); }
    __device__ __forceinline__ void load(int j, uint32_t o, Raw& w) const { w.v = rv.load(o, this->so(j)); }
    __device__ __forceinline__ T value(int, const Raw& w, T) const { return w.v; }
    __device__ __forceinline__ void keep(int j, Own& w) const {
        if constexpr (!FIRST) {
            w.p = pold.load(this->ro, this->so(j));
            w.q = qv.load(this->ro, this->so(j));
        }
    }
    __device__ __forceinline__ double use(int j, const T* st, const Own& w) const {
        T pn = st[threadIdx.x], qn = lds_row_product<T, W>(this->mv, this->l, st);
        if constexpr (!FIRST) {
            const T bet = beta[j];
            pn += bet * w.p;
            qn += bet * w.q;
        }
        pnew.store(pn, this->ro, this->so(j));
        qv.store(qn, this->ro, this->so(j));
        return (double)pn * (double)qn;
    }
};

// cg_b staged: stage p
template <typename T, int W>
struct CgBStaged : StagedRow<T, W> {
    static constexpr bool kDots = true;
    struct Own { T r; };
    struct Raw { T v; };
    T mrow;
    BufVec<T> pn, rv;
    const T* alpha;  // LDS copy
    __device__ __forceinline__ T pre(uint32_t) const { return T(0); }
    __device__ __forceinline__ void load(int j, uint32_t o, Raw& w) const { w.v = pn.load(o, this->so(j)); }
    __device__ __forceinline__ T value(int, const Raw& w, T) const { return w.v; }
    __device__ __forceinline__ void keep(int j, Own& w) const { w.r = rv.load(this->ro, this->so(j)); }
    __device__ __forceinline__ double use(int j, const T* st, const Own& w) const {
        const T qq = lds_row_product<T, W>(this->mv, this->l, st);
        const T al = alpha[j];
        const T res = w.r - al * qq;
        rv.store(res, this->ro, this->so(j));
        return (double)res * (double)res * (double)mrow;
    }
};

// Chebyshev first iterate staged: stage rhs / m
template <typename T, int W>
struct ChebFirstStaged : StagedRow<T, W> {
    static constexpr bool kDots = false;
    struct Own { T rhs; };
    struct Raw { T v; };
    T mrow;
    BufVec<T> rhs, minv, x0, x1;
    T gamma;
    __device__ __forceinline__ T pre(uint32_t o) const { return minv.load(o, 0); }
    __device__ __forceinline__ void load(int j, uint32_t o, Raw& w) const { w.v = rhs.load(o, this->so(j)); }
    __device__ __forceinline__ T value(int, const Raw& w, T mg) const { return w.v * mg; }
    __device__ __forceinline__ void keep(int j, Own& w) const { w.rhs = rhs.load(this->ro, this->so(j)); }
    __device__ __forceinline__ double use(int j, const T* st, const Own& w) const {
        const T acc = lds_row_product<T, W>(this->mv, this->l, st);
        const T xa = w.rhs * mrow;
        x0.store(xa, this->ro, this->so(j));
        x1.store(xa + gamma * ((w.rhs - acc) * mrow), this->ro, this->so(j));
        return 0.0;
    }
};

// Chebyshev iterate staged: stage x_k
template <typename T, int W>
struct ChebStaged : StagedRow<T, W> {
    static constexpr bool kDots = false;
    struct Own { T b, xp; };
    struct Raw { T v; };
    T mrow;
    BufVec<T> rhs, xk, xp;
    T omega, gamma;
    __device__ __forceinline__ T pre(uint32_t) const { return T(0); }
    __device__ __forceinline__ void load(int j, uint32_t o, Raw& w) const { w.v = xk.load(o, this->so(j)); }
    __device__ __forceinline__ T value(int, const Raw& w, T) const { return w.v; }
    __device__ __forceinline__ void keep(int j, Own& w) const {
        w.b = rhs.load(this->ro, this->so(j));
        w.xp = xp.load(this->ro, this->so(j));
    }
    __device__ __forceinline__ double use(int j, const T* st, const Own& w) const {
        const T acc = lds_row_product<T, W>(this->mv, this->l, st);
        const T z = (w.b - acc) * mrow;
        xp.store(omega * (gamma * z + st[threadIdx.x] - w.xp) + w.xp, this->ro, this->so(j));
        return 0.0;
    }
};

template <typename T, int W, int HR, class B>
__device__ __forceinline__ void staged_row_setup(B& b, const DevLayout& L, int64_t R, int row) {
    b.l.load(HR == 0 ? L.wlcol : L.lcol, R, row);
#pragma unroll
    for (int k = 0; k < W; k++) b.mv[k] = gat(reinterpret_cast<const T*>(L.Mval) + k * R, row);
    b.ro = (uint32_t)row * (uint32_t)sizeof(T);
    b.sR = (uint32_t)R * (uint32_t)sizeof(T);
}

// bytes of a [NP][R] vector of T (the host keeps it below 4 GiB for the
// staged forms) and of the [R] inverse masses
template <typename T, int NP>
__device__ __forceinline__ uint32_t vec_bytes(const DevLayout& L) {
    return (uint32_t)NP * (uint32_t)L.R * (uint32_t)sizeof(T);
}
template <typename T>
__device__ __forceinline__ uint32_t row_bytes(const DevLayout& L) {
    return (uint32_t)L.R * (uint32_t)sizeof(T);
}

template <typename T, int W, int NP, int CH, int HR>
__global__ __launch_bounds__(TILE) void k_cg_init_lds(DevLayout L, int tile_begin) {
    FEL_ROW_LAYOUT();
    extern __shared__ __align__(16) unsigned char fel_smem[];
    CgInitStaged<T, W> b;
    staged_row_setup<T, W, HR>(b, L, R, row);
    const uint32_t vb = vec_bytes<T, NP>(L);
    b.minv.bind(reinterpret_cast<const T*>(L.minv), row_bytes<T>(L));
    b.mrow = ld<T>(L.minv, row);
    b.rhs.bind(vec<T>(L.Pb), vb);
    b.rv.bind(vec<T>(L.Rv), vb);
    FEL_REDUCER(red, NP);
    run_staged<T, NP, CH, HR>(b, L, tile, row, reinterpret_cast<T*>(fel_smem), &red);
    red.finish(L, tile);
}

template <typename T, int W, int NP, int CH, int HR>
__global__ __launch_bounds__(TILE) void k_cg_a_lds(DevLayout L, int tile_begin, int first, int it) {
    FEL_ROW_LAYOUT();
    extern __shared__ __align__(16) unsigned char fel_smem[];
    const int inst = L.tile_inst[tile];
    T* sh = reinterpret_cast<T*>(fel_smem);
    FEL_REDUCER(red, NP);
    // beta of the instance in LDS: read where the staged values are formed
    __shared__ T sbeta[NP];
    if (threadIdx.x < NP) sbeta[threadIdx.x] = (T)L.beta[inst * NP + threadIdx.x];
    __syncthreads();
    const uint32_t vb = vec_bytes<T, NP>(L);
    auto setup = [&](auto& b) {
        staged_row_setup<T, W, HR>(b, L, R, row);
        b.rv.bind(vec<T>(L.Rv), vb);
        b.pold.bind(ph<T, NP>(L, it > 0 ? it - 1 : 0), vb);  // unread on the first iteration
        b.pnew.bind(ph<T, NP>(L, it), vb);
        b.beta = sbeta;
    };
    if constexpr (q_recurrence<W>()) {
        auto setup_q = [&](auto& b) {
            setup(b);
            b.qv.bind(vec<T>(L.Pa), vb);
        };
        if (first) {
            CgAQStaged<T, W, true> b;
            setup_q(b);
            run_staged<T, NP, CH, HR>(b, L, tile, row, sh, &red);
        } else {
            CgAQStaged<T, W, false> b;
            setup_q(b);
            run_staged<T, NP, CH, HR>(b, L, tile, row, sh, &red);
        }
    } else {
        auto setup_m = [&](auto& b) {
            setup(b);
            b.minv.bind(reinterpret_cast<const T*>(L.minv), row_bytes<T>(L));
        };
        if (first) {
            CgAStaged<T, W, true> b;
            setup_m(b);
            run_staged<T, NP, CH, HR>(b, L, tile, row, sh, &red);
        } else {
            CgAStaged<T, W, false> b;
            setup_m(b);
            run_staged<T, NP, CH, HR>(b, L, tile, row, sh, &red);
        }
    }
    red.finish(L, tile);
}

template <typename T, int W, int NP, int CH, int HR>
__global__ __launch_bounds__(TILE) void k_cg_b_lds(DevLayout L, int tile_begin, int it) {
    FEL_ROW_LAYOUT();
    extern __shared__ __align__(16) unsigned char fel_smem[];
    const int inst = L.tile_inst[tile];
    FEL_REDUCER(red, NP);
    if constexpr (q_recurrence<W>()) {
        // nothing to stage in the recurrence form (the host never selects
        // this kernel there); the direct rows keep it well defined
        CgBQRows<T> b;
        b.Qv = vec<T>(L.Pa);
        b.Rv = vec<T>(L.Rv);
        b.alpha = alpha_of<NP>(L, it, inst);
        b.mrow = ld<T>(L.minv, row);
        b.R = R;
        b.row = row;
        run_rows<NP, CH>(b, &red);
    } else {
        // alpha of the instance in LDS
        __shared__ T salpha[NP];
        if (threadIdx.x < NP) salpha[threadIdx.x] = (T)alpha_of<NP>(L, it, inst)[threadIdx.x];
        __syncthreads();
        CgBStaged<T, W> b;
        staged_row_setup<T, W, HR>(b, L, R, row);
        const uint32_t vb = vec_bytes<T, NP>(L);
        b.mrow = ld<T>(L.minv, row);
        b.pn.bind(ph<T, NP>(L, it), vb);
        b.rv.bind(vec<T>(L.Rv), vb);
        b.alpha = salpha;
        run_staged<T, NP, CH, HR>(b, L, tile, row, reinterpret_cast<T*>(fel_smem), &red);
    }
    red.finish(L, tile);
}

template <typename T, int W, int NP, int CH, int HR>
__global__ __launch_bounds__(TILE) void k_cheb_first_lds(DevLayout L, int tile_begin, int out0,
                                                         double gamma_d) {
    FEL_ROW_LAYOUT();
    extern __shared__ __align__(16) unsigned char fel_smem[];
    ChebFirstStaged<T, W> b;
    staged_row_setup<T, W, HR>(b, L, R, row);
    const uint32_t vb = vec_bytes<T, NP>(L);
    b.minv.bind(reinterpret_cast<const T*>(L.minv), row_bytes<T>(L));
    b.mrow = ld<T>(L.minv, row);
    b.rhs.bind(vec<T>(L.Pb), vb);
    b.x0.bind(cheb_buf<T>(L, out0), vb);
    b.x1.bind(cheb_buf<T>(L, 1 - out0), vb);
    b.gamma = (T)gamma_d;
    run_staged<T, NP, CH, HR>(b, L, tile, row, reinterpret_cast<T*>(fel_smem), (TileReducer<NP>*)nullptr);
}

template <typename T, int W, int NP, int CH, int HR>
__global__ __launch_bounds__(TILE) void k_cheb_lds(DevLayout L, int tile_begin, int cur, double omega_d,
                                                   double gamma_d) {
    FEL_ROW_LAYOUT();
    extern __shared__ __align__(16) unsigned char fel_smem[];
    ChebStaged<T, W> b;
    staged_row_setup<T, W, HR>(b, L, R, row);
    const uint32_t vb = vec_bytes<T, NP>(L);
    b.mrow = ld<T>(L.minv, row);
    b.rhs.bind(vec<T>(L.Pb), vb);
    b.xk.bind(cheb_buf<T>(L, cur), vb);
    b.xp.bind(cheb_buf<T>(L, 1 - cur), vb);
    b.omega = (T)omega_d;
    b.gamma = (T)gamma_d;
    run_staged<T, NP, CH, HR>(b, L, tile, row, reinterpret_cast<T*>(fel_smem), (TileReducer<NP>*)nullptr);
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
// dispatch

// dynamic LDS a staged launch may use
constexpr size_t kMaxStageBytes = kStageBytes;  // plus the static reducer buffer

// halo rounds of the staged instantiation a layout runs (its stage row is
// TILE plus the largest halo, rounded up to 64)
inline int staged_halo_rounds(const DevLayout& L) { return L.sw - TILE <= 2 * TILE ? 2 : 4; }

// Launches kernel K<T, W, NP, CH> (or, when staged, K_lds with 2 ch stage
// rows of dynamic LDS) for the context's value type and the population
// batch ch (1, 2 or 4).
#define FEL_SOLVER_LAUNCH_T(K, T, SH, ch, s, nt, ...)                                    \
    do {                                                                               \
        switch (ch) {                                                                  \
        case 4:                                                                        \
            if constexpr (direct_max_batch(W, sizeof(T)) >= 4)                         \
                FEL_LAUNCH((K<T, W, NP, 4>), dim3(nt), dim3(TILE), SH, s, __VA_ARGS__); \
            else                                                                       \
                return hipErrorInvalidValue;                                           \
            break;                                                                     \
        case 2: FEL_LAUNCH((K<T, W, NP, 2>), dim3(nt), dim3(TILE), SH, s, __VA_ARGS__); break; \
        default: FEL_LAUNCH((K<T, W, NP, 1>), dim3(nt), dim3(TILE), SH, s, __VA_ARGS__);       \
        }                                                                              \
    } while (0)

// The staged kernels' halo registers are sized for HR rounds of TILE
// entries: 2 when the layout's largest halo fits (smaller register
// footprint, more resident blocks), else 4; HR = 0 is the per-wavefront
// form (kWaveHaloRounds rounds of 64 entries), built for ELL width 7.
#define FEL_STAGED_LAUNCH_HR(K, T, SH, C, hr, s, nt, ...)                                          \
    do {                                                                                           \
        if (hr == 0) {                                                                             \
            if constexpr (W == 7) FEL_LAUNCH((K<T, W, NP, C, 0>), dim3(nt), dim3(TILE), SH, s, __VA_ARGS__); \
            else return hipErrorInvalidValue;                                                      \
        } else if (hr == 2) {                                                                      \
            FEL_LAUNCH((K<T, W, NP, C, 2>), dim3(nt), dim3(TILE), SH, s, __VA_ARGS__);              \
        } else {                                                                                   \
            FEL_LAUNCH((K<T, W, NP, C, 4>), dim3(nt), dim3(TILE), SH, s, __VA_ARGS__);              \
        }                                                                                          \
    } while (0)
#define FEL_STAGED_LAUNCH_T(K, T, SH, ch, hr, s, nt, ...)                  \
    do {                                                                   \
        switch (ch) {                                                      \
        case 4: FEL_STAGED_LAUNCH_HR(K, T, SH, 4, hr, s, nt, __VA_ARGS__); break; \
        case 2: FEL_STAGED_LAUNCH_HR(K, T, SH, 2, hr, s, nt, __VA_ARGS__); break; \
        default: FEL_STAGED_LAUNCH_HR(K, T, SH, 1, hr, s, nt, __VA_ARGS__);       \
        }                                                                  \
    } while (0)

// stage: 1 direct, 2 per tile, 3 per wavefront
#define FEL_SOLVER_LAUNCH(K, ch, stage, s, nt, ...)                                   \
    do {                                                                              \
        const bool f64_ = L.precision == 0;                                           \
        if (stage == 2 || stage == 3) {                                               \
            const bool wave_ = stage == 3;                                            \
            const size_t sh_ = 2 * (size_t)(ch) * (wave_ ? kWaveStageWidth : L.sw) * (f64_ ? 8 : 4); \
            if (sh_ > kMaxStageBytes || L.sw > TILE + kHaloRounds * TILE ||          \
                !staged_vectors_fit(NP, L.R, L.precision) || (wave_ && !L.wlcol))     \
                return hipErrorInvalidValue;                                          \
            const int hr_ = wave_ ? 0 : staged_halo_rounds(L);                        \
            if (f64_) FEL_STAGED_LAUNCH_T(K##_lds, double, sh_, ch, hr_, s, nt, __VA_ARGS__); \
            else FEL_STAGED_LAUNCH_T(K##_lds, float, sh_, ch, hr_, s, nt, __VA_ARGS__);       \
        } else if (stage == 1) {                                                      \
            if (f64_) FEL_SOLVER_LAUNCH_T(K, double, 0, ch, s, nt, __VA_ARGS__);          \
            else FEL_SOLVER_LAUNCH_T(K, float, 0, ch, s, nt, __VA_ARGS__);                \
        } else {                                                                      \
            return hipErrorInvalidValue;                                              \
        }                                                                             \
    } while (0)

template <int Q, int W> struct CgInitBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, int ch, int st, hipStream_t s) {
        constexpr int NP = 2 * (Q - 1);
        FEL_SOLVER_LAUNCH(k_cg_init, ch, st, s, nt, L, tb);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct CgABody {
    static hipError_t run(const DevLayout& L, int tb, int nt, bool first, int it, int ch, int st, hipStream_t s) {
        constexpr int NP = 2 * (Q - 1);
        FEL_SOLVER_LAUNCH(k_cg_a, ch, st, s, nt, L, tb, (int)first, it);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct CgBBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, int it, int ch, int st, hipStream_t s) {
        constexpr int NP = 2 * (Q - 1);
        FEL_SOLVER_LAUNCH(k_cg_b, ch, st, s, nt, L, tb, it);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct ChebFirstBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, int out0, double gamma, int ch,
                          int st, hipStream_t s) {
        constexpr int NP = 2 * (Q - 1);
        FEL_SOLVER_LAUNCH(k_cheb_first, ch, st, s, nt, L, tb, out0, gamma);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct ChebBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, int cur, double omega, double gamma,
                          int ch, int st, hipStream_t s) {
        constexpr int NP = 2 * (Q - 1);
        FEL_SOLVER_LAUNCH(k_cheb, ch, st, s, nt, L, tb, cur, omega, gamma);
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

hipError_t launch_cg_init(const DevLayout& L, int tb, int nt, int batch, int stage, hipStream_t s) {
    return dispatch_qw<CgInitBody>(L, tb, nt, batch, stage, s);
}
hipError_t launch_cg_a(const DevLayout& L, int tb, int nt, bool first, int it, int batch, int stage,
                       hipStream_t s) {
    if (it < 0 || it >= L.K || (!first && it == 0)) return hipErrorInvalidValue;
    return dispatch_qw<CgABody>(L, tb, nt, first, it, batch, stage, s);
}
hipError_t launch_cg_b(const DevLayout& L, int tb, int nt, int it, int batch, int stage, hipStream_t s) {
    if (it < 0 || it >= L.K) return hipErrorInvalidValue;
    return dispatch_qw<CgBBody>(L, tb, nt, it, batch, stage, s);
}
hipError_t launch_cg_x(const DevLayout& L, int tb, int nt, bool check, hipStream_t s) {
    (void)hipGetLastError();
    // the residual check reads the fused CG's partials, which exist for the 2-D lattice only
    if (nt <= 0 || (check && (L.Q != 9 || L.nfb <= 0))) return hipErrorInvalidValue;
    const bool f64 = L.precision == 0;
    const int ck = check ? 1 : 0;
    if (L.Q == 9) {
        if (f64) FEL_LAUNCH((k_cg_x<double, 16>), dim3(nt), dim3(TILE), 0, s, L, tb, ck);
        else FEL_LAUNCH((k_cg_x<float, 16>), dim3(nt), dim3(TILE), 0, s, L, tb, ck);
    } else if (L.Q == 19) {
        if (f64) FEL_LAUNCH((k_cg_x<double, 36>), dim3(nt), dim3(TILE), 0, s, L, tb, ck);
        else FEL_LAUNCH((k_cg_x<float, 36>), dim3(nt), dim3(TILE), 0, s, L, tb, ck);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
hipError_t launch_cheb_first(const DevLayout& L, int tb, int nt, int out0, double gamma, int batch,
                             int stage, hipStream_t s) {
    return dispatch_qw<ChebFirstBody>(L, tb, nt, out0, gamma, batch, stage, s);
}
hipError_t launch_cheb(const DevLayout& L, int tb, int nt, int cur, double omega, double gamma,
                       int batch, int stage, hipStream_t s) {
    return dispatch_qw<ChebBody>(L, tb, nt, cur, omega, gamma, batch, stage, s);
}
hipError_t launch_lumped(const DevLayout& L, int tb, int nt, hipStream_t s) {
    return dispatch_qw<LumpedBody>(L, tb, nt, s);
}

// Fused kernels: D2Q9 layouts of ELL width 7 only (the host enables the
// path there; at width 12 their rows would spill registers).  Their
// 1024-thread blocks cap a thread at 128 VGPRs, so only the population
// batches that fit without spilling are built (fused_max_batch: cg_init 4
// in FP32 / 2 in FP64, cg_a 1, cg_b 4 / 1); a larger batch runs as the
// largest built one.
#define FEL_FUSED_W7(K, T, B, s, ...) FEL_LAUNCH((K<T, 7, 16, B>), g_, b_, 0, s, __VA_ARGS__)
#define FEL_FUSED_LAUNCH(K, ch, MAX32, MAX64, s, ...)                                                 \
    do {                                                                                              \
        if (L.Q != 9 || L.nfb <= 0) return hipErrorInvalidValue;                                     \
        const bool f64_ = L.precision == 0;                                                           \
        const int c_ = min(ch, f64_ ? MAX64 : MAX32);                                                 \
        const dim3 g_(L.nfb), b_(FB_THREADS);                                                         \
        if (L.W == 7) {                                                                               \
            if (f64_) {                                                                               \
                if (MAX64 >= 4 && c_ == 4) FEL_FUSED_W7(K, double, (MAX64 >= 4 ? 4 : 1), s, __VA_ARGS__); \
                else if (MAX64 >= 2 && c_ == 2) FEL_FUSED_W7(K, double, (MAX64 >= 2 ? 2 : 1), s, __VA_ARGS__); \
                else FEL_FUSED_W7(K, double, 1, s, __VA_ARGS__);                                      \
            } else {                                                                                  \
                if (MAX32 >= 4 && c_ == 4) FEL_FUSED_W7(K, float, (MAX32 >= 4 ? 4 : 1), s, __VA_ARGS__); \
                else if (MAX32 >= 2 && c_ == 2) FEL_FUSED_W7(K, float, (MAX32 >= 2 ? 2 : 1), s, __VA_ARGS__); \
                else FEL_FUSED_W7(K, float, 1, s, __VA_ARGS__);                                       \
            }                                                                                         \
        } else {                                                                                      \
            return hipErrorInvalidValue;                                                              \
        }                                                                                             \
    } while (0)

int fused_max_batch(int cls, int precision) {
    const bool f64 = precision == 0;
    if (cls == KC_CG_INIT) return f64 ? 2 : 4;
    if (cls == KC_CG_B) return f64 ? 1 : 4;
    return 1;
}

hipError_t launch_cg_init_fused(const DevLayout& L, int batch, hipStream_t s) {
    (void)hipGetLastError();
    FEL_FUSED_LAUNCH(k_cg_init_fused, batch, 4, 2, s, L);
    return hipGetLastError();
}
hipError_t launch_cg_a_fused(const DevLayout& L, int it, int batch, hipStream_t s) {
    (void)hipGetLastError();
    if (it < 0 || it >= L.K) return hipErrorInvalidValue;
    FEL_FUSED_LAUNCH(k_cg_a_fused, batch, 1, 1, s, L, it);
    return hipGetLastError();
}
hipError_t launch_cg_b_fused(const DevLayout& L, int it, int batch, hipStream_t s) {
    (void)hipGetLastError();
    if (it < 0 || it >= L.K) return hipErrorInvalidValue;
    FEL_FUSED_LAUNCH(k_cg_b_fused, batch, 4, 1, s, L, it);
    return hipGetLastError();
}

hipError_t launch_finalize(const DevLayout& L, int inst_begin, int ninst, int op, int nvals, hipStream_t s,
                           int it) {
    (void)hipGetLastError();
    if (op == FIN_CG_A && (it < 0 || it >= L.K)) return hipErrorInvalidValue;
    const dim3 grid(ninst, nvals), block(FIN_THREADS);
    if (nvals == 16)
        FEL_LAUNCH((k_finalize<16>), grid, block, 0, s, L, inst_begin, op, it);
    else if (nvals == 36)
        FEL_LAUNCH((k_finalize<36>), grid, block, 0, s, L, inst_begin, op, it);
    else if (nvals == 8)
        FEL_LAUNCH((k_finalize<8>), grid, block, 0, s, L, inst_begin, op, it);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace fel
