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
// in a fixed order (wavefront shuffles, then LDS), and the last block of
// each instance to finish sums that instance's partials in a fixed order,
// so results are bitwise reproducible and no extra launch is needed.
#include "felbm_internal.h"

namespace fel {

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
                                          "grad", "div", "collide", "init", "sums"};
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

template <typename T> __device__ __forceinline__ T ld(const void* p, int64_t i) {
    return reinterpret_cast<const T*>(p)[i];
}
template <typename T> __device__ __forceinline__ void st(void* p, int64_t i, T v) {
    reinterpret_cast<T*>(p)[i] = v;
}

// Per-tile partial sums of NP values, then the instance's last block sums
// all its tiles (fixed order) and calls op(inst, j, total) for j < NP.
template <int NP, typename Op>
__device__ __forceinline__ void reduce_finalize(const DevLayout& L, int tile, int inst, double (&part)[NP],
                                                Op op) {
    static_assert(NP <= TILE, "too many reduction values");
    __shared__ double lds[TILE / 64][NP];
    __shared__ double fin[TILE];
    __shared__ int s_last;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NP; j++) {
        const double v = wave_sum(part[j]);
        if (lane == 0) lds[wave][j] = v;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < NP; j += TILE) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < TILE / 64; w++) s += lds[w][j];
        L.partial[(int64_t)tile * NP + j] = s;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const int prev = atomicAdd(&L.counter[inst], 1);
        s_last = (prev == L.params[inst].tile_count - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    const int tb = L.params[inst].tile_begin, nt = L.params[inst].tile_count;
    constexpr int G = TILE / NP;
    const int j = threadIdx.x % NP, g = threadIdx.x / NP;
    double s = 0.0;
    if (g < G)
        for (int t = g; t < nt; t += G)
            s += __hip_atomic_load(&L.partial[(int64_t)(tb + t) * NP + j], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    fin[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < NP) {
        double tot = 0.0;
        for (int gg = 0; gg < G; gg++) tot += fin[gg * NP + threadIdx.x];
        op(inst, (int)threadIdx.x, tot);
    }
    if (threadIdx.x == 0) atomicExch(&L.counter[inst], 0);
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

template <typename T, int W, int NP>
__global__ __launch_bounds__(TILE) void k_cg_init(DevLayout L, int tile_begin) {
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int inst = L.tile_inst[tile];
    const int64_t R = L.R;
    const int64_t row = (int64_t)tile * TILE + threadIdx.x;
    const T* rhs = reinterpret_cast<const T*>(L.Pb);
    const T* minv = reinterpret_cast<const T*>(L.minv);
    int64_t c[W];
    T mv[W], mi[W];
#pragma unroll
    for (int k = 0; k < W; k++) {
        c[k] = L.col[k * R + row];
        mv[k] = ld<T>(L.Mval, k * R + row);
        mi[k] = minv[c[k]];
    }
    const T mrow = minv[row];
    double part[NP];
#pragma unroll
    for (int j = 0; j < NP; j++) {
        const T* b = rhs + (int64_t)j * R;
        T acc = 0;
#pragma unroll
        for (int k = 0; k < W; k++) acc += mv[k] * (b[c[k]] * mi[k]);
        const T bj = b[row];
        const T r = bj - acc;
        st<T>(L.X, (int64_t)j * R + row, bj * mrow);
        st<T>(L.Rv, (int64_t)j * R + row, r);
        part[j] = (double)r * (double)r * (double)mrow;
    }
    reduce_finalize<NP>(L, tile, inst, part, [&](int in, int j, double tot) {
        L.rz[in * NP + j] = tot;
        L.rz0[in * NP + j] = tot;
        L.beta[in * NP + j] = 0.0;
    });
}

// p_new = r / m + beta p_old (p_old unread on the first iteration),
// q = M p_new recomputed from neighbour values; reduces p.q -> alpha.
template <typename T, int W, int NP>
__global__ __launch_bounds__(TILE) void k_cg_a(DevLayout L, int tile_begin, int first, int flip) {
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int inst = L.tile_inst[tile];
    const int64_t R = L.R;
    const int64_t row = (int64_t)tile * TILE + threadIdx.x;
    const T* Rv = reinterpret_cast<const T*>(L.Rv);
    const T* Pold = reinterpret_cast<const T*>(flip ? L.Pa : L.Pb);
    T* Pnew = reinterpret_cast<T*>(flip ? L.Pb : L.Pa);
    const T* minv = reinterpret_cast<const T*>(L.minv);
    int64_t c[W];
    T mv[W], mi[W];
#pragma unroll
    for (int k = 0; k < W; k++) {
        c[k] = L.col[k * R + row];
        mv[k] = ld<T>(L.Mval, k * R + row);
        mi[k] = minv[c[k]];
    }
    const T mrow = minv[row];
    double part[NP];
#pragma unroll
    for (int j = 0; j < NP; j++) {
        const T* r = Rv + (int64_t)j * R;
        const T* po = Pold + (int64_t)j * R;
        T acc = 0, pown;
        if (first) {
#pragma unroll
            for (int k = 0; k < W; k++) acc += mv[k] * (r[c[k]] * mi[k]);
            pown = r[row] * mrow;
        } else {
            const T bet = (T)L.beta[inst * NP + j];
#pragma unroll
            for (int k = 0; k < W; k++) acc += mv[k] * (r[c[k]] * mi[k] + bet * po[c[k]]);
            pown = r[row] * mrow + bet * po[row];
        }
        Pnew[(int64_t)j * R + row] = pown;
        part[j] = (double)pown * (double)acc;
    }
    reduce_finalize<NP>(L, tile, inst, part, [&](int in, int j, double tot) {
        const double rz = L.rz[in * NP + j];
        L.alpha[in * NP + j] = (tot != 0.0) ? rz / tot : 0.0;
    });
}

// x += alpha p, r -= alpha M p (M p recomputed), reduces r.z -> beta;
// on the last iteration checks r.z / r0.z0 against the tolerance instead.
template <typename T, int W, int NP>
__global__ __launch_bounds__(TILE) void k_cg_b(DevLayout L, int tile_begin, int last, int flip) {
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int inst = L.tile_inst[tile];
    const int64_t R = L.R;
    const int64_t row = (int64_t)tile * TILE + threadIdx.x;
    const T* Pn = reinterpret_cast<const T*>(flip ? L.Pb : L.Pa);
    T* X = reinterpret_cast<T*>(L.X);
    T* Rv = reinterpret_cast<T*>(L.Rv);
    const T* minv = reinterpret_cast<const T*>(L.minv);
    int64_t c[W];
    T mv[W];
#pragma unroll
    for (int k = 0; k < W; k++) {
        c[k] = L.col[k * R + row];
        mv[k] = ld<T>(L.Mval, k * R + row);
    }
    const T mrow = minv[row];
    double part[NP];
#pragma unroll
    for (int j = 0; j < NP; j++) {
        const T* p = Pn + (int64_t)j * R;
        T q = 0;
#pragma unroll
        for (int k = 0; k < W; k++) q += mv[k] * p[c[k]];
        const T al = (T)L.alpha[inst * NP + j];
        const int64_t i = (int64_t)j * R + row;
        const T x = X[i] + al * p[row];
        const T r = Rv[i] - al * q;
        X[i] = x;
        Rv[i] = r;
        part[j] = (double)r * (double)r * (double)mrow;
    }
    if (last) {
        reduce_finalize<NP>(L, tile, inst, part, [&](int in, int j, double tot) {
            const double r0 = L.rz0[in * NP + j];
            if (r0 > 0.0 && !(tot <= L.cg_tol2 * r0)) atomicOr(L.status, 2u);
        });
    } else {
        reduce_finalize<NP>(L, tile, inst, part, [&](int in, int j, double tot) {
            const double rz = L.rz[in * NP + j];
            L.beta[in * NP + j] = (rz != 0.0) ? tot / rz : 0.0;
            L.rz[in * NP + j] = tot;
        });
    }
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
    reduce_finalize<8>(L, tile, inst, part, [&](int in, int j, double tot) { L.sums[in * 8 + j] = tot; });
}

// ---------------------------------------------------------------------------
// dispatch

#define FEL_CHECK_LAUNCH() return hipGetLastError()

// run body<Q, W>() for the context's lattice and ELL width
template <template <int, int> class Body, typename... A>
static hipError_t dispatch_qw(const DevLayout& L, A... args) {
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
        if (L.precision == 0) {
            hipLaunchKernelGGL((k_stream_plain<Q, W>), dim3(nt), dim3(TILE), 0, s, L, tb);
            FEL_CHECK_LAUNCH();
        }
        return hipErrorInvalidValue;
    }
};
template <int Q, int W> struct CgInitBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        constexpr int NP = 2 * (Q - 1);
        if (L.precision == 0)
            hipLaunchKernelGGL((k_cg_init<double, W, NP>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else
            hipLaunchKernelGGL((k_cg_init<float, W, NP>), dim3(nt), dim3(TILE), 0, s, L, tb);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct CgABody {
    static hipError_t run(const DevLayout& L, int tb, int nt, bool first, bool flip, hipStream_t s) {
        constexpr int NP = 2 * (Q - 1);
        if (L.precision == 0)
            hipLaunchKernelGGL((k_cg_a<double, W, NP>), dim3(nt), dim3(TILE), 0, s, L, tb, (int)first, (int)flip);
        else
            hipLaunchKernelGGL((k_cg_a<float, W, NP>), dim3(nt), dim3(TILE), 0, s, L, tb, (int)first, (int)flip);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct CgBBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, bool last, bool flip, hipStream_t s) {
        constexpr int NP = 2 * (Q - 1);
        if (L.precision == 0)
            hipLaunchKernelGGL((k_cg_b<double, W, NP>), dim3(nt), dim3(TILE), 0, s, L, tb, (int)last, (int)flip);
        else
            hipLaunchKernelGGL((k_cg_b<float, W, NP>), dim3(nt), dim3(TILE), 0, s, L, tb, (int)last, (int)flip);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct LumpedBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        constexpr int NP = 2 * (Q - 1);
        if (L.precision == 0)
            hipLaunchKernelGGL((k_lumped<double, NP>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else
            hipLaunchKernelGGL((k_lumped<float, NP>), dim3(nt), dim3(TILE), 0, s, L, tb);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct MomentsBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        if (L.precision == 0) {
            hipLaunchKernelGGL((k_moments_plain<Q>), dim3(nt), dim3(TILE), 0, s, L, tb);
            FEL_CHECK_LAUNCH();
        }
        return hipErrorInvalidValue;
    }
};
template <int Q, int W> struct GradBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        constexpr int D = Lat<Q>::D;
        if (L.precision == 0)
            hipLaunchKernelGGL((k_grad<double, W, D>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else
            hipLaunchKernelGGL((k_grad<float, W, D>), dim3(nt), dim3(TILE), 0, s, L, tb);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct DivBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        constexpr int D = Lat<Q>::D;
        if (L.precision == 0)
            hipLaunchKernelGGL((k_div<double, W, D>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else
            hipLaunchKernelGGL((k_div<float, W, D>), dim3(nt), dim3(TILE), 0, s, L, tb);
        FEL_CHECK_LAUNCH();
    }
};
template <int Q, int W> struct CollideBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        if (L.precision == 0) {
            hipLaunchKernelGGL((k_collide_plain<Q, W>), dim3(nt), dim3(TILE), 0, s, L, tb);
            FEL_CHECK_LAUNCH();
        }
        return hipErrorInvalidValue;
    }
};
template <int Q, int W> struct InitBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        if (L.precision == 0) {
            hipLaunchKernelGGL((k_init_plain<Q, W>), dim3(nt), dim3(TILE), 0, s, L, tb);
            FEL_CHECK_LAUNCH();
        }
        return hipErrorInvalidValue;
    }
};
template <int Q, int W> struct SumsBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, hipStream_t s) {
        if (L.precision == 0) {
            hipLaunchKernelGGL((k_sums_plain<Q>), dim3(nt), dim3(TILE), 0, s, L, tb);
            FEL_CHECK_LAUNCH();
        }
        return hipErrorInvalidValue;
    }
};

hipError_t launch_stream(const DevLayout& L, int tb, int nt, hipStream_t s) {
    return dispatch_qw<StreamBody>(L, tb, nt, s);
}
hipError_t launch_cg_init(const DevLayout& L, int tb, int nt, hipStream_t s) {
    return dispatch_qw<CgInitBody>(L, tb, nt, s);
}
hipError_t launch_cg_a(const DevLayout& L, int tb, int nt, bool first, bool flip, hipStream_t s) {
    return dispatch_qw<CgABody>(L, tb, nt, first, flip, s);
}
hipError_t launch_cg_b(const DevLayout& L, int tb, int nt, bool last, bool flip, hipStream_t s) {
    return dispatch_qw<CgBBody>(L, tb, nt, last, flip, s);
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
