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
// This file holds the streaming right-hand side (direct, and LDS-staged for
// 2-D grids), moments, recovery, collision, initialisation and conserved
// sums; the mass solve is in felbm_solver.hip.  Reductions (conserved sums, CG dot products) are FP64:
// per-tile partials in a fixed order (wavefront shuffles, then LDS), summed
// per instance in a fixed order, so results are bitwise reproducible.
#include "felbm_device.h"
namespace fel {

thread_local LaunchEvents g_launch_events;

const char* kernel_class_name(int k) {
    static const char* names[KC_COUNT] = {"stream", "cg_init", "cg_a", "cg_b", "lumped", "moments", "grad",
                                          "div", "collide", "init", "sums", "finalize", "cheb", "cg_x"};
    return (k >= 0 && k < KC_COUNT) ? names[k] : "?";
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
    // one slot at a time: the accumulators and a slot's 2(Q-1) gathers fill
    // the registers (unrolling the slots too ran one wave per SIMD in 2-D
    // and spilled in 3-D)
#pragma unroll 1
    for (int k = 0; k < W; k++) {
        const int64_t c = ell_col(L, k, row);
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
// walls + density moment, FP64 populations
// (LAST: the collision, the last reader in the step: non-temporal loads)
template <int Q, bool LAST = false>
__device__ __forceinline__ void streamed_plain(const DevLayout& L, int64_t row, int base, double (&v)[Q]) {
    // base = 0 for f, Q for g; X holds Delta for populations 1..Q-1 of each
    const int64_t R = L.R;
    const double* psi = reinterpret_cast<const double*>(L.psi);
    const double* X = reinterpret_cast<const double*>(L.X);
    auto ld = [](const double* p) { return LAST ? __builtin_nontemporal_load(p) : *p; };
    const int xb = base ? (Q - 1) : 0;
    v[0] = ld(&psi[(int64_t)base * R + row]);
#pragma unroll
    for (int a = 1; a < Q; a++) v[a] = ld(&psi[(int64_t)(base + a) * R + row]) + ld(&X[(int64_t)(xb + a - 1) * R + row]);
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
        const T v = rho[ell_col(L, k, row)];
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
        const int64_t c = ell_col(L, k, row);
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
        const double v = mu[ell_col(L, k, row)];
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
    streamed_plain<Q, true>(L, row, 0, f);
    streamed_plain<Q, true>(L, row, Q, g);
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
    // slot 0 is the row itself, whose differences are exactly 0: it adds
    // nothing to the sums, so it is skipped
#pragma unroll
    for (int k = 1; k < W; k++) {
        // pattern and basis values stream through once: non-temporal, so they
        // do not evict the population rows that neighbouring tiles gather
        const int c = __builtin_nontemporal_load(&L.col[k * R + row]);
        float b[NB];
#pragma unroll
        for (int n = 0; n < NB; n++) b[n] = __builtin_nontemporal_load(&B[((int64_t)n * W + k) * R + row]);
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
// a stored value as float, non-temporal when NT (FP16 through its bits)
// The streaming step with neighbour values read from LDS (2-D grids,
// ELL width 7).  The block stages the two node references at its rows and
// its halo once, then, one lattice direction a per pass, the stored
// deviations of f_a and g_a (own rows with coalesced loads, one load per
// halo entry); every row forms its sums through the 16-bit local columns,
// slot by slot in the direct kernel's order (the same values and the same
// operations).  The basis values of the row's slots stay in registers for
// all directions.  Passes are double-buffered as in the staged solver
// kernels: the next direction's loads are issued right after the barrier
// that publishes the current one.  Dynamic LDS: 6 sw floats (references,
// and 2 buffers of 2 stage rows).  Each thread stages at most HR halo
// entries (the host checks).
template <int Q, typename S, int HR>
__global__ __launch_bounds__(TILE) void k_stream_dev_lds(DevLayout L, int tile_begin) {
    using LT = Lat<Q>;
    constexpr int W = 7, NB = LT::NB;
    static_assert(LT::D == 2, "staged streaming is built for the 2-D lattice");
    extern __shared__ __align__(16) unsigned char fel_smem[];
    float* rs = reinterpret_cast<float*>(fel_smem);  // [2][sw] references
    float* st = rs + 2 * L.sw;                         // [2 buffers][2][sw]
    const int sw = L.sw;
    const int tile = tile_begin + tile_of_block(blockIdx.x, gridDim.x);
    const int64_t R = L.R;
    const int lr = threadIdx.x;
    const int row = tile * TILE + lr;
    const InstParams& P = L.params[L.tile_inst[tile]];
    const float dt = (float)P.dt, h2 = 0.5f * dt * dt, sc = (float)P.scale;
    const int hb = L.halo_ptr[tile], hn = L.halo_ptr[tile + 1] - hb;
    int hg[HR];
#pragma unroll
    for (int i = 0; i < HR; i++) {
        const int h = lr + i * TILE;
        hg[i] = h < hn ? L.halo_col[hb + h] : -1;
    }
    const float* reff = L.ref;
    const float* refg = L.ref + R;
    const float rf0 = reff[row], rg0 = refg[row];
    rs[lr] = rf0;
    rs[sw + lr] = rg0;
#pragma unroll
    for (int i = 0; i < HR; i++) {
        if (hg[i] >= 0) {
            rs[TILE + i * TILE + lr] = reff[hg[i]];
            rs[sw + TILE + i * TILE + lr] = refg[hg[i]];
        }
    }
    // the row's slots: local columns and basis values, read once
    const float* B = reinterpret_cast<const float*>(L.basis);
    int lc[W];
    float b[W][NB];
#pragma unroll
    for (int k = 1; k < W; k++) {
        lc[k] = __builtin_nontemporal_load(&L.lcol[k * R + row]);
#pragma unroll
        for (int n = 0; n < NB; n++) b[k][n] = __builtin_nontemporal_load(&B[((int64_t)n * W + k) * R + row]);
    }
    // the stored values as loaded; converted when the stage is written (a
    // conversion where the halo is loaded would wait for the loads inside
    // the halo branch, before the current direction is used)
    const S* ps = reinterpret_cast<const S*>(L.psi);
    S v[2], vh[HR][2];
    auto fetch = [&](int a) {
        v[0] = ps[(int64_t)a * R + row];
        v[1] = ps[(int64_t)(Q + a) * R + row];
#pragma unroll
        for (int i = 0; i < HR; i++) {
            if (hg[i] >= 0) {
                vh[i][0] = ps[(int64_t)a * R + hg[i]];
                vh[i][1] = ps[(int64_t)(Q + a) * R + hg[i]];
            }
        }
    };
    fetch(1);
    __syncthreads();  // references published
    float drf[W], drg[W];
#pragma unroll
    for (int k = 1; k < W; k++) {
        drf[k] = rs[lc[k]] - rf0;
        drg[k] = rs[sw + lc[k]] - rg0;
    }
    float* rhs = reinterpret_cast<float*>(L.Pb);
#pragma unroll
    for (int a = 1; a < Q; a++) {
        float* buf = st + ((a - 1) & 1) * 2 * sw;
        buf[lr] = (float)v[0];
        buf[sw + lr] = (float)v[1];
#pragma unroll
        for (int i = 0; i < HR; i++) {
            if (hg[i] >= 0) {
                buf[TILE + i * TILE + lr] = (float)vh[i][0];
                buf[sw + TILE + i * TILE + lr] = (float)vh[i][1];
            }
        }
        __syncthreads();
        if (a + 1 < Q) fetch(a + 1);
        const float ex = LT::e(a, 0), ey = LT::e(a, 1);
        const float f0 = buf[lr], g0 = buf[sw + lr];
        float af = 0.0f, ag = 0.0f;
#pragma unroll
        for (int k = 1; k < W; k++) {
            const float coef = dt * (ex * b[k][0] + ey * b[k][1]) +
                               h2 * (ex * ex * b[k][2] + ey * ey * b[k][3] + ex * ey * b[k][4]);
            const float df = buf[lc[k]] - f0;
            const float dg = buf[sw + lc[k]] - g0;
            af += coef * (drf[k] + sc * df);
            ag += coef * (drg[k] + sc * dg);
        }
        const float w = (float)LT::w(a);
        rhs[(int64_t)(a - 1) * R + row] = -w * af;
        rhs[(int64_t)(Q - 1 + a - 1) * R + row] = -w * ag;
        // keep the next direction's conversions (and the waits for its loads)
        // behind this direction's rows
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <bool NT, typename V>
__device__ __forceinline__ float ldf(const V* p) {
    if constexpr (!NT) {
        return (float)*p;
    } else if constexpr (std::is_same<V, __half>::value) {
        const unsigned short b = __builtin_nontemporal_load(reinterpret_cast<const unsigned short*>(p));
        return __half2float(__ushort_as_half(b));
    } else {
        return (float)__builtin_nontemporal_load(p);
    }
}

// (LAST: the collision, the last reader of these values in the step, which
// reads them non-temporally)
template <int Q, typename S, bool LAST = false>
__device__ __forceinline__ void streamed_dev(const DevLayout& L, int row, int base, float sc, float (&e)[Q]) {
    using LT = Lat<Q>;
    const int64_t R = L.R;
    const float* X = reinterpret_cast<const float*>(L.X);
    const S* psi = reinterpret_cast<const S*>(L.psi);
    const int xb = base ? (Q - 1) : 0;
    e[0] = sc * ldf<LAST>(&psi[(int64_t)base * R + row]);
#pragma unroll
    for (int a = 1; a < Q; a++)
        e[a] = sc * ldf<LAST>(&psi[(int64_t)(base + a) * R + row]) +
               ldf<LAST>(&X[(int64_t)(xb + a - 1) * R + row]) * (float)(1.0 / LT::w(a));
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
        const T v = gat(f, ell_col(L, k, row));
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
    streamed_dev<Q, S, true>(L, row, 0, sc, ef);
    streamed_dev<Q, S, true>(L, row, Q, sc, eg);
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

template <int Q, int W> struct StreamBody {
    static hipError_t run(const DevLayout& L, int tb, int nt, bool staged, hipStream_t s) {
        if constexpr (Q == 9 && W == 7) {
            if (staged) {
                // 2 reference rows and 2 buffers of 2 stage rows
                const size_t sh = 6 * (size_t)L.sw * sizeof(float);
                if (L.precision == 0 || L.sw > TILE + kHaloRounds * TILE || sh > (size_t)kStageBytes)
                    return hipErrorInvalidValue;
                const bool hr2 = L.sw - TILE <= 2 * TILE;
                if (L.precision == 1) {
                    if (hr2) FEL_LAUNCH((k_stream_dev_lds<Q, float, 2>), dim3(nt), dim3(TILE), sh, s, L, tb);
                    else FEL_LAUNCH((k_stream_dev_lds<Q, float, 4>), dim3(nt), dim3(TILE), sh, s, L, tb);
                } else {
                    if (hr2) FEL_LAUNCH((k_stream_dev_lds<Q, __half, 2>), dim3(nt), dim3(TILE), sh, s, L, tb);
                    else FEL_LAUNCH((k_stream_dev_lds<Q, __half, 4>), dim3(nt), dim3(TILE), sh, s, L, tb);
                }
                FEL_CHECK_LAUNCH();
            }
        }
        if (staged) return hipErrorInvalidValue;
        if (L.precision == 0)
            FEL_LAUNCH((k_stream_plain<Q, W>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else if (L.precision == 1)
            FEL_LAUNCH((k_stream_dev<Q, W, float>), dim3(nt), dim3(TILE), 0, s, L, tb);
        else
            FEL_LAUNCH((k_stream_dev<Q, W, __half>), dim3(nt), dim3(TILE), 0, s, L, tb);
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

hipError_t launch_stream(const DevLayout& L, int tb, int nt, bool staged, hipStream_t s) {
    return dispatch_qw<StreamBody>(L, tb, nt, staged, s);
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
