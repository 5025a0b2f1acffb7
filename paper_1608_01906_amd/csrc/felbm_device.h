// Device-side helpers shared by the kernel translation units of the FE
// lattice Boltzmann step (gfx950): launch wrapper, lattice tables, the
// XCD-aware tile mapping, wavefront/tile reductions, ELL gathers and the
// (lattice, ELL width) dispatch.
#pragma once

#include "felbm_internal.h"

#include <hip/hip_ext.h>

namespace fel {

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
template <int NP, int NW = TILE / 64>
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
    // the tile's partials, population-major: partial[j][tile]
    __device__ __forceinline__ void finish(const DevLayout& L, int tile) {
        __syncthreads();
        for (int j = threadIdx.x; j < NP; j += NW * 64) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < NW; w++) s += lds[w][j];
            L.partial[(int64_t)j * L.ntiles + tile] = s;
        }
    }
    // the block's partials over its first nw waves: dst[j * stride + index]
    __device__ __forceinline__ void finish_to(double* dst, int stride, int index, int nw) {
        __syncthreads();
        for (int j = threadIdx.x; j < NP; j += NW * 64) {
            double s = 0.0;
            for (int w = 0; w < nw; w++) s += lds[w][j];
            dst[(int64_t)j * stride + index] = s;
        }
    }
};

#define FEL_REDUCER(NAME, NP)                         \
    __shared__ double NAME##_buf[TILE / 64][NP];      \
    TileReducer<NP> NAME(NAME##_buf)

#define FEL_REDUCER_N(NAME, NP, NW)                   \
    __shared__ double NAME##_buf[NW][NP];             \
    TileReducer<NP, NW> NAME(NAME##_buf)

// Column of ELL slot k of a row.  Slot 0 is the diagonal in every pattern
// row (padding rows included), so it is the row itself and is not loaded;
// with k a compile-time constant the test folds away.
__device__ __forceinline__ int ell_col(const DevLayout& L, int k, int64_t row) {
    return k == 0 ? (int)row : L.col[k * L.R + row];
}

// gathers through a uniform base and a 32-bit byte offset
template <typename T>
__device__ __forceinline__ T gat(const T* base, int idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)idx * (uint32_t)sizeof(T));
}
// the store of the same form
template <typename T>
__device__ __forceinline__ void sto(T* base, int idx, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)idx * (uint32_t)sizeof(T)) = v;
}

// A population-major vector [n][R] of T (4 or 8 bytes) through a buffer
// resource (raw buffer: stride 0, byte offsets).  An access takes the row's
// byte offset in a VGPR and the population's slice offset (j R sizeof(T),
// uniform) in an SGPR, so one offset register serves every population of a
// row and no 64-bit address is formed per access.  The resource covers the
// whole vector; a row offset at or past its size (kIdleRow) is out of range:
// the load returns 0 and touches no memory.
constexpr uint32_t kIdleRow = 0xFFFFFFF0u;
template <typename T>
struct BufVec {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit elements");
    typedef unsigned U2 __attribute__((ext_vector_type(2)));
    __amdgpu_buffer_rsrc_t rs;
    __device__ __forceinline__ void bind(const T* base, uint32_t bytes) {
        rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0, (int)bytes, 0x00020000);
    }
    __device__ __forceinline__ T load(uint32_t voff, uint32_t soff) const {
        if constexpr (sizeof(T) == 4)
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
        else
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
    }
    __device__ __forceinline__ void store(T v, uint32_t voff, uint32_t soff) const {
        if constexpr (sizeof(T) == 4)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, voff, soff, 0);
        else
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), rs, voff, soff, 0);
    }
};

// ---------------------------------------------------------------------------
// dispatch

#define FEL_CHECK_LAUNCH() return hipGetLastError()

// run body<Q, W>() for the context's lattice and ELL width
template <template <int, int> class Body, typename... A>
inline hipError_t dispatch_qw(const DevLayout& L, A... args) {
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

}  // namespace fel
