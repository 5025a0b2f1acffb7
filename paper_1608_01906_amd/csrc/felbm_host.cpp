// Host side of the felbm C ABI: mesh validation and P1 assembly, device
// layout, workspace sub-allocation, step scheduling (HIP graph replay) and
// read-back.  See include/felbm.h for the contract of each entry point.
#include "../../include/felbm.h"
#include "felbm_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace fel;

namespace {


struct LatticeInfo {
    int Q, D, NB;
    int e[19][3];
    double w[19];
};

LatticeInfo make_lattice_info(int Q) {
    LatticeInfo L{};
    L.Q = Q;
    if (Q == 9) {
        const int E[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                             {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
        L.D = 2;
        L.NB = 5;
        for (int a = 0; a < 9; a++) {
            for (int r = 0; r < 3; r++) L.e[a][r] = E[a][r];
            L.w[a] = a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        }
    } else {
        const int E[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                              {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                              {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                              {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
        L.D = 3;
        L.NB = 9;
        for (int a = 0; a < 19; a++) {
            for (int r = 0; r < 3; r++) L.e[a][r] = E[a][r];
            L.w[a] = a == 0 ? 1.0 / 3.0 : (a < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
        }
    }
    return L;
}

// Assembled operators of one instance in local node numbering, row-major
// ELL with the diagonal in slot 0.
struct HostMesh {
    bool present = false;
    int dim = 0;
    int64_t N = 0;
    int W = 0;                    // max row length
    std::vector<int32_t> col;     // [N][W] (-1 = empty slot)
    std::vector<double> M;        // [N][W]
    std::vector<double> basis;    // [NB][N][W]
    std::vector<double> m;        // [N] lumped mass
    std::vector<uint32_t> wmask;  // [N]
    std::vector<int64_t> perm;    // [N] device order -> caller node index
};

struct Instance {
    HostMesh mesh;
    bool have_phys = false;
    fel_phys phys{};
    InstParams P{};
};

struct ProfEvent {
    int cls;
    hipEvent_t a, b;
};

}  // namespace

struct fel_ctx {
    fel_options opt{};
    LatticeInfo lat{};
    std::vector<Instance> inst;
    int ninst = 0;
    // layout
    bool bound = false;
    int W = 0, NB = 0, NP = 0;
    int64_t R = 0;
    int ntiles = 0;
    size_t ws_bytes = 0;
    int cg_iters = 0;
    double cg_tol = 0.0;
    DevLayout L{};
    hipStream_t stream = nullptr;
    char* dev = nullptr;
    std::vector<int32_t> tile_inst;
    // offsets in the workspace
    // LDS staging: per-tile halos and local columns (built with the layout)
    std::vector<int32_t> halo_ptr, halo_col;
    std::vector<uint16_t> lcol;
    int hmax = 0, sw = 0;
    int64_t halo_total = 0;
    // LDS staging per wavefront (ELL width 7 layouts whose wavefront halos
    // fit kWaveHaloRounds * 64): halos and local columns, wave_ok when built
    std::vector<int32_t> whalo_ptr, whalo_col;
    std::vector<uint16_t> wlcol;
    int whmax = 0;
    bool wave_ok = false;
    struct Off {
        size_t lcol, halo_ptr, halo_col, wlcol, whalo_ptr, whalo_col, fblocks, fpart0, fpart1, srz, col, Mval, basis, minv, mlump, wmask, tile_inst, params, psi, ref, X, Rv, Pa, Pb, Ph, rho, grad,
            mu, S, u, p, partial, rz, rz0, alpha, beta, sums, status, end;
    } off{};
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    bool use_graph = true;
    // schedule of each kernel class: population batch (see run_rows) and
    // LDS staging (1 direct gathers, 2 a stage per tile, 3 a stage per
    // wavefront); 0 = not yet tuned
    int batch[KC_COUNT] = {};
    int stage[KC_COUNT] = {};
    // fused-reduction CG: 0 = not yet chosen, 1 = finalize launches, 2 = fused
    // (fbatch: the fused kernels' population batches); fblocks in dispatch order
    int fused = 0;
    int fbatch[KC_COUNT] = {};
    bool fused_ok = false;
    bool refined = false;  // schedule refined by timing whole solves (refine_schedule)
    int static_dev = -1;   // device whose static workspace the context is bound to (-1: caller's buffer)
    std::vector<int32_t> fblocks;  // 4 ints per block
    int nfb = 0;
    // profiling
    bool profiling = false;
    std::vector<ProfEvent> pending;
    std::vector<hipEvent_t> event_pool;
    int64_t prof_count[KC_COUNT] = {};
    double prof_ms[KC_COUNT] = {};
    std::string err;
};

namespace {

fel_status fail(fel_ctx* c, fel_status s, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

#define HIP_TRY(ctx, call)                                                                    \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(ctx, FEL_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

int elem_size(int precision) { return precision == 0 ? 8 : 4; }

// Element volume and shape-function gradients from the unwrapped vertices:
// 2-D: grad N_1 = (y_2 - y_0, x_0 - x_2) / 2A, grad N_2 = (y_0 - y_1, x_1 - x_0) / 2A;
// 3-D: grad N_1 = (x_2 - x_0) x (x_3 - x_0) / 6V and cyclic; grad N_0 = -sum.
bool element_gradients(int dim, const double X[4][3], double* vol, double g[4][3]) {
    if (dim == 2) {
        const double ax = X[1][0] - X[0][0], ay = X[1][1] - X[0][1];
        const double bx = X[2][0] - X[0][0], by = X[2][1] - X[0][1];
        const double twoA = ax * by - ay * bx;
        if (!(twoA > 0.0) || !std::isfinite(twoA)) return false;
        *vol = 0.5 * twoA;
        g[1][0] = by / twoA;
        g[1][1] = -bx / twoA;
        g[2][0] = -ay / twoA;
        g[2][1] = ax / twoA;
        g[0][0] = -(g[1][0] + g[2][0]);
        g[0][1] = -(g[1][1] + g[2][1]);
        return true;
    }
    double a[3], b[3], c[3];
    for (int r = 0; r < 3; r++) {
        a[r] = X[1][r] - X[0][r];
        b[r] = X[2][r] - X[0][r];
        c[r] = X[3][r] - X[0][r];
    }
    auto cross = [](const double* u, const double* v, double* o) {
        o[0] = u[1] * v[2] - u[2] * v[1];
        o[1] = u[2] * v[0] - u[0] * v[2];
        o[2] = u[0] * v[1] - u[1] * v[0];
    };
    double bc[3], ca[3], ab[3];
    cross(b, c, bc);
    cross(c, a, ca);
    cross(a, b, ab);
    const double sixV = a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2];
    if (!(sixV > 0.0) || !std::isfinite(sixV)) return false;
    *vol = sixV / 6.0;
    for (int r = 0; r < 3; r++) {
        g[1][r] = bc[r] / sixV;
        g[2][r] = ca[r] / sixV;
        g[3][r] = ab[r] / sixV;
        g[0][r] = -(g[1][r] + g[2][r] + g[3][r]);
    }
    return true;
}

int supported_width(int Q, int w) {
    if (Q == 9) {
        if (w <= 7) return 7;
        if (w <= 12) return 12;
    } else {
        if (w <= 15) return 15;
        if (w <= 24) return 24;
    }
    return -1;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

uint64_t spread_bits(uint64_t v, int dim) {
    uint64_t r = 0;
    const int nbits = dim == 2 ? 31 : 21;
    for (int b = 0; b < nbits; b++) r |= ((v >> b) & 1ull) << (b * dim);
    return r;
}

// Device node order: Z-order (Morton) of the nodes quantised to the mesh
// spacing h, so that a wavefront's 64 consecutive rows are a compact patch
// and a 256-row tile is a block (16 x 16 on a 2-D grid, 8 x 8 x 4 in 3-D)
// whose halo is its boundary layer.  h is the median, over the element
// edges that do not wrap around a periodic box, of the significant edge
// components (those at least half the edge's largest one): on a jittered
// grid each is one grid step plus symmetric noise, whatever the edge kind
// (axis, face or body diagonal), so the quantised points fall on the
// lattice and the Morton blocks align with it.
std::vector<int64_t> locality_order(int dim, int64_t n, const double* xyz, int64_t n_elems, const int32_t* conn,
                                    const int8_t* shift) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t k = 0; k < n; k++)
        for (int r = 0; r < dim; r++) {
            lo[r] = std::min(lo[r], xyz[k * dim + r]);
            hi[r] = std::max(hi[r], xyz[k * dim + r]);
        }
    const int nv = dim + 1;
    std::vector<double> ext;
    ext.reserve(n_elems * nv * (nv - 1) / 2);
    for (int64_t e = 0; e < n_elems; e++) {
        bool wraps = false;
        if (shift)
            for (int i = 0; i < nv * dim; i++) wraps |= shift[e * nv * dim + i] != 0;
        if (wraps) continue;
        for (int a = 0; a < nv; a++)
            for (int b = a + 1; b < nv; b++) {
                const int64_t p = conn[e * nv + a], q = conn[e * nv + b];
                double d[3] = {0.0, 0.0, 0.0}, m = 0.0;
                for (int r = 0; r < dim; r++) m = std::max(m, d[r] = std::fabs(xyz[p * dim + r] - xyz[q * dim + r]));
                for (int r = 0; r < dim; r++)
                    if (m > 0.0 && d[r] >= 0.5 * m) ext.push_back(d[r]);
            }
    }
    double h;
    if (!ext.empty()) {
        std::nth_element(ext.begin(), ext.begin() + ext.size() / 2, ext.end());
        h = ext[ext.size() / 2];
    } else {
        double vol = 1.0;
        for (int r = 0; r < dim; r++) vol *= std::max(hi[r] - lo[r], 1e-300);
        h = std::pow(vol / (double)n, 1.0 / dim);
    }
    h = std::max(h, 1e-300);
    const double cap = dim == 2 ? 2147483647.0 : 2097151.0;
    std::vector<uint64_t> key(n);
    for (int64_t k = 0; k < n; k++) {
        uint64_t code = 0;
        for (int r = 0; r < dim; r++) {
            double q = std::floor((xyz[k * dim + r] - lo[r]) / h + 0.5);
            q = std::min(std::max(q, 0.0), cap);
            code |= spread_bits((uint64_t)q, dim) << r;
        }
        key[k] = code;
    }
    std::vector<int64_t> perm(n);
    for (int64_t k = 0; k < n; k++) perm[k] = k;
    std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
    return perm;
}

}  // namespace

// ---------------------------------------------------------------------------

extern "C" {

const char* fel_version(void) { return "felbm 0.1 (gfx950)"; }

const char* fel_last_error(const fel_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

fel_status fel_create(const fel_options* opt, fel_ctx** out) {
    if (!opt || !out) return FEL_EINVAL;
    *out = nullptr;
    if (opt->lattice != 9 && opt->lattice != 19) return FEL_EINVAL;
    if (opt->precision < 0 || opt->precision > 2) return FEL_EINVAL;
    if (opt->mass_mode < 0 || opt->mass_mode > 2) return FEL_EINVAL;
    if (opt->laplacian_mode != 0 && opt->laplacian_mode != 1) return FEL_EINVAL;
    if (opt->max_instances < 1 || opt->max_instances > 65536) return FEL_EINVAL;
    if (opt->cg_iters < 0 || opt->cg_iters > 1000 || opt->cg_tol < 0.0) return FEL_EINVAL;
    if (opt->node_order != FEL_ORDER_CALLER && opt->node_order != FEL_ORDER_ZCURVE) return FEL_EINVAL;
    const int nb = opt->solver_batch;
    if (nb != 0 && nb != 1 && nb != 2 && nb != 4) return FEL_EINVAL;
    if (opt->lds_staging < 0 || opt->lds_staging > 3) return FEL_EINVAL;
    if (opt->fused_reductions < 0 || opt->fused_reductions > 2) return FEL_EINVAL;
    fel_ctx* c = new (std::nothrow) fel_ctx();
    if (!c) return FEL_ENOMEM;
    c->opt = *opt;
    c->lat = make_lattice_info(opt->lattice);
    c->inst.resize(opt->max_instances);
    const bool fp64 = opt->precision == 0;
    const bool d2 = opt->lattice == 9;
    c->cg_iters = opt->cg_iters ? opt->cg_iters : (d2 ? (fp64 ? 30 : 15) : (fp64 ? 34 : 17));
    c->cg_tol = opt->cg_tol > 0.0 ? opt->cg_tol : (fp64 ? 1e-11 : 1e-5);
    c->NP = 2 * (opt->lattice - 1);
    c->NB = c->lat.NB;
    for (int k = 0; k < KC_COUNT; k++) c->batch[k] = 1;
    for (int k = 0; k < KC_COUNT; k++) c->stage[k] = 1;
    for (int k : {KC_CG_INIT, KC_CG_A, KC_CG_B, KC_CHEB}) {
        c->batch[k] = nb;
        c->stage[k] = opt->lds_staging;
    }
    // the streaming kernel's batch is always 1; its staged form is per tile
    c->stage[KC_STREAM] = opt->lds_staging == 3 ? 2 : opt->lds_staging;
    c->fused = opt->fused_reductions;
    *out = c;
    return FEL_OK;
}

}  // extern "C"

static fel_status assemble(fel_ctx* c, int inst, int dim, int64_t n_nodes, const double* xyz, int64_t n_elems,
                           const int32_t* conn, const int8_t* shift, const double* box, const uint8_t* wall,
                           const double* wall_normal, std::vector<int64_t>&& perm) {
    const int nv = dim + 1;
    const int NB = c->NB;
    HostMesh hm;
    hm.dim = dim;
    hm.N = n_nodes;
    // node -> elements
    std::vector<int64_t> cnt(n_nodes + 1, 0);
    for (int64_t e = 0; e < n_elems; e++)
        for (int a = 0; a < nv; a++) {
            const int32_t k = conn[e * nv + a];
            if (k < 0 || k >= n_nodes) return fail(c, FEL_EINVAL, "element %lld vertex index %d out of range",
                                                   (long long)e, k);
            cnt[k + 1]++;
        }
    for (int64_t k = 0; k < n_nodes; k++) cnt[k + 1] += cnt[k];
    std::vector<int64_t> n2e(cnt[n_nodes]);
    {
        std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
        for (int64_t e = 0; e < n_elems; e++)
            for (int a = 0; a < nv; a++) n2e[pos[conn[e * nv + a]]++] = e;
    }
    // pattern: neighbours of each node (diagonal first, then ascending)
    std::vector<std::vector<int32_t>> nbr(n_nodes);
    int W = 0;
    std::vector<int32_t> tmp;
    for (int64_t k = 0; k < n_nodes; k++) {
        tmp.clear();
        for (int64_t i = cnt[k]; i < cnt[k + 1]; i++)
            for (int a = 0; a < nv; a++) {
                const int32_t v = conn[n2e[i] * nv + a];
                if (v != k) tmp.push_back(v);
            }
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        nbr[k].reserve(tmp.size() + 1);
        nbr[k].push_back((int32_t)k);
        nbr[k].insert(nbr[k].end(), tmp.begin(), tmp.end());
        W = std::max<int>(W, (int)nbr[k].size());
    }
    hm.W = W;
    hm.col.assign(n_nodes * W, -1);
    for (int64_t k = 0; k < n_nodes; k++)
        for (size_t s = 0; s < nbr[k].size(); s++) hm.col[k * W + s] = nbr[k][s];
    nbr.clear();
    nbr.shrink_to_fit();
    hm.M.assign(n_nodes * W, 0.0);
    hm.basis.assign((size_t)NB * n_nodes * W, 0.0);
    hm.m.assign(n_nodes, 0.0);
    const double mdiag = 2.0 / (nv * (nv + 1)), moff = 1.0 / (nv * (nv + 1));
    for (int64_t e = 0; e < n_elems; e++) {
        double X[4][3] = {{0}};
        int32_t v[4];
        for (int a = 0; a < nv; a++) {
            v[a] = conn[e * nv + a];
            for (int r = 0; r < dim; r++) {
                const double s = shift ? (double)shift[(e * nv + a) * dim + r] * box[r] : 0.0;
                X[a][r] = xyz[(int64_t)v[a] * dim + r] + s;
            }
        }
        double vol, g[4][3] = {{0}};
        if (!element_gradients(dim, X, &vol, g))
            return fail(c, FEL_EINVAL, "element %lld has non-positive volume", (long long)e);
        for (int a = 0; a < nv; a++) {
            const int64_t rowk = v[a];
            hm.m[rowk] += vol / nv;
            for (int b = 0; b < nv; b++) {
                int slot = -1;
                for (int s = 0; s < W; s++)
                    if (hm.col[rowk * W + s] == v[b]) {
                        slot = s;
                        break;
                    }
                const int64_t i = rowk * W + slot;
                hm.M[i] += vol * (a == b ? mdiag : moff);
                // G_r[a][b] = int N_a d_r N_b = V / (d+1) d_r N_b
                for (int r = 0; r < dim; r++) hm.basis[((size_t)r * n_nodes) * W + i] += vol / nv * g[b][r];
                // K_rr and symmetrised K_rs + K_sr
                int n = dim;
                for (int r = 0; r < dim; r++) hm.basis[((size_t)(n++) * n_nodes) * W + i] += vol * g[a][r] * g[b][r];
                for (int r = 0; r < dim; r++)
                    for (int s = r + 1; s < dim; s++)
                        hm.basis[((size_t)(n++) * n_nodes) * W + i] +=
                            vol * (g[a][r] * g[b][s] + g[a][s] * g[b][r]);
            }
        }
    }
    // bounce-back masks at wall nodes
    hm.wmask.assign(n_nodes, 0u);
    if (wall) {
        for (int64_t k = 0; k < n_nodes; k++) {
            if (!wall[k]) continue;
            uint32_t mask = 0;
            for (int a = 0; a < c->lat.Q; a++) {
                double cn = 0.0;
                for (int r = 0; r < dim; r++) cn += c->lat.e[a][r] * wall_normal[k * dim + r];
                if (cn > 1e-12) mask |= 1u << a;
            }
            hm.wmask[k] = mask;
        }
    }
    hm.present = true;
    hm.perm = std::move(perm);
    c->inst[inst].mesh = std::move(hm);
    return FEL_OK;
}

extern "C" {

fel_status fel_upload_mesh(fel_ctx* c, int inst, int dim, int64_t n_nodes, const double* xyz, int64_t n_elems,
                           const int32_t* conn, const int8_t* shift, const double* box, const uint8_t* wall,
                           const double* wall_normal) {
    if (!c) return FEL_EINVAL;
    if (c->bound) return fail(c, FEL_EINVAL, "upload after bind");
    if (inst < 0 || inst >= (int)c->inst.size()) return fail(c, FEL_EINVAL, "instance %d out of range", inst);
    if (dim != c->lat.D) return fail(c, FEL_EINVAL, "dim %d does not match lattice D%dQ%d", dim, c->lat.D, c->lat.Q);
    if (n_nodes <= 0 || n_elems <= 0 || !xyz || !conn) return fail(c, FEL_EINVAL, "empty mesh");
    if (n_nodes > (int64_t)1 << 30) return fail(c, FEL_EINVAL, "too many nodes");
    if (shift && !box) return fail(c, FEL_EINVAL, "shift given without box");
    if (wall && !wall_normal) return fail(c, FEL_EINVAL, "wall flags given without normals");
    const int nv = dim + 1;
    for (int64_t i = 0; i < n_elems * nv; i++)
        if (conn[i] < 0 || conn[i] >= n_nodes)
            return fail(c, FEL_EINVAL, "element %lld vertex index %d out of range", (long long)(i / nv), conn[i]);
    // renumber into the device order and assemble there
    std::vector<int64_t> perm;
    if (c->opt.node_order == FEL_ORDER_ZCURVE) {
        perm = locality_order(dim, n_nodes, xyz, n_elems, conn, shift);
    } else {
        perm.resize(n_nodes);
        for (int64_t k = 0; k < n_nodes; k++) perm[k] = k;
    }
    std::vector<int32_t> inv(n_nodes);
    for (int64_t k = 0; k < n_nodes; k++) inv[perm[k]] = (int32_t)k;
    std::vector<double> pxyz(n_nodes * dim), pwn(wall ? n_nodes * dim : 0);
    std::vector<uint8_t> pwall(wall ? n_nodes : 0);
    for (int64_t k = 0; k < n_nodes; k++) {
        const int64_t o = perm[k];
        for (int r = 0; r < dim; r++) pxyz[k * dim + r] = xyz[o * dim + r];
        if (wall) {
            pwall[k] = wall[o];
            for (int r = 0; r < dim; r++) pwn[k * dim + r] = wall_normal[o * dim + r];
        }
    }
    std::vector<int32_t> pconn(n_elems * nv);
    for (int64_t i = 0; i < n_elems * nv; i++) pconn[i] = inv[conn[i]];
    return assemble(c, inst, dim, n_nodes, pxyz.data(), n_elems, pconn.data(), shift, box,
                    wall ? pwall.data() : nullptr, wall ? pwn.data() : nullptr, std::move(perm));
}

// Per tile: the columns its rows reference outside the tile (the halo,
// ascending, unique) and every slot column as a tile-local index, so a
// kernel can stage a tile's neighbourhood in LDS with coalesced own-row
// loads plus one load per halo entry.  Padding slots and rows reference
// their own row.
static void build_halos(fel_ctx* c) {
    const int64_t R = c->R;
    const int W = c->W, nt = c->ntiles;
    c->halo_ptr.assign(nt + 1, 0);
    c->halo_col.clear();
    c->lcol.assign((size_t)W * R, 0);
    for (int64_t r = 0; r < R; r++)
        for (int k = 0; k < W; k++) c->lcol[k * R + r] = (uint16_t)(r % TILE);
    c->hmax = 0;
    std::vector<int32_t> cols;
    for (int t = 0; t < nt; t++) {
        c->halo_ptr[t] = (int32_t)c->halo_col.size();
        const Instance& I = c->inst[c->tile_inst[t]];
        const HostMesh& hm = I.mesh;
        const int64_t rb = I.P.row_begin, t0 = (int64_t)t * TILE;
        cols.clear();
        for (int64_t r = t0; r < t0 + TILE; r++) {
            const int64_t k = r - rb;
            if (k >= hm.N) continue;
            for (int sl = 0; sl < hm.W; sl++) {
                const int32_t cl = hm.col[k * hm.W + sl];
                if (cl < 0) continue;
                const int64_t g = rb + cl;
                if (g < t0 || g >= t0 + TILE) cols.push_back((int32_t)g);
            }
        }
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        for (int64_t r = t0; r < t0 + TILE; r++) {
            const int64_t k = r - rb;
            if (k >= hm.N) continue;
            for (int sl = 0; sl < hm.W; sl++) {
                const int32_t cl = hm.col[k * hm.W + sl];
                if (cl < 0) continue;
                const int64_t g = rb + cl;
                int loc;
                if (g >= t0 && g < t0 + TILE)
                    loc = (int)(g - t0);
                else
                    loc = TILE + (int)(std::lower_bound(cols.begin(), cols.end(), (int32_t)g) - cols.begin());
                c->lcol[sl * R + r] = (uint16_t)loc;
            }
        }
        c->hmax = std::max(c->hmax, (int)cols.size());
        c->halo_col.insert(c->halo_col.end(), cols.begin(), cols.end());
    }
    c->halo_ptr[nt] = (int32_t)c->halo_col.size();
    c->halo_total = (int64_t)c->halo_col.size();
    // whole wavefronts of halo entries: a staging wavefront with any entry in
    // a round writes all 64 of its slots
    c->sw = (TILE + c->hmax + 63) / 64 * 64;
}

// The same per 64-row wavefront of a tile (the per-wavefront LDS form):
// its halo holds every column outside its own 64 rows (rows of the other
// wavefronts of the tile included), and its slot columns index its own rows
// by their tile-local position and halo entry h by TILE + w * 3 * 64 + h
// (w = the wavefront within the tile).  Built for ELL width 7; wave_ok
// stays false when a wavefront's halo exceeds kWaveHaloRounds * 64.
static void build_wave_halos(fel_ctx* c) {
    constexpr int WV = TILE / 64, HW = kWaveHaloRounds * 64;
    c->wave_ok = false;
    c->whmax = 0;
    std::vector<int32_t>().swap(c->whalo_ptr);
    std::vector<int32_t>().swap(c->whalo_col);
    std::vector<uint16_t>().swap(c->wlcol);
    bool wanted = c->opt.mass_mode != FEL_MASS_LUMPED;  // (a schedule left to the tuner or forced to 3)
    bool any = false;
    for (int k : {KC_CG_INIT, KC_CG_A, KC_CG_B, KC_CHEB}) any |= c->stage[k] == 0 || c->stage[k] == 3;
    if (c->W != 7 || !wanted || !any) return;
    const int64_t R = c->R;
    const int W = c->W, nw = c->ntiles * WV;
    std::vector<int32_t> ptr(nw + 1, 0), hcol;
    std::vector<uint16_t> wl((size_t)W * R);
    for (int64_t r = 0; r < R; r++)
        for (int k = 0; k < W; k++) wl[k * R + r] = (uint16_t)(r % TILE);
    std::vector<int32_t> cols;
    for (int w = 0; w < nw; w++) {
        ptr[w] = (int32_t)hcol.size();
        const int t = w / WV;
        const Instance& I = c->inst[c->tile_inst[t]];
        const HostMesh& hm = I.mesh;
        const int64_t rb = I.P.row_begin, w0 = (int64_t)w * 64, t0 = (int64_t)t * TILE;
        cols.clear();
        for (int64_t r = w0; r < w0 + 64; r++) {
            const int64_t k = r - rb;
            if (k >= hm.N) continue;
            for (int sl = 0; sl < hm.W; sl++) {
                const int32_t cl = hm.col[k * hm.W + sl];
                if (cl < 0) continue;
                const int64_t g = rb + cl;
                if (g < w0 || g >= w0 + 64) cols.push_back((int32_t)g);
            }
        }
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        c->whmax = std::max(c->whmax, (int)cols.size());
        if ((int)cols.size() > HW) return;  // no per-wavefront form for this layout
        const int slot0 = TILE + (w % WV) * HW;
        for (int64_t r = w0; r < w0 + 64; r++) {
            const int64_t k = r - rb;
            if (k >= hm.N) continue;
            for (int sl = 0; sl < hm.W; sl++) {
                const int32_t cl = hm.col[k * hm.W + sl];
                if (cl < 0) continue;
                const int64_t g = rb + cl;
                int loc;
                if (g >= w0 && g < w0 + 64)
                    loc = (int)(g - t0);
                else
                    loc = slot0 + (int)(std::lower_bound(cols.begin(), cols.end(), (int32_t)g) - cols.begin());
                wl[sl * R + r] = (uint16_t)loc;
            }
        }
        hcol.insert(hcol.end(), cols.begin(), cols.end());
    }
    ptr[nw] = (int32_t)hcol.size();
    c->whalo_ptr.swap(ptr);
    c->whalo_col.swap(hcol);
    c->wlcol.swap(wl);
    c->wave_ok = true;
}

// Blocks of the fused-reduction CG: each instance's tiles in groups of
// kFusedTiles (the last group may be short), listed in dispatch order so
// that, with block b running on XCD b % 8, each XCD receives a contiguous
// range of blocks (as tile_of_block does for the one-tile blocks).  The
// path is available for D2Q9 layouts of ELL width 7 whose instances have at
// most kFusedMaxBlocks blocks.
static void build_fused_blocks(fel_ctx* c) {
    std::vector<int32_t> order;
    c->fused_ok = c->opt.lattice == 9 && c->W == 7;
    for (int i = 0; i < c->ninst; i++) {
        InstParams& P = c->inst[i].P;
        const int nb = (P.tile_count + kFusedTiles - 1) / kFusedTiles;
        P.fb_begin = (int)(order.size() / 4);
        P.fb_count = nb;
        c->fused_ok = c->fused_ok && nb <= kFusedMaxBlocks;
        for (int k = 0; k < nb; k++) {
            order.push_back(P.tile_begin + k * kFusedTiles);
            order.push_back(std::min(kFusedTiles, P.tile_count - k * kFusedTiles));
            order.push_back(i);
            order.push_back(k);
        }
    }
    const int nb = (int)(order.size() / 4);
    c->nfb = nb;
    c->fblocks.assign(order.size(), 0);
    constexpr int NX = 8;
    const int base = nb / NX, extra = nb % NX;
    for (int b = 0; b < nb; b++) {
        const int xcd = b % NX, idx = b / NX;
        const int src = xcd * base + std::min(xcd, extra) + idx;
        for (int q = 0; q < 4; q++) c->fblocks[4 * b + q] = order[4 * src + q];
    }
}

static fel_status plan_layout(fel_ctx* c) {
    int n = 0;
    while (n < (int)c->inst.size() && c->inst[n].mesh.present) n++;
    for (int i = n; i < (int)c->inst.size(); i++)
        if (c->inst[i].mesh.present) return fail(c, FEL_EINVAL, "instances must be uploaded as 0..n-1");
    if (n == 0) return fail(c, FEL_ESTATE, "no mesh uploaded");
    c->ninst = n;
    int wmax = 0;
    for (int i = 0; i < n; i++) wmax = std::max(wmax, c->inst[i].mesh.W);
    c->W = supported_width(c->opt.lattice, wmax);
    if (c->W < 0) return fail(c, FEL_EINVAL, "mesh valence %d above the supported ELL width", wmax);
    if (c->W >= kQRecurrenceWidth) c->stage[KC_CG_B] = 1;  // recurrence form: cg_b has no staged form
    // a fixed direct schedule runs at the largest batch built for it
    for (int k : {KC_CG_INIT, KC_CG_A, KC_CG_B, KC_CHEB})
        if (c->stage[k] == 1) c->batch[k] = std::min(c->batch[k], direct_max_batch(c->W, (int)elem_size(c->opt.precision)));
    int64_t rows = 0;
    c->tile_inst.clear();
    for (int i = 0; i < n; i++) {
        InstParams& P = c->inst[i].P;
        const int64_t N = c->inst[i].mesh.N;
        const int64_t tiles = (N + TILE - 1) / TILE;
        P.row_begin = (int)rows;
        P.row_end = (int)(rows + N);
        P.tile_begin = (int)(rows / TILE);
        P.tile_count = (int)tiles;
        for (int64_t t = 0; t < tiles; t++) c->tile_inst.push_back(i);
        rows += tiles * TILE;
    }
    // gathers address one population's vector with 32-bit byte offsets
    if (rows >= ((int64_t)1 << 31) || rows * elem_size(c->opt.precision) >= ((int64_t)1 << 32))
        return fail(c, FEL_EINVAL, "too many rows (%lld)", (long long)rows);
    c->R = rows;
    c->ntiles = (int)(rows / TILE);
    build_halos(c);
    build_wave_halos(c);
    build_fused_blocks(c);
    const size_t R = (size_t)rows;
    const int W = c->W, NB = c->NB, NP = c->NP, Q = c->opt.lattice, D = c->lat.D;
    const size_t s = elem_size(c->opt.precision);
    const size_t sp = c->opt.precision == 0 ? 8 : (c->opt.precision == 1 ? 4 : 2);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    auto& f = c->off;
    f.lcol = take(2 * W * R);
    f.halo_ptr = take(4 * ((size_t)c->ntiles + 1));
    f.halo_col = take(4 * std::max<size_t>(c->halo_col.size(), 1));
    f.wlcol = take(2 * c->wlcol.size());
    f.whalo_ptr = take(4 * c->whalo_ptr.size());
    f.whalo_col = take(4 * c->whalo_col.size());
    f.col = take(4 * W * R);
    f.Mval = take(s * W * R);
    f.basis = take(s * NB * W * R);
    f.minv = take(s * R);
    f.mlump = take(8 * R);
    f.wmask = take(4 * R);
    f.tile_inst = take(4 * (size_t)c->ntiles);
    f.params = take(sizeof(InstParams) * n);
    f.psi = take(sp * 2 * Q * R);
    f.ref = take(c->opt.precision == 0 ? 0 : 4 * 2 * R);
    f.X = take(s * NP * R);
    f.Rv = take(s * NP * R);
    f.Pa = take(s * NP * R);
    f.Pb = take(s * NP * R);
    // the consistent-mass CG keeps every iteration's search direction
    const size_t K = c->opt.mass_mode == FEL_MASS_CONSISTENT ? (size_t)c->cg_iters : 0;
    f.Ph = take(s * NP * R * K);
    f.rho = take(s * R);
    f.grad = take(s * D * R);
    f.mu = take(s * R);
    f.S = take(s * D * R);
    f.u = take(s * D * R);
    f.p = take(s * R);
    f.partial = take(8 * (size_t)c->ntiles * std::max(NP, 8));
    f.rz = take(8 * (size_t)n * NP);
    f.rz0 = take(8 * (size_t)n * NP);
    f.alpha = take(8 * std::max<size_t>(K, 1) * n * NP);
    f.beta = take(8 * (size_t)n * NP);
    f.sums = take(8 * 8 * (size_t)n);
    f.fblocks = take(16 * (size_t)std::max(c->nfb, 1));
    f.fpart0 = take(8 * (size_t)NP * std::max(c->nfb, 1));
    f.fpart1 = take(8 * (size_t)NP * std::max(c->nfb, 1));
    f.srz = take(8 * 2 * (size_t)n * NP);
    f.status = take(4);
    f.end = o;
    c->ws_bytes = o;
    return FEL_OK;
}

fel_status fel_workspace_size(fel_ctx* c, size_t* bytes) {
    if (!c || !bytes) return FEL_EINVAL;
    if (!c->bound) {
        fel_status st = plan_layout(c);
        if (st != FEL_OK) return st;
    }
    *bytes = c->ws_bytes;
    return FEL_OK;
}

static fel_status upload_operators(fel_ctx* c) {
    const size_t R = c->R;
    const int W = c->W, NB = c->NB;
    const bool fp64 = c->opt.precision == 0;
    const size_t s = elem_size(c->opt.precision);
    std::vector<int32_t> col(W * R);
    std::vector<double> Mv(W * R, 0.0), basis((size_t)NB * W * R, 0.0), minv(R, 1.0), mlump(R, 0.0);
    std::vector<uint32_t> wmask(R, 0u);
    for (size_t r = 0; r < R; r++)
        for (int k = 0; k < W; k++) col[k * R + r] = (int32_t)r;
    for (int i = 0; i < c->ninst; i++) {
        const HostMesh& hm = c->inst[i].mesh;
        const int64_t rb = c->inst[i].P.row_begin;
        for (int64_t k = 0; k < hm.N; k++) {
            const size_t row = rb + k;
            for (int sl = 0; sl < hm.W; sl++) {
                const int32_t cl = hm.col[k * hm.W + sl];
                if (cl < 0) continue;
                col[sl * R + row] = (int32_t)(rb + cl);
                Mv[sl * R + row] = hm.M[k * hm.W + sl];
                for (int n = 0; n < NB; n++)
                    basis[((size_t)n * W + sl) * R + row] = hm.basis[((size_t)n * hm.N + k) * hm.W + sl];
            }
            minv[row] = 1.0 / hm.m[k];
            mlump[row] = hm.m[k];
            wmask[row] = hm.wmask[k];
        }
    }
    auto put = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
        return hipMemcpyAsync(c->dev + off, src, bytes, hipMemcpyHostToDevice, c->stream);
    };
    auto put_t = [&](size_t off, const std::vector<double>& v) -> hipError_t {
        if (fp64) return put(off, v.data(), v.size() * 8);
        std::vector<float> t(v.size());
        for (size_t i = 0; i < v.size(); i++) t[i] = (float)v[i];
        hipError_t e = put(off, t.data(), t.size() * 4);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        return e;
    };
    (void)s;
    HIP_TRY(c, put(c->off.col, col.data(), col.size() * 4));
    HIP_TRY(c, put(c->off.lcol, c->lcol.data(), c->lcol.size() * 2));
    HIP_TRY(c, put(c->off.halo_ptr, c->halo_ptr.data(), c->halo_ptr.size() * 4));
    if (!c->halo_col.empty()) HIP_TRY(c, put(c->off.halo_col, c->halo_col.data(), c->halo_col.size() * 4));
    if (c->wave_ok) {
        HIP_TRY(c, put(c->off.wlcol, c->wlcol.data(), c->wlcol.size() * 2));
        HIP_TRY(c, put(c->off.whalo_ptr, c->whalo_ptr.data(), c->whalo_ptr.size() * 4));
        if (!c->whalo_col.empty()) HIP_TRY(c, put(c->off.whalo_col, c->whalo_col.data(), c->whalo_col.size() * 4));
    }
    HIP_TRY(c, put_t(c->off.Mval, Mv));
    HIP_TRY(c, put_t(c->off.basis, basis));
    HIP_TRY(c, put_t(c->off.minv, minv));
    HIP_TRY(c, put(c->off.mlump, mlump.data(), R * 8));
    HIP_TRY(c, put(c->off.wmask, wmask.data(), R * 4));
    HIP_TRY(c, put(c->off.tile_inst, c->tile_inst.data(), c->tile_inst.size() * 4));
    if (c->nfb) HIP_TRY(c, put(c->off.fblocks, c->fblocks.data(), c->fblocks.size() * 4));
    HIP_TRY(c, hipMemsetAsync(c->dev + c->off.status, 0, 4, c->stream));
    // padding rows of every vector start at zero
    HIP_TRY(c, hipMemsetAsync(c->dev + c->off.psi, 0, c->off.X - c->off.psi, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->dev + c->off.X, 0, c->off.partial - c->off.X, c->stream));
    // reduction scratch too: a reused workspace (the static one) keeps an earlier context's values
    HIP_TRY(c, hipMemsetAsync(c->dev + c->off.partial, 0, c->off.fblocks - c->off.partial, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->dev + c->off.fpart0, 0, c->off.status - c->off.fpart0, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return FEL_OK;
}

static void set_pointers(fel_ctx* c) {
    DevLayout& L = c->L;
    char* d = c->dev;
    const auto& f = c->off;
    L.R = c->R;
    L.W = c->W;
    L.NB = c->NB;
    L.Q = c->opt.lattice;
    L.dim = c->lat.D;
    L.ninst = c->ninst;
    L.ntiles = c->ntiles;
    L.precision = c->opt.precision;
    L.col = reinterpret_cast<const int32_t*>(d + f.col);
    L.lcol = reinterpret_cast<const uint16_t*>(d + f.lcol);
    L.halo_ptr = reinterpret_cast<const int32_t*>(d + f.halo_ptr);
    L.halo_col = reinterpret_cast<const int32_t*>(d + f.halo_col);
    L.sw = c->sw;
    L.wlcol = c->wave_ok ? reinterpret_cast<const uint16_t*>(d + f.wlcol) : nullptr;
    L.whalo_ptr = c->wave_ok ? reinterpret_cast<const int32_t*>(d + f.whalo_ptr) : nullptr;
    L.whalo_col = c->wave_ok ? reinterpret_cast<const int32_t*>(d + f.whalo_col) : nullptr;
    L.Mval = d + f.Mval;
    L.basis = d + f.basis;
    L.minv = d + f.minv;
    L.mlump = reinterpret_cast<const double*>(d + f.mlump);
    L.wmask = reinterpret_cast<const uint32_t*>(d + f.wmask);
    L.tile_inst = reinterpret_cast<const int32_t*>(d + f.tile_inst);
    L.params = reinterpret_cast<const InstParams*>(d + f.params);
    L.psi = d + f.psi;
    L.ref = c->opt.precision == 0 ? nullptr : reinterpret_cast<float*>(d + f.ref);
    L.X = d + f.X;
    L.Rv = d + f.Rv;
    L.Pa = d + f.Pa;
    L.Pb = d + f.Pb;
    L.Ph = d + f.Ph;
    L.K = c->opt.mass_mode == FEL_MASS_CONSISTENT ? c->cg_iters : 0;
    L.rho = d + f.rho;
    L.grad = d + f.grad;
    L.mu = d + f.mu;
    L.S = d + f.S;
    L.u = d + f.u;
    L.p = d + f.p;
    L.partial = reinterpret_cast<double*>(d + f.partial);
    L.rz = reinterpret_cast<double*>(d + f.rz);
    L.rz0 = reinterpret_cast<double*>(d + f.rz0);
    L.alpha = reinterpret_cast<double*>(d + f.alpha);
    L.beta = reinterpret_cast<double*>(d + f.beta);
    L.sums = reinterpret_cast<double*>(d + f.sums);
    L.status = reinterpret_cast<uint32_t*>(d + f.status);
    L.fblocks = reinterpret_cast<const int4*>(d + f.fblocks);
    L.nfb = c->nfb;
    L.fpart0 = reinterpret_cast<double*>(d + f.fpart0);
    L.fpart1 = reinterpret_cast<double*>(d + f.fpart1);
    L.srz = reinterpret_cast<double*>(d + f.srz);
    L.cg_tol2 = c->cg_tol * c->cg_tol;
    L.lap_mode = c->opt.laplacian_mode;
}

}  // extern "C"

namespace {
bool stream_stage_ok(const fel_ctx* c);
}  // namespace

// Binds the context to the device range [dev_ptr, dev_ptr + bytes): lays
// out the workspace, uploads the operators and clears the state.  Shared by
// fel_bind (a caller's buffer) and fel_bind_static (the library's own
// array); `stat` names the static case in the size error.
static fel_status bind_range(fel_ctx* c, void* dev_ptr, size_t bytes, void* hip_stream, bool stat) {
    if (!c || !dev_ptr) return FEL_EINVAL;
    if (c->bound) return fail(c, FEL_ESTATE, "already bound");
    if (((uintptr_t)dev_ptr) & 255) return fail(c, FEL_EINVAL, "workspace must be 256-byte aligned");
    fel_status st = plan_layout(c);
    if (st != FEL_OK) return st;
    // staging asked of every kernel: the streaming kernel stages where it can
    if (!stream_stage_ok(c)) c->stage[KC_STREAM] = 1;
    if (bytes < c->ws_bytes)
        return fail(c, FEL_ENOMEM, stat ? "the meshes need %2$zu workspace bytes, above the %1$zu bytes of the "
                                          "static workspace"
                                        : "workspace of %zu bytes, %zu needed",
                    bytes, c->ws_bytes);
    c->dev = static_cast<char*>(dev_ptr);
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (c->fused == 2 && !c->fused_ok && c->opt.mass_mode == FEL_MASS_CONSISTENT)
        return fail(c, FEL_EINVAL, "fused reductions need a D2Q9 layout of ELL width 7 with at most %d "
                    "blocks of %d tiles per instance", kFusedMaxBlocks, kFusedTiles);
    set_pointers(c);
    st = upload_operators(c);
    if (st != FEL_OK) return st;
    // host copies of the assembled operators are no longer needed
    for (int i = 0; i < c->ninst; i++) {
        HostMesh& hm = c->inst[i].mesh;
        std::vector<int32_t>().swap(hm.col);
        std::vector<double>().swap(hm.M);
        std::vector<double>().swap(hm.basis);
        std::vector<uint32_t>().swap(hm.wmask);
    }
    std::vector<uint16_t>().swap(c->lcol);
    std::vector<int32_t>().swap(c->halo_col);
    std::vector<uint16_t>().swap(c->wlcol);
    std::vector<int32_t>().swap(c->whalo_ptr);
    std::vector<int32_t>().swap(c->whalo_col);
    c->bound = true;
    // graphs cannot be captured on the legacy default stream
    c->use_graph = c->stream != nullptr;
    return FEL_OK;
}

extern "C" fel_status fel_bind(fel_ctx* c, void* dev_ptr, size_t bytes, void* hip_stream) {
    return bind_range(c, dev_ptr, bytes, hip_stream, false);
}

// ---------------------------------------------------------------------------
// the static workspace (fel_bind_static, felbm_static.hip)

namespace {
std::mutex g_static_mu;
fel_ctx* g_static_owner[fel::kMaxDevices] = {};

// true when the context was bound to a device's static workspace that a
// later fel_bind_static has taken over
bool static_stale(fel_ctx* c) {
    if (c->static_dev < 0) return false;
    std::lock_guard<std::mutex> lk(g_static_mu);
    return g_static_owner[c->static_dev] != c;
}
}  // namespace

#define STATIC_CHECK(c)                                                                                    \
    do {                                                                                                   \
        if (static_stale(c))                                                                               \
            return fail(c, FEL_ESTATE, "the static workspace of device %d was bound to another context", \
                        (c)->static_dev);                                                                  \
    } while (0)

fel_status fel::set_error(fel_ctx* c, fel_status st, const char* msg) { return fail(c, st, "%s", msg); }

fel_status fel::bind_static_workspace(fel_ctx* c, void* ptr, size_t bytes, void* hip_stream, int device) {
    if (!c) return FEL_EINVAL;
    if (c->bound) return fail(c, FEL_ESTATE, "already bound");
    // no timing (it creates events and graphs): schedules left open take fixed
    // defaults, and steps launch directly, with no graph of the library's own
    for (int k : {KC_CG_INIT, KC_CG_A, KC_CG_B, KC_CHEB}) {
        if (!c->batch[k]) c->batch[k] = 2;
        if (!c->stage[k]) c->stage[k] = 1;
    }
    if (c->W >= kQRecurrenceWidth) c->stage[KC_CG_B] = 1;
    if (!c->fused) c->fused = 1;
    c->stage[KC_STREAM] = 1;
    c->refined = true;
    fel_status st = bind_range(c, ptr, bytes, hip_stream, true);
    if (st != FEL_OK) return st;
    if (c->fused == 2)
        for (int k : {KC_CG_INIT, KC_CG_A, KC_CG_B})
            c->fbatch[k] = std::min(c->batch[k], fused_max_batch(k, c->opt.precision));
    c->use_graph = false;
    c->static_dev = device;
    std::lock_guard<std::mutex> lk(g_static_mu);
    g_static_owner[device] = c;
    return FEL_OK;
}

// ---------------------------------------------------------------------------
// launches

namespace {

hipEvent_t get_event(fel_ctx* c) {
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

template <typename F>
hipError_t timed(fel_ctx* c, int cls, F&& launch) {
    (void)hipGetLastError();  // launches report hipGetLastError: clear anything left by earlier calls
    if (!c->profiling) return launch();
    ProfEvent pe{cls, get_event(c), get_event(c)};
    if (pe.a && pe.b) g_launch_events = LaunchEvents{pe.a, pe.b};
    hipError_t e = launch();
    g_launch_events = LaunchEvents{};
    c->pending.push_back(pe);
    return e;
}

// Whether a class runs its LDS-staged kernel (the streaming kernel's one
// staged form is per tile; the solver classes pass their stage on).
bool staged(const fel_ctx* c, int cls) { return c->stage[cls] == 2; }
// The streaming kernel's staged form: 2-D layouts of ELL width 7 in
// deviation storage, 2 reference rows and 2 x 2 stage rows of sw floats.
bool stream_stage_ok(const fel_ctx* c) {
    return c->opt.lattice == 9 && c->W == 7 && c->opt.precision != 0 && c->hmax <= kHaloRounds * TILE &&
           6 * (size_t)c->sw * sizeof(float) <= (size_t)kStageBytes;
}
// Whether batch ch fits a solver kernel's staged form (stage 2 per tile, 3
// per wavefront): its dynamic LDS holds 2 ch stage rows (sw values, or
// kWaveStageWidth), a thread stages at most kHaloRounds halo entries (the
// per-wavefront tables exist only where every wavefront halo fits), and the
// CG vectors fit one buffer resource.
bool stage_fits(const fel_ctx* c, int ch, int stage) {
    const size_t row = stage == 3 ? (size_t)kWaveStageWidth : (size_t)c->sw;
    return (stage == 3 ? c->wave_ok : c->hmax <= kHaloRounds * TILE) &&
           staged_vectors_fit(c->NP, c->R, c->opt.precision) &&
           2 * (size_t)ch * row * (size_t)elem_size(c->opt.precision) <= (size_t)kStageBytes;
}

hipError_t enqueue_solve(fel_ctx* c) {
    const DevLayout& L = c->L;
    hipStream_t s = c->stream;
    const int tb = 0, nt = c->ntiles;
    hipError_t e;
    if (c->opt.mass_mode == FEL_MASS_LUMPED) return timed(c, KC_LUMPED, [&] { return launch_lumped(L, tb, nt, s); });
    if (c->opt.mass_mode == FEL_MASS_CHEBYSHEV) {
        // spectrum of m^-1 M in [1/(d+2), 1]; iterate count cg_iters
        const double a = 1.0 / (c->lat.D + 2), b = 1.0;
        const double theta = 0.5 * (b + a), sigma = (b - a) / (b + a), gamma = 1.0 / theta;
        const int K = c->cg_iters, ch = c->batch[KC_CHEB];
        const int st = c->stage[KC_CHEB];
        const int out0 = (K % 2 == 0) ? 0 : 1;  // x_K must land in buffer 0 (X)
        if ((e = timed(c, KC_CHEB, [&] { return launch_cheb_first(L, tb, nt, out0, gamma, ch, st, s); })) != hipSuccess)
            return e;
        double omega = 1.0;
        int cur = 1 - out0;  // buffer holding x_1
        for (int k = 1; k < K; k++) {
            omega = (k == 1) ? 1.0 / (1.0 - 0.5 * sigma * sigma) : 1.0 / (1.0 - 0.25 * sigma * sigma * omega);
            if ((e = timed(c, KC_CHEB, [&] { return launch_cheb(L, tb, nt, cur, omega, gamma, ch, st, s); })) !=
                hipSuccess)
                return e;
            cur = 1 - cur;
        }
        return hipSuccess;
    }
    if (c->fused == 2) {
        if ((e = timed(c, KC_CG_INIT, [&] { return launch_cg_init_fused(L, c->fbatch[KC_CG_INIT], s); })) !=
            hipSuccess)
            return e;
        for (int it = 0; it < c->cg_iters; it++) {
            if ((e = timed(c, KC_CG_A, [&] { return launch_cg_a_fused(L, it, c->fbatch[KC_CG_A], s); })) !=
                hipSuccess)
                return e;
            if ((e = timed(c, KC_CG_B, [&] { return launch_cg_b_fused(L, it, c->fbatch[KC_CG_B], s); })) !=
                hipSuccess)
                return e;
        }
        // cg_x also runs the final residual check on the last cg_b's partials
        return timed(c, KC_CG_X, [&] { return launch_cg_x(L, tb, nt, true, s); });
    }
    const int ni = c->ninst, np = c->NP;
    auto fin = [&](int op, int it = 0) {
        return timed(c, KC_FINALIZE, [&] { return launch_finalize(L, 0, ni, op, np, s, it); });
    };
    if ((e = timed(c, KC_CG_INIT, [&] {
             return launch_cg_init(L, tb, nt, c->batch[KC_CG_INIT], c->stage[KC_CG_INIT], s);
         })) != hipSuccess)
        return e;
    if ((e = fin(0)) != hipSuccess) return e;
    for (int it = 0; it < c->cg_iters; it++) {
        if ((e = timed(c, KC_CG_A, [&] {
                 return launch_cg_a(L, tb, nt, it == 0, it, c->batch[KC_CG_A], c->stage[KC_CG_A], s);
             })) != hipSuccess)
            return e;
        if ((e = fin(1, it)) != hipSuccess) return e;
        if ((e = timed(c, KC_CG_B, [&] {
                 return launch_cg_b(L, tb, nt, it, c->batch[KC_CG_B], c->stage[KC_CG_B], s);
             })) != hipSuccess)
            return e;
        if ((e = fin(it == c->cg_iters - 1 ? 3 : 2)) != hipSuccess) return e;
    }
    return timed(c, KC_CG_X, [&] { return launch_cg_x(L, tb, nt, false, s); });
}

// Times one launch kind with HIP events: kWarm untimed then kReps timed.
template <typename F>
hipError_t time_launches(fel_ctx* c, hipEvent_t a, hipEvent_t b, F&& run, float* ms) {
    constexpr int kWarm = 2, kReps = 8;
    (void)hipGetLastError();
    hipError_t e = hipSuccess;
    for (int r = 0; r < kWarm && e == hipSuccess; r++) e = run();
    if (e == hipSuccess) e = hipEventRecord(a, c->stream);
    for (int r = 0; r < kReps && e == hipSuccess; r++) e = run();
    if (e == hipSuccess) e = hipEventRecord(b, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    return e;
}

// Chooses the schedule of each solver kernel left to the tuner: the
// population batch (1, 2 or 4: how many populations' loads its pipeline
// issues ahead, or stages per LDS pass) and direct gathers vs LDS staging
// per tile (block barriers) vs per wavefront (no barriers, larger halos),
// by timing every allowed candidate on the bound layout; and whether the
// streaming kernel runs direct or staged, where it has a staged form.  The
// launches only touch the solve's scratch (X, Rv, Pa, Pb: the streaming
// kernel's right-hand sides, the stored directions, the alpha history, tile
// partials), which the next step rewrites before reading.
fel_status tune_schedule(fel_ctx* c) {
    const DevLayout& L = c->L;
    hipStream_t s = c->stream;
    const int nt = c->ntiles;
    const int tit = L.K > 1 ? 1 : 0;  // a CG iteration to time (the second, if there is one)
    const double gamma = 2.0 / (1.0 + 1.0 / (c->lat.D + 2));
    hipEvent_t a = get_event(c), b = get_event(c);
    if (!a || !b) return fail(c, FEL_EDEVICE, "event creation failed");
    auto run = [&](int cls, int t, int st) -> hipError_t {
        switch (cls) {
            case KC_CG_INIT: return launch_cg_init(L, 0, nt, t, st, s);
            case KC_CG_A: return launch_cg_a(L, 0, nt, tit == 0, tit, t, st, s);
            case KC_CG_B: return launch_cg_b(L, 0, nt, tit, t, st, s);
            default: return launch_cheb(L, 0, nt, 1, 1.0, gamma, t, st, s);
        }
    };
    // kernels the mass mode never launches keep the direct batch-1 form
    const int mode = c->opt.mass_mode;
    for (int cls : {KC_CG_INIT, KC_CG_A, KC_CG_B, KC_CHEB}) {
        const bool used = cls == KC_CHEB ? mode == FEL_MASS_CHEBYSHEV : mode == FEL_MASS_CONSISTENT;
        if (!used) {
            if (c->batch[cls] == 0) c->batch[cls] = 1;
            if (c->stage[cls] == 0) c->stage[cls] = 1;
        }
    }
    constexpr int kWarm = 2, kReps = 8;
    fel_status st = FEL_OK;
    // the streaming kernel: direct or staged, where the staged form exists
    if (!stream_stage_ok(c)) c->stage[KC_STREAM] = 1;
    if (c->stage[KC_STREAM] == 0) {
        float ms[2] = {0.0f, 0.0f};
        for (int sg : {1, 2}) {
            const hipError_t e =
                time_launches(c, a, b, [&] { return launch_stream(L, 0, nt, sg == 2, s); }, &ms[sg - 1]);
            if (e != hipSuccess) {
                st = fail(c, FEL_EDEVICE, "tuning launch failed: %s", hipGetErrorString(e));
                break;
            }
        }
        c->stage[KC_STREAM] = ms[1] < ms[0] ? 2 : 1;
    }
    for (int cls : {KC_CG_INIT, KC_CG_A, KC_CG_B, KC_CHEB}) {
        if (st != FEL_OK) break;
        if (c->batch[cls] != 0 && c->stage[cls] != 0) continue;
        int best_b = 0, best_s = 0;
        float best_ms = 0.0f;
        for (int sg : {1, 2, 3}) {
            if (c->stage[cls] != 0 && c->stage[cls] != sg) continue;
            for (int t : {1, 2, 4}) {
                if (c->batch[cls] != 0 && c->batch[cls] != t) continue;
                if (sg >= 2 && !stage_fits(c, t, sg)) continue;
                if (sg == 1 && t > direct_max_batch(c->W, (int)elem_size(c->opt.precision))) continue;
                (void)hipGetLastError();
                hipError_t e = hipSuccess;
                for (int r = 0; r < kWarm && e == hipSuccess; r++) e = run(cls, t, sg);
                if (e == hipSuccess) e = hipEventRecord(a, s);
                for (int r = 0; r < kReps && e == hipSuccess; r++) e = run(cls, t, sg);
                if (e == hipSuccess) e = hipEventRecord(b, s);
                if (e == hipSuccess) e = hipEventSynchronize(b);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
                if (e != hipSuccess) {
                    st = fail(c, FEL_EDEVICE, "tuning launch failed: %s", hipGetErrorString(e));
                    break;
                }
                if (best_b == 0 || ms < best_ms) best_b = t, best_s = sg, best_ms = ms;
            }
            if (st != FEL_OK) break;
        }
        if (st != FEL_OK) break;
        if (best_b == 0) {  // a fixed staged batch whose stage does not fit
            if (c->stage[cls] == 3)
                st = fail(c, FEL_EINVAL, "no per-wavefront LDS stage of batch %d (wavefront halo %d, ELL width %d)",
                          c->batch[cls], c->whmax, c->W);
            else
                st = fail(c, FEL_EINVAL, "LDS stage of 2 x %d rows of %d values (halo %d) does not fit",
                          c->batch[cls], c->sw, c->hmax);
            break;
        }
        c->batch[cls] = best_b;
        c->stage[cls] = best_s;
    }
    c->event_pool.push_back(a);
    c->event_pool.push_back(b);
    return st;
}

// Population batches of the fused kernels (1, 2, 4), by
// timing, unless solver_batch fixes them.
fel_status tune_fused_batches(fel_ctx* c) {
    const DevLayout& L = c->L;
    hipStream_t s = c->stream;
    const int tit = L.K > 1 ? 1 : 0;
    const int prec = c->opt.precision;
    if (c->opt.solver_batch) {
        for (int cls : {KC_CG_INIT, KC_CG_A, KC_CG_B})
            c->fbatch[cls] = std::min(c->opt.solver_batch, fused_max_batch(cls, prec));
        return FEL_OK;
    }
    hipEvent_t a = get_event(c), b = get_event(c);
    if (!a || !b) return fail(c, FEL_EDEVICE, "event creation failed");
    fel_status st = FEL_OK;
    for (int cls : {KC_CG_INIT, KC_CG_A, KC_CG_B}) {
        int best = 0;
        float best_ms = 0.0f;
        for (int t : {1, 2, 4}) {
            if (t > fused_max_batch(cls, prec)) continue;
            float ms = 0.0f;
            hipError_t e = time_launches(c, a, b, [&] {
                return cls == KC_CG_INIT ? launch_cg_init_fused(L, t, s)
                       : cls == KC_CG_A  ? launch_cg_a_fused(L, tit, t, s)
                                         : launch_cg_b_fused(L, tit, t, s);
            }, &ms);
            if (e != hipSuccess) {
                st = fail(c, FEL_EDEVICE, "fused tuning launch failed: %s", hipGetErrorString(e));
                break;
            }
            if (best == 0 || ms < best_ms) best = t, best_ms = ms;
        }
        if (st != FEL_OK) break;
        c->fbatch[cls] = best;
    }
    c->event_pool.push_back(a);
    c->event_pool.push_back(b);
    return st;
}

// Chooses between the finalize-launch and the fused-reduction CG when the
// option left it open: graphs of the whole mass solve are built both ways
// and timed, and the faster is kept (without graphs, fused: fewer launches
// is then the whole gain).  Like the other tuning it touches only the
// solve's scratch; the status word, which the final residual check may set
// on that scratch, is restored afterwards.
// Times the whole mass solve as a graph of the current schedule (kWarm
// untimed and kReps timed replays).
hipError_t time_solve(fel_ctx* c, hipEvent_t a, hipEvent_t b, float* ms) {
    hipStream_t s = c->stream;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        e = enqueue_solve(c);
        hipError_t e2 = hipStreamEndCapture(s, &g);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e == hipSuccess) e = time_launches(c, a, b, [&] { return hipGraphLaunch(ge, s); }, ms);
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

fel_status choose_fused(fel_ctx* c) {
    if (!c->use_graph) {
        c->fused = 2;
        return FEL_OK;
    }
    hipStream_t s = c->stream;
    uint32_t saved = 0;
    HIP_TRY(c, hipStreamSynchronize(s));
    HIP_TRY(c, hipMemcpy(&saved, c->dev + c->off.status, 4, hipMemcpyDeviceToHost));
    hipEvent_t a = get_event(c), b = get_event(c);
    if (!a || !b) return fail(c, FEL_EDEVICE, "event creation failed");
    // per-launch profiling events cannot be recorded inside a capture
    const bool profiling = c->profiling;
    c->profiling = false;
    fel_status st = FEL_OK;
    int best = 1;
    float best_ms = 0.0f;
    for (int mode : {1, 2}) {
        c->fused = mode;
        float ms = 0.0f;
        hipError_t e = time_solve(c, a, b, &ms);
        if (e != hipSuccess) {
            st = fail(c, FEL_EDEVICE, "solve timing failed: %s", hipGetErrorString(e));
            break;
        }
        if (mode == 1 || ms < best_ms) best = mode, best_ms = ms;
    }
    c->fused = st == FEL_OK ? best : 1;
    c->profiling = profiling;
    c->event_pool.push_back(a);
    c->event_pool.push_back(b);
    if (st != FEL_OK) return st;
    HIP_TRY(c, hipStreamSynchronize(s));
    HIP_TRY(c, hipMemcpy(c->dev + c->off.status, &saved, 4, hipMemcpyHostToDevice));
    return FEL_OK;
}

// Refines the schedule in context.  The first tuning times each kernel
// alone, repeated on warm caches; here each solver class's allowed
// schedules are timed as the whole mass solve (graph-replayed, the other
// classes as chosen so far), one class at a time, and the fastest is kept.
// Like the other tuning it touches only the solve's scratch, and the status
// word is restored afterwards.
fel_status refine_schedule(fel_ctx* c) {
    if (!c->use_graph || c->opt.mass_mode == FEL_MASS_LUMPED) return FEL_OK;
    const bool fused = c->fused == 2;
    const int sb = c->opt.solver_batch, ls = c->opt.lds_staging;
    if (sb && (fused || ls)) return FEL_OK;  // the options fix every choice
    hipStream_t s = c->stream;
    uint32_t saved = 0;
    HIP_TRY(c, hipStreamSynchronize(s));
    HIP_TRY(c, hipMemcpy(&saved, c->dev + c->off.status, 4, hipMemcpyDeviceToHost));
    hipEvent_t a = get_event(c), b = get_event(c);
    if (!a || !b) return fail(c, FEL_EDEVICE, "event creation failed");
    const bool profiling = c->profiling;  // no per-launch events inside a capture
    c->profiling = false;
    float cur = 0.0f;
    hipError_t e = time_solve(c, a, b, &cur);
    std::vector<int> classes;
    if (c->opt.mass_mode == FEL_MASS_CHEBYSHEV) classes = {KC_CHEB};
    else classes = {KC_CG_B, KC_CG_A, KC_CG_INIT};
    for (int cls : classes) {
        if (e != hipSuccess) break;
        int* bt = fused ? &c->fbatch[cls] : &c->batch[cls];
        int* sg = fused ? nullptr : &c->stage[cls];
        const int keep_b = *bt, keep_s = sg ? *sg : 1;
        int best_b = keep_b, best_s = keep_s;
        float best = cur;
        // the recurrence form's cg_b has no staged form
        const int fixed_st = (cls == KC_CG_B && c->W >= kQRecurrenceWidth) ? 1 : ls;
        for (int st : {1, 2, 3}) {
            if (fused && st >= 2) continue;  // the fused kernels gather directly
            if (!fused && fixed_st && st != fixed_st) continue;
            for (int t : {1, 2, 4}) {
                if (sb && t != sb) continue;
                if (fused && t > fused_max_batch(cls, c->opt.precision)) continue;
                if (!fused && st == 1 && t > direct_max_batch(c->W, (int)elem_size(c->opt.precision))) continue;
                if (st >= 2 && !stage_fits(c, t, st)) continue;
                if (t == keep_b && st == keep_s) continue;
                *bt = t;
                if (sg) *sg = st;
                float ms = 0.0f;
                e = time_solve(c, a, b, &ms);
                if (e != hipSuccess) break;
                if (ms < best) best = ms, best_b = t, best_s = st;
            }
            if (e != hipSuccess) break;
        }
        *bt = best_b;
        if (sg) *sg = best_s;
        cur = best;
    }
    c->profiling = profiling;
    c->event_pool.push_back(a);
    c->event_pool.push_back(b);
    if (e != hipSuccess) return fail(c, FEL_EDEVICE, "solve timing failed: %s", hipGetErrorString(e));
    HIP_TRY(c, hipStreamSynchronize(s));
    HIP_TRY(c, hipMemcpy(c->dev + c->off.status, &saved, 4, hipMemcpyHostToDevice));
    return FEL_OK;
}

hipError_t enqueue_step(fel_ctx* c) {
    const DevLayout& L = c->L;
    hipStream_t s = c->stream;
    const int nt = c->ntiles;
    hipError_t e;
    if ((e = timed(c, KC_STREAM, [&] { return launch_stream(L, 0, nt, staged(c, KC_STREAM), s); })) != hipSuccess)
        return e;
    if ((e = enqueue_solve(c)) != hipSuccess) return e;
    if ((e = timed(c, KC_MOMENTS, [&] { return launch_moments(L, 0, nt, s); })) != hipSuccess) return e;
    if ((e = timed(c, KC_GRAD, [&] { return launch_grad(L, 0, nt, s); })) != hipSuccess) return e;
    if ((e = timed(c, KC_DIV, [&] { return launch_div(L, 0, nt, s); })) != hipSuccess) return e;
    if ((e = timed(c, KC_COLLIDE, [&] { return launch_collide(L, 0, nt, s); })) != hipSuccess) return e;
    return hipSuccess;
}

fel_status drain_profile(fel_ctx* c) {
    if (c->pending.empty()) return FEL_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (auto& pe : c->pending) {
        float ms = 0.0f;
        if (pe.a && pe.b && hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
            c->prof_ms[pe.cls] += ms;
            c->prof_count[pe.cls]++;
        } else {
            (void)hipGetLastError();
        }
        if (pe.a) c->event_pool.push_back(pe.a);
        if (pe.b) c->event_pool.push_back(pe.b);
    }
    c->pending.clear();
    return FEL_OK;
}

bool all_initialised(const fel_ctx* c) {
    for (int i = 0; i < c->ninst; i++)
        if (!c->inst[i].have_phys) return false;
    return true;
}

}  // namespace

extern "C" {

fel_status fel_init_fields(fel_ctx* c, int inst, const fel_phys* ph, const double* rho, const double* u,
                           const double* p) {
    if (!c || !ph || !rho) return FEL_EINVAL;
    if (!c->bound) return fail(c, FEL_ESTATE, "init_fields before bind");
    STATIC_CHECK(c);
    if (inst < 0 || inst >= c->ninst) return fail(c, FEL_EINVAL, "instance %d out of range", inst);
    const double drho = ph->rho_l - ph->rho_v;
    if (!(drho > 0.0) || !(ph->rho_v > 0.0) || !(ph->tau_l > 0.0) || !(ph->tau_v > 0.0) || !(ph->dt > 0.0) ||
        !(ph->xi > 0.0) || !(ph->sigma >= 0.0))
        return fail(c, FEL_EINVAL, "invalid physical parameters");
    Instance& I = c->inst[inst];
    const int64_t N = I.mesh.N;
    const int D = c->lat.D;
    for (int64_t k = 0; k < N; k++)
        if (!std::isfinite(rho[k]) || !(rho[k] > 0.0)) return fail(c, FEL_EINVAL, "rho must be finite and positive");
    I.phys = *ph;
    InstParams& P = I.P;
    P.rho_l = ph->rho_l;
    P.rho_v = ph->rho_v;
    P.tau_l = ph->tau_l;
    P.tau_v = ph->tau_v;
    P.dt = ph->dt;
    for (int r = 0; r < 3; r++) P.grav[r] = r < D ? ph->grav[r] : 0.0;
    P.beta = 12.0 * ph->sigma / (ph->xi * drho * drho * drho * drho);
    P.kappa = 1.5 * ph->xi * ph->sigma / (drho * drho);
    // deviation scale: FP16 deviations are stored times 2^8 (|deviation| up to ~250 fits)
    P.scale = c->opt.precision == 2 ? 1.0 / 256.0 : 1.0;
    HIP_TRY(c, hipMemcpyAsync(c->dev + c->off.params + sizeof(InstParams) * inst, &P, sizeof(InstParams),
                              hipMemcpyHostToDevice, c->stream));
    const bool fp64 = c->opt.precision == 0;
    const size_t R = c->R;
    // upload rho, u, p into the field arrays at the instance rows
    auto put_field = [&](size_t off, int comp, const double* src, int stride) -> hipError_t {
        std::vector<double> v(N);
        const std::vector<int64_t>& perm = I.mesh.perm;
        for (int64_t k = 0; k < N; k++) v[k] = src ? src[perm[k] * stride + comp] : 0.0;
        const size_t at = off + ((size_t)comp * R + P.row_begin) * (fp64 ? 8 : 4);
        if (fp64) {
            hipError_t e = hipMemcpyAsync(c->dev + at, v.data(), N * 8, hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            return e;
        }
        std::vector<float> t(N);
        for (int64_t k = 0; k < N; k++) t[k] = (float)v[k];
        hipError_t e = hipMemcpyAsync(c->dev + at, t.data(), N * 4, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        return e;
    };
    HIP_TRY(c, put_field(c->off.rho, 0, rho, 1));
    for (int r = 0; r < D; r++) HIP_TRY(c, put_field(c->off.u, r, u, D));
    HIP_TRY(c, put_field(c->off.p, 0, p, 1));
    const int tb = P.tile_begin, nt = P.tile_count;
    HIP_TRY(c, launch_grad(c->L, tb, nt, c->stream));
    HIP_TRY(c, launch_div(c->L, tb, nt, c->stream));
    HIP_TRY(c, launch_init(c->L, tb, nt, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    I.have_phys = true;
    return FEL_OK;
}

fel_status fel_step(fel_ctx* c, int n_steps) {
    if (!c || n_steps < 0) return FEL_EINVAL;
    if (!c->bound || !all_initialised(c)) return fail(c, FEL_ESTATE, "step before bind/init_fields");
    STATIC_CHECK(c);
    if (n_steps == 0) return FEL_OK;
    // a staged schedule the options fix completely but the layout cannot run
    for (int cls : {KC_CG_INIT, KC_CG_A, KC_CG_B, KC_CHEB}) {
        const int mode = c->opt.mass_mode;
        const bool used = cls == KC_CHEB ? mode == FEL_MASS_CHEBYSHEV : (mode == FEL_MASS_CONSISTENT && c->fused != 2);
        if (used && c->batch[cls] && c->stage[cls] >= 2 && !stage_fits(c, c->batch[cls], c->stage[cls]))
            return fail(c, FEL_EINVAL, "%s LDS stage (form %d, batch %d) does not fit this layout (halo %d, "
                        "wavefront halo %d, ELL width %d)", kernel_class_name(cls), c->stage[cls], c->batch[cls],
                        c->hmax, c->whmax, c->W);
    }
    bool untuned = false;
    for (int k : {KC_CG_INIT, KC_CG_A, KC_CG_B, KC_CHEB}) untuned |= !c->batch[k] || !c->stage[k];
    untuned |= !c->stage[KC_STREAM];
    if (untuned) {
        fel_status st = tune_schedule(c);
        if (st != FEL_OK) return st;
    }
    if (c->fused != 1 && !c->fbatch[KC_CG_A]) {
        if (!c->fused_ok || c->opt.mass_mode != FEL_MASS_CONSISTENT) {
            c->fused = 1;  // the fused path needs a 2-D layout, small instances and the CG solve
        } else {
            fel_status st = tune_fused_batches(c);
            if (st == FEL_OK && c->fused == 0) st = choose_fused(c);
            if (st != FEL_OK) return st;
        }
    }
    if (!c->refined) {
        fel_status st = refine_schedule(c);
        if (st != FEL_OK) return st;
        c->refined = true;
    }
    if (c->profiling || !c->use_graph) {
        // profiling launches directly: each kernel's events are stamped by its own dispatch
        for (int i = 0; i < n_steps; i++) {
            hipError_t e = enqueue_step(c);
            if (e != hipSuccess) return fail(c, FEL_EDEVICE, "launch failed: %s", hipGetErrorString(e));
            if (c->profiling && c->pending.size() > 4096) {
                fel_status st = drain_profile(c);
                if (st != FEL_OK) return st;
            }
        }
        return c->profiling ? drain_profile(c) : FEL_OK;
    }
    if (!c->graph_exec) {
        HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_step(c);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(c, FEL_EDEVICE, "graph capture failed: %s",
                        hipGetErrorString(e != hipSuccess ? e : e2));
        }
        c->graph = g;
        HIP_TRY(c, hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
    }
    for (int i = 0; i < n_steps; i++) HIP_TRY(c, hipGraphLaunch(c->graph_exec, c->stream));
    return FEL_OK;
}

fel_status fel_sync(fel_ctx* c) {
    if (!c) return FEL_EINVAL;
    if (!c->bound) return fail(c, FEL_ESTATE, "sync before bind");
    STATIC_CHECK(c);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    uint32_t st = 0;
    HIP_TRY(c, hipMemcpy(&st, c->dev + c->off.status, 4, hipMemcpyDeviceToHost));
    if (st) {
        const uint32_t zero = 0;
        HIP_TRY(c, hipMemcpy(c->dev + c->off.status, &zero, 4, hipMemcpyHostToDevice));
    }
    if (st & 1u) return fail(c, FEL_ENONFINITE, "non-finite population or field");
    if (st & 2u) return fail(c, FEL_ENOTCONV, "CG residual above tolerance after %d iterations", c->cg_iters);
    return FEL_OK;
}

}  // extern "C"

namespace {

// copy `count` rows of a device array of element size s (8 or 4) into doubles
// (device rows first..first+count-1 land at caller indices perm[k])
fel_status read_rows(fel_ctx* c, size_t off, int64_t first, int64_t count, double* out, int stride, int comp,
                     const std::vector<int64_t>& perm) {
    const bool fp64 = c->opt.precision == 0;
    const size_t es = fp64 ? 8 : 4;
    if (fp64) {
        std::vector<double> v(count);
        HIP_TRY(c, hipMemcpy(v.data(), c->dev + off + first * es, count * es, hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < count; k++) out[perm[k] * stride + comp] = v[k];
    } else {
        std::vector<float> v(count);
        HIP_TRY(c, hipMemcpy(v.data(), c->dev + off + first * es, count * es, hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < count; k++) out[perm[k] * stride + comp] = v[k];
    }
    return FEL_OK;
}

}  // namespace

extern "C" {

fel_status fel_read_fields(fel_ctx* c, int inst, double* rho, double* u, double* p, double* C) {
    if (!c) return FEL_EINVAL;
    if (!c->bound) return fail(c, FEL_ESTATE, "read before bind");
    STATIC_CHECK(c);
    if (inst < 0 || inst >= c->ninst) return fail(c, FEL_EINVAL, "instance %d out of range", inst);
    const Instance& I = c->inst[inst];
    if (!I.have_phys) return fail(c, FEL_ESTATE, "instance %d not initialised", inst);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int64_t N = I.mesh.N, rb = I.P.row_begin;
    const int D = c->lat.D;
    const size_t R = c->R;
    fel_status st;
    const std::vector<int64_t>& perm = I.mesh.perm;
    std::vector<double> r(N);
    if ((st = read_rows(c, c->off.rho, rb, N, r.data(), 1, 0, perm)) != FEL_OK) return st;
    if (rho) std::copy(r.begin(), r.end(), rho);
    if (C)
        for (int64_t k = 0; k < N; k++) C[k] = (r[k] - I.phys.rho_v) / (I.phys.rho_l - I.phys.rho_v);
    if (u)
        for (int d = 0; d < D; d++)
            if ((st = read_rows(c, c->off.u, (int64_t)d * R + rb, N, u, D, d, perm)) != FEL_OK) return st;
    if (p && (st = read_rows(c, c->off.p, rb, N, p, 1, 0, perm)) != FEL_OK) return st;
    return FEL_OK;
}

fel_status fel_conserved_sums(fel_ctx* c, int inst, double out[6]) {
    if (!c || !out) return FEL_EINVAL;
    if (!c->bound) return fail(c, FEL_ESTATE, "sums before bind");
    STATIC_CHECK(c);
    if (inst < 0 || inst >= c->ninst) return fail(c, FEL_EINVAL, "instance %d out of range", inst);
    const InstParams& P = c->inst[inst].P;
    if (!c->inst[inst].have_phys) return fail(c, FEL_ESTATE, "instance %d not initialised", inst);
    HIP_TRY(c, launch_sums(c->L, P.tile_begin, P.tile_count, c->stream));
    HIP_TRY(c, launch_finalize(c->L, inst, 1, 4, 8, c->stream));
    double v[8];
    HIP_TRY(c, hipMemcpyAsync(v, c->dev + c->off.sums + 64 * inst, 64, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < 6; i++) out[i] = v[i];
    return FEL_OK;
}

fel_status fel_get_state(fel_ctx* c, int inst, double* psibar) {
    if (!c || !psibar) return FEL_EINVAL;
    if (!c->bound) return fail(c, FEL_ESTATE, "get_state before bind");
    STATIC_CHECK(c);
    if (inst < 0 || inst >= c->ninst) return fail(c, FEL_EINVAL, "instance %d out of range", inst);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const Instance& I = c->inst[inst];
    const int64_t N = I.mesh.N, rb = I.P.row_begin;
    const int Q = c->opt.lattice;
    const size_t R = c->R;
    std::vector<double> v(N);
    if (c->opt.precision == 0) {
        for (int a = 0; a < 2 * Q; a++) {
            HIP_TRY(c, hipMemcpy(v.data(), c->dev + c->off.psi + ((size_t)a * R + rb) * 8, N * 8,
                                 hipMemcpyDeviceToHost));
            for (int64_t k = 0; k < N; k++) psibar[a * N + I.mesh.perm[k]] = v[k];
        }
        return FEL_OK;
    }
    // deviations: psi_a = w_a (ref + s d_a)
    std::vector<float> ref(2 * N);
    for (int h = 0; h < 2; h++)
        HIP_TRY(c, hipMemcpy(ref.data() + h * N, c->dev + c->off.ref + ((size_t)h * R + rb) * 4, N * 4,
                             hipMemcpyDeviceToHost));
    const bool half = c->opt.precision == 2;
    std::vector<float> d(N);
    std::vector<__half> dh(half ? N : 0);
    for (int a = 0; a < 2 * Q; a++) {
        if (half) {
            HIP_TRY(c, hipMemcpy(dh.data(), c->dev + c->off.psi + ((size_t)a * R + rb) * 2, N * 2,
                                 hipMemcpyDeviceToHost));
            for (int64_t k = 0; k < N; k++) d[k] = __half2float(dh[k]);
        } else {
            HIP_TRY(c, hipMemcpy(d.data(), c->dev + c->off.psi + ((size_t)a * R + rb) * 4, N * 4,
                                 hipMemcpyDeviceToHost));
        }
        const double w = c->lat.w[a % Q];
        const float* rf = ref.data() + (a < Q ? 0 : N);
        for (int64_t k = 0; k < N; k++)
            psibar[a * N + I.mesh.perm[k]] = w * ((double)rf[k] + I.P.scale * (double)d[k]);
    }
    return FEL_OK;
}

fel_status fel_set_state(fel_ctx* c, int inst, const double* psibar) {
    if (!c || !psibar) return FEL_EINVAL;
    if (!c->bound) return fail(c, FEL_ESTATE, "set_state before bind");
    STATIC_CHECK(c);
    if (inst < 0 || inst >= c->ninst) return fail(c, FEL_EINVAL, "instance %d out of range", inst);
    if (!c->inst[inst].have_phys) return fail(c, FEL_ESTATE, "set_state needs init_fields first");
    const Instance& I = c->inst[inst];
    const int64_t N = I.mesh.N, rb = I.P.row_begin;
    const int Q = c->opt.lattice;
    const size_t R = c->R;
    std::vector<double> v(N);
    if (c->opt.precision == 0) {
        for (int a = 0; a < 2 * Q; a++) {
            for (int64_t k = 0; k < N; k++) v[k] = psibar[a * N + I.mesh.perm[k]];
            HIP_TRY(c, hipMemcpy(c->dev + c->off.psi + ((size_t)a * R + rb) * 8, v.data(), N * 8,
                                 hipMemcpyHostToDevice));
        }
        return FEL_OK;
    }
    // references: density and p / cs^2 (zeroth moments), deviations relative to them
    std::vector<float> ref(2 * N, 0.0f);
    for (int h = 0; h < 2; h++)
        for (int64_t k = 0; k < N; k++) {
            double sum = 0.0;
            for (int a = 0; a < Q; a++) sum += psibar[(h * Q + a) * N + I.mesh.perm[k]];
            ref[h * N + k] = (float)sum;
        }
    for (int h = 0; h < 2; h++)
        HIP_TRY(c, hipMemcpy(c->dev + c->off.ref + ((size_t)h * R + rb) * 4, ref.data() + h * N, N * 4,
                             hipMemcpyHostToDevice));
    const bool half = c->opt.precision == 2;
    std::vector<float> d(N);
    std::vector<__half> dh(half ? N : 0);
    for (int a = 0; a < 2 * Q; a++) {
        const double w = c->lat.w[a % Q];
        const float* rf = ref.data() + (a < Q ? 0 : N);
        for (int64_t k = 0; k < N; k++)
            d[k] = (float)((psibar[a * N + I.mesh.perm[k]] / w - (double)rf[k]) / I.P.scale);
        if (half) {
            for (int64_t k = 0; k < N; k++) dh[k] = __float2half(d[k]);
            HIP_TRY(c, hipMemcpy(c->dev + c->off.psi + ((size_t)a * R + rb) * 2, dh.data(), N * 2,
                                 hipMemcpyHostToDevice));
        } else {
            HIP_TRY(c, hipMemcpy(c->dev + c->off.psi + ((size_t)a * R + rb) * 4, d.data(), N * 4,
                                 hipMemcpyHostToDevice));
        }
    }
    return FEL_OK;
}

fel_status fel_read_aux(fel_ctx* c, int inst, int which, double* out) {
    if (!c || !out) return FEL_EINVAL;
    if (!c->bound) return fail(c, FEL_ESTATE, "read_aux before bind");
    STATIC_CHECK(c);
    if (inst < 0 || inst >= c->ninst) return fail(c, FEL_EINVAL, "instance %d out of range", inst);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const Instance& I = c->inst[inst];
    const int64_t N = I.mesh.N, rb = I.P.row_begin;
    const int D = c->lat.D, Q = c->opt.lattice;
    const size_t R = c->R;
    const std::vector<int64_t>& perm = I.mesh.perm;
    fel_status st = FEL_OK;
    switch (which) {
    case FEL_AUX_GRADRHO:
        for (int d = 0; d < D && st == FEL_OK; d++) st = read_rows(c, c->off.grad, (int64_t)d * R + rb, N, out, D, d, perm);
        return st;
    case FEL_AUX_MU:
        return read_rows(c, c->off.mu, rb, N, out, 1, 0, perm);
    case FEL_AUX_S:
        for (int d = 0; d < D && st == FEL_OK; d++) st = read_rows(c, c->off.S, (int64_t)d * R + rb, N, out, D, d, perm);
        return st;
    case FEL_AUX_DELTA:
        for (int64_t k = 0; k < N; k++) {
            out[k] = 0.0;
            out[Q * N + k] = 0.0;
        }
        for (int j = 0; j < c->NP && st == FEL_OK; j++) {
            const int pop = j < Q - 1 ? j + 1 : Q + (j - (Q - 1)) + 1;
            st = read_rows(c, c->off.X, (int64_t)j * R + rb, N, out + pop * N, 1, 0, perm);
        }
        return st;
    default:
        return fail(c, FEL_EINVAL, "unknown aux field %d", which);
    }
}

fel_status fel_profile(fel_ctx* c, int enable) {
    if (!c) return FEL_EINVAL;
    if (!enable) {
        drain_profile(c);
        for (int k = 0; k < KC_COUNT; k++) {
            c->prof_count[k] = 0;
            c->prof_ms[k] = 0.0;
        }
    }
    c->profiling = enable != 0;
    return FEL_OK;
}

fel_status fel_profile_read(fel_ctx* c, int max_classes, int* n_classes, int64_t* counts, double* total_ms,
                            const char** names) {
    if (!c || !n_classes) return FEL_EINVAL;
    fel_status st = drain_profile(c);
    if (st != FEL_OK) return st;
    *n_classes = KC_COUNT;
    for (int k = 0; k < KC_COUNT && k < max_classes; k++) {
        if (counts) counts[k] = c->prof_count[k];
        if (total_ms) total_ms[k] = c->prof_ms[k];
        if (names) names[k] = kernel_class_name(k);
    }
    return FEL_OK;
}

fel_status fel_layout_info(fel_ctx* c, int64_t* rows, int* ell_width, int* pops, int* cg_iters, int* halo_max,
                           double* halo_mean) {
    if (!c) return FEL_EINVAL;
    if (!c->bound) {
        fel_status st = plan_layout(c);
        if (st != FEL_OK) return st;
    }
    if (rows) *rows = c->R;
    if (ell_width) *ell_width = c->W;
    if (pops) *pops = 2 * c->opt.lattice;
    if (cg_iters) *cg_iters = c->opt.mass_mode == FEL_MASS_LUMPED ? 0 : c->cg_iters;
    if (halo_max) *halo_max = c->hmax;
    if (halo_mean) *halo_mean = c->ntiles ? (double)c->halo_total / c->ntiles : 0.0;
    return FEL_OK;
}

fel_status fel_stage_tables(fel_ctx* c, int form, int64_t* n_lists, int64_t* n_cols, uint16_t* lcol,
                            int32_t* list_ptr, int32_t* list_col) {
    if (!c || !n_lists || !n_cols || (form != 2 && form != 3)) return FEL_EINVAL;
    if (c->bound) return fail(c, FEL_ESTATE, "the staging tables are freed at binding");
    fel_status st = plan_layout(c);
    if (st != FEL_OK) return st;
    if (form == 3 && !c->wave_ok)
        return fail(c, FEL_EINVAL, "no per-wavefront staging (ELL width %d, largest wavefront halo %d)", c->W,
                    c->whmax);
    const auto& lc = form == 3 ? c->wlcol : c->lcol;
    const auto& ptr = form == 3 ? c->whalo_ptr : c->halo_ptr;
    const auto& col = form == 3 ? c->whalo_col : c->halo_col;
    *n_lists = (int64_t)ptr.size() - 1;
    *n_cols = (int64_t)col.size();
    if (lcol) std::copy(lc.begin(), lc.end(), lcol);
    if (list_ptr) std::copy(ptr.begin(), ptr.end(), list_ptr);
    if (list_col) std::copy(col.begin(), col.end(), list_col);
    return FEL_OK;
}

fel_status fel_tuning(fel_ctx* c, int max_classes, int* n_classes, int* batch, int* staging, int* fused) {
    if (!c || !n_classes) return FEL_EINVAL;
    *n_classes = KC_COUNT;
    const bool f = c->fused == 2;
    if (fused) *fused = c->fused;
    for (int k = 0; k < KC_COUNT && k < max_classes; k++) {
        const bool fk = f && (k == KC_CG_INIT || k == KC_CG_A || k == KC_CG_B);
        if (batch) batch[k] = fk ? c->fbatch[k] : c->batch[k];
        if (staging) staging[k] = fk ? 1 : c->stage[k];
    }
    return FEL_OK;
}

fel_status fel_destroy(fel_ctx* c) {
    if (!c) return FEL_OK;
    if (c->bound && c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_owner[c->static_dev] == c) g_static_owner[c->static_dev] = nullptr;
    }
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    for (auto& pe : c->pending) {
        if (pe.a) (void)hipEventDestroy(pe.a);
        if (pe.b) (void)hipEventDestroy(pe.b);
    }
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    delete c;
    return FEL_OK;
}

}  // extern "C"
