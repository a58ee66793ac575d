// C ABI of the as-S_N library: problem set-up, device memory layout, stepping.
#include "../../include/asn.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "asn_host.hpp"
#include "asn_implicit.hpp"
#include "asn_kernels.hpp"

using asn::QInfo;
using asn::StepArgs;

namespace {

thread_local std::string g_last_error;

asn_status fail(asn_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ASN_E_HIP, std::string(#expr ": ") + hipGetErrorString(e_));         \
    } while (0)

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

constexpr int kGmresRestart = 30;

struct Layout {
    int Q = 0, Qp = 0, G = 1, qchunk = 1, tiles_x = 1, tiles_y = 1, fin_blocks = 1;
    int64_t C = 0, P = 0;
    bool lowp = false, fused = false;
    bool flat = false;   // separate-kernel stencil over flat cell chunks (not column strips)
    bool banded = false; // banded step: one kernel per step for a product ordinate set
    int ktab_len = 0;
    size_t off_psi0, off_psi1, off_Y, off_Kt, off_Klp, off_rdef, off_ktab, off_qi, off_coef, off_iso,
        off_band, off_brange, off_bcoef, off_bfrag,
        off_phi64, off_phipart, off_blk, off_fin, off_ypart, off_fix, off_delta, off_bmax0, off_bmax1, off_rec,
        off_tab, off_off, off_base, off_left, off_imp,
        total;
};

// Coefficients the banded form of a set of `levels` polar levels of `azim` azimuths
// can need at most (reach up to kBandMaxReach, runs padded to 4).
static size_t band_coef_capacity(int levels, int azim) {
    const int span = 2 * asn::kBandMaxReach + 1;
    return (size_t)levels * span * (size_t)round_up(azim, 4);
}

// log2 of an accepted operand scale block (0 selects the default), else -1.
int scale_block_log(int32_t n) {
    if (n == 0) n = asn::kScaleBlock;
    if (n < asn::kScaleBlockMin || n > asn::kScaleBlockMax || (n & (n - 1)) != 0) return -1;
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

Layout make_layout(int nx, int ny, int Q, int dtype, int scheme, bool fused, int band_levels = 0,
                   int band_azim = 0) {
    Layout L;
    L.banded = band_levels > 0;
    // the banded reduced-precision step keeps the fused form's pending correction
    if (L.banded) fused = dtype != ASN_GEMM_F32;
    L.fused = fused;
    L.Q = Q;
    L.Qp = (int)round_up(Q, asn::kGemmBM);
    L.C = (int64_t)nx * ny;
    L.P = round_up(L.C, asn::kScaleBlock);
    L.lowp = dtype != ASN_GEMM_F32;
    const int strip = scheme == ASN_SCHEME_HEUN ? asn::kStripXM : asn::kStripX;
    L.tiles_x = (nx + strip - 1) / strip;
    L.tiles_y = (ny + asn::kTileY - 1) / asn::kTileY;
    // Separate stencils up to a width run over flat cell chunks, wider grids over
    // column strips; the ordinates are split into chunks sized to the grid below.
    L.flat = !fused && !L.banded && ((scheme == ASN_SCHEME_EULER && nx <= asn::kFlatMaxNx) ||
                                     (scheme == ASN_SCHEME_HEUN && nx <= asn::kFlatMaxNxM));
    if (L.flat) {
        L.tiles_x = (int)((L.P + asn::kFlatCells - 1) / asn::kFlatCells);
        L.tiles_y = 1;
    }
    int tiles = L.tiles_x * L.tiles_y;
    if (L.banded) {
        // one block per kBandCells (kBandLpCells) cells, every ordinate: each cell's Phi
        // complete
        const int cells = L.lowp ? asn::kBandLpCells : asn::kBandCells;
        L.tiles_x = (int)((L.C + cells - 1) / cells);
        L.tiles_y = 1;
        tiles = L.tiles_x;
        L.qchunk = Q;
        L.G = 1;
    } else if (fused) {
        // the stencil runs in the contraction's epilogue: its blocks are the
        // contraction's 128 x 128 tiles, one Phi partial per ordinate tile
        L.tiles_x = (int)(L.P / asn::kGemmBN);
        L.tiles_y = 1;
        tiles = L.tiles_x;
        L.qchunk = asn::kGemmBM;
        L.G = L.Qp / asn::kGemmBM;
    } else {
        // strip blocks: about four rounds of the 1024 resident; flat-chunk blocks: one
        // round of the 512 resident (a partial last round would cost a whole one, and
        // fewer chunks leave fewer Phi partials to sum)
        int G = L.flat ? asn::kFlatResident / tiles : (int)std::lround(4096.0 / tiles);
        G = std::max(1, std::min(G, std::min(64, std::max(1, Q / 2))));
        L.qchunk = (Q + G - 1) / G;
        L.G = (Q + L.qchunk - 1) / L.qchunk;
    }
    L.fin_blocks = (int)((L.C + 255) / 256);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (size_t)round_up((int64_t)bytes, 256);
        return o;
    };
    const size_t plane = (size_t)L.P;
    L.off_psi0 = take((size_t)Q * plane * 4);
    L.off_psi1 = take((size_t)Q * plane * 4);
    // the fused and banded steps keep Y in registers
    L.off_Y = take(fused || L.banded ? 0 : (size_t)Q * plane * 4);
    L.off_Kt = take((size_t)L.Qp * L.Qp * 4);
    L.off_Klp = take(L.lowp ? (size_t)L.Qp * L.Qp * 2 : 0);
    L.off_rdef = take((size_t)L.Qp * 4);
    {
        const int mt = L.Qp / asn::kGemmBM;
        const int bk = L.lowp ? asn::kBK_LP : asn::kBK_F32;
        L.ktab_len = mt + 1 + 2 * mt * (L.Qp / bk);   // offsets, k-steps, sub-block masks
        L.off_ktab = take((size_t)L.ktab_len * 4);
    }
    // level descriptors, 8 words, and 8 zero words after them (the kernel may read one
    // descriptor word past the last level's)
    L.off_band = take(L.banded ? (size_t)(band_levels + 1) * 32 : 0);
    L.off_brange = take(L.banded ? (size_t)band_levels * 8 : 0);    // coefficient ranges, int2
    L.off_bcoef = take(L.banded && !L.lowp ? band_coef_capacity(band_levels, band_azim) * 4 : 0);
    // reduced-precision banded step: per level and one more, 2 kBandLpMaxReach + 1 pair
    // slots of n_az / 16 A operands of 1 KiB and a (cx, cy) table of n_az float pairs, and
    // 1 KiB after them
    L.off_bfrag = take(L.banded && L.lowp
                           ? (size_t)(band_levels + 1) *
                                     ((2 * asn::kBandLpMaxReach + 1) * (band_azim / 16) * 1024 + band_azim * 8) +
                                 1024
                           : 0);
    L.off_qi = take((size_t)Q * sizeof(QInfo));
    L.off_coef = take(plane * 16);
    L.off_iso = take(plane * 4);
    L.off_phi64 = take(plane * 8);
    L.off_phipart = take((size_t)L.G * plane * 8);
    L.off_blk = take((size_t)tiles * L.G * 2 * 8);
    L.off_fin = take((size_t)L.fin_blocks * 4 * 8);
    L.off_ypart = take(L.lowp ? (size_t)(L.Qp / asn::kGemmBM) * plane * 8 : 0);
    L.off_fix = take(L.lowp && !fused ? plane * 4 : 0);
    L.off_delta = take(L.lowp && fused ? plane * 4 : 0);
    // block maxima for the smallest scale block (any block size a problem takes fits)
    L.off_bmax0 = take((size_t)asn::scale_blocks(L.P, scale_block_log(asn::kScaleBlockMin)) * 4);
    L.off_bmax1 = take((size_t)asn::scale_blocks(L.P, scale_block_log(asn::kScaleBlockMin)) * 4);
    L.off_rec = take(asn::REC_LEN * 8);
    // the problem as a batch of one: step arguments for both buffers, block offsets,
    // buffer base and step counter
    L.off_tab = take(2 * sizeof(StepArgs));
    L.off_off = take(asn::KT_COUNT * 2 * sizeof(int));
    L.off_base = take(sizeof(int));
    L.off_left = take(sizeof(int));
    // FP64 state and iteration vectors of the implicit scheme
    size_t imp = 0;
    if (scheme == ASN_SCHEME_IMPLICIT) {
        asn::ImplicitParams ip{};
        ip.nx = nx;
        ip.ny = ny;
        ip.Q = Q;
        ip.C = L.C;
        ip.P = L.P;
        ip.gmres_restart = kGmresRestart;
        imp = asn::ImplicitSolver::bytes(ip);
    }
    L.off_imp = take(imp);
    L.total = off;
    return L;
}

}  // namespace

struct asn_problem_s {
    int nx = 0, ny = 0;
    Layout L;
    double dx = 0, dy = 0, dt = 0, W = 0, eps = 0, stability = 0;
    int64_t n_to_tfinal = 0, steps_done = 0;
    int dtype = 0, norm = 0, scheme = 0;
    int sb_log = 8;   // log2 of the cells per operand scale block
    hipStream_t stream = nullptr;
    int device = 0;
    bool owns = false;
    char* base = nullptr;
    int cur = 0;  // which psi buffer holds the current state
    std::vector<double> w;
    double tile_entries = 0;  // K entries inside the multiplied tiles (real rows/cols)
    double nonzero_entries = 0;   // nonzero entries of K in the stored operand type
    StepArgs tab[2];          // step arguments when psi buffer 0 / 1 holds the state
    int blocks[asn::KT_COUNT];
    std::unique_ptr<asn::ImplicitSolver> imp;   // the implicit scheme's solver (else null)
    int band_levels = 0, band_azim = 0, band_reach = 0, band_cmax = 0;   // banded step (else 0)
    size_t band_lds() const {
        return dtype == ASN_GEMM_F32 ? asn::band_lds_bytes(band_azim, band_reach, band_cmax)
                                     : asn::band_lp_lds_bytes(band_azim, band_reach, dtype);
    }
    bool band_wide_rows() const { return nx >= asn::kBandWideRowCells; }
};

struct asn_batch_s {
    std::vector<asn_problem> probs;
    int n = 0, dtype = 0, scheme = 0;
    int launch_scheme = 0;   // scheme, or its flat-chunk stencil form
    int band_az = 0;         // banded batches: the azimuth count and LDS bytes per block
    size_t band_lds = 0;
    int band_reach = 0;      // the largest reach of a banded reduced-precision batch
    bool band_wide = false;  // every problem's rows are wide (asn::kBandWideRowCells)
    hipStream_t stream = nullptr;
    std::vector<StepArgs> tab;
    std::vector<int> off;
    char* dev = nullptr;
    asn::BatchArgs args{};
    int grid[asn::KT_COUNT] = {0, 0, 0, 0, 0};
    std::map<int64_t, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
};

namespace {

StepArgs make_args(asn_problem p, int cur) {
    const Layout& L = p->L;
    char* b = p->base;
    StepArgs a{};
    a.nx = p->nx;
    a.ny = p->ny;
    a.Q = L.Q;
    a.Qp = L.Qp;
    a.C = L.C;
    a.P = L.P;
    a.G = L.G;
    a.qchunk = L.qchunk;
    a.tiles_x = L.tiles_x;
    a.tiles_y = L.tiles_y;
    a.fin_blocks = L.fin_blocks;
    a.dtype = p->dtype;
    a.sb_log = p->sb_log;
    a.fused = L.fused ? 1 : 0;
    a.W = p->W;
    a.area = p->dx * p->dy;
    float* psi0 = reinterpret_cast<float*>(b + L.off_psi0);
    float* psi1 = reinterpret_cast<float*>(b + L.off_psi1);
    a.psi = cur == 0 ? psi0 : psi1;
    a.psi_new = cur == 0 ? psi1 : psi0;
    a.Y = reinterpret_cast<float*>(b + L.off_Y);
    a.Kt = reinterpret_cast<const float*>(b + L.off_Kt);
    a.Klp = reinterpret_cast<const uint16_t*>(b + L.off_Klp);
    a.rdef = reinterpret_cast<const float*>(b + L.off_rdef);
    a.ktab = reinterpret_cast<const int*>(b + L.off_ktab);
    a.qi = reinterpret_cast<const QInfo*>(b + L.off_qi);
    a.coef = reinterpret_cast<const float4*>(b + L.off_coef);
    a.iso = reinterpret_cast<float*>(b + L.off_iso);
    a.phi64 = reinterpret_cast<double*>(b + L.off_phi64);
    a.phi_part = reinterpret_cast<double*>(b + L.off_phipart);
    a.blk_part = reinterpret_cast<double*>(b + L.off_blk);
    a.fin_part = reinterpret_cast<double*>(b + L.off_fin);
    a.ypart = reinterpret_cast<double*>(b + L.off_ypart);
    a.fix = reinterpret_cast<float*>(b + L.off_fix);
    a.delta = reinterpret_cast<float*>(b + L.off_delta);
    unsigned* bm0 = reinterpret_cast<unsigned*>(b + L.off_bmax0);
    unsigned* bm1 = reinterpret_cast<unsigned*>(b + L.off_bmax1);
    a.bmax_cur = cur == 0 ? bm0 : bm1;
    a.bmax_next = cur == 0 ? bm1 : bm0;
    a.rec = reinterpret_cast<double*>(b + L.off_rec);
    if (L.banded) {
        a.band = reinterpret_cast<const uint4*>(b + L.off_band);   // two per level
        a.brange = reinterpret_cast<const int2*>(b + L.off_brange);
        a.bcoef = reinterpret_cast<const float*>(b + L.off_bcoef);
        a.bfrag = reinterpret_cast<const uint4*>(b + L.off_bfrag);
        a.n_lev = p->band_levels;
        a.n_az = p->band_azim;
        a.reach = p->band_reach;
        a.bcmax = p->band_cmax;
    }
    return a;
}

// The problem as a batch of one (tables in its workspace).
asn::BatchArgs single_batch(asn_problem p) {
    const Layout& L = p->L;
    asn::BatchArgs b{};
    b.tab = reinterpret_cast<const StepArgs*>(p->base + L.off_tab);
    b.off = reinterpret_cast<const int*>(p->base + L.off_off);
    b.base = reinterpret_cast<const int*>(p->base + L.off_base);
    b.steps_left = reinterpret_cast<int*>(p->base + L.off_left);
    b.n = 1;
    b.s_par = 0;
    return b;
}

hipError_t arm_single(asn_problem p, int64_t limit) {
    asn::ArmArgs v{};
    v.limit[0] = (int)std::min<int64_t>(limit, 1 << 30);
    v.cur[0] = p->cur;
    const Layout& L = p->L;
    return asn::launch_arm(reinterpret_cast<int*>(p->base + L.off_left),
                           reinterpret_cast<int*>(p->base + L.off_base), 1, v, p->stream);
}

// K of a quadrature/width/normalisation, cached across problems (set-up is O(Q^2)
// with a scaling loop; serving creates many problems with the same ordinates).
bool cached_kernel(int Q, const std::vector<double>& om, const std::vector<double>& w, double eps,
                   int mode, std::vector<double>& K, std::string& err) {
    static std::mutex mu;
    static std::vector<std::pair<std::vector<double>, std::vector<double>>> cache;  // key, K
    std::vector<double> key(om);
    key.insert(key.end(), w.begin(), w.end());
    key.push_back(eps);
    key.push_back((double)mode);
    {
        std::lock_guard<std::mutex> g(mu);
        for (auto& e : cache)
            if (e.first == key) {
                K = e.second;
                return true;
            }
    }
    if (!asn::kernel_matrix(Q, om.data(), w.data(), eps, mode, K, err)) return false;
    std::lock_guard<std::mutex> g(mu);
    if (cache.size() >= 8) cache.erase(cache.begin());
    cache.emplace_back(std::move(key), K);
    return true;
}

asn_status check_grid(const asn_grid* g) {
    if (!g) return fail(ASN_E_INVALID, "grid is NULL");
    if (g->nx < 1 || g->ny < 1) return fail(ASN_E_INVALID, "nx and ny must be >= 1");
    if (!(g->x_max > g->x_min) || !(g->y_max > g->y_min) || !std::isfinite(g->x_max - g->x_min) ||
        !std::isfinite(g->y_max - g->y_min))
        return fail(ASN_E_INVALID, "empty or non-finite domain");
    // plane byte offsets are 32-bit in the stencil's buffer addressing
    if ((int64_t)g->nx * g->ny > (int64_t)1 << 29) return fail(ASN_E_INVALID, "grid too large");
    return ASN_OK;
}

asn_status resolve_quadrature(const asn_quadrature* q, std::vector<double>& om,
                              std::vector<double>& w) {
    if (!q) return fail(ASN_E_INVALID, "quadrature is NULL");
    if (q->q_custom > 0) {
        if (!q->omega_xyz || !q->weights)
            return fail(ASN_E_INVALID, "custom quadrature needs omega_xyz and weights");
        const int Q = q->q_custom;
        om.assign(q->omega_xyz, q->omega_xyz + 3 * (size_t)Q);
        w.assign(q->weights, q->weights + Q);
        for (int i = 0; i < Q; ++i) {
            const double n = std::sqrt(om[3 * i] * om[3 * i] + om[3 * i + 1] * om[3 * i + 1] +
                                       om[3 * i + 2] * om[3 * i + 2]);
            if (!(std::fabs(n - 1.0) <= 1e-12)) return fail(ASN_E_INVALID, "ordinate not unit length");
            if (!(w[i] > 0.0) || !std::isfinite(w[i])) return fail(ASN_E_INVALID, "weight must be > 0");
        }
        return ASN_OK;
    }
    if (q->icosahedron_order > 0) {
        if (q->icosahedron_order < 2 || q->icosahedron_order > 41)
            return fail(ASN_E_INVALID, "icosahedron_order must be in [2, 41]");
        asn::icosahedron_quadrature(q->icosahedron_order, om, w);
        return ASN_OK;
    }
    if (q->n_polar < 1 || q->n_azim < 1) return fail(ASN_E_INVALID, "n_polar and n_azim must be >= 1");
    if ((int64_t)q->n_polar * q->n_azim > 16384) return fail(ASN_E_INVALID, "too many ordinates");
    asn::product_quadrature(q->n_polar, q->n_azim, om, w);
    return ASN_OK;
}

// T(fp32(K)) as 16-bit patterns in a ld x ld zero-padded row-major array, and the
// row defects r_q = fp32(1 - sum_p T(K)_qp) with the sum taken in FP64.
void quantise_kernel(int Q, const double* K, int dtype, int ld, uint16_t* out, float* rdef) {
    for (int q = 0; q < Q; ++q) {
        double sum = 0.0;
        for (int k = 0; k < Q; ++k) {
            const float f = (float)K[(size_t)q * Q + k];
            uint16_t h;
            double back;
            if (dtype == ASN_GEMM_BF16) {
                h = asn::float_to_bf16_rne(f);
                back = asn::bf16_to_float(h);
            } else {
                h = asn::float_to_half_rne(f);
                back = asn::half_to_float(h);
            }
            out[(size_t)q * ld + k] = h;
            sum += back;
        }
        rdef[q] = (float)(1.0 - sum);
    }
}

int quad_size(const asn_quadrature* q) {
    if (q->q_custom > 0) return q->q_custom;
    if (q->icosahedron_order > 0) return 10 * (q->icosahedron_order - 1) * (q->icosahedron_order - 1) + 2;
    return q->n_polar * q->n_azim;
}

asn_status check_field(const float* f, int64_t n, const char* name, bool allow_null) {
    if (!f) return allow_null ? ASN_OK : fail(ASN_E_INVALID, std::string(name) + " is NULL");
    for (int64_t i = 0; i < n; ++i)
        if (!(f[i] >= 0.f) || !std::isfinite(f[i]))
            return fail(ASN_E_INVALID, std::string(name) + " must be finite and >= 0");
    return ASN_OK;
}

// Whether forward-Euler steps run fused (stencil in the contraction's epilogue).
// ASN_FORM_AUTO: 16-bit operands always fuse; FP32 fuses problems below 2^25
// cell-ordinates and runs the separate contraction (four blocks per CU) and flat
// stencil above, where they are faster (400^2 x 512: 0.48 vs 0.50 ms per step;
// 700^2 x 1152: 2.98 vs 3.32 ms; 1024^2 x 2048: 11.9 vs 15.8 ms; 128^2 x 512: 0.093 vs
// 0.078 ms).  Wider grids than the flat stencil takes fuse.
bool use_fused(int dtype, int scheme, int form, int nx, int ny, int Q) {
    if (!asn::can_fuse(dtype, scheme) || form == ASN_FORM_SEPARATE) return false;
    if (form == ASN_FORM_BANDED) return false;
    if (form == ASN_FORM_FUSED || dtype != ASN_GEMM_F32) return true;
    return !(nx <= asn::kFlatMaxNx && (double)nx * ny * Q >= 33554432.0);
}

// Whether a problem may take the banded step: forward Euler on a product set whose
// azimuth count has a kernel instance (FP32: 8 .. 64 in steps of 8; BF16 / FP16: 32 or
// 64) (ASN_FORM_AUTO or ASN_FORM_BANDED); the stored K must then also have the banded
// form (band_form).
bool band_candidate(int dtype, int scheme, int form, const asn_quadrature* q, int64_t C) {
    // the kernel addresses one polar level of planes (n_azim * P floats) with byte
    // offsets below 2^31
    const int64_t P = round_up(C, asn::kScaleBlock);
    const bool az_ok = dtype == ASN_GEMM_F32 ? asn::band_azimuths_supported(q->n_azim)
                                             : asn::band_lp_azimuths_supported(q->n_azim);
    return az_ok && scheme == ASN_SCHEME_EULER &&
           (int64_t)std::max(q->n_azim, 1) * P * 4 < ((int64_t)1 << 31) &&
           (form == ASN_FORM_AUTO || form == ASN_FORM_BANDED) && q->q_custom == 0 &&
           q->icosahedron_order == 0 && q->n_polar >= 1;
}

}  // namespace

extern "C" {

asn_status asn_options_default(asn_options* opt) {
    if (!opt) return fail(ASN_E_INVALID, "options is NULL");
    std::memset(opt, 0, sizeof(*opt));
    opt->gemm_dtype = ASN_GEMM_F32;
    opt->normalization = ASN_NORM_SYM;
    opt->cfl = 0.95;
    opt->scale_block = asn::kScaleBlock;
    return ASN_OK;
}

asn_status asn_workspace_size(const asn_grid* grid, const asn_quadrature* quad,
                              const asn_options* opt, size_t* bytes) {
    asn_status s = check_grid(grid);
    if (s != ASN_OK) return s;
    if (!quad || !bytes) return fail(ASN_E_INVALID, "NULL argument");
    const int Q = quad_size(quad);
    if (Q < 1) return fail(ASN_E_INVALID, "Q must be >= 1");
    asn_options d;
    asn_options_default(&d);
    const int dtype = opt ? opt->gemm_dtype : d.gemm_dtype;
    const int scheme = opt ? opt->scheme : d.scheme;
    const int form = opt ? opt->step_form : d.step_form;
    if (scale_block_log(opt ? opt->scale_block : d.scale_block) < 0)
        return fail(ASN_E_INVALID, "scale_block must be a power of two from 64 to 4096 (or 0)");
    if (form < ASN_FORM_AUTO || form > ASN_FORM_BANDED)
        return fail(ASN_E_INVALID, "step_form must be ASN_FORM_AUTO, _SEPARATE, _FUSED or _BANDED");
    if (form == ASN_FORM_BANDED) {
        if (!band_candidate(dtype, scheme, form, quad, (int64_t)grid->nx * grid->ny))
            return fail(ASN_E_UNSUPPORTED, "ASN_FORM_BANDED needs forward Euler on a product set "
                                           "with n_azim in {8, 16, ..., 64} (FP32) or {32, 48, 64} "
                                           "(BF16, FP16)");
        *bytes = make_layout(grid->nx, grid->ny, Q, dtype, scheme, false, quad->n_polar,
                             quad->n_azim).total;
        return ASN_OK;
    }
    const bool fused = use_fused(dtype, scheme, form, grid->nx, grid->ny, Q);
    size_t total = make_layout(grid->nx, grid->ny, Q, dtype, scheme, fused).total;
    // whether K has the banded form is known only once K is built: cover both layouts
    if (band_candidate(dtype, scheme, form, quad, (int64_t)grid->nx * grid->ny))
        total = std::max(total, make_layout(grid->nx, grid->ny, Q, dtype, scheme, false, quad->n_polar,
                                            quad->n_azim).total);
    *bytes = total;
    return ASN_OK;
}

asn_status asn_create(const asn_grid* grid, const asn_quadrature* quad, const float* sigma_s,
                      const float* sigma_a, const float* sigma_as, const float* source,
                      double kernel_beta, double t_final, const asn_options* opt_in,
                      void* hip_stream, void* workspace, size_t workspace_bytes,
                      asn_problem* out) {
    if (!out) return fail(ASN_E_INVALID, "out is NULL");
    *out = nullptr;
    asn_status s = check_grid(grid);
    if (s != ASN_OK) return s;
    asn_options opt;
    if (opt_in) opt = *opt_in;
    else asn_options_default(&opt);
    if (opt.gemm_dtype < ASN_GEMM_F32 || opt.gemm_dtype > ASN_GEMM_F16)
        return fail(ASN_E_INVALID, "unknown gemm_dtype");
    if (opt.normalization != ASN_NORM_SYM && opt.normalization != ASN_NORM_ROW)
        return fail(ASN_E_INVALID, "unknown normalization");
    const int sb_log = scale_block_log(opt.scale_block);
    if (sb_log < 0)
        return fail(ASN_E_INVALID, "scale_block must be a power of two from 64 to 4096 (or 0)");
    if (opt.scheme != ASN_SCHEME_EULER && opt.scheme != ASN_SCHEME_HEUN &&
        opt.scheme != ASN_SCHEME_IMPLICIT)
        return fail(ASN_E_INVALID, "unknown scheme");
    const bool implicit = opt.scheme == ASN_SCHEME_IMPLICIT;
    if (opt.step_form < ASN_FORM_AUTO || opt.step_form > ASN_FORM_BANDED)
        return fail(ASN_E_INVALID, "step_form must be ASN_FORM_AUTO, _SEPARATE, _FUSED or _BANDED");
    if (opt.source_test != ASN_SOURCE_TEST_ABSOLUTE && opt.source_test != ASN_SOURCE_TEST_RELATIVE)
        return fail(ASN_E_INVALID, "source_test must be ASN_SOURCE_TEST_ABSOLUTE or ASN_SOURCE_TEST_RELATIVE");
    if (opt.dt_rule != ASN_DT_STREAMING && opt.dt_rule != ASN_DT_STIFF)
        return fail(ASN_E_INVALID, "unknown dt_rule");
    if (!(opt.cfl > 0.0)) return fail(ASN_E_INVALID, "cfl must be > 0");
    if (opt.cfl > 1.0 && !implicit)
        return fail(ASN_E_UNSTABLE, "cfl above 1 is unstable for the explicit step");
    if (!(t_final > 0.0) || !std::isfinite(t_final)) return fail(ASN_E_INVALID, "t_final must be > 0");
    if (!(kernel_beta > 0.0) && !(opt.eps_override > 0.0))
        return fail(ASN_E_INVALID, "kernel_beta must be > 0");

    std::vector<double> om, w;
    s = resolve_quadrature(quad, om, w);
    if (s != ASN_OK) return s;
    const int Q = (int)w.size();
    const int64_t C = (int64_t)grid->nx * grid->ny;
    if ((s = check_field(sigma_s, C, "sigma_s", false)) != ASN_OK) return s;
    if ((s = check_field(sigma_a, C, "sigma_a", false)) != ASN_OK) return s;
    if ((s = check_field(sigma_as, C, "sigma_as", false)) != ASN_OK) return s;
    if ((s = check_field(source, C, "source", true)) != ASN_OK) return s;

    auto* p = new asn_problem_s();
    p->nx = grid->nx;
    p->ny = grid->ny;
    p->dx = (grid->x_max - grid->x_min) / grid->nx;
    p->dy = (grid->y_max - grid->y_min) / grid->ny;
    p->dtype = opt.gemm_dtype;
    p->sb_log = sb_log;
    p->norm = opt.normalization;
    p->scheme = opt.scheme;
    p->stream = reinterpret_cast<hipStream_t>(hip_stream);
    p->w = w;
    double W = 0.0;
    for (double v : w) W += v;
    p->W = W;
    p->eps = opt.eps_override > 0.0 ? opt.eps_override : kernel_beta / Q;

    // kernel matrix
    std::vector<double> K;
    std::string err;
    if (!cached_kernel(Q, om, w, p->eps, p->norm == ASN_NORM_SYM ? 0 : 1, K, err)) {
        delete p;
        return fail(ASN_E_UNSUPPORTED, err);
    }

    // time step
    const double srate = asn::stability_rate(Q, om.data(), K.data(), p->dx, p->dy, C, sigma_a,
                                             sigma_s, sigma_as);
    if (opt.dt_rule == ASN_DT_STIFF)
        asn::stiff_time_step(Q, om.data(), p->dx, p->dy, srate, opt.cfl, t_final, p->dt,
                             p->n_to_tfinal);
    else
        asn::cfl_time_step(Q, om.data(), p->dx, p->dy, opt.cfl, t_final, p->dt, p->n_to_tfinal);
    if (opt.dt_override > 0.0) {
        double rate = 0.0;
        for (int q = 0; q < Q; ++q)
            rate = std::fmax(rate, std::fabs(om[3 * q]) / p->dx + std::fabs(om[3 * q + 1]) / p->dy);
        if (!implicit && opt.dt_override * rate > opt.cfl * (1.0 + 1e-12)) {
            delete p;
            return fail(ASN_E_UNSTABLE, "dt_override exceeds the CFL bound");
        }
        p->dt = opt.dt_override;
        p->n_to_tfinal = (int64_t)std::llround(t_final / p->dt);
    }
    p->stability = p->dt * srate;

    // banded step when K has that form (ASN_FORM_AUTO) or on request (ASN_FORM_BANDED)
    asn::BandForm bf;
    bool banded = false;
    if (band_candidate(p->dtype, p->scheme, opt.step_form, quad, C)) {
        // the values the kernel multiplies: FP32 K, or its BF16 / FP16 rounding
        std::vector<float> K32((size_t)Q * Q);
        if (p->dtype == ASN_GEMM_F32) {
            for (size_t i = 0; i < K32.size(); ++i) K32[i] = (float)K[i];
        } else {
            std::vector<uint16_t> kq((size_t)Q * Q);
            std::vector<float> rd((size_t)Q);
            quantise_kernel(Q, K.data(), p->dtype, Q, kq.data(), rd.data());
            for (size_t i = 0; i < K32.size(); ++i)
                K32[i] = p->dtype == ASN_GEMM_BF16 ? asn::bf16_to_float(kq[i]) : asn::half_to_float(kq[i]);
        }
        banded = asn::band_form(quad->n_polar, quad->n_azim, K32.data(), asn::kBandMaxReach,
                                asn::kBandNarrow, bf);
        if (banded && p->dtype != ASN_GEMM_F32) {
            // the reduced-precision kernel takes one row defect per level (the rows of a
            // level hold the same values, so their FP64 sums agree; checked) and must fit
            // its LDS
            if (asn::band_lp_lds_bytes(bf.azim, bf.reach, p->dtype) > asn::kMaxBlockLds) banded = false;
            std::vector<uint16_t> kq((size_t)Q * Q);
            std::vector<float> rd((size_t)Q);
            quantise_kernel(Q, K.data(), p->dtype, Q, kq.data(), rd.data());
            for (int q = 0; banded && q < Q; ++q)
                if (rd[(size_t)q] != rd[(size_t)(q / quad->n_azim) * quad->n_azim]) banded = false;
        }
    }
    if (opt.step_form == ASN_FORM_BANDED && !banded) {
        delete p;
        return fail(ASN_E_UNSUPPORTED,
                    "ASN_FORM_BANDED needs forward Euler on a product set with n_azim in "
                    "{8, 16, ..., 64} (FP32) or {32, 48, 64} (BF16, FP16), n_azim * cells below 2^29, "
                    "and a stored K that couples polar levels at most 3 apart (BF16 at 48 or "
                    "64 azimuths: 2) and is circulant along the azimuth");
    }
    if (banded) {
        p->band_levels = bf.levels;
        p->band_azim = bf.azim;
        p->band_reach = bf.reach;
        p->band_cmax = bf.cmax;
        p->L = make_layout(p->nx, p->ny, Q, p->dtype, p->scheme, false, bf.levels, bf.azim);
    } else {
        p->L = make_layout(p->nx, p->ny, Q, p->dtype, p->scheme,
                           use_fused(p->dtype, p->scheme, opt.step_form, p->nx, p->ny, Q));
    }
    const Layout& L = p->L;
    if (workspace) {
        if (workspace_bytes < L.total) {
            delete p;
            return fail(ASN_E_OOM, "workspace smaller than asn_workspace_size");
        }
        p->base = static_cast<char*>(workspace);
        p->owns = false;
    } else {
        void* m = nullptr;
        if (hipMalloc(&m, L.total) != hipSuccess) {
            delete p;
            return fail(ASN_E_OOM, "hipMalloc of the problem memory failed");
        }
        p->base = static_cast<char*>(m);
        p->owns = true;
    }
    (void)hipGetDevice(&p->device);

    // host-side tables
    std::vector<float> Kt((size_t)L.Qp * L.Qp, 0.f);
    for (int q = 0; q < Q; ++q)
        for (int k = 0; k < Q; ++k) Kt[(size_t)k * L.Qp + q] = (float)K[(size_t)q * Q + k];
    std::vector<uint16_t> Klp;
    std::vector<float> rdef((size_t)L.Qp, 0.f);
    if (L.lowp) {
        Klp.assign((size_t)L.Qp * L.Qp, 0);
        quantise_kernel(Q, K.data(), p->dtype, L.Qp, Klp.data(), rdef.data());
    }
    // k-steps per M-tile whose tile of the stored K (FP32 or 16-bit) has a nonzero entry.
    // Steps inside the tile's own ordinate range come last: the fused epilogue then
    // reads rows that the block (and its neighbours) has just streamed through L2.
    // After the k-step list, one mask per entry.  FP32: bit 4 s + g is set when rows
    // m0 + 16 s .. m0 + 16 s + 15 and columns k0 + 4 g .. k0 + 4 g + 3 of the step's K tile
    // (one MFMA operand block) have a nonzero entry; the kernel skips the products of the
    // other blocks.  16-bit operands: bit s for the 16-row sub-block (the kernel
    // multiplies whole tiles).
    std::vector<int> ktab((size_t)L.ktab_len, 0);
    {
        const int mt_n = L.Qp / asn::kGemmBM;
        const int bk = L.lowp ? asn::kBK_LP : asn::kBK_F32;
        const int nk = (Q + bk - 1) / bk;
        std::vector<int> entries, masks;
        double cover = 0;
        for (int mt = 0; mt < mt_n; ++mt) {
            ktab[mt] = (int)entries.size();
            const int m0 = mt * asn::kGemmBM, m1 = std::min(Q, m0 + asn::kGemmBM);
            std::vector<int> own, own_mask;
            for (int kt = 0; kt < nk; ++kt) {
                const int k0 = kt * bk, k1 = std::min(Q, k0 + bk);
                uint32_t mask = 0;
                for (int m = m0; m < m1; ++m)
                    for (int k = k0; k < k1; ++k)
                        if (L.lowp ? (Klp[(size_t)m * L.Qp + k] & 0x7FFFu) != 0
                                   : Kt[(size_t)k * L.Qp + m] != 0.f)
                            mask |= L.lowp ? 1u << ((m - m0) / 16) : 1u << (4 * ((m - m0) / 16) + (k - k0) / 4);
                if (mask) {
                    const bool is_own = L.fused && k0 >= m0 && k0 < m0 + asn::kGemmBM;
                    (is_own ? own : entries).push_back(kt);
                    (is_own ? own_mask : masks).push_back((int)mask);
                    // K entries the kernel multiplies: whole tiles (16-bit operands) or
                    // the nonzero 16 x 4 blocks (FP32)
                    if (L.lowp) {
                        cover += (double)(m1 - m0) * (k1 - k0);
                    } else {
                        for (int b = 0; b < 32; ++b) {
                            if (!(mask & (1u << b))) continue;
                            const int r0 = m0 + 16 * (b / 4), c0 = k0 + 4 * (b % 4);
                            cover += (double)std::max(0, std::min(m1, r0 + 16) - r0) *
                                     std::max(0, std::min(k1, c0 + 4) - c0);
                        }
                    }
                }
            }
            entries.insert(entries.end(), own.begin(), own.end());
            masks.insert(masks.end(), own_mask.begin(), own_mask.end());
        }
        ktab[mt_n] = (int)entries.size();
        std::copy(entries.begin(), entries.end(), ktab.begin() + mt_n + 1);
        std::copy(masks.begin(), masks.end(), ktab.begin() + mt_n + 1 + entries.size());
        p->tile_entries = cover;
    }
    {   // the method's own products: nonzeros of the stored K
        double nz = 0;
        for (int q = 0; q < Q; ++q)
            for (int k = 0; k < Q; ++k)
                nz += L.lowp ? ((Klp[(size_t)q * L.Qp + k] & 0x7FFFu) != 0)
                             : (Kt[(size_t)k * L.Qp + q] != 0.f);
        p->nonzero_entries = nz;
    }
    if (banded) {   // the banded step multiplies each pair's run (wide runs padded to 4);
                    // the reduced-precision one each pair's whole n_az x n_az block
        double ex = 0;
        for (int i = 0; i < bf.levels; ++i) {
            const int n = (int)bf.desc[(size_t)i * 8];
            for (int t = 0; t < n; ++t) {
                const uint32_t code = bf.desc[(size_t)i * 8 + 1 + t];
                int lo = 0, len = 0;
                asn::band_run(code, bf.azim, lo, len);
                ex += L.lowp ? (double)bf.azim * bf.azim
                             : (double)bf.azim * ((code & 64u) ? (len + 3) / 4 * 4 : len);
            }
        }
        p->tile_entries = ex;
    }
    std::vector<QInfo> qi(Q);
    for (int q = 0; q < Q; ++q) {
        const double xi = om[3 * q], eta = om[3 * q + 1];
        qi[q].cx = (float)(p->dt * std::fabs(xi) / p->dx);
        qi[q].cy = (float)(p->dt * std::fabs(eta) / p->dy);
        qi[q].wf = (float)w[q];
        qi[q].dir = (xi > 0 ? 1 : 0) | (xi < 0 ? 2 : 0) | (eta > 0 ? 4 : 0) | (eta < 0 ? 8 : 0);
        qi[q].w = w[q];
    }
    std::vector<float4> coef((size_t)L.P, make_float4(0.f, 0.f, 0.f, 0.f));
    for (int64_t c = 0; c < C; ++c) {
        coef[c].x = (float)(p->dt * (double)sigma_a[c]);
        coef[c].y = (float)(p->dt * (double)sigma_s[c]);
        coef[c].z = (float)(p->dt * (double)sigma_as[c]);
        coef[c].w = source ? (float)(p->dt * (double)source[c]) : 0.f;
    }

    // the banded kernel's descriptors: counts as built, pair codes in its decoded form
    std::vector<uint32_t> ddesc;
    std::vector<uint16_t> bfrag;
    if (banded && !L.lowp) {
        ddesc = bf.desc;
        for (int i = 0; i < bf.levels; ++i)
            for (int t = 0; t < (int)bf.desc[(size_t)i * 8]; ++t)
                ddesc[(size_t)i * 8 + 1 + t] =
                    asn::band_device_code(bf.desc[(size_t)i * 8 + 1 + t], i, bf.reach, bf.azim);
    } else if (banded) {
        // per level and one more {pairs, first uint4 of its block, the level offsets k of its
        // pair slots (4 bits each), 0}.  Block l: 2 kBandLpMaxReach + 1 pair slots of
        // n_az / 16 A operands of MFMA 16x16x32 (band_lp_fragments), the coupled pairs of
        // level l first, then zero operands whose partner is the level itself (the kernel
        // runs the first 2 reach + 1 slots of its launch's largest reach, with no count);
        // then (cx, cy) of level l - 1's ordinates as FP32 pairs (its update runs a level
        // behind); block n_lev holds only the last level's table
        constexpr int slots = 2 * asn::kBandLpMaxReach + 1;
        const int per_slot = bf.azim / 16;
        const size_t block = (size_t)slots * per_slot * 512 + (size_t)bf.azim * 4;   // 16-bit words
        ddesc.assign((size_t)(bf.levels + 1) * 8, 0u);
        for (int i = 0; i <= bf.levels; ++i) {
            const int n = i < bf.levels ? (int)bf.desc[(size_t)i * 8] : 0;
            uint32_t kc = 0;
            for (int t = 0; t < slots; ++t)
                kc |= (t < n ? ((bf.desc[(size_t)i * 8 + 1 + t] >> 8) & 7u) : (uint32_t)bf.reach)
                      << (4 * t);
            ddesc[(size_t)i * 8] = (uint32_t)n;
            ddesc[(size_t)i * 8 + 1] = (uint32_t)(i * block / 8);
            ddesc[(size_t)i * 8 + 2] = kc;
            for (int t = 0; t < n; ++t) asn::band_lp_fragments(bf, i, t, p->dtype, bfrag);
            bfrag.resize((size_t)i * block + (size_t)slots * per_slot * 512, 0);
            for (int az = 0; az < bf.azim; ++az) {
                float c[2] = {0.f, 0.f};
                if (i > 0) {
                    c[0] = qi[(size_t)(i - 1) * bf.azim + az].cx;
                    c[1] = qi[(size_t)(i - 1) * bf.azim + az].cy;
                }
                uint16_t w[4];
                std::memcpy(w, c, sizeof(c));
                bfrag.insert(bfrag.end(), w, w + 4);
            }
        }
    }
    auto bail = [&](asn_status st) {
        if (p->owns) (void)hipFree(p->base);
        delete p;
        return st;
    };
    char* b = p->base;
    if (hipMemsetAsync(b, 0, L.total, p->stream) != hipSuccess ||
        hipMemcpyAsync(b + L.off_Kt, Kt.data(), Kt.size() * 4, hipMemcpyHostToDevice, p->stream) !=
            hipSuccess ||
        hipMemcpyAsync(b + L.off_qi, qi.data(), qi.size() * sizeof(QInfo), hipMemcpyHostToDevice,
                       p->stream) != hipSuccess ||
        hipMemcpyAsync(b + L.off_rdef, rdef.data(), rdef.size() * 4, hipMemcpyHostToDevice,
                       p->stream) != hipSuccess ||
        hipMemcpyAsync(b + L.off_ktab, ktab.data(), ktab.size() * 4, hipMemcpyHostToDevice,
                       p->stream) != hipSuccess ||
        (banded && !L.lowp &&
         (hipMemcpyAsync(b + L.off_band, ddesc.data(), ddesc.size() * 4, hipMemcpyHostToDevice,
                         p->stream) != hipSuccess ||
          hipMemcpyAsync(b + L.off_brange, bf.range.data(), bf.range.size() * 4,
                         hipMemcpyHostToDevice, p->stream) != hipSuccess ||
          hipMemcpyAsync(b + L.off_bcoef, bf.coef.data(), bf.coef.size() * 4, hipMemcpyHostToDevice,
                         p->stream) != hipSuccess ||
          asn::prepare_banded(bf.azim, p->band_lds()) != hipSuccess)) ||
        (banded && L.lowp &&
         (hipMemcpyAsync(b + L.off_band, ddesc.data(), ddesc.size() * 4, hipMemcpyHostToDevice,
                         p->stream) != hipSuccess ||
          hipMemcpyAsync(b + L.off_bfrag, bfrag.data(), bfrag.size() * 2, hipMemcpyHostToDevice,
                         p->stream) != hipSuccess ||
          asn::prepare_banded_lp(bf.azim, p->dtype, bf.reach, p->band_lds()) != hipSuccess)) ||
        (L.lowp && hipMemcpyAsync(b + L.off_Klp, Klp.data(), Klp.size() * 2,
                                  hipMemcpyHostToDevice, p->stream) != hipSuccess) ||
        hipMemcpyAsync(b + L.off_coef, coef.data(), coef.size() * 16, hipMemcpyHostToDevice,
                       p->stream) != hipSuccess)
        return bail(fail(ASN_E_HIP, "copying the problem tables to the device failed"));
    p->cur = 0;
    p->steps_done = 0;
    p->tab[0] = make_args(p, 0);
    p->tab[1] = make_args(p, 1);
    asn::blocks_per_kind(p->tab[0], p->blocks);
    int off1[asn::KT_COUNT * 2];
    for (int k = 0; k < asn::KT_COUNT; ++k) {
        off1[2 * k] = 0;
        off1[2 * k + 1] = p->blocks[k];
    }
    if (hipMemcpyAsync(b + L.off_tab, p->tab, sizeof(p->tab), hipMemcpyHostToDevice, p->stream) !=
            hipSuccess ||
        hipMemcpyAsync(b + L.off_off, off1, sizeof(off1), hipMemcpyHostToDevice, p->stream) !=
            hipSuccess)
        return bail(fail(ASN_E_HIP, "copying the step tables to the device failed"));
    if (arm_single(p, 1) != hipSuccess ||
        asn::launch_init(p->tab[0], single_batch(p), p->stream) != hipSuccess)
        return bail(fail(ASN_E_HIP, "initial moment kernels failed to launch"));
    if (implicit) {
        asn::ImplicitParams ip{};
        ip.nx = p->nx;
        ip.ny = p->ny;
        ip.Q = Q;
        ip.C = C;
        ip.P = L.P;
        ip.dx = p->dx;
        ip.dy = p->dy;
        ip.dt = p->dt;
        ip.W = p->W;
        ip.gmres_tol = opt.implicit_tol > 0.0 ? opt.implicit_tol : 1.5e-8;
        ip.source_tol = opt.source_tol > 0.0 ? opt.source_tol : 1e-4;
        ip.source_relative = opt.source_test == ASN_SOURCE_TEST_RELATIVE;
        ip.gmres_restart = kGmresRestart;
        p->imp.reset(new asn::ImplicitSolver());
        std::string ierr;
        if (!p->imp->init(ip, om.data(), w.data(), K.data(), sigma_s, sigma_a, sigma_as, source,
                          b + L.off_imp, p->stream, ierr))
            return bail(fail(ierr.find("nx must") != std::string::npos ? ASN_E_UNSUPPORTED : ASN_E_HIP,
                             ierr));
        if (!p->imp->set_state(reinterpret_cast<const float*>(b + L.off_psi0),
                               reinterpret_cast<double*>(b + L.off_phi64), ierr))
            return bail(fail(ASN_E_HIP, ierr));
    }
    if (hipStreamSynchronize(p->stream) != hipSuccess)
        return bail(fail(ASN_E_HIP, "synchronising after set-up failed"));
    *out = p;
    return ASN_OK;
}

static asn_status finish_set_state(asn_problem p) {
    p->steps_done = 0;
    HIP_TRY(arm_single(p, 1));
    HIP_TRY(asn::launch_init(p->tab[p->cur], single_batch(p), p->stream));
    if (p->imp) {
        const Layout& L = p->L;
        std::string ierr;
        if (!p->imp->set_state(reinterpret_cast<const float*>(p->base + (p->cur == 0 ? L.off_psi0 : L.off_psi1)),
                               reinterpret_cast<double*>(p->base + L.off_phi64), ierr))
            return fail(ASN_E_HIP, ierr);
    }
    return ASN_OK;
}

asn_status asn_set_state(asn_problem p, const float* psi, int32_t on_device) {
    if (!p || !psi) return fail(ASN_E_INVALID, "NULL argument");
    const Layout& L = p->L;
    float* dst = reinterpret_cast<float*>(p->base + (p->cur == 0 ? L.off_psi0 : L.off_psi1));
    HIP_TRY(hipMemcpy2DAsync(dst, L.P * 4, psi, L.C * 4, L.C * 4, L.Q,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                             p->stream));
    if (!on_device) HIP_TRY(hipStreamSynchronize(p->stream));
    return finish_set_state(p);
}

asn_status asn_set_state_isotropic(asn_problem p, const float* cell, int32_t on_device) {
    if (!p || !cell) return fail(ASN_E_INVALID, "NULL argument");
    const Layout& L = p->L;
    float* dst = reinterpret_cast<float*>(p->base + (p->cur == 0 ? L.off_psi0 : L.off_psi1));
    // stage the cell values in the iso buffer (recomputed from the new state below)
    float* stage = reinterpret_cast<float*>(p->base + L.off_iso);
    HIP_TRY(hipMemcpyAsync(stage, cell, L.C * 4,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, p->stream));
    HIP_TRY(asn::launch_broadcast(dst, stage, L.Q, L.C, L.P, p->stream));
    if (!on_device) HIP_TRY(hipStreamSynchronize(p->stream));
    return finish_set_state(p);
}

asn_status asn_get_state(asn_problem p, float* psi, int32_t on_device) {
    if (!p || !psi) return fail(ASN_E_INVALID, "NULL argument");
    const Layout& L = p->L;
    if (p->L.lowp && p->L.fused)   // fold the pending correction into the stored state
        HIP_TRY(asn::launch_materialize(p->tab[p->cur], p->stream));
    if (p->imp) {          // the implicit state is FP64: round it into the FP32 buffer first
        std::string ierr;
        if (!p->imp->get_state(reinterpret_cast<float*>(p->base + (p->cur == 0 ? L.off_psi0 : L.off_psi1)),
                               ierr))
            return fail(ASN_E_HIP, ierr);
    }
    const float* src = reinterpret_cast<const float*>(p->base + (p->cur == 0 ? L.off_psi0 : L.off_psi1));
    HIP_TRY(hipMemcpy2DAsync(psi, L.C * 4, src, L.P * 4, L.C * 4, L.Q,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    return ASN_OK;
}

// The scheme the kernels are launched with: a separate-kernel step whose stencil
// runs over flat cell chunks (Euler or Heun) has a launch form of its own.
static int launch_scheme(asn_problem p) {
    if (p->L.banded) return asn::SCHEME_EULER_BANDED;
    if (!p->L.flat) return p->scheme;
    return p->scheme == ASN_SCHEME_HEUN ? asn::SCHEME_HEUN_FLAT : asn::SCHEME_EULER_FLAT;
}

// An Euler step moves the state to the other buffer; a Heun step brings it back.
static int state_flip(int scheme, int64_t n_steps) {
    return scheme == ASN_SCHEME_HEUN ? 0 : (int)(n_steps & 1);
}

asn_status asn_step(asn_problem p, int64_t n_steps) {
    if (!p) return fail(ASN_E_INVALID, "problem is NULL");
    if (n_steps < 0 || n_steps > (1 << 30)) return fail(ASN_E_INVALID, "n_steps must be in [0, 2^30]");
    if (n_steps == 0) return ASN_OK;
    if (p->imp) {
        std::string ierr;
        if (!p->imp->step(n_steps, reinterpret_cast<double*>(p->base + p->L.off_phi64), ierr))
            return fail(ASN_E_HIP, ierr);
        p->steps_done += n_steps;
        return ASN_OK;
    }
    HIP_TRY(arm_single(p, n_steps));
    asn::BatchArgs b = single_batch(p);
    const size_t lds = p->L.banded ? p->band_lds() : 0;
    for (int64_t i = 0; i < n_steps; ++i) {
        b.s_par = (int)(i & 1);
        HIP_TRY(asn::launch_step(b, p->blocks, p->dtype, launch_scheme(p), p->stream, nullptr,
                                 p->band_azim, lds, p->band_wide_rows(), p->band_reach));
    }
    p->cur ^= state_flip(p->scheme, n_steps);
    p->steps_done += n_steps;
    return ASN_OK;
}

asn_status asn_step_timed(asn_problem p, int64_t n_steps, double kernel_ms[5]) {
    if (!p || !kernel_ms) return fail(ASN_E_INVALID, "NULL argument");
    if (n_steps < 1 || n_steps > (1 << 20)) return fail(ASN_E_INVALID, "n_steps must be in [1, 2^20]");
    if (p->imp) {          // iterative steps: only the span of a whole step is reported
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        HIP_TRY(hipEventRecord(e0, p->stream));
        const asn_status st = asn_step(p, n_steps);
        HIP_TRY(hipEventRecord(e1, p->stream));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != ASN_OK) return st;
        for (int k = 0; k < 4; ++k) kernel_ms[k] = 0.0;
        kernel_ms[4] = ms / (double)n_steps;
        return ASN_OK;
    }
    const int passes = asn::passes_per_step(p->scheme);
    const size_t per = 5 * (size_t)passes;
    std::vector<hipEvent_t> ev((size_t)n_steps * per, nullptr);
    asn_status st = ASN_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            st = fail(ASN_E_HIP, "hipEventCreate failed");
            break;
        }
    if (st == ASN_OK && arm_single(p, n_steps) != hipSuccess)
        st = fail(ASN_E_HIP, "arming the step counter failed");
    asn::BatchArgs bt = single_batch(p);
    for (int64_t i = 0; st == ASN_OK && i < n_steps; ++i) {
        bt.s_par = (int)(i & 1);
        const hipError_t e = asn::launch_step(
            bt, p->blocks, p->dtype, launch_scheme(p), p->stream, &ev[(size_t)i * per], p->band_azim,
            p->L.banded ? p->band_lds() : 0, p->band_wide_rows(), p->band_reach);
        if (e != hipSuccess) {
            st = fail(ASN_E_HIP, std::string("step launch failed: ") + hipGetErrorString(e));
            break;
        }
    }
    if (st == ASN_OK) {
        p->cur ^= state_flip(p->scheme, n_steps);
        p->steps_done += n_steps;
    }
    double acc[5] = {0, 0, 0, 0, 0};
    if (st == ASN_OK && hipEventSynchronize(ev.back()) != hipSuccess)
        st = fail(ASN_E_HIP, "hipEventSynchronize failed");
    for (int64_t i = 0; st == ASN_OK && i < n_steps; ++i)
        for (int pass = 0; st == ASN_OK && pass < passes; ++pass) {
            hipEvent_t* e = &ev[(size_t)i * per + 5 * (size_t)pass];
            for (int k = 0; k < 5; ++k) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, e[k == 4 ? 0 : k], e[k == 4 ? 4 : k + 1]) != hipSuccess) {
                    st = fail(ASN_E_HIP, "hipEventElapsedTime failed");
                    break;
                }
                acc[k] += ms;
            }
        }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (st != ASN_OK) return st;
    for (int k = 0; k < 5; ++k) kernel_ms[k] = acc[k] / (double)n_steps;
    return ASN_OK;
}

// Whether problems may step together (shared operand type, scheme, kernel form,
// stream; no repeats, no implicit problems).
static asn_status check_batch(asn_problem* probs, int32_t n) {
    if (!probs || n < 1 || n > asn::kMaxArm)
        return fail(ASN_E_INVALID, "a batch holds 1 to 64 problems");
    for (int32_t i = 0; i < n; ++i) {
        if (!probs[i]) return fail(ASN_E_INVALID, "NULL problem in batch");
        if (probs[i]->dtype != probs[0]->dtype)
            return fail(ASN_E_INVALID, "problems of a batch must share the operand type");
        if (probs[i]->scheme != probs[0]->scheme)
            return fail(ASN_E_INVALID, "problems of a batch must share the time scheme");
        if (probs[i]->imp)
            return fail(ASN_E_UNSUPPORTED, "implicit problems step alone (asn_step)");
        if (probs[i]->L.fused != probs[0]->L.fused)
            return fail(ASN_E_INVALID, "problems of a batch must share the kernel form "
                                       "(asn_step_form; ask for ASN_FORM_FUSED or ASN_FORM_SEPARATE "
                                       "when their sizes differ)");
        if (probs[i]->L.banded != probs[0]->L.banded ||
            probs[i]->band_azim != probs[0]->band_azim)
            return fail(ASN_E_INVALID, "problems of a banded batch must share the azimuth count "
                                       "(and a batch is banded for all its problems or none)");
        if (probs[i]->L.flat != probs[0]->L.flat)
            return fail(ASN_E_INVALID, std::string("problems of a batch must share the stencil form: ") +
                                       "separate-kernel steps use flat cell chunks up to nx = " +
                                       std::to_string(asn::kFlatMaxNx) + " (Euler) or " +
                                       std::to_string(asn::kFlatMaxNxM) + " (Heun), strips beyond");
        if (probs[i]->stream != probs[0]->stream)
            return fail(ASN_E_INVALID, "problems of a batch must share the HIP stream");
        for (int32_t j = 0; j < i; ++j)
            if (probs[j] == probs[i]) return fail(ASN_E_INVALID, "a problem appears twice");
    }
    return ASN_OK;
}

asn_status asn_batch_create(asn_problem* probs, int32_t n, asn_batch* out) {
    if (!out) return fail(ASN_E_INVALID, "out is NULL");
    *out = nullptr;
    const asn_status cs = check_batch(probs, n);
    if (cs != ASN_OK) return cs;
    auto* b = new asn_batch_s();
    b->probs.assign(probs, probs + n);
    b->n = n;
    b->dtype = probs[0]->dtype;
    b->scheme = probs[0]->scheme;
    b->launch_scheme = launch_scheme(probs[0]);
    b->band_az = probs[0]->band_azim;
    b->band_wide = true;
    for (int32_t i = 0; i < n; ++i) {
        if (probs[i]->L.banded)
            b->band_lds = std::max(b->band_lds, probs[i]->band_lds());
        b->band_wide = b->band_wide && probs[i]->band_wide_rows();
        b->band_reach = std::max(b->band_reach, probs[i]->band_reach);
    }
    b->stream = probs[0]->stream;
    b->tab.resize(2 * (size_t)n);
    b->off.assign((size_t)asn::KT_COUNT * (n + 1), 0);
    for (int32_t i = 0; i < n; ++i) {
        b->tab[2 * i] = probs[i]->tab[0];
        b->tab[2 * i + 1] = probs[i]->tab[1];
        for (int k = 0; k < asn::KT_COUNT; ++k)
            b->off[(size_t)k * (n + 1) + i + 1] = b->off[(size_t)k * (n + 1) + i] + probs[i]->blocks[k];
    }
    for (int k = 0; k < asn::KT_COUNT; ++k) b->grid[k] = b->off[(size_t)k * (n + 1) + n];
    const size_t tab_b = b->tab.size() * sizeof(StepArgs);
    const size_t off_b = b->off.size() * sizeof(int);
    const size_t bytes = tab_b + off_b + 2 * asn::kMaxArm * sizeof(int);
    void* m = nullptr;
    if (hipMalloc(&m, bytes) != hipSuccess) {
        delete b;
        return fail(ASN_E_OOM, "hipMalloc of the batch tables failed");
    }
    b->dev = static_cast<char*>(m);
    if (hipMemcpyAsync(b->dev, b->tab.data(), tab_b, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipMemcpyAsync(b->dev + tab_b, b->off.data(), off_b, hipMemcpyHostToDevice, b->stream) !=
            hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        (void)hipFree(b->dev);
        delete b;
        return fail(ASN_E_HIP, "copying the batch tables failed");
    }
    b->args.tab = reinterpret_cast<const StepArgs*>(b->dev);
    b->args.off = reinterpret_cast<const int*>(b->dev + tab_b);
    b->args.base = reinterpret_cast<const int*>(b->dev + tab_b + off_b);
    b->args.steps_left = reinterpret_cast<int*>(b->dev + tab_b + off_b + asn::kMaxArm * sizeof(int));
    b->args.n = n;
    b->args.s_par = 0;
    *out = b;
    return ASN_OK;
}

asn_status asn_batch_step(asn_batch b, int64_t n_steps, const int64_t* limit) {
    if (!b) return fail(ASN_E_INVALID, "batch is NULL");
    if (n_steps < 0 || n_steps > (1 << 20)) return fail(ASN_E_INVALID, "n_steps must be in [0, 2^20]");
    asn::ArmArgs v{};
    std::vector<int64_t> take(b->n);
    bool any = false;
    for (int i = 0; i < b->n; ++i) {
        take[i] = limit ? std::max<int64_t>(0, std::min<int64_t>(limit[i], n_steps)) : n_steps;
        v.limit[i] = (int)take[i];
        v.cur[i] = b->probs[i]->cur;
        any = any || take[i] > 0;
    }
    if (!any) return ASN_OK;
    int* left = b->args.steps_left;
    HIP_TRY(asn::launch_arm(left, const_cast<int*>(b->args.base), b->n, v, b->stream));
    asn::BatchArgs args = b->args;
    if (b->stream != nullptr && n_steps >= 2) {
        // Capture the step sequence once per length; later calls replay it.
        auto it = b->graphs.find(n_steps);
        if (it == b->graphs.end()) {
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
            hipError_t e = hipSuccess;
            for (int64_t j = 0; j < n_steps && e == hipSuccess; ++j) {
                args.s_par = (int)(j & 1);
                e = asn::launch_step(args, b->grid, b->dtype, b->launch_scheme, b->stream, nullptr,
                                     b->band_az, b->band_lds, b->band_wide, b->band_reach);
            }
            const hipError_t e2 = hipStreamEndCapture(b->stream, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return fail(ASN_E_HIP, std::string("capturing the step graph failed: ") +
                                           hipGetErrorString(e != hipSuccess ? e : e2));
            }
            if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGraphDestroy(g);
                return fail(ASN_E_HIP, "instantiating the step graph failed");
            }
            it = b->graphs.emplace(n_steps, std::make_pair(g, ge)).first;
        }
        HIP_TRY(hipGraphLaunch(it->second.second, b->stream));
    } else {
        for (int64_t j = 0; j < n_steps; ++j) {
            args.s_par = (int)(j & 1);
            HIP_TRY(asn::launch_step(args, b->grid, b->dtype, b->launch_scheme, b->stream, nullptr,
                                     b->band_az, b->band_lds, b->band_wide, b->band_reach));
        }
    }
    for (int i = 0; i < b->n; ++i) {
        b->probs[i]->cur ^= state_flip(b->scheme, take[i]);
        b->probs[i]->steps_done += take[i];
    }
    return ASN_OK;
}

asn_status asn_batch_destroy(asn_batch b) {
    if (!b) return ASN_OK;
    asn_status st = ASN_OK;
    if (hipStreamSynchronize(b->stream) != hipSuccess)
        st = fail(ASN_E_HIP, "synchronising before destroying the batch failed");
    for (auto& kv : b->graphs) {
        (void)hipGraphExecDestroy(kv.second.second);
        (void)hipGraphDestroy(kv.second.first);
    }
    if (b->dev) (void)hipFree(b->dev);
    delete b;
    return st;
}

// asn_step_batch_noalloc: the batch tables (step arguments of both buffers, block
// offsets per kernel kind, buffer bases, step counters) live in this file-scope device
// array instead of a hipMalloc'd block.  In host code the array's name is no device
// address: each device's copy is reached through the pointer hipGetSymbolAddress
// returns for it (kept per device at the first call there).
constexpr size_t kNoAllocBytes = 64 * 1024;
static __device__ __align__(256) unsigned char noalloc_scratch[kNoAllocBytes];

static std::mutex g_scratch_mu;
static std::map<int, char*> g_scratch_ptr;

static asn_status scratch_on_device(char** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch)));
        it = g_scratch_ptr.emplace(dev, static_cast<char*>(ptr)).first;
    }
    *out = it->second;
    return ASN_OK;
}

asn_status asn_step_batch_noalloc(asn_problem* probs, int32_t n, int64_t n_steps) {
    const asn_status cs = check_batch(probs, n);
    if (cs != ASN_OK) return cs;
    if (n_steps < 0 || n_steps > (1 << 20)) return fail(ASN_E_INVALID, "n_steps must be in [0, 2^20]");
    // the tables, laid out as in asn_batch_create, in host arrays of fixed size
    constexpr int kN = asn::kMaxArm;
    StepArgs tab[2 * kN];
    int off[asn::KT_COUNT * (kN + 1)];
    const size_t tab_b = 2 * (size_t)n * sizeof(StepArgs);
    const size_t off_b = (size_t)asn::KT_COUNT * (n + 1) * sizeof(int);
    const size_t bytes = tab_b + off_b + 2 * (size_t)kN * sizeof(int);
    if (bytes > kNoAllocBytes)
        return fail(ASN_E_INVALID, "batch tables exceed the no-allocation scratch (" +
                                       std::to_string(kNoAllocBytes) + " bytes)");
    int grid[asn::KT_COUNT];
    for (int k = 0; k < asn::KT_COUNT; ++k) off[k * (n + 1)] = 0;
    size_t band_lds = 0;
    bool band_wide = true;
    int band_reach = 0;
    for (int32_t i = 0; i < n; ++i) {
        tab[2 * i] = probs[i]->tab[0];
        tab[2 * i + 1] = probs[i]->tab[1];
        for (int k = 0; k < asn::KT_COUNT; ++k)
            off[k * (n + 1) + i + 1] = off[k * (n + 1) + i] + probs[i]->blocks[k];
        if (probs[i]->L.banded) band_lds = std::max(band_lds, probs[i]->band_lds());
        band_wide = band_wide && probs[i]->band_wide_rows();
        band_reach = std::max(band_reach, probs[i]->band_reach);
    }
    for (int k = 0; k < asn::KT_COUNT; ++k) grid[k] = off[k * (n + 1) + n];
    if (n_steps == 0) return ASN_OK;
    char* dev = nullptr;
    const asn_status ss = scratch_on_device(&dev);
    if (ss != ASN_OK) return ss;
    hipStream_t stream = probs[0]->stream;
    // stream order: earlier work on this stream that read the tables has finished
    // before the copies land; the host arrays must outlive the copies, hence the wait
    HIP_TRY(hipMemcpyAsync(dev, tab, tab_b, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(dev + tab_b, off, off_b, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    asn::BatchArgs args{};
    args.tab = reinterpret_cast<const StepArgs*>(dev);
    args.off = reinterpret_cast<const int*>(dev + tab_b);
    args.base = reinterpret_cast<const int*>(dev + tab_b + off_b);
    args.steps_left = reinterpret_cast<int*>(dev + tab_b + off_b + kN * sizeof(int));
    args.n = n;
    asn::ArmArgs v{};
    for (int i = 0; i < n; ++i) {
        v.limit[i] = (int)n_steps;
        v.cur[i] = probs[i]->cur;
    }
    HIP_TRY(asn::launch_arm(args.steps_left, const_cast<int*>(args.base), n, v, stream));
    const int scheme = launch_scheme(probs[0]);
    for (int64_t j = 0; j < n_steps; ++j) {
        args.s_par = (int)(j & 1);
        HIP_TRY(asn::launch_step(args, grid, probs[0]->dtype, scheme, stream, nullptr,
                                 probs[0]->band_azim, band_lds, band_wide, band_reach));
    }
    for (int i = 0; i < n; ++i) {
        probs[i]->cur ^= state_flip(probs[i]->scheme, n_steps);
        probs[i]->steps_done += n_steps;
    }
    // the next call overwrites the tables: let this one's kernels finish first
    HIP_TRY(hipStreamSynchronize(stream));
    return ASN_OK;
}

asn_status asn_step_batch(asn_problem* probs, int32_t n, int64_t n_steps) {
    asn_batch b = nullptr;
    asn_status s = asn_batch_create(probs, n, &b);
    if (s != ASN_OK) return s;
    s = asn_batch_step(b, n_steps, nullptr);
    const asn_status s2 = asn_batch_destroy(b);
    return s != ASN_OK ? s : s2;
}

asn_status asn_scalar_flux(asn_problem p, double* phi_host) {
    if (!p || !phi_host) return fail(ASN_E_INVALID, "NULL argument");
    HIP_TRY(hipMemcpyAsync(phi_host, p->base + p->L.off_phi64, p->L.C * 8, hipMemcpyDeviceToHost,
                           p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    return ASN_OK;
}

asn_status asn_mass_budget(asn_problem p, double out[ASN_BUDGET_LEN]) {
    if (!p || !out) return fail(ASN_E_INVALID, "NULL argument");
    if (p->imp) {
        HIP_TRY(hipStreamSynchronize(p->stream));
        for (int k = 0; k < ASN_BUDGET_LEN; ++k) out[k] = p->imp->budget[k];
        if (!std::isfinite(out[0])) return fail(ASN_E_UNSTABLE, "mass is not finite");
        return ASN_OK;
    }
    double rec[asn::REC_LEN];
    HIP_TRY(hipMemcpyAsync(rec, p->base + p->L.off_rec, sizeof(rec), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    out[0] = rec[asn::REC_MASS];
    out[1] = rec[asn::REC_MASS0];
    out[2] = rec[asn::REC_ABS];
    out[3] = rec[asn::REC_OUT];
    out[4] = rec[asn::REC_SRC];
    out[5] = rec[asn::REC_DEF];
    out[6] = rec[asn::REC_RES];
    out[7] = rec[asn::REC_STEPS];
    if (!std::isfinite(out[0])) return fail(ASN_E_UNSTABLE, "mass is not finite");
    return ASN_OK;
}

asn_status asn_info(asn_problem p, double* dt, int64_t* steps_done, int64_t* steps_to_tfinal,
                    int32_t* q) {
    if (!p) return fail(ASN_E_INVALID, "problem is NULL");
    if (dt) *dt = p->dt;
    if (steps_done) *steps_done = p->steps_done;
    if (steps_to_tfinal) *steps_to_tfinal = p->n_to_tfinal;
    if (q) *q = p->L.Q;
    return ASN_OK;
}

asn_status asn_step_form(asn_problem p, int32_t* form) {
    if (!p || !form) return fail(ASN_E_INVALID, "NULL argument");
    *form = p->L.banded ? ASN_FORM_BANDED : p->L.fused ? ASN_FORM_FUSED : ASN_FORM_SEPARATE;
    return ASN_OK;
}

asn_status asn_iteration_counts(asn_problem p, int64_t* sweeps, int64_t* matvecs) {
    if (!p) return fail(ASN_E_INVALID, "problem is NULL");
    if (sweeps) *sweeps = p->imp ? p->imp->sweeps : 0;
    if (matvecs) *matvecs = p->imp ? p->imp->matvecs : 0;
    return ASN_OK;
}

asn_status asn_stability(asn_problem p, double* z) {
    if (!p || !z) return fail(ASN_E_INVALID, "NULL argument");
    *z = p->stability;
    return ASN_OK;
}

asn_status asn_contraction_work(asn_problem p, double* dense_flops, double* tile_flops) {
    if (!p) return fail(ASN_E_INVALID, "problem is NULL");
    const double C = (double)p->L.C, Q = (double)p->L.Q;
    if (dense_flops) *dense_flops = 2.0 * Q * Q * C;
    if (tile_flops) *tile_flops = 2.0 * p->tile_entries * C;
    return ASN_OK;
}

asn_status asn_contraction_nonzero(asn_problem p, double* nonzero_flops) {
    if (!p || !nonzero_flops) return fail(ASN_E_INVALID, "NULL argument");
    *nonzero_flops = 2.0 * p->nonzero_entries * (double)p->L.C;
    return ASN_OK;
}

asn_status asn_destroy(asn_problem p) {
    if (!p) return ASN_OK;
    asn_status s = ASN_OK;
    if (hipStreamSynchronize(p->stream) != hipSuccess)
        s = fail(ASN_E_HIP, "synchronising before destroy failed");
    if (p->owns && p->base) (void)hipFree(p->base);
    delete p;
    return s;
}

const char* asn_status_string(asn_status s) {
    switch (s) {
        case ASN_OK: return "ok";
        case ASN_E_INVALID: return "invalid argument";
        case ASN_E_OOM: return "out of memory";
        case ASN_E_HIP: return "HIP runtime error";
        case ASN_E_UNSTABLE: return "unstable";
        case ASN_E_STATE: return "invalid state";
        case ASN_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* asn_last_error(void) { return g_last_error.c_str(); }

asn_status asn_build_quadrature(int32_t n_polar, int32_t n_azim, double* omega_xyz,
                                double* weights) {
    if (n_polar < 1 || n_azim < 1 || !omega_xyz || !weights)
        return fail(ASN_E_INVALID, "invalid quadrature request");
    std::vector<double> om, w;
    asn::product_quadrature(n_polar, n_azim, om, w);
    std::memcpy(omega_xyz, om.data(), om.size() * 8);
    std::memcpy(weights, w.data(), w.size() * 8);
    return ASN_OK;
}

asn_status asn_build_icosahedron(int32_t order, double* omega_xyz, double* weights) {
    if (order < 2 || order > 41 || !omega_xyz || !weights)
        return fail(ASN_E_INVALID, "invalid icosahedron request");
    std::vector<double> om, w;
    asn::icosahedron_quadrature(order, om, w);
    std::memcpy(omega_xyz, om.data(), om.size() * 8);
    std::memcpy(weights, w.data(), w.size() * 8);
    return ASN_OK;
}

asn_status asn_build_kernel(int32_t q, const double* omega_xyz, const double* weights, double eps,
                            int32_t normalization, double* k_out) {
    if (q < 1 || !omega_xyz || !weights || !k_out || !(eps > 0.0))
        return fail(ASN_E_INVALID, "invalid kernel request");
    if (normalization != ASN_NORM_SYM && normalization != ASN_NORM_ROW)
        return fail(ASN_E_INVALID, "unknown normalization");
    std::vector<double> K;
    std::string err;
    if (!asn::kernel_matrix(q, omega_xyz, weights, eps, normalization == ASN_NORM_SYM ? 0 : 1, K, err))
        return fail(ASN_E_UNSUPPORTED, err);
    std::memcpy(k_out, K.data(), K.size() * 8);
    return ASN_OK;
}

asn_status asn_build_kernel_lowp(int32_t q, const double* k_in, int32_t gemm_dtype,
                                 uint16_t* k_bits, float* row_defect) {
    if (q < 1 || !k_in || !k_bits || !row_defect)
        return fail(ASN_E_INVALID, "invalid reduced-precision kernel request");
    if (gemm_dtype != ASN_GEMM_BF16 && gemm_dtype != ASN_GEMM_F16)
        return fail(ASN_E_INVALID, "gemm_dtype must be ASN_GEMM_BF16 or ASN_GEMM_F16");
    quantise_kernel(q, k_in, gemm_dtype, q, k_bits, row_defect);
    return ASN_OK;
}

asn_status asn_band_expand(int32_t n_polar, int32_t n_azim, const double* k_in, float* k_out,
                           int32_t* reach) {
    if (n_polar < 1 || n_azim < 1 || (int64_t)n_polar * n_azim > 16384 || !k_in || !k_out || !reach)
        return fail(ASN_E_INVALID, "invalid band request");
    const int Q = n_polar * n_azim;
    std::vector<float> K32((size_t)Q * Q);
    for (size_t i = 0; i < K32.size(); ++i) K32[i] = (float)k_in[i];
    asn::BandForm bf;
    if (!asn::band_form(n_polar, n_azim, K32.data(), asn::kBandMaxReach, asn::kBandNarrow, bf))
        return fail(ASN_E_UNSUPPORTED, "K has no banded form");
    // decode the per-level descriptors the kernel reads
    std::fill(k_out, k_out + (size_t)Q * Q, 0.f);
    auto put_run = [&](int i, int k, int lo, int len, int first) {
        const int j = i + k - bf.reach;
        for (int t = 0; t < len; ++t) {
            const int delta = lo + t;
            for (int kk = 0; kk < n_azim; ++kk) {
                const int kp = ((kk + delta) % n_azim + n_azim) % n_azim;
                k_out[(size_t)(i * n_azim + kk) * Q + j * n_azim + kp] = bf.coef[first + t];
            }
        }
    };
    for (int i = 0; i < n_polar; ++i) {
        const int n = (int)bf.desc[(size_t)i * 8];
        for (int p = 0; p < n; ++p) {
            const uint32_t c = bf.desc[(size_t)i * 8 + 1 + p];
            int lo = 0, len = 0;
            asn::band_run(c, n_azim, lo, len);
            put_run(i, (int)((c >> 8) & 7u), lo, len, bf.range[2 * (size_t)i] + 4 * (int)(c >> 11));
        }
    }
    *reach = bf.reach;
    return ASN_OK;
}

asn_status asn_time_step(const asn_grid* grid, int32_t q, const double* omega_xyz, double cfl,
                         double t_final, double* dt, int64_t* n_steps) {
    asn_status s = check_grid(grid);
    if (s != ASN_OK) return s;
    if (q < 1 || !omega_xyz || !dt || !n_steps || !(t_final > 0.0) || !(cfl > 0.0))
        return fail(ASN_E_INVALID, "invalid time-step request");
    if (cfl > 1.0) return fail(ASN_E_UNSTABLE, "cfl above 1 is unstable for the explicit step");
    const double dx = (grid->x_max - grid->x_min) / grid->nx;
    const double dy = (grid->y_max - grid->y_min) / grid->ny;
    asn::cfl_time_step(q, omega_xyz, dx, dy, cfl, t_final, *dt, *n_steps);
    return ASN_OK;
}

}  // extern "C"
