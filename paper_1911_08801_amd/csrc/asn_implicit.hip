// Device kernels and host driver of the implicit as-S_N step (FP64).  See
// asn_implicit.hpp.  Faces carry 3/2 psi_up - 1/2 psi_upup (paper Section 3.5,
// no limiter); cells outside the grid are 0 (vacuum).
#include "asn_implicit.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace asn {

namespace {

constexpr int kT = 64;      // GEMM tile (ordinates x cells)
constexpr int kTK = 16;     // GEMM k-step
constexpr int kVecBlock = 1024;   // vector elements per reduction block

inline int64_t rup(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
inline unsigned ndiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

struct RhsArgs {
    const double* K;        // [Q][Q]
    const double* psi;      // [Q][P]
    const double* psi_old;  // [Q][P]
    const double* phi;      // [P] or null
    const float4* coef;     // per cell {sigma_a, sigma_s, sigma_as, q}
    double* rhs;            // [Q][P]
    int Q;
    int64_t C, P;
    double alpha, beta, inv_dt, inv_W;
    const int* stop;        // nonzero *stop: the source iteration has converged, do nothing
};

// rhs[q][c] = sigma_as (K psi)[q][c] + alpha sigma_s phi_c / W + beta (q_c + psi_old[q][c] / dt)
__global__ __launch_bounds__(256) void imp_rhs_kernel(RhsArgs a) {
    if (a.stop != nullptr && *a.stop) return;   // block-uniform, before any barrier
    __shared__ double Ks[kTK][kT + 1];
    __shared__ double Ps[kTK][kT];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int q0 = blockIdx.x * kT;
    const int64_t c0 = (int64_t)blockIdx.y * kT;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    // the next k-step's tiles are fetched into registers while this one is multiplied
    double kr[4], pr[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int idx = tid + 256 * l;
            const int r = idx >> 4, kk = idx & 15;
            const int q = q0 + r, k = k0 + kk;
            kr[l] = (q < a.Q && k < a.Q) ? a.K[(size_t)q * a.Q + k] : 0.0;
            const int pk = idx >> 6, cc = idx & 63;
            pr[l] = (k0 + pk < a.Q) ? a.psi[(size_t)(k0 + pk) * a.P + c0 + cc] : 0.0;
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < a.Q; k0 += kTK) {
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int idx = tid + 256 * l;
            Ks[idx & 15][idx >> 4] = kr[l];
            Ps[idx >> 6][idx & 63] = pr[l];
        }
        __syncthreads();
        if (k0 + kTK < a.Q) fetch(k0 + kTK);
#pragma unroll
        for (int kk = 0; kk < kTK; ++kk) {
            double kv[4], pv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) kv[i] = Ks[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) pv[j] = Ps[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(kv[i], pv[j], acc[i][j]);
        }
        __syncthreads();
    }
    // the thread's four consecutive cells (32 bytes of each ordinate's row, read and
    // written as one piece; cb + 3 < P since the pitch is a multiple of the tile)
    const int64_t cb = c0 + tx * 4;
    float4 cf[4];
    double iso[4];
    bool cok[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t c = cb + j;
        cok[j] = c < a.C;
        cf[j] = cok[j] ? a.coef[c] : make_float4(0.f, 0.f, 0.f, 0.f);
        iso[j] = (cok[j] && a.phi) ? a.alpha * (double)cf[j].y * a.phi[c] * a.inv_W : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = q0 + ty * 4 + i;
        if (q >= a.Q) continue;
        const size_t o = (size_t)q * a.P + cb;
        const double2 o01 = *reinterpret_cast<const double2*>(a.psi_old + o);
        const double2 o23 = *reinterpret_cast<const double2*>(a.psi_old + o + 2);
        const double old[4] = {o01.x, o01.y, o23.x, o23.y};
        double v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            v[j] = cok[j] ? (double)cf[j].z * acc[i][j] + iso[j] +
                                a.beta * ((double)cf[j].w + old[j] * a.inv_dt)
                          : 0.0;
        *reinterpret_cast<double2*>(a.rhs + o) = make_double2(v[0], v[1]);
        *reinterpret_cast<double2*>(a.rhs + o + 2) = make_double2(v[2], v[3]);
    }
}

struct SweepArgs {
    const double* rhs;      // [Q][P]
    const double* dir;      // per ordinate {|xi|/dx, |eta|/dy, sign xi, sign eta}
    const double* sig;      // per cell sigma_a + sigma_s + sigma_as + 1/dt
    double* out;            // [Q][P]
    int nx, ny;
    int64_t P;
    const int* stop;        // as in RhsArgs
};

// Lane l receives the value of lane l - 1 (lane 0 receives 0): DPP wave_shr:1, one
// VALU move per 32-bit half, no LDS round trip.
__device__ __forceinline__ double wave_shr1(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// One block per ordinate.  The grid is walked in strips of 64 rows from the upwind
// side; lane j of a wave holds row j of its strip and, at its step t, the cell t - j
// positions from the upwind x boundary, so its x-upwind neighbours are its own two
// previous results and its y-upwind neighbours are those of lanes j - 1 and j - 2:
// lane j - 1's value comes by a lane shift of the current step, lane j - 2's is what
// lane j - 1 received one step earlier.  The block's W waves take W consecutive strips
// at once, wave w starting 72 steps after wave w - 1 (a wavefront over strips): the
// rows 62 and 63 of wave w - 1 that lane 0 of wave w needs in a window of 8 steps were
// written to an LDS ring at least two block steps before the window starts, so lane 0
// reads them at the window start and the block synchronises once per window, not per
// step.  The last strip of a round of W strips keeps its two downwind rows for the
// next round.
// The cells a wave touches in one step lie on a diagonal (one per row), so its inputs
// (right-hand side and rate) and outputs go through LDS in windows of 8 steps: for each
// row the 8 cells of a window are consecutive, and 8 lanes move them as one 64-byte
// segment (a window is loaded 8 steps before it is used and its results are stored 8
// steps after), instead of every load and store of a step touching 64 cache lines.
// Block barrier that orders LDS only: the sweep's waves exchange rows through LDS, and
// a full barrier would also wait for every global load in flight (the next window).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int kSweepAhead = 8;    // steps per staged window
constexpr int kSweepWaves = 8;    // strips in flight per ordinate (at most)
constexpr int kSweepRing = 32;    // columns of a strip's rows 62, 63 kept for the next wave
constexpr int kSweepLag = 64 + kSweepAhead;   // steps between the starts of waves w - 1, w
constexpr int kSweepWinPitch = kSweepAhead + 1;                  // padded LDS row (doubles)
constexpr int kSweepWinDoubles = 3 * 64 * kSweepWinPitch;        // inputs x 2, outputs
__global__ __launch_bounds__(64 * kSweepWaves) void imp_sweep_kernel(SweepArgs a) {
    extern __shared__ double smem[];   // [2 parity][2 rows][nx], then [W][3][64][pitch]
    __shared__ double ring[kSweepWaves][2][kSweepRing];
    __shared__ double spare[64];   // targets of the stores of lanes that keep nothing
    constexpr int D = kSweepAhead, DP = kSweepWinPitch;
    // the slot u = tau mod D is the same for every wave (kSweepLag is a multiple of D);
    // wave w - 1 writes ring column k + kSweepRing 23 block steps after wave w read k
    static_assert(kSweepLag % D == 0 && kSweepRing >= 4 * D, "ring slots must outlive their reads");
    if (a.stop != nullptr && *a.stop) return;   // block-uniform, before any barrier
    const int q = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int W = blockDim.x >> 6;
    const int nx = a.nx, ny = a.ny;
    const double ax = a.dir[4 * q + 0], ay = a.dir[4 * q + 1];
    const bool xpos = a.dir[4 * q + 2] > 0.0, ypos = a.dir[4 * q + 3] > 0.0;
    const double* rhs = a.rhs + (size_t)q * a.P;
    double* out = a.out + (size_t)q * a.P;
    const double dflux = 1.5 * (ax + ay);
    const int nstrips = (ny + 63) / 64;
    const int Tw = nx + 63;   // steps of one strip
    double* rowbuf = smem;
    double* win_r = smem + 4 * (size_t)nx + (size_t)w * kSweepWinDoubles;   // this wave's
    double* win_s = win_r + 64 * DP;
    double* win_o = win_s + 64 * DP;
    // window lanes: lane l moves column l % 8 of strip rows l / 8 + 8 i, i = 0..7
    const int wrow = lane >> 3, wcol = lane & 7;
    int par = 0;
    for (int g0 = 0; g0 < nstrips; g0 += W) {
        const int Wg = min(W, nstrips - g0);   // strips of this round
        const int s = g0 + w;                  // this wave's strip (idle if w >= Wg)
        const bool wave_on = w < Wg;
        const bool last_wave = w == Wg - 1;
        const int r = s * 64 + lane;           // row in sweep order
        const bool valid = wave_on && r < ny;
        const double* prev_top = rowbuf + (size_t)(par ^ 1) * 2 * nx;   // previous round
        double* cur_top = rowbuf + (size_t)par * 2 * nx;
        auto grid_y = [&](int row) { return ypos ? row : ny - 1 - row; };
        auto grid_x = [&](int k) { return xpos ? k : nx - 1 - k; };
        // Window of steps T0 .. T0 + 7: strip row rl needs columns T0 - rl .. T0 - rl + 7.
        // Loads at clamped in-range addresses (values outside the grid are not used).
        double nr[8], ns[8];
        auto load_win = [&](int T0) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int rl = wrow + 8 * i;
                const int yc = grid_y(min(s * 64 + rl, ny - 1));
                const int kc = min(max(T0 + wcol - rl, 0), nx - 1);
                const size_t c = (size_t)yc * nx + grid_x(kc);
                nr[i] = rhs[c];
                ns[i] = a.sig[c];
            }
        };
        auto stage_win = [&]() {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                win_r[(wrow + 8 * i) * DP + wcol] = nr[i];
                win_s[(wrow + 8 * i) * DP + wcol] = ns[i];
            }
        };
        auto flush_win = [&](int T0) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int rl = wrow + 8 * i, row = s * 64 + rl;
                const int k = T0 + wcol - rl;
                const double v = win_o[rl * DP + wcol];
                if (wave_on && row < ny && k >= 0 && k < nx)
                    out[(size_t)grid_y(row) * nx + grid_x(k)] = v;
            }
        };
        load_win(0);
        double er = 0.0, es = 0.0;         // this lane's inputs of its current step
        double t62r[8], t63r[8];           // lane 0: rows 62, 63 above, columns of the window
        double last1 = 0.0, last2 = 0.0;   // x ghosts
        double y1prev = 0.0;               // y-upwind value this lane received last step
        auto step = [&](int tau, int u) {
            const int k = tau - lane;
            double yn1 = wave_shr1(last1);    // lane - 1: row r - 1, column k
            double yn2 = wave_shr1(y1prev);   // lane - 2: row r - 2, column k
            if (lane == 0) {   // rows 63 and 62 of the strip above (read at the window start)
                yn1 = t63r[u];
                yn2 = t62r[u];
            }
            y1prev = yn1;
            // Branch-free: every lane computes (the window's inputs are staged for every
            // lane, at clamped in-grid cells, so the division is well defined) and the
            // results are selected.  A lane's slot of a step before its start is never
            // stored to memory; rows 62 and 63 keep their results for the strip below,
            // the other lanes write a spare slot.  The history shifts every step once the
            // lane has started, also past the end of its row: the lane two rows up reads
            // this lane's previous value one step later than the lane just above.
            const bool started = k >= 0;
            const bool live = valid && started && k < nx;
            const double num = er + ax * (2.0 * last1 - 0.5 * last2) + ay * (2.0 * yn1 - 0.5 * yn2);
            const double v = live ? num / (dflux + es) : 0.0;
            win_o[lane * DP + u] = v;
            const bool keep = lane >= 62 && started && k < nx;
            const int kr = max(lane - 62, 0);
            *(keep ? &ring[w][kr][k & (kSweepRing - 1)] : &spare[lane]) = v;
            if (last_wave) *(keep ? &cur_top[(size_t)kr * nx + k] : &spare[lane]) = v;
            last2 = started ? last1 : last2;
            last1 = started ? v : last1;
        };
        // Block step t: wave w runs its step tau = t - 72 w (slot u = tau mod 8, fixed at
        // compile time in the unrolled loops since 72 w is a multiple of 8).  At a window
        // start the wave stores the results of the window before, puts this window's
        // inputs into LDS and loads the next window.  A lane reads the inputs of its next
        // step from LDS while the current one runs (off the steps' dependent chain).  The
        // barrier at each window start orders the LDS traffic between waves; within a
        // wave, LDS operations run in program order.
        auto block_step = [&](int t, int u) {
            const int tau = t - kSweepLag * w;
            if (u == 0) {   // u is the same for every wave: all of them reach this barrier
                const bool win_on = tau >= 0 && tau < Tw + D;
                if (win_on) {
                    if (tau >= D) flush_win(tau - D);
                    if (tau < Tw) {
                        stage_win();
                        load_win(tau + D);
                    }
                }
                lds_barrier();
                er = win_r[lane * DP];
                es = win_s[lane * DP];
                // rows 63 and 62 of the strip above for the window's columns tau .. tau + 7:
                // wave w - 1 (its ring), the last strip of the previous round, or ghosts
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const int k = tau + i;
                    double t63 = 0.0, t62 = 0.0;
                    if (w > 0) {
                        t63 = ring[w - 1][1][k & (kSweepRing - 1)];
                        t62 = ring[w - 1][0][k & (kSweepRing - 1)];
                    } else if (g0 > 0) {
                        t63 = prev_top[nx + min(max(k, 0), nx - 1)];
                        t62 = prev_top[min(max(k, 0), nx - 1)];
                    }
                    const bool kin = k >= 0 && k < nx;
                    t63r[i] = kin ? t63 : 0.0;
                    t62r[i] = kin ? t62 : 0.0;
                }
            }
            // inputs of the next step of this window (slot u + 1), read now
            const double er1 = u + 1 < D ? win_r[lane * DP + u + 1] : 0.0;
            const double es1 = u + 1 < D ? win_s[lane * DP + u + 1] : 0.0;
            if (wave_on && tau >= 0 && tau < Tw) step(tau, u);
            er = er1;
            es = es1;
        };
        const int T = Tw + kSweepLag * (Wg - 1);
        int t0 = 0;
        for (; t0 + D <= T; t0 += D) {
#pragma unroll
            for (int u = 0; u < D; ++u) block_step(t0 + u, u);
        }
#pragma unroll
        for (int u = 0; u < D; ++u)
            if (t0 + u < T) block_step(t0 + u, u);
        // the window of the wave's last block step has not been stored yet (for a window
        // past the row's end every column is outside the grid and nothing is stored)
        const int tau_end = T - kSweepLag * w;
        if (tau_end > 0) flush_win(((tau_end - 1) / D) * D);
        lds_barrier();
        par ^= 1;
    }
}

// Dynamic LDS of the sweep: two parities of two carried rows, then W wave windows.
size_t sweep_lds_bytes(int nx, int W) {
    return ((size_t)4 * nx + (size_t)W * kSweepWinDoubles) * sizeof(double);
}
// Strips in flight per ordinate: at most kSweepWaves, and as many as the LDS holds next to
// the carried rows (nx <= 2048 keeps those within 64 KB, so one wave always fits).
int sweep_waves(int nx, int ny) {
    constexpr size_t kLdsBudget = 156 * 1024;   // of 160 KB, the rest for the static ring
    int W = std::min((ny + 63) / 64, kSweepWaves);
    while (W > 1 && sweep_lds_bytes(nx, W) > kLdsBudget) --W;
    return W;
}

// part[b] = {sum (x - y)^2, sum x^2} over this block's elements of [n]; nothing once
// *stop is set
__global__ __launch_bounds__(256) void imp_diff_kernel(const double* x, const double* y, int64_t n,
                                                       double* part, const int* stop) {
    if (*stop) return;
    double d = 0.0, m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kVecBlock + threadIdx.x;
         i < std::min<int64_t>(n, (int64_t)(blockIdx.x + 1) * kVecBlock); i += 256) {
        const double e = x[i] - y[i];
        d += e * e;
        m += x[i] * x[i];
    }
    __shared__ double red[2][256];
    red[0][threadIdx.x] = d;
    red[1][threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = red[0][0];
        part[2 * blockIdx.x + 1] = red[1][0];
    }
}

// The stopping test of a source iteration, on the device: ||x - y|| < thr (absolute) or
// ||x - y|| < thr ||x|| (relative) over the difference partials of imp_diff_kernel
// (strided shares, then a fixed-order tree).  stat = {done, iteration that met the test};
// once done is set, nothing changes it.
__global__ __launch_bounds__(256) void imp_test_kernel(const double* part, int nb, double thr,
                                                       int relative, int it, int* stat) {
    if (stat[0]) return;
    double d = 0.0, m = 0.0;
    const double2* p2 = reinterpret_cast<const double2*>(part);
    for (int b0 = threadIdx.x; b0 < nb; b0 += 256 * 8) {   // eight loads in flight
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p2[min(b0 + 256 * u, nb - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (b0 + 256 * u < nb) {
                d += v[u].x;
                m += v[u].y;
            }
    }
    __shared__ double red[2][256];
    red[0][threadIdx.x] = d;
    red[1][threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && !(sqrt(red[0][0]) >= thr * (relative ? sqrt(red[1][0]) : 1.0))) {
        stat[0] = 1;
        stat[1] = it;
    }
}

__global__ void imp_stat_clear_kernel(int* stat) {
    if (threadIdx.x < 2) stat[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void imp_dot_kernel(const double* x, const double* y, int64_t n,
                                                      double* part) {
    double d = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kVecBlock + threadIdx.x;
         i < std::min<int64_t>(n, (int64_t)(blockIdx.x + 1) * kVecBlock); i += 256)
        d += x[i] * y[i];
    __shared__ double red[256];
    red[threadIdx.x] = d;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void imp_axpy_kernel(double* y, double alpha, const double* x, double beta, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = beta * y[i] + alpha * x[i];
}

// phi[c] = sum_q w_q psi[q][c] (c < C; padding 0)
__global__ void imp_moments_kernel(const double* psi, const double* w, int Q, int64_t C, int64_t P,
                                   double* phi) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P) return;
    double s = 0.0;
    if (c < C)
        for (int q = 0; q < Q; ++q) s += w[q] * psi[(size_t)q * P + c];
    phi[c] = s;
}

__global__ void imp_to64_kernel(const float* src, double* dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (double)src[i];
}

__global__ void imp_to32_kernel(const double* src, float* dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

__global__ void imp_copy_kernel(const double* src, double* dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

struct BudgetArgs {
    const double* psi;      // [Q][P]
    const double* w;        // [Q]
    const double* dq;       // [Q]: (w^T K)_q - w_q
    const double* dir;
    const float4* coef;
    int nx, ny, Q;
    int64_t C, P;
    double dx, dy;
    double* part;           // [blocks][4]: Phi, sigma_a Phi, defect, outflow
};

// Per-block partials of the particle balance at the new level; the outflow
// through a boundary face is the face flux 3/2 psi_last - 1/2 psi_before_last.
__global__ __launch_bounds__(256) void imp_budget_kernel(BudgetArgs a) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (c < a.C) {
        const int y = (int)(c / a.nx), x = (int)(c - (int64_t)y * a.nx);
        const float4 cf = a.coef[c];
        double phi = 0.0, dd = 0.0, out = 0.0;
        const bool edge = x == 0 || x == a.nx - 1 || y == 0 || y == a.ny - 1;
        for (int q = 0; q < a.Q; ++q) {
            const double p = a.psi[(size_t)q * a.P + c];
            phi += a.w[q] * p;
            dd += a.dq[q] * p;
            if (!edge) continue;
            const double ax = a.dir[4 * q], ay = a.dir[4 * q + 1];
            const bool xp = a.dir[4 * q + 2] > 0.0, yp = a.dir[4 * q + 3] > 0.0;
            double f = 0.0;
            if (ax > 0.0 && ((xp && x == a.nx - 1) || (!xp && x == 0))) {
                const int xb = xp ? x - 1 : x + 1;
                const double pb = (xb >= 0 && xb < a.nx) ? a.psi[(size_t)q * a.P + (int64_t)y * a.nx + xb] : 0.0;
                f += ax * a.dx * a.dy * (1.5 * p - 0.5 * pb);
            }
            if (ay > 0.0 && ((yp && y == a.ny - 1) || (!yp && y == 0))) {
                const int yb = yp ? y - 1 : y + 1;
                const double pb = (yb >= 0 && yb < a.ny) ? a.psi[(size_t)q * a.P + (int64_t)yb * a.nx + x] : 0.0;
                f += ay * a.dx * a.dy * (1.5 * p - 0.5 * pb);
            }
            out += a.w[q] * f;
        }
        v[0] = phi;
        v[1] = (double)cf.x * phi;
        v[2] = (double)cf.z * dd;
        v[3] = out;
    }
    __shared__ double red[4][256];
#pragma unroll
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) a.part[4 * blockIdx.x + k] = red[k][0];
}

}  // namespace

#define IMP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) {                                                                \
            err = std::string(#expr ": ") + hipGetErrorString(e_);                             \
            return false;                                                                      \
        }                                                                                      \
    } while (0)

// Slots of four doubles in the partials buffer: one per reduction block of the widest
// user, the difference/dot kernels (kVecBlock elements of Q * P or P) and the budget
// kernel (256 cells of C), plus spare.
static int64_t partial_blocks(const ImplicitParams& p) {
    const int64_t vec = ndiv(std::max<int64_t>((int64_t)p.Q * p.P, p.P), kVecBlock);
    const int64_t bud = ndiv(p.C, 256);
    return std::max(vec, bud) + 8;
}

static size_t take(size_t& off, size_t bytes) {
    const size_t o = off;
    off += (size_t)rup((int64_t)bytes, 256);
    return o;
}

size_t ImplicitSolver::bytes(const ImplicitParams& p) {
    size_t off = 0;
    const size_t plane = (size_t)p.Q * p.P * 8;
    for (int i = 0; i < 4; ++i) take(off, plane);                 // psi_old, psi_a, psi_b, rhs
    take(off, (size_t)p.Q * p.Q * 8);                             // K
    take(off, (size_t)p.Q * 8 * 6);                               // w, dq, dir
    take(off, (size_t)p.P * 16);                                  // coef
    take(off, (size_t)p.P * 8);                                   // sig
    take(off, (size_t)p.P * 8);                                   // phi
    take(off, (size_t)(p.gmres_restart + 6) * p.P * 8);           // GMRES vectors
    take(off, (size_t)partial_blocks(p) * 4 * 8);                 // partials
    take(off, 256);                                               // stopping-test status
    return off;
}

bool ImplicitSolver::init(const ImplicitParams& p, const double* omega, const double* w,
                          const double* K, const float* sigma_s, const float* sigma_a,
                          const float* sigma_as, const float* source, char* base, hipStream_t s,
                          std::string& err) {
    p_ = p;
    s_ = s;
    if (p.nx > 2048) {
        err = "the implicit sweep keeps two grid rows in LDS: nx must be <= 2048";
        return false;
    }
    size_t off = 0;
    const size_t plane = (size_t)p.Q * p.P * 8;
    psi_old_ = reinterpret_cast<double*>(base + take(off, plane));
    psi_a_ = reinterpret_cast<double*>(base + take(off, plane));
    psi_b_ = reinterpret_cast<double*>(base + take(off, plane));
    rhs_ = reinterpret_cast<double*>(base + take(off, plane));
    K_ = reinterpret_cast<double*>(base + take(off, (size_t)p.Q * p.Q * 8));
    double* small = reinterpret_cast<double*>(base + take(off, (size_t)p.Q * 8 * 6));
    wq_ = small;
    dq_ = small + p.Q;
    dir_ = small + 2 * p.Q;
    coef_ = reinterpret_cast<float4*>(base + take(off, (size_t)p.P * 16));
    sig_ = reinterpret_cast<double*>(base + take(off, (size_t)p.P * 8));
    phi_ = reinterpret_cast<double*>(base + take(off, (size_t)p.P * 8));
    vecs_ = reinterpret_cast<double*>(base + take(off, (size_t)(p.gmres_restart + 6) * p.P * 8));
    nparts_ = partial_blocks(p);
    part_ = reinterpret_cast<double*>(base + take(off, (size_t)nparts_ * 4 * 8));
    hpart_.assign((size_t)nparts_ * 4, 0.0);
    stat_ = reinterpret_cast<int*>(base + take(off, 256));

    // host tables
    std::vector<double> small_h((size_t)p.Q * 6, 0.0);
    double tmax = 0.0;
    for (int q = 0; q < p.Q; ++q) {
        small_h[q] = w[q];
        double col = 0.0;
        for (int r = 0; r < p.Q; ++r) col += w[r] * K[(size_t)r * p.Q + q];
        small_h[p.Q + q] = col - w[q];
        const double xi = omega[3 * q], eta = omega[3 * q + 1];
        small_h[2 * p.Q + 4 * q + 0] = std::fabs(xi) / p.dx;
        small_h[2 * p.Q + 4 * q + 1] = std::fabs(eta) / p.dy;
        small_h[2 * p.Q + 4 * q + 2] = xi >= 0.0 ? 1.0 : -1.0;
        small_h[2 * p.Q + 4 * q + 3] = eta >= 0.0 ? 1.0 : -1.0;
    }
    std::vector<float4> coef((size_t)p.P, make_float4(0.f, 0.f, 0.f, 0.f));
    // total rate of the implicit update per cell, sigma_a + sigma_s + sigma_as + 1/dt
    std::vector<double> sig((size_t)p.P, 0.0);
    for (int64_t c = 0; c < p.C; ++c) {
        coef[c] = make_float4(sigma_a[c], sigma_s[c], sigma_as[c], source ? source[c] : 0.f);
        sig[c] = (double)sigma_a[c] + (double)sigma_s[c] + (double)sigma_as[c] + 1.0 / p.dt;
        const double st = (double)sigma_a[c] + sigma_s[c] + sigma_as[c] + 1.0 / p.dt;
        tmax = std::max(tmax, (double)sigma_as[c] / st);
    }
    T_ = tmax;
    double qs = 0.0;
    if (source)
        for (int64_t c = 0; c < p.C; ++c) qs += (double)source[c];
    src_rate_ = p.dx * p.dy * p.W * qs;
    IMP_TRY(hipMemcpyAsync(K_, K, (size_t)p.Q * p.Q * 8, hipMemcpyHostToDevice, s_));
    IMP_TRY(hipMemcpyAsync(small, small_h.data(), small_h.size() * 8, hipMemcpyHostToDevice, s_));
    IMP_TRY(hipMemcpyAsync(coef_, coef.data(), coef.size() * 16, hipMemcpyHostToDevice, s_));
    IMP_TRY(hipMemcpyAsync(sig_, sig.data(), sig.size() * 8, hipMemcpyHostToDevice, s_));
    if ((size_t)4 * p.nx * 8 > 65536) {
        err = "sweep LDS request too large";
        return false;
    }
    IMP_TRY(hipFuncSetAttribute((const void*)imp_sweep_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sweep_lds_bytes(p.nx, sweep_waves(p.nx, p.ny))));
    return true;
}

bool ImplicitSolver::set_state(const float* psi32, double* phi64_out, std::string& err) {
    const int64_t n = (int64_t)p_.Q * p_.P;
    imp_to64_kernel<<<ndiv(n, 256), 256, 0, s_>>>(psi32, psi_old_, n);
    IMP_TRY(hipGetLastError());
    if (!moments(psi_old_, phi_, err)) return false;
    IMP_TRY(hipMemcpyAsync(phi64_out, phi_, (size_t)p_.C * 8, hipMemcpyDeviceToDevice, s_));
    // budget start: M^0
    std::vector<double> h((size_t)p_.P);
    IMP_TRY(hipMemcpyAsync(h.data(), phi_, (size_t)p_.C * 8, hipMemcpyDeviceToHost, s_));
    IMP_TRY(hipStreamSynchronize(s_));
    double m = 0.0;
    for (int64_t c = 0; c < p_.C; ++c) m += h[c];
    m *= p_.dx * p_.dy;
    std::memset(budget, 0, sizeof(budget));
    budget[0] = m;
    budget[1] = m;
    sweeps = matvecs = 0;
    return true;
}

bool ImplicitSolver::get_state(float* psi32, std::string& err) {
    const int64_t n = (int64_t)p_.Q * p_.P;
    imp_to32_kernel<<<ndiv(n, 256), 256, 0, s_>>>(psi_old_, psi32, n);
    IMP_TRY(hipGetLastError());
    return true;
}

bool ImplicitSolver::sweep_once(const double* psi_in, double* psi_out, const double* phi,
                                double alpha, double beta, std::string& err, const int* stop) {
    RhsArgs r{K_, psi_in, psi_old_, phi, coef_, rhs_, p_.Q, p_.C, p_.P, alpha, beta,
              1.0 / p_.dt, 1.0 / p_.W, stop};
    dim3 g(ndiv(p_.Q, kT), (unsigned)(p_.P / kT));
    imp_rhs_kernel<<<g, 256, 0, s_>>>(r);
    IMP_TRY(hipGetLastError());
    SweepArgs sa{rhs_, dir_, sig_, psi_out, p_.nx, p_.ny, p_.P, stop};
    const int W = sweep_waves(p_.nx, p_.ny);
    imp_sweep_kernel<<<p_.Q, 64 * W, sweep_lds_bytes(p_.nx, W), s_>>>(sa);
    IMP_TRY(hipGetLastError());
    if (stop == nullptr) ++sweeps;   // queued sweeps are counted once the test has run
    return true;
}

double* ImplicitSolver::source_iteration(const double* phi, double alpha, double beta,
                                         std::string& err, bool& ok) {
    ok = false;
    const double c = T_ > 0.0 ? (1.0 - T_) / T_ : 0.0;
    const double* prev = psi_old_;
    double* bufs[2] = {psi_a_, psi_b_};
    int cur = 0;
    if (!sweep_once(prev, bufs[cur], phi, alpha, beta, err)) return nullptr;
    if (T_ == 0.0) {       // no artificial scattering: one sweep is the exact inverse
        ok = true;
        return bufs[cur];
    }
    const int64_t n = (int64_t)p_.Q * p_.P;
    const unsigned nb = ndiv(n, kVecBlock);
    const double thr = p_.source_tol * c;
    // Iteration it compares sweep it with sweep it - 1 and stops when the change is below
    // the tolerance.  The test runs on the device, so iterations are queued in groups with
    // no host round trip between them; the kernels of iterations after the one that met
    // the test exit at once, leaving its result in place.  The host reads the status once
    // per group.
    constexpr int kGroup = 4, kMaxIt = 500;
    imp_stat_clear_kernel<<<1, 64, 0, s_>>>(stat_);
    int it = 1;
    while (it < kMaxIt) {
        const int end = std::min(it + kGroup, kMaxIt);
        for (; it < end; ++it) {
            imp_diff_kernel<<<nb, 256, 0, s_>>>(bufs[cur], prev, n, part_, stat_);
            imp_test_kernel<<<1, 256, 0, s_>>>(part_, (int)nb, thr, p_.source_relative ? 1 : 0,
                                               it, stat_);
            prev = bufs[cur];
            cur ^= 1;
            if (!sweep_once(prev, bufs[cur], phi, alpha, beta, err, stat_)) return nullptr;
        }
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(hstat_, stat_, sizeof(hstat_), hipMemcpyDeviceToHost, s_) != hipSuccess ||
            hipStreamSynchronize(s_) != hipSuccess) {
            err = "source-iteration test failed";
            return nullptr;
        }
        if (hstat_[0]) {                 // met at iteration k: sweeps 1 .. k ran
            const int k = hstat_[1];
            sweeps += k - 1;
            ok = true;
            return bufs[(k - 1) & 1];
        }
    }
    sweeps += kMaxIt - 1;
    ok = true;
    return bufs[cur];
}

bool ImplicitSolver::moments(const double* psi, double* phi, std::string& err) {
    imp_moments_kernel<<<ndiv(p_.P, 256), 256, 0, s_>>>(psi, wq_, p_.Q, p_.C, p_.P, phi);
    IMP_TRY(hipGetLastError());
    return true;
}

bool ImplicitSolver::dot(const double* a, const double* b, double& out, std::string& err) {
    const unsigned nb = ndiv(p_.P, kVecBlock);
    imp_dot_kernel<<<nb, 256, 0, s_>>>(a, b, p_.P, part_);
    IMP_TRY(hipGetLastError());
    IMP_TRY(hipMemcpyAsync(hpart_.data(), part_, (size_t)nb * 8, hipMemcpyDeviceToHost, s_));
    IMP_TRY(hipStreamSynchronize(s_));
    out = 0.0;
    for (unsigned i = 0; i < nb; ++i) out += hpart_[i];
    return true;
}

bool ImplicitSolver::axpy(double* y, double alpha, const double* x, std::string& err) {
    imp_axpy_kernel<<<ndiv(p_.P, 256), 256, 0, s_>>>(y, alpha, x, 1.0, p_.P);
    IMP_TRY(hipGetLastError());
    return true;
}

bool ImplicitSolver::scale_copy(double* y, double alpha, const double* x, std::string& err) {
    imp_axpy_kernel<<<ndiv(p_.P, 256), 256, 0, s_>>>(y, alpha, x, 0.0, p_.P);
    IMP_TRY(hipGetLastError());
    return true;
}

// out = v - M L~^-1 (sigma_s v / W), L~ = L - sigma_as K (Algorithm 2)
bool ImplicitSolver::lhs(const double* v, double* out, std::string& err) {
    bool ok = false;
    double* psi = source_iteration(v, 1.0, 0.0, err, ok);
    if (!ok) return false;
    if (!moments(psi, out, err)) return false;
    // out = v - out
    imp_axpy_kernel<<<ndiv(p_.P, 256), 256, 0, s_>>>(out, 1.0, v, -1.0, p_.P);
    IMP_TRY(hipGetLastError());
    ++matvecs;
    return true;
}

bool ImplicitSolver::fold_budget(const double* psi_new, double mass_prev, std::string& err) {
    const unsigned nb = ndiv(p_.C, 256);
    if ((int64_t)nb > nparts_) {
        err = "implicit budget: more blocks than partial slots";
        return false;
    }
    BudgetArgs b{psi_new, wq_, dq_, dir_, coef_, p_.nx, p_.ny, p_.Q, p_.C, p_.P, p_.dx, p_.dy, part_};
    imp_budget_kernel<<<nb, 256, 0, s_>>>(b);
    IMP_TRY(hipGetLastError());
    std::vector<double> h((size_t)nb * 4);
    IMP_TRY(hipMemcpyAsync(h.data(), part_, h.size() * 8, hipMemcpyDeviceToHost, s_));
    IMP_TRY(hipStreamSynchronize(s_));
    double t[4] = {0, 0, 0, 0};
    for (unsigned i = 0; i < nb; ++i)
        for (int k = 0; k < 4; ++k) t[k] += h[4 * i + k];
    const double area = p_.dx * p_.dy;
    const double m_next = area * t[0], absr = area * t[1], def = area * t[2], out = t[3];
    const double src = src_rate_;
    const double pred = mass_prev + p_.dt * (-absr - out + src + def);
    const double ref = std::max(budget[1], mass_prev);
    const double rel = ref > 0.0 ? std::fabs(m_next - pred) / ref : std::fabs(m_next - pred);
    budget[0] = m_next;
    budget[2] += p_.dt * absr;
    budget[3] += p_.dt * out;
    budget[4] += p_.dt * src;
    budget[5] += p_.dt * def;
    budget[6] = std::max(budget[6], rel);
    budget[7] += 1.0;
    return true;
}

bool ImplicitSolver::step(int64_t n, double* phi64_out, std::string& err) {
    const int m = p_.gmres_restart;
    double* V = vecs_;                  // V_0 .. V_m
    double* wv = vec(m + 1);
    double* bv = vec(m + 2);
    double* xv = vec(m + 3);
    double* rv = vec(m + 4);
    double* tmp = vec(m + 5);
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    auto Hat = [&](int i, int k) -> double& { return H[(size_t)i * m + k]; };
    for (int64_t step = 0; step < n; ++step) {
        const double mass_prev = budget[0];
        bool ok = false;
        // b = M L~^-1 (q + psi_old / dt)
        double* psi = source_iteration(nullptr, 0.0, 1.0, err, ok);
        if (!ok || !moments(psi, bv, err)) return false;
        // GMRES on A phi = b from the previous scalar flux (Algorithm 3)
        IMP_TRY(hipMemcpyAsync(xv, phi_, (size_t)p_.P * 8, hipMemcpyDeviceToDevice, s_));
        double bnorm = 0.0;
        if (!dot(bv, bv, bnorm, err)) return false;
        bnorm = std::sqrt(bnorm);
        const int max_mv = 300;
        int n_mv = 0;
        bool done = bnorm == 0.0;
        if (done) IMP_TRY(hipMemsetAsync(xv, 0, (size_t)p_.P * 8, s_));
        while (!done && n_mv < max_mv) {
            if (!lhs(xv, wv, err)) return false;
            ++n_mv;
            if (!scale_copy(rv, 1.0, bv, err) || !axpy(rv, -1.0, wv, err)) return false;
            double beta = 0.0;
            if (!dot(rv, rv, beta, err)) return false;
            beta = std::sqrt(beta);
            if (beta <= p_.gmres_tol * bnorm) break;
            if (!scale_copy(V, 1.0 / beta, rv, err)) return false;
            std::fill(H.begin(), H.end(), 0.0);
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int kd = 0;
            for (int k = 0; k < m; ++k) {
                double* Vk = V + (size_t)k * p_.P;
                if (!lhs(Vk, wv, err)) return false;
                ++n_mv;
                for (int i = 0; i <= k; ++i) {
                    double h = 0.0;
                    if (!dot(wv, V + (size_t)i * p_.P, h, err)) return false;
                    Hat(i, k) = h;
                    if (!axpy(wv, -h, V + (size_t)i * p_.P, err)) return false;
                }
                double hn = 0.0;
                if (!dot(wv, wv, hn, err)) return false;
                hn = std::sqrt(hn);
                Hat(k + 1, k) = hn;
                for (int i = 0; i < k; ++i) {
                    const double t = cs[i] * Hat(i, k) + sn[i] * Hat(i + 1, k);
                    Hat(i + 1, k) = -sn[i] * Hat(i, k) + cs[i] * Hat(i + 1, k);
                    Hat(i, k) = t;
                }
                const double den = std::hypot(Hat(k, k), Hat(k + 1, k));
                cs[k] = Hat(k, k) / den;
                sn[k] = Hat(k + 1, k) / den;
                Hat(k, k) = den;
                Hat(k + 1, k) = 0.0;
                g[k + 1] = -sn[k] * g[k];
                g[k] = cs[k] * g[k];
                kd = k + 1;
                if (std::fabs(g[k + 1]) <= p_.gmres_tol * bnorm || hn == 0.0 || n_mv >= max_mv) break;
                if (!scale_copy(V + (size_t)(k + 1) * p_.P, 1.0 / hn, wv, err)) return false;
            }
            for (int i = kd - 1; i >= 0; --i) {       // back substitution
                double s = g[i];
                for (int j = i + 1; j < kd; ++j) s -= Hat(i, j) * y[j];
                y[i] = s / Hat(i, i);
            }
            for (int i = 0; i < kd; ++i)
                if (!axpy(xv, y[i], V + (size_t)i * p_.P, err)) return false;
            if (std::fabs(g[kd]) <= p_.gmres_tol * bnorm) break;
        }
        // psi^{n+1} = L~^-1 (sigma_s phi / W + q + psi_old / dt)
        psi = source_iteration(xv, 1.0, 1.0, err, ok);
        if (!ok) return false;
        IMP_TRY(hipMemcpyAsync(psi_old_, psi, (size_t)p_.Q * p_.P * 8, hipMemcpyDeviceToDevice, s_));
        IMP_TRY(hipMemcpyAsync(phi_, xv, (size_t)p_.P * 8, hipMemcpyDeviceToDevice, s_));
        if (!moments(psi_old_, tmp, err)) return false;
        IMP_TRY(hipMemcpyAsync(phi64_out, tmp, (size_t)p_.C * 8, hipMemcpyDeviceToDevice, s_));
        if (!fold_budget(psi_old_, mass_prev, err)) return false;
    }
    return true;
}

}  // namespace asn
