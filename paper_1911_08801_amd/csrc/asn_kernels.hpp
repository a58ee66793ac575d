// Device kernels of the as-S_N step and their launchers (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace asn {

// Per-ordinate constants of the streaming update, read with uniform (scalar) loads.
struct QInfo {
    float cx;     // dt |xi_q| / dx
    float cy;     // dt |eta_q| / dy
    float wf;     // w_q in FP32
    int32_t dir;  // bit0 xi > 0, bit1 xi < 0, bit2 eta > 0, bit3 eta < 0
    double w;     // w_q in FP64 (moment and budget accumulation)
};

// Device-side particle budget record (FP64), updated once per step.
enum {
    REC_MASS = 0,      // M at the current level
    REC_MASS0 = 1,     // M at set_state
    REC_ABS = 2,       // cumulative absorption increments
    REC_OUT = 3,       // cumulative outflow increments
    REC_SRC = 4,       // cumulative source increments
    REC_DEF = 5,       // cumulative collision defect increments
    REC_RES = 6,       // max relative residual
    REC_STEPS = 7,     // steps covered
    REC_ABS_NEXT = 8,  // absorption increment of the current level
    REC_SRC_STEP = 9,  // source increment per step (constant)
    REC_HALF = 10,     // Heun: half of the first stage's mass increment
    REC_ABS_STAGE = 11,  // Heun: absorption increment of the intermediate level
    REC_LEN = 16
};

// Time schemes: forward Euler + donor cell; Heun + minmod-limited fluxes.
enum { SCHEME_EULER = 0, SCHEME_HEUN = 1 };
// Launch form of a forward-Euler step with separate kernels whose stencil runs over
// flat cell chunks (see kFlatCells); the scheme is Euler.
constexpr int SCHEME_EULER_FLAT = 3;

// Separate forward-Euler stencil over flat chunks of kFlatCells consecutive cells (512
// threads, 4 cells each): each ordinate's plane segment, with the row below or above it,
// is staged in LDS in rounds of 2048 floats, at most kFlatRounds.  Used when
// nx <= kFlatMaxNx.
constexpr int kFlatThreads = 512;
constexpr int kFlatCells = 4 * kFlatThreads;
constexpr int kFlatRounds = 3;
constexpr int kFlatMaxNx = kFlatRounds * kFlatCells - kFlatCells - 8;
// Heun passes in the same form: the limited stencil reads two rows on one side and one
// on the other, so the segment is kFlatCells + 3 nx + 8 floats.
constexpr int SCHEME_HEUN_FLAT = 4;
// Flat-chunk stencil blocks the chip keeps resident at once: 256 CUs x 2 blocks of
// 8 waves (at most 4 waves per SIMD at their register use, 48 KB of LDS each).
constexpr int kFlatResident = 512;
constexpr int kFlatMaxNxM = (kFlatRounds * kFlatCells - kFlatCells - 8) / 3;

// Banded forward-Euler step (product ordinate sets, FP32): one kernel per step does
// the contraction, the stream + collide update, the moments and the budget partials.
// A block owns kBandCells consecutive cells (flat index) and every ordinate: it walks
// the polar levels in order with a ring of 2 reach + 2 level slots in LDS, each slot
// kBandLead + n_az + kBandTrail azimuth rows (wrapped copies of the last kBandLead and
// the first kBandTrail azimuths around the n_az rows) of kBandStride floats (the cells
// plus one neighbour on each side, padded), and the current level's coefficients
// staged in LDS.  Lane (wave w, half h, cell c) produces azimuths (2 w + h) kBandO ..
// + kBandO - 1 of every level for cell c, so a block has n_az / (2 kBandO) waves.
// Level pairs coupling azimuths at most kBandNarrow apart are unrolled per width;
// wider ones run in steps of four offsets.
constexpr int SCHEME_EULER_BANDED = 5;
constexpr int kBandCells = 32;
constexpr int kBandO = 4;
constexpr int kBandNarrow = 8;
// Rows before azimuth 0 and after the last azimuth.  A narrow pair of width s reads
// the azimuths a0 - s .. a0 + kBandO - 1 + s of outputs a0 .. a0 + kBandO - 1, a wide
// step the rows m .. m + kBandO + 2 from a wrapped start m in [0, n_az).
constexpr int kBandLead = kBandNarrow;
constexpr int kBandTrail = kBandNarrow > kBandO + 2 ? kBandNarrow : kBandO + 2;
static_assert(kBandLead >= kBandNarrow && kBandTrail >= kBandNarrow && kBandTrail >= kBandO + 2,
              "banded ring rows must cover every narrow and wide read");
constexpr int kBandStride = 40;
constexpr int kBandMaxReach = 3;
// Azimuth counts with a kernel instance.
inline bool band_azimuths_supported(int az) { return az >= 8 && az <= 64 && az % 8 == 0; }
// Floats of one ring slot of the banded kernel.
inline int band_slot_floats(int az) { return (kBandLead + az + kBandTrail) * kBandStride; }
// The kernel's form of a pair code of band_form (asn_host.hpp), decoded on the host so the
// kernel spends few scalar instructions per pair:
//   bits 0-16   byte offset of the partner level's ring slot (level j sits in slot j mod
//               (2 reach + 2); at most 8 slots of (16 + 64) x 40 floats: < 2^17)
//   bits 17-23  start of the pair's run in the level's staged coefficients, in units of 4
//   bits 24-31  narrow run: its half-width s (<= kBandNarrow); wider run: kBandWideTag + s;
//               whole ring: kBandRingTag
constexpr uint32_t kBandWideTag = 32, kBandRingTag = 128;
inline uint32_t band_device_code(uint32_t code, int level, int reach, int az) {
    const int s = (int)(code & 63u), k = (int)((code >> 8) & 7u);
    const int j = level + k - reach;
    const uint32_t slot = (uint32_t)(j % (2 * reach + 2)) * (uint32_t)band_slot_floats(az) * 4u;
    const uint32_t w = (code & 128u) ? kBandRingTag : ((code & 64u) ? kBandWideTag + (uint32_t)s
                                                                     : (uint32_t)s);
    return slot | ((code >> 11) & 127u) << 17 | w << 24;
}
// Dynamic LDS of a banded block: the ring, then two level-coefficient buffers of cmax
// floats (cmax a multiple of 4) and two tables of the level's (cx, cy).
inline size_t band_lds_bytes(int az, int reach, int cmax) {
    return (size_t)(2 * reach + 2) * (kBandLead + az + kBandTrail) * kBandStride * 4 +
           2 * (size_t)((cmax + 1) & ~1) * 4 + 2 * (size_t)az * 8;
}

// Banded reduced-precision step (BF16 / FP16 operands on MFMA 16x16x32, FP32 accumulate)
// for product sets of 32, 48 or 64 azimuths: a block owns kBandLpCells consecutive cells and
// every ordinate; wave (m, n) produces azimuths 16 m .. 16 m + 15 of cells 16 n .. 16 n + 15.
// Per level pair (i, j) the circulant block of the stored K is multiplied as A operands
// of 16 x 32 (one per 16-azimuth offset, built on the host: band_lp_fragments) with the
// quantised partner level as B operand.
constexpr int kBandLpCells = 64;
constexpr int kBandLpMaxReach = 3;
inline bool band_lp_azimuths_supported(int az) { return az == 32 || az == 48 || az == 64; }
// k-steps of 32 azimuths a level pair takes (48 azimuths: two, the second half-padded)
__host__ __device__ constexpr int band_lp_ksteps(int az) { return (az + 31) / 32; }
__host__ __device__ constexpr int band_lp_threads(int az) { return (az / 16) * (kBandLpCells / 16) * 64; }
// 16-bit elements of a slot of the quantised-level ring (one level, one operand term): the
// 8-azimuth chunks of every k-step (the padding past n_az held at zero), each chunk the
// block's cells in a row ([chunk][cell][8]: 16 lanes reading one chunk of 16 cells read
// 256 contiguous bytes)
__host__ __device__ constexpr int band_lp_slot(int az) { return 4 * band_lp_ksteps(az) * kBandLpCells * 8; }
// Dynamic LDS of a banded reduced-precision block: the ring of 2 reach + 2 quantised
// levels (two operand terms for BF16), two buffers of a level's A operands (at most
// 2 reach + 1 pairs, n_az / 16 fragments of 1 KiB each, and the previous level's
// (cx, cy)), the ring of tile-edge values (reach + 3 levels).
inline size_t band_lp_lds_bytes(int az, int reach, int dtype) {
    const int terms = dtype == 1 ? 2 : 1, mt = az / 16, nt = kBandLpCells / 16;
    return (size_t)(2 * reach + 2) * terms * band_lp_slot(az) * 2 +
           (size_t)2 * ((2 * reach + 1) * mt * 1024 + az * 8) + (size_t)(reach + 3) * 2 * nt * az * 4;
}
// Largest dynamic LDS a block may take.
constexpr size_t kMaxBlockLds = 160 * 1024 - 1024;

// Modes of the budget kernel.
enum { BUD_STEP = 0, BUD_INIT = 1, BUD_STAGE1 = 2, BUD_STAGE2 = 3 };

// Cells per block of the reduced-precision operand scale: the default, and the range
// of powers of two a problem may choose (StepArgs::sb_log).  A block holds at least 64
// cells, so the 64 cells of one wave of the contraction's epilogue or of a flat-chunk
// stencil lie in one block.
constexpr int kScaleBlock = 256;
constexpr int kScaleBlockMin = 64;
constexpr int kScaleBlockMax = 4096;
// Blocks of 2^sb_log cells covering a plane of P cells.
__host__ __device__ inline int64_t scale_blocks(int64_t P, int sb_log) { return (P + (1 << sb_log) - 1) >> sb_log; }
// Scaled operands satisfy |x| < 2^(kScaleExp + 1).
constexpr int kScaleExp = 14;

// GEMM tiles (rows of K x cells x contraction step).
constexpr int kGemmBM = 128;
constexpr int kGemmBN = 128;

// Contraction depth per k-step: FP32 path and reduced-precision path.
constexpr int kBK_F32 = 16;
constexpr int kBK_LP = 32;

// Stencil tile: a strip of 62 updated columns (one wavefront of 64 lanes, the two
// outer lanes read the neighbouring columns) x 4 wavefronts x kRows rows each.
constexpr int kRows = 4;
constexpr int kStripX = 62;
// The limited (two-cell) stencil: 60 updated columns, two halo lanes per side.
constexpr int kStripXM = 60;
constexpr int kTileY = 4 * kRows;

struct StepArgs {
    // geometry
    int nx, ny, Q, Qp;
    int64_t C, P;  // cells, plane pitch (multiple of 256 cells)
    // stencil decomposition
    int G, qchunk, tiles_x, tiles_y;
    int fin_blocks;
    // operand type: 0 FP32, 1 BF16, 2 FP16
    int dtype;
    // log2 of the cells per block of the reduced-precision operand scale
    int sb_log;
    // 1: the stencil runs in the contraction's epilogue (forward Euler); the
    // stencil decomposition is then the contraction's: tiles_x = P / kGemmBN cell
    // tiles, tiles_y = 1, G = Qp / kGemmBM ordinate tiles
    int fused;
    double W, area;
    // buffers
    const float* psi;
    float* psi_new;
    float* Y;
    const float* Kt;        // FP32 K transposed, [Qp][Qp]
    const uint16_t* Klp;    // reduced-precision K, [Qp][Qp] row-major (K[m][k])
    const float* rdef;      // row defect of the reduced-precision K, [Qp]
    const int* ktab;        // per M-tile k-steps with a nonzero K tile: offsets[mtiles + 1],
                            // then the k-step indices (steps of kBK_F32 or kBK_LP ordinates)
    const QInfo* qi;
    const float4* coef;     // per cell {dt sigma_a, dt sigma_s, dt sigma_as, dt q}
    float* iso;             // Phi / W (FP32)
    double* phi64;          // Phi (FP64)
    double* phi_part;       // [G][P]
    double* blk_part;       // stencil block partials [G * tiles][2]
    double* fin_part;       // finalize block partials [fin_blocks][4]
    double* ypart;          // [Qp / kGemmBM][P] weighted row sums of Y (reduced precision)
    float* fix;             // [P] per-cell particle correction of the reduced-precision Y
    float* delta;           // [P] fused reduced precision: pending isotropic correction of the
                            // stored state (true state = psi + delta); iso then holds Phi^ / W
                            // of the stored state and phi64 the true Phi
    unsigned* bmax_cur;     // block max |psi^n| (read by the GEMM), follows the psi buffer
    unsigned* bmax_next;    // block max |psi^{n+1}| (written by the stencil)
    double* rec;
    // banded step (product ordinate sets): n_lev levels of n_az azimuths, coupling
    // levels up to `reach` apart; per level the descriptor (band, two uint4), the
    // coefficient range {first, count} (brange) and the coefficients (bcoef) as built by
    // band_form (asn_host.hpp); bcmax the largest count of a level
    const uint4* band;
    const int2* brange;
    const float* bcoef;
    int n_lev, n_az, reach, bcmax;
    // banded reduced-precision step: per level pair and 16-azimuth offset the A operand
    // of MFMA 16x16x32 as 64 lanes x 8 16-bit values (band_lp_fragments); band then holds
    // per level {pairs, first fragment, level offsets k of the pairs (4 bits each), 0}
    const uint4* bfrag;
};

// Kernel kinds of one step, each with its own block decomposition.
enum { KT_GEMM = 0, KT_FIX = 1, KT_SC = 2, KT_FIN = 3, KT_BUDGET = 4, KT_COUNT = 5 };

// Launch view of a batch of problems that share Q, K and the operand type.
// Every kernel covers all problems in one launch: block b of kernel kind k
// belongs to problem i with off[k * (n + 1) + i] <= b < off[k * (n + 1) + i + 1].
// tab[2 i + c] are the step arguments of problem i when psi buffer c holds its
// current state; at batch step s problem i uses c = base[i] ^ s_par.  A problem
// whose steps_left[i] is not positive is skipped (its blocks exit at once); the
// budget kernel decrements steps_left[i] after each step.  A single problem is a
// batch of one, so a problem computes bitwise the same alone and in a batch.
struct BatchArgs {
    const StepArgs* tab;
    const int* off;
    const int* base;
    int* steps_left;
    int n;
    int s_par;
};

// Blocks of each kernel kind for one problem.
void blocks_per_kind(const StepArgs& a, int out[KT_COUNT]);

// Whether a problem runs the stencil inside the FP32 contraction.
inline bool can_fuse(int dtype, int scheme) { (void)dtype; return scheme == SCHEME_EULER; }

// One step for every problem of the batch.  Euler: one pass of contraction,
// stream + collide, finalize and budget, on the buffers selected by b.s_par.
// Heun: two such passes (s_par 0, then 1), so the state returns to its buffer.
// If ev is given, ev[5 k .. 5 k + 4] are recorded before, between and after
// the four kernels of pass k.
// band_az / band_lds: the banded step's azimuth count and dynamic LDS bytes (every
// problem of a banded batch has that azimuth count); band_wide_rows: every problem's
// rows hold at least kBandWideRowCells cells (selects the FP32 banded kernel's instance
// that reads the y-upwind rows non-temporally); band_reach: the reach the banded
// reduced-precision kernel is instantiated for (at least every problem's).
hipError_t launch_step(const BatchArgs& b, const int* grid, int dtype, int scheme, hipStream_t s,
                       hipEvent_t* ev = nullptr, int band_az = 0, size_t band_lds = 0,
                       bool band_wide_rows = false, int band_reach = 0);
// Rows from this many cells on: the banded kernel's y-upwind row belongs to a block at
// least 32 blocks away, which runs about half a block's time apart on its XCD.
constexpr int kBandWideRowCells = 32 * kBandCells;
// Raise the dynamic LDS limit of the banded kernel for an azimuth count (once per device).
hipError_t prepare_banded(int band_az, size_t band_lds);
// The same for the banded reduced-precision kernel of an azimuth count, operand type
// and reach.
hipError_t prepare_banded_lp(int band_az, int dtype, int reach, size_t band_lds);
// Passes per step of a scheme.
inline int passes_per_step(int scheme) {
    return scheme == SCHEME_HEUN || scheme == SCHEME_HEUN_FLAT ? 2 : 1;
}
// Arm a batch: steps_left[i] = limit[i] and base[i] = cur[i], i < n <= kMaxArm.
constexpr int kMaxArm = 64;
struct ArmArgs {
    int limit[kMaxArm];
    int cur[kMaxArm];
};
hipError_t launch_arm(int* steps_left, int* base, int n, const ArmArgs& v, hipStream_t s);
// Moments of the current state (after set_state): phi64, iso, bmax, budget record.
hipError_t launch_init(const StepArgs& a, const BatchArgs& one, hipStream_t s);
// Fused reduced precision: fold the pending correction into the stored state.
hipError_t launch_materialize(const StepArgs& a, hipStream_t s);
// psi[q][c] = cell[c] for all q (pitch P), zero padding.
hipError_t launch_broadcast(float* psi, const float* cell, int Q, int64_t C, int64_t P,
                            hipStream_t s);

}  // namespace asn
