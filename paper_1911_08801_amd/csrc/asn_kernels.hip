// Device kernels of the explicit as-S_N step (gfx950, wave64).
//
// One step (paper Section 3.2, eq. asSNeq; forward Euler + donor cell, or the
// paper's Heun + minmod scheme of Section 3.1 as two such passes):
//   1. contraction  Y = K Psi  over ordinates, every cell      (MFMA, gemm_*)
//   2. stream + collide psi^{n+1} from psi^n, Y, Phi^n          (HBM, stream_collide)
//      also emits partial moments Phi^{n+1} and budget partials
//   3. finalize: Phi^{n+1} = sum of partials, Phi/W, mass partials
//   4. budget: one block folds the partials into the FP64 record
// All reductions have a fixed order (no floating-point atomics), so a step is
// bitwise reproducible.
#include "asn_kernels.hpp"

namespace asn {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Buffers are reached through pointers stored in the device argument table, which
// carry no address space; qualifying them as global keeps loads and stores on the
// global path (flat accesses would also tie up the LDS counter).
#if defined(__HIP_DEVICE_COMPILE__)
#define ASN_G __attribute__((address_space(1)))
#else
#define ASN_G
#endif
template <typename T>
__device__ __forceinline__ ASN_G T* gp(T* p) {
    return (ASN_G T*)p;
}

// Consecutive workgroups are dispatched round-robin over the 8 XCDs.  Map the
// hardware block id to a logical tile id so that logical neighbours share an
// XCD (and its L2): XCD x receives logical ids [start_x, start_x + count_x).
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
    constexpr int X = 8;
    const int per = nb / X, rem = nb % X;
    const int xcd = bid % X, slot = bid / X;
    return xcd * per + (xcd < rem ? xcd : rem) + slot;
}

// Problem i and its local block for hardware block b of kernel kind `kind`;
// false if that problem has no steps left in this batch.
__device__ __forceinline__ bool locate(const BatchArgs& B, int kind, int b, int& i, int& local) {
    const ASN_G int* off = gp(B.off) + kind * (B.n + 1);
    int lo = 0, hi = B.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    i = lo;
    local = b - off[lo];
    return gp(B.steps_left)[lo] > 0;
}

__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, off, 64));
    return v;
}

__device__ __forceinline__ StepArgs args_of(const BatchArgs& B, int i) {
    return gp(B.tab)[2 * i + (gp(B.base)[i] ^ B.s_par)];
}

// ---------------------------------------------------------------------------
// 1a. FP32 contraction Y[q][c] = sum_p K[q][p] psi[p][c] on MFMA 16x16x4 f32.
//     Block tile 128 (ordinates) x 128 (cells), k-step 16, 4 waves of 64x64.
//     Kt is K transposed and zero-padded to Qp x Qp; psi rows >= Q meet zero rows
//     of Kt.  Only k-steps whose K tile has a nonzero are visited, and in those
//     each wave multiplies only the 16-ordinate x 4 blocks of its 64 rows that
//     have one.  The products are taken with the operands swapped (Y^T = Psi^T
//     K^T), so each lane's accumulator holds four consecutive cells of one
//     ordinate: Y is stored as float4 rows.
//     FUSED: the forward-Euler stream + collide update is applied in the
//     epilogue instead of storing Y: the lane reads the old values and upwind
//     neighbours of its cells as aligned float4 rows, writes psi^{n+1} as a float4
//     (two cell groups, the halves of one 128-byte line, stored together), and
//     the block emits the Phi partial of its 128 ordinates for its 128 cells
//     plus its budget partials.  Y never reaches memory.
// ---------------------------------------------------------------------------
constexpr int kBK = kBK_F32;
constexpr int kLdsPad = 16;

template <int NV, typename OutPtr>
__device__ __forceinline__ void block_sum_256(double (&v)[NV], OutPtr out);

#ifndef ASN_F32_FUSED_WAVES
#define ASN_F32_FUSED_WAVES 2
#endif
// The fused epilogue needs more registers (two resident blocks per CU); the plain
// contraction fits four, whose loads then hide behind the others' products.
template <bool FUSED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FUSED ? ASN_F32_FUSED_WAVES : 4)))
void gemm_f32_kernel(BatchArgs B) {
    __shared__ float As[2][kBK][kGemmBM + kLdsPad];
    __shared__ float Bs[2][kBK][kGemmBN + kLdsPad];
    int pi, tile;
    if (!locate(B, KT_GEMM, xcd_remap(blockIdx.x, gridDim.x), pi, tile)) return;
    const StepArgs a = args_of(B, pi);   // by value: no reloads after stores
    const ASN_G float* __restrict__ Kt = gp(a.Kt);
    const ASN_G float* __restrict__ psi = gp(a.psi);
    ASN_G float* __restrict__ Y = gp(a.Y);
    const ASN_G int* __restrict__ ktab = gp(a.ktab);
    const int Q = a.Q, Qp = a.Qp;
    const int64_t P = a.P;
    const int mtiles = Qp / kGemmBM;
    const int mt = tile % mtiles;
    const int nt = tile / mtiles;
    const int m0 = mt * kGemmBM;
    const int64_t n0 = (int64_t)nt * kGemmBN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;

    // Staging of one k-step (kBK ordinates): thread t moves float4 number t + 256 r
    // (r < kBK / 8) of the A tile (Kt rows) and of the B tile (psi rows).  Steps past
    // row Q - 1 of psi read that row again: the matching rows of Kt are zero, so they
    // add exact zeros (a conditional overwrite of the loaded value would make the
    // wait for it count all loads in flight).
    constexpr int kNR = kBK / 8;
    const int kk0 = tid >> 5, c4 = (tid & 31) << 2;
#define ASN_GL1(S, r, k0)                                                                      \
    do {                                                                                       \
        const int ka = (k0) + kk0 + 8 * (r);                                                   \
        ra##S##r = *reinterpret_cast<const ASN_G float4*>(Kt + (size_t)ka * Qp + m0 + c4);     \
        rb##S##r = *reinterpret_cast<const ASN_G float4*>(psi + (size_t)min(ka, Q - 1) * P + n0 + c4); \
    } while (0)
#define ASN_LS1(S, r, b)                                                                       \
    do {                                                                                       \
        *reinterpret_cast<float4*>(&As[b][kk0 + 8 * (r)][c4]) = ra##S##r;                      \
        *reinterpret_cast<float4*>(&Bs[b][kk0 + 8 * (r)][c4]) = rb##S##r;                      \
    } while (0)
    static_assert(kNR == 2, "staging of 16-row k-steps");
    // register set X, and (plain contraction) set Y for a second step in flight
    float4 raX0, raX1, rbX0, rbX1, raY0, raY1, rbY0, rbY1;
    auto gloadX = [&](int k0) { ASN_GL1(X, 0, k0); ASN_GL1(X, 1, k0); };
    auto gloadY = [&](int k0) { ASN_GL1(Y, 0, k0); ASN_GL1(Y, 1, k0); };
    auto lstoreX = [&](int b) { ASN_LS1(X, 0, b); ASN_LS1(X, 1, b); };
    auto lstoreY = [&](int b) { ASN_LS1(Y, 0, b); ASN_LS1(Y, 1, b); };
#undef ASN_GL1
#undef ASN_LS1

    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // Only k-steps whose K tile has a nonzero entry, and in those only the 16 x 4 operand
    // blocks of the wave with a nonzero entry (the skipped products are +0).
    const ASN_G int* __restrict__ klist = ktab + (mtiles + 1) + ktab[mt];
    const ASN_G int* __restrict__ mlist = klist + ktab[mtiles];
    const int nkt = ktab[mt + 1] - ktab[mt];
    // products of visited step kt from LDS buffer b (none for kt = nkt, the padding
    // step of an odd count)
    // mask of visited step kt (0 for the padding step kt = nkt)
    auto step_mask = [&](int kt) { return kt < nkt ? (unsigned)mlist[kt] : 0u; };
    auto mma = [&](unsigned m, int b) {
        // this wave's 64 ordinates: bit 4 i + g for sub-block i and k-group g (4 k each)
        // (wave-uniform: kept in a scalar register, tested with scalar branches)
        const unsigned wmask =
            (unsigned)__builtin_amdgcn_readfirstlane((int)((m >> (16 * (wave & 1))) & 0xFFFFu));
#pragma unroll
        for (int kk = 0; kk < kBK; kk += 4) {
            float av[4], bv[4];
            const int kr = kk + (lane >> 4), cl = lane & 15;
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = As[b][kr][wm + i * 16 + cl];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = Bs[b][kr][wn + j * 16 + cl];
            // rows = cells (bv), columns = ordinates (av): acc[i][j] holds cells block i of
            // ordinate block j, four consecutive cells of one ordinate per lane
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (wmask & (1u << (4 * j + kk / 4)))
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[i], av[j], acc[i][j], 0, 0, 0);
        }
    };
    if constexpr (FUSED) {
        // one step in flight: loaded during the products of the previous one
        if (nkt > 0) {
            gloadX(klist[0] * kBK);
            lstoreX(0);
        }
        __syncthreads();
        for (int kt = 0; kt < nkt; ++kt) {
            const int b = kt & 1;
            if (kt + 1 < nkt) gloadX(klist[kt + 1] * kBK);
            mma(step_mask(kt), b);
            if (kt + 1 < nkt) lstoreX(b ^ 1);
            __syncthreads();
        }
    } else {
        // two steps in flight: set X holds even steps, set Y odd ones; a step's
        // registers are loaded two product phases before they go to LDS.  The loop is
        // entered, and goes round, with both sets in flight, the one stored next the
        // older, and has no conditional store or exit, so every wait counts only the
        // older set.  Loads past the last step repeat it; an odd count ends with a
        // padding step that multiplies nothing.
        // The step numbers and masks (scalar loads) are fetched one use ahead, so no
        // step waits on a scalar load issued in it.
        if (nkt > 0) {
            gloadX(klist[0] * kBK);
            gloadY(klist[min(1, nkt - 1)] * kBK);
        }
        int kx = klist[min(2, max(nkt - 1, 0))], ky = klist[min(3, max(nkt - 1, 0))];
        unsigned mx = step_mask(0), my = step_mask(1);
        for (int kt = 0; kt < nkt; kt += 2) {
            lstoreX(0);
            __syncthreads();
            gloadX(kx * kBK);
            kx = klist[min(kt + 4, nkt - 1)];
            mma(mx, 0);
            mx = step_mask(kt + 2);
            lstoreY(1);
            __syncthreads();
            gloadY(ky * kBK);
            ky = klist[min(kt + 5, nkt - 1)];
            mma(my, 1);
            my = step_mask(kt + 3);
        }
    }
    // D layout of the 16x16 MFMA: lane holds rows 4 (lane / 16) + v, column lane % 16, so
    // acc[i][j] is cells n0 + wn + 16 i + 4 (lane / 16) + v of ordinate m0 + wm + 16 j +
    // lane % 16.
    if constexpr (!FUSED) {
        // one float4 store per cell group; groups i and i + 1 (the halves of a 128-byte
        // line of the ordinate's row) back to back
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int q = m0 + wm + j * 16 + (lane & 15);
            if (q < Q) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t c0 = n0 + wn + i * 16 + 4 * (lane >> 4);
                    *reinterpret_cast<ASN_G float4*>(Y + (size_t)q * P + c0) =
                        make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
                }
            }
        }
    } else {
        const int nx = a.nx, ny = a.ny;
        const int64_t C = a.C;
        const ASN_G QInfo* __restrict__ qtab = gp(a.qi);
        const ASN_G float* __restrict__ isop = gp(a.iso);
        const ASN_G float4* __restrict__ coef = gp(a.coef);
        ASN_G float* __restrict__ out = gp(a.psi_new);
        const bool rows4 = (nx & 3) == 0;   // then a float4 of cells never crosses a grid row
        // The lane's four ordinates (columns j).  Padding ordinates (q >= Q) read row 0
        // and store nothing.
        QInfo qi[4];
        bool qok[4];
        const ASN_G float* rowp[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int q = m0 + wm + j * 16 + (lane & 15);
            qok[j] = q < Q;
            qi[j] = qtab[qok[j] ? q : 0];
            rowp[j] = psi + (size_t)(qok[j] ? q : 0) * P;
        }
        __shared__ double phred[2][kGemmBN];
        double defect = 0.0, outflow = 0.0;
        float4 held[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            // four consecutive cells c0 .. c0 + 3 (c0 a multiple of 4, c0 + 3 < P)
            const int64_t c0 = n0 + wn + i * 16 + 4 * (lane >> 4);
            // All loads of this cell group first, at clamped in-range addresses, so that
            // they are in flight together; ghost and padding values are masked below.
            const float4 iso4 = *reinterpret_cast<const ASN_G float4*>(isop + c0);
            float4 cf[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) cf[k] = coef[c0 + k];
            float4 v4[4], u4[4];
            float xs[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const ASN_G float* row = rowp[j];
                v4[j] = *reinterpret_cast<const ASN_G float4*>(row + c0);
                // the x-upwind cell outside the float4: just before (xi > 0) or after it
                const int64_t xi = (qi[j].dir & 1) ? c0 - 1 : c0 + 4;
                xs[j] = row[min(max(xi, (int64_t)0), P - 1)];
                // the y-upwind row: below (eta > 0) or above; one aligned float4 when nx
                // is a multiple of 4, else four scalars
                const int64_t yi = c0 + ((qi[j].dir & 4) ? -(int64_t)nx : (int64_t)nx);
                if (rows4) {
                    u4[j] = *reinterpret_cast<const ASN_G float4*>(row + min(max(yi, (int64_t)0), P - 4));
                } else {
                    u4[j].x = row[min(max(yi, (int64_t)0), P - 1)];
                    u4[j].y = row[min(max(yi + 1, (int64_t)0), P - 1)];
                    u4[j].z = row[min(max(yi + 2, (int64_t)0), P - 1)];
                    u4[j].w = row[min(max(yi + 3, (int64_t)0), P - 1)];
                }
            }
            // Per cell: live (a grid cell, not padding) and its boundary faces as the bits
            // of the direction code (bit0 x = 0, bit1 x = nx - 1, bit2 y = 0, bit3
            // y = ny - 1): the upwind neighbour of ordinate class d is a ghost where
            // d & in_edge != 0 and the cell has an outflow face where d & out_edge != 0.
            int in_edge[4], out_edge[4];
            bool ck[4];
            {
                const int y0 = (int)(c0 / nx);
                int x = (int)(c0 - (int64_t)y0 * nx), y = y0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    ck[k] = c0 + k < C;
                    const int e = (x == 0 ? 1 : 0) | (x == nx - 1 ? 2 : 0) | (y == 0 ? 4 : 0) |
                                  (y == ny - 1 ? 8 : 0);
                    in_edge[k] = e;
                    out_edge[k] = ((e & 5) << 1) | ((e & 10) >> 1);
                    x = x + 1 == nx ? 0 : x + 1;
                    y = x == 0 ? y + 1 : y;
                }
            }
            const float isv[4] = {iso4.x, iso4.y, iso4.z, iso4.w};
            double ph[4] = {0.0, 0.0, 0.0, 0.0};
            // An interior group (four live cells off the domain boundary) needs no ghost,
            // padding or outflow handling.
            bool interior = true;
#pragma unroll
            for (int k = 0; k < 4; ++k) interior = interior && ck[k] && in_edge[k] == 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const QInfo& qj = qi[j];
                const int d = qj.dir;
                const float vv[4] = {v4[j].x, v4[j].y, v4[j].z, v4[j].w};
                const float uu[4] = {u4[j].x, u4[j].y, u4[j].z, u4[j].w};
                const float lft[4] = {xs[j], vv[0], vv[1], vv[2]};
                const float rgt[4] = {vv[1], vv[2], vv[3], xs[j]};
                float nv[4];
                float colsum = 0.f, o = 0.f;
                if (interior) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        // (cx = 0 when d & 3 = 0 and cy = 0 when d & 12 = 0)
                        const float ux = (d & 1) ? lft[k] : rgt[k];
                        const float v = vv[k];
                        const float col = cf[k].z * (acc[i][j][k] - v) + cf[k].y * (isv[k] - v);
                        nv[k] = v - qj.cx * (v - ux) - qj.cy * (v - uu[k]) - cf[k].x * v + col + cf[k].w;
                        colsum += col;
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int gi = d & in_edge[k], go = d & out_edge[k];
                        const float ux = (gi & 3) ? 0.f : ((d & 1) ? lft[k] : rgt[k]);
                        const float uy = (gi & 12) ? 0.f : uu[k];
                        const float v = vv[k];
                        const float col = cf[k].z * (acc[i][j][k] - v) + cf[k].y * (isv[k] - v);
                        const float r = v - qj.cx * (v - ux) - qj.cy * (v - uy) - cf[k].x * v + col + cf[k].w;
                        nv[k] = ck[k] ? r : 0.f;   // padding cells stay zero
                        colsum += ck[k] ? col : 0.f;
                        o += ck[k] ? ((go & 3) ? qj.cx * v : 0.f) + ((go & 12) ? qj.cy * v : 0.f) : 0.f;
                    }
                }
                const double wj = qok[j] ? qj.w : 0.0;   // padding ordinates add nothing
#pragma unroll
                for (int k = 0; k < 4; ++k) ph[k] += wj * (double)nv[k];
                // Groups i and i + 1 are the two halves of a 128-byte line of the row: the
                // even group's result is held and both are stored together.
                const float4 res = make_float4(nv[0], nv[1], nv[2], nv[3]);
                if ((i & 1) == 0) {
                    held[j] = res;
                } else if (qok[j]) {
                    ASN_G float* o = out + (size_t)(m0 + wm + j * 16 + (lane & 15)) * P + c0;
                    *reinterpret_cast<ASN_G float4*>(o - 16) = held[j];
                    *reinterpret_cast<ASN_G float4*>(o) = res;
                }
                defect += wj * (double)colsum;
                outflow += wj * (double)o;
            }
            // Phi partial of this wave's 64 ordinates: the 16 lanes of a row group
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ph[k] += __shfl_xor(ph[k], 1, 64);
                ph[k] += __shfl_xor(ph[k], 2, 64);
                ph[k] += __shfl_xor(ph[k], 4, 64);
                ph[k] += __shfl_xor(ph[k], 8, 64);
                if ((lane & 15) == 0) phred[wave & 1][wn + i * 16 + 4 * (lane >> 4) + k] = ph[k];
            }
        }
        // then the two waves that share the cells (fixed order)
        double sums[2] = {defect, outflow};
        block_sum_256<2>(sums, gp(a.blk_part) + 2 * (size_t)tile);   // synchronises the block
        if (tid < kGemmBN)
            gp(a.phi_part)[(size_t)mt * P + n0 + tid] = phred[0][tid] + phred[1][tid];
    }
}

// ---------------------------------------------------------------------------
// 1b. Reduced-precision contraction (BF16 or FP16 operands, FP32 accumulate) on
//     MFMA 16x16x32.  Only the anisotropic part of psi is rounded:
//       iso_c = Phi_c / W,  dev = psi - iso,  s = dev * 2^(E - e_b)
//       x = T(s) for FP16; for BF16 x = hi + lo, hi = T(s), lo = T(s - hi), two
//       MFMAs per k-step (a single BF16 term biases quasi-steady regions)
//       Y = iso + 2^(e_b - E) (T(K) x) + r_q dev,   r_q = 1 - sum_p T(K)_qp
//     with e_b the exponent of the block max |psi| over 256 cells (the N tile
//     lies inside one such block).  The epilogue also writes, per cell, the
//     w-weighted sum of this tile's Y rows (FP64) for the per-cell particle fix
//     applied in stream + collide.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int kBKL = kBK_LP;
constexpr int kRowL = kBKL + 8;  // LDS row length in 16-bit elements (padded)

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// Two FP32 values rounded to nearest even in the operand type, packed (lo in bits
// 0..15): one v_cvt_pk_bf16_f32 / v_cvt_pk_f16_f32 on gfx950.
template <int DT>
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    const f32x2_t w = {lo, hi};
    if constexpr (DT == 1) return __builtin_bit_cast(uint32_t, __builtin_convertvector(w, bf16x2_t));
    else return __builtin_bit_cast(uint32_t, __builtin_convertvector(w, f16x2_t));
}

// BF16 residual terms of a packed pair p = pack2<1>(lo, hi): s - T(s) is exact in FP32;
// the residuals are rounded to BF16 and packed as well.
__device__ __forceinline__ uint32_t bf16_residual2(uint32_t p, float lo, float hi) {
    return pack2<1>(lo - __uint_as_float(p << 16), hi - __uint_as_float(p & 0xFFFF0000u));
}

template <int DT>
__device__ __forceinline__ f32x4 mfma_lp(const uint4& av, const uint4& bv, const f32x4& c) {
    if constexpr (DT == 1)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                       __builtin_bit_cast(bf16x8, bv), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, av),
                                                      __builtin_bit_cast(f16x8, bv), c, 0, 0, 0);
}

template <int DT, bool FUSED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((FUSED || DT == 1) ? 2 : 3, 3)))
void gemm_lp_kernel(BatchArgs B) {
    __shared__ __attribute__((aligned(16))) uint16_t As[2][kGemmBM][kRowL];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][kGemmBN][kRowL];
    __shared__ __attribute__((aligned(16))) uint16_t Bl[DT == 1 ? 2 : 1][DT == 1 ? kGemmBN : 1][kRowL];
    __shared__ double red[2][kGemmBN];
    __shared__ double yred[FUSED ? 2 : 1][FUSED ? kGemmBN : 1];
    int pi, tile;
    if (!locate(B, KT_GEMM, xcd_remap(blockIdx.x, gridDim.x), pi, tile)) return;
    const StepArgs a = args_of(B, pi);   // by value: no reloads after stores
    const ASN_G uint16_t* __restrict__ Klp = gp(a.Klp);
    const ASN_G float* __restrict__ psi = gp(a.psi);
    const ASN_G float* __restrict__ iso = gp(a.iso);
    const ASN_G float* __restrict__ rdef = gp(a.rdef);
    const ASN_G QInfo* __restrict__ qinfo = gp(a.qi);
    const ASN_G int* __restrict__ ktab = gp(a.ktab);
    ASN_G float* __restrict__ Yo = gp(a.Y);
    ASN_G double* __restrict__ ypart = gp(a.ypart);
    const int mtiles = a.Qp / kGemmBM;
    const int mt = tile % mtiles;
    const int nt = tile / mtiles;
    const int m0 = mt * kGemmBM;
    const int64_t n0 = (int64_t)nt * kGemmBN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
    const int Q = a.Q, Qp = a.Qp;
    const int64_t P = a.P;

    // Operand scale 2^(E - e_b) of scale block b (at least 64 cells): the four cells a
    // thread stages (n0 + 4 cg ..) lie in one block, and so do the 64 output cells of a
    // wave (n0 + wn ..); with blocks of 128 or more the tile has one scale.
    auto block_exp = [&](int64_t c) {
        const float bm = __uint_as_float(gp(a.bmax_cur)[c >> a.sb_log]);
        int e = 0;
        if (bm > 0.f) (void)frexpf(bm, &e);
        return max(e, -100);
    };
    const float s_in = ldexpf(1.f, kScaleExp - block_exp(n0 + 4 * (tid & 31)));
    const float s_out = ldexpf(1.f, block_exp(n0 + __builtin_amdgcn_readfirstlane(wn)) - kScaleExp);

    // Staging of one k-step (32 ordinates).  A: thread t moves 16-byte pieces t and
    // t + 256 of the T(K) tile.  B: thread t loads ordinates k0 + 4 kg .. + 3 of cells
    // n0 + 4 cg .. + 3 (four float4), subtracts iso, scales, rounds, and writes each
    // cell's four values as one 8-byte group of its LDS row.
    const int arow0 = tid >> 2, arow1 = arow0 + 64, akq = (tid & 3) * 8;
    const int cg = tid & 31, kg = tid >> 5;
    const float4 iso4 = *reinterpret_cast<const ASN_G float4*>(iso + n0 + 4 * cg);
    uint4 ra0, ra1;
    float4 rb[4];
#define ASN_GLOAD_LP(k0)                                                                       \
    do {                                                                                       \
        ra0 = *reinterpret_cast<const ASN_G uint4*>(Klp + (size_t)(m0 + arow0) * Qp + (k0) + akq); \
        ra1 = *reinterpret_cast<const ASN_G uint4*>(Klp + (size_t)(m0 + arow1) * Qp + (k0) + akq); \
        _Pragma("unroll") for (int j = 0; j < 4; ++j) {                                        \
            const int kr = (k0) + 4 * kg + j;                                                  \
            rb[j] = *reinterpret_cast<const ASN_G float4*>(psi + (size_t)min(kr, Q - 1) * P +  \
                                                           n0 + 4 * cg);                       \
            if (kr >= Q) rb[j] = iso4; /* T(K) is zero there; keep the operand finite */       \
        }                                                                                      \
    } while (0)
    auto lstore = [&](int b) {
        *reinterpret_cast<uint4*>(&As[b][arow0][akq]) = ra0;
        *reinterpret_cast<uint4*>(&As[b][arow1][akq]) = ra1;
        // (v - iso) 2^(E - e_b): the scale is a power of two, so one FMA with the
        // scaled iso rounds exactly as the difference would
        const float ivs[4] = {iso4.x * s_in, iso4.y * s_in, iso4.z * s_in, iso4.w * s_in};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            float x[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float v = c == 0 ? rb[j].x : c == 1 ? rb[j].y : c == 2 ? rb[j].z : rb[j].w;
                x[j] = __builtin_fmaf(v, s_in, -ivs[c]);
            }
            uint2 pk;
            pk.x = pack2<DT>(x[0], x[1]);
            pk.y = pack2<DT>(x[2], x[3]);
            *reinterpret_cast<uint2*>(&Bs[b][4 * cg + c][4 * kg]) = pk;
            if constexpr (DT == 1) {
                uint2 pl;
                pl.x = bf16_residual2(pk.x, x[0], x[1]);
                pl.y = bf16_residual2(pk.y, x[2], x[3]);
                *reinterpret_cast<uint2*>(&Bl[b][4 * cg + c][4 * kg]) = pl;
            }
        }
    };

    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // Only k-steps whose T(K) tile has a nonzero entry (whole tiles are multiplied:
    // tests per operand block cost more issue slots than the products they skip).
    const ASN_G int* __restrict__ klist = ktab + (mtiles + 1) + ktab[mt];
    const int nkt = ktab[mt + 1] - ktab[mt];
    if (nkt > 0) {
        ASN_GLOAD_LP(klist[0] * kBKL);
        lstore(0);
    }
    __syncthreads();
    for (int kt = 0; kt < nkt; ++kt) {
        const int b = kt & 1;
        if (kt + 1 < nkt) ASN_GLOAD_LP(klist[kt + 1] * kBKL);
        const int r16 = lane & 15, kofs = 8 * (lane >> 4);
        uint4 av[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = *reinterpret_cast<const uint4*>(&As[b][wm + i * 16 + r16][kofs]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint4 bv = *reinterpret_cast<const uint4*>(&Bs[b][wn + j * 16 + r16][kofs]);
            // FUSED: rows = cells (bv), columns = ordinates (av): acc[cell block][ordinate block]
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if constexpr (FUSED) acc[j][i] = mfma_lp<DT>(bv, av[i], acc[j][i]);
                else acc[i][j] = mfma_lp<DT>(av[i], bv, acc[i][j]);
            }
            if constexpr (DT == 1) {
                const uint4 bl = *reinterpret_cast<const uint4*>(&Bl[b][wn + j * 16 + r16][kofs]);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if constexpr (FUSED) acc[j][i] = mfma_lp<DT>(bl, av[i], acc[j][i]);
                    else acc[i][j] = mfma_lp<DT>(av[i], bl, acc[i][j]);
                }
            }
        }
        if (kt + 1 < nkt) lstore(b ^ 1);
        __syncthreads();
    }
#undef ASN_GLOAD_LP

    if constexpr (!FUSED) {
    double part[4] = {0.0, 0.0, 0.0, 0.0};
    #pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t n = n0 + wn + j * 16 + (lane & 15);
            const float iso_n = iso[n];
    #pragma unroll
            for (int i = 0; i < 4; ++i)
    #pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int m = m0 + wm + i * 16 + 4 * (lane >> 4) + v;
                    if (m < Q) {
                        const float dev = psi[(size_t)m * P + n] - iso_n;
                        const float y = iso_n + s_out * acc[i][j][v] + rdef[m] * dev;
                        Yo[(size_t)m * P + n] = y;
                        part[j] += qinfo[m].w * (double)y;
                    }
                }
            part[j] += __shfl_xor(part[j], 16, 64);
            part[j] += __shfl_xor(part[j], 32, 64);
            if (lane < 16) red[wave & 1][wn + j * 16 + lane] = part[j];
        }
        __syncthreads();
        if (tid < kGemmBN) ypart[(size_t)mt * P + n0 + tid] = red[0][tid] + red[1][tid];
    } else {
        // Stream + collide with the stored state psi^ and the per-cell pending particle
        // correction delta: the true state is psi^ + delta (delta is isotropic, so it
        // drops out of the quantised deviation psi^ - iso^; iso^ = Phi^ / W).
        //   Y^  = (iso^ + delta) + 2^(e - E) T(K) x + r_q (psi^ - iso^)
        //   new = psi - cx (psi - up_x) - cy (psi - up_y) - dt sigma_a psi + col^ + dt q
        //   col^ = dt sigma_as (Y^ - psi) + dt sigma_s (iso - psi)
        // The block writes psi^{n+1} without its own correction and the per-cell
        // partials of Phi^, of sum_q w_q Y^ (for the next correction) and the budget.
        const int nx = a.nx, ny = a.ny;
        const int64_t C = a.C;
        ASN_G float* __restrict__ out = gp(a.psi_new);
        const ASN_G float* __restrict__ dl = gp(a.delta);
        const bool rows4 = (nx & 3) == 0;
        float rq[4], cxq[4], cyq[4];
        int dq[4];
        double wq[4];
        bool qok[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int q = m0 + wm + j * 16 + (lane & 15);
            qok[j] = q < Q;
            const QInfo qi = qinfo[qok[j] ? q : 0];
            rq[j] = rdef[qok[j] ? q : 0];
            cxq[j] = qi.cx;
            cyq[j] = qi.cy;
            dq[j] = qi.dir;
            wq[j] = qi.w;
        }
        double defect = 0.0, outflow = 0.0;
        float mx = 0.f;
        const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
        float4 held[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t c0 = n0 + wn + i * 16 + 4 * (lane >> 4);
            // Groups i and i + 1 are the two halves of a 128-byte line of the row: the
            // even group's result is held and both are stored together.
            auto emit = [&](int j, int q, const float4& res) {
                if ((i & 1) == 0) {
                    held[j] = res;
                } else {
                    ASN_G float* o = out + (size_t)q * P + c0;
                    *reinterpret_cast<ASN_G float4*>(o - 16) = held[j];
                    *reinterpret_cast<ASN_G float4*>(o) = res;
                }
            };
            float aa[4], bs[4], gs[4], ss[4];
            int xk[4], yk[4];
            bool ck[4];
            const float4 ih4 = *reinterpret_cast<const ASN_G float4*>(iso + c0);
            const float4 d4 = *reinterpret_cast<const ASN_G float4*>(dl + c0);
            const float ihv[4] = {ih4.x, ih4.y, ih4.z, ih4.w};
            const float dv[4] = {d4.x, d4.y, d4.z, d4.w};
            {
                const int y0 = (int)(c0 / nx);
                int x = (int)(c0 - (int64_t)y0 * nx), y = y0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    ck[k] = c0 + k < C;
                    xk[k] = x;
                    yk[k] = y;
                    if (++x == nx) {
                        x = 0;
                        ++y;
                    }
                    const float4 cf = ck[k] ? gp(a.coef)[c0 + k] : z4;
                    aa[k] = cf.x;
                    bs[k] = cf.y;
                    gs[k] = cf.z;
                    ss[k] = cf.w;
                }
            }
            // pending corrections of the neighbouring cells
            const float dprev = c0 >= 4 ? dl[c0 - 1] : 0.f;
            const float dnext = c0 + 4 < P ? dl[c0 + 4] : 0.f;
            double ph[4] = {0.0, 0.0, 0.0, 0.0}, yp[4] = {0.0, 0.0, 0.0, 0.0};
            // An interior group (four live cells of one grid row, off the domain
            // boundary) needs no ghost, padding or outflow handling.
            const bool interior = ck[3] && xk[0] >= 1 && xk[3] == xk[0] + 3 && xk[3] <= nx - 2 &&
                                  yk[0] >= 1 && yk[0] <= ny - 2;
            if (interior) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (!qok[j]) continue;
                const int q = m0 + wm + j * 16 + (lane & 15);
                const ASN_G float* row = psi + (size_t)q * P;
                const float4 v4 = *reinterpret_cast<const ASN_G float4*>(row + c0);
                const float vh[4] = {v4.x, v4.y, v4.z, v4.w};
                // x-upwind value outside the group (before it for xi > 0, else after it)
                // and the y-upwind row; for xi = 0 (eta = 0) cx (cy) is 0 and any finite
                // value serves
                const bool xp = dq[j] & 1;
                const float xsv = row[xp ? c0 - 1 : c0 + 4] + (xp ? dprev : dnext);
                const int64_t sh = (dq[j] & 4) ? -(int64_t)nx : (int64_t)nx;
                float uy[4];
                if (rows4) {
                    const float4 u4 = *reinterpret_cast<const ASN_G float4*>(row + c0 + sh);
                    const float4 e4 = *reinterpret_cast<const ASN_G float4*>(dl + c0 + sh);
                    uy[0] = u4.x + e4.x;
                    uy[1] = u4.y + e4.y;
                    uy[2] = u4.z + e4.z;
                    uy[3] = u4.w + e4.w;
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) uy[k] = row[c0 + k + sh] + dl[c0 + k + sh];
                }
                float tv[4];   // true state psi^ + delta
#pragma unroll
                for (int k = 0; k < 4; ++k) tv[k] = vh[k] + dv[k];
                const float lft[4] = {xsv, tv[0], tv[1], tv[2]};
                const float rgt[4] = {tv[1], tv[2], tv[3], xsv};
                float nv[4];
                float colsum = 0.f;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float v = tv[k];
                    const float ux = xp ? lft[k] : rgt[k];
                    const float dev = vh[k] - ihv[k];
                    const float ya = s_out * acc[i][j][k] + rq[j] * dev;   // Y^ - iso
                    const float col = gs[k] * ((ihv[k] + ya) - vh[k]) + bs[k] * (ihv[k] - vh[k]);
                    nv[k] = v - cxq[j] * (v - ux) - cyq[j] * (v - uy[k]) - aa[k] * v + col + ss[k];
                    ph[k] += wq[j] * (double)nv[k];
                    yp[k] += wq[j] * ((double)(ihv[k] + dv[k]) + (double)ya);
                    colsum += col;
                    mx = fmaxf(mx, fabsf(nv[k]));
                }
                emit(j, q, make_float4(nv[0], nv[1], nv[2], nv[3]));
                defect += wq[j] * (double)colsum;
            }
            } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (!qok[j]) continue;
                const int q = m0 + wm + j * 16 + (lane & 15);
                const ASN_G float* row = psi + (size_t)q * P;
                const float4 v4 = *reinterpret_cast<const ASN_G float4*>(row + c0);
                const float vh[4] = {v4.x, v4.y, v4.z, v4.w};
                float ux[4] = {0.f, 0.f, 0.f, 0.f};
                if (dq[j] & 1) {
                    ux[0] = (c0 >= 4 ? row[c0 - 1] : 0.f) + dprev;
#pragma unroll
                    for (int k = 1; k < 4; ++k) ux[k] = vh[k - 1] + dv[k - 1];
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (xk[k] == 0) ux[k] = 0.f;
                } else if (dq[j] & 2) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) ux[k] = vh[k + 1] + dv[k + 1];
                    ux[3] = (c0 + 4 < P ? row[c0 + 4] : 0.f) + dnext;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (xk[k] == nx - 1) ux[k] = 0.f;
                }
                float uy[4] = {0.f, 0.f, 0.f, 0.f};
                if (dq[j] & 12) {
                    const int64_t sh = (dq[j] & 4) ? -(int64_t)nx : (int64_t)nx;
                    if (rows4) {
                        const bool has = (dq[j] & 4) ? yk[0] > 0 : yk[0] < ny - 1;
                        if (has && ck[0]) {
                            const float4 u4 = *reinterpret_cast<const ASN_G float4*>(row + c0 + sh);
                            const float4 e4 = *reinterpret_cast<const ASN_G float4*>(dl + c0 + sh);
                            uy[0] = u4.x + e4.x;
                            uy[1] = u4.y + e4.y;
                            uy[2] = u4.z + e4.z;
                            uy[3] = u4.w + e4.w;
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const bool has = ck[k] && ((dq[j] & 4) ? yk[k] > 0 : yk[k] < ny - 1);
                            uy[k] = has ? row[c0 + k + sh] + dl[c0 + k + sh] : 0.f;
                        }
                    }
                }
                float nv[4];
                float colsum = 0.f, o = 0.f;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float v = vh[k] + dv[k];
                    const float dev = vh[k] - ihv[k];
                    const float ya = s_out * acc[i][j][k] + rq[j] * dev;   // Y^ - iso
                    const float col = gs[k] * ((ihv[k] + ya) - vh[k]) + bs[k] * (ihv[k] - vh[k]);
                    const float r = v - cxq[j] * (v - ux[k]) - cyq[j] * (v - uy[k]) - aa[k] * v + col + ss[k];
                    nv[k] = ck[k] ? r : 0.f;
                    ph[k] += wq[j] * (double)nv[k];
                    yp[k] += ck[k] ? wq[j] * ((double)(ihv[k] + dv[k]) + (double)ya) : 0.0;
                    colsum += ck[k] ? col : 0.f;
                    mx = fmaxf(mx, fabsf(nv[k]));
                    if (ck[k]) {
                        if (((dq[j] & 1) && xk[k] == nx - 1) || ((dq[j] & 2) && xk[k] == 0)) o += cxq[j] * v;
                        if (((dq[j] & 4) && yk[k] == ny - 1) || ((dq[j] & 8) && yk[k] == 0)) o += cyq[j] * v;
                    }
                }
                emit(j, q, make_float4(nv[0], nv[1], nv[2], nv[3]));
                defect += wq[j] * (double)colsum;
                outflow += wq[j] * (double)o;
            }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
#pragma unroll
                for (int sft = 1; sft < 16; sft <<= 1) {
                    ph[k] += __shfl_xor(ph[k], sft, 64);
                    yp[k] += __shfl_xor(yp[k], sft, 64);
                }
                if ((lane & 15) == 0) {
                    red[wave & 1][wn + i * 16 + 4 * (lane >> 4) + k] = ph[k];
                    yred[wave & 1][wn + i * 16 + 4 * (lane >> 4) + k] = yp[k];
                }
            }
        }
        // block max |psi^{n+1}| of the next operand scale: the wave's 64 cells lie in
        // one block
        const unsigned mbits = wave_max_u32(__float_as_uint(mx));
        if (lane == 0 && mbits) atomicMax(&a.bmax_next[(n0 + wn) >> a.sb_log], mbits);
        double sums[2] = {defect, outflow};
        block_sum_256<2>(sums, gp(a.blk_part) + 2 * (size_t)tile);   // synchronises the block
        if (tid < kGemmBN) {
            gp(a.phi_part)[(size_t)mt * P + n0 + tid] = red[0][tid] + red[1][tid];
            ypart[(size_t)mt * P + n0 + tid] = yred[0][tid] + yred[1][tid];
        }
    }
}

// ---------------------------------------------------------------------------
// Block-level FP64 sum in a fixed order (wave butterflies, then wave 0).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int NV, typename OutPtr>
__device__ __forceinline__ void block_sum_256(double (&v)[NV], OutPtr out) {
    __shared__ double red[4][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) out[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
}
// The same for a block of NW waves (block size 64 NW).
template <int NW, int NV, typename OutPtr>
__device__ __forceinline__ void block_sum_waves(double (&v)[NV], OutPtr out) {
    __shared__ double red[NW][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double t = red[0][k];
#pragma unroll
            for (int w = 1; w < NW; ++w) t += red[w][k];
            out[k] = t;
        }
}

// ---------------------------------------------------------------------------
// 2. Stream + collide.  Block = 4 waves; wave w owns rows y0 + w R .. + R - 1
//    of a strip of 62 columns: lane l holds column x0 + l - 1, lanes 0 and 63
//    only read the neighbouring columns (halo), lanes 1..62 update.  The block
//    loops over a chunk of ordinates and loads plane q + 1 while it updates
//    plane q.  Upwind neighbour along y: the lane's previous (or next) row, plus
//    one halo row per wave; along x: the neighbouring lane (shuffle).
//    Memory goes through buffer descriptors of one ordinate plane each: offsets
//    outside the grid read as 0 (the vacuum ghost value) and stores to them are
//    dropped, so the loop has no per-cell branches.  Runs for grids wider than the
//    flat-chunk form takes (stream_collide_flat_kernel, below).
//      col  = dt sigma_as (Y - fix - psi) + dt sigma_s (Phi/W - psi)
//      new  = psi - cx (psi - up_x) - cy (psi - up_y) - dt sigma_a psi + col + dt q
//    LP: fix is the per-cell particle correction of the reduced-precision Y, and
//    the block max |new| for the next step's operand scale is reduced per wave.
// ---------------------------------------------------------------------------
constexpr uint32_t kOOB = 0x80000000u;   // byte offset beyond every plane
constexpr int kRsrcWord3 = 0x00020000;   // raw buffer, 32-bit data (gfx9 family)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float* base, int64_t C) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, (int)(C * 4),
                                             kRsrcWord3);
}

// The raw buffer builtins move 32-bit patterns; reinterpret, never convert.
__device__ __forceinline__ float load_plane(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void store_plane(float v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, 0);
}
// Non-temporal forms (cache policy NT) for data the kernel touches once and that no
// later kernel of the step reads from the caches (the flat stencil's Y and new state:
// 400^2 x 512 0.193 -> 0.186 ms, 700^2 x 1152 1.26 -> 1.22 ms; its staged state rows
// stay cached, a neighbouring block reads them again).
constexpr int kCachePolicyNT = 2;
__device__ __forceinline__ float load_plane_nt(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kCachePolicyNT));
}
__device__ __forceinline__ void store_plane_nt(float v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, kCachePolicyNT);
}


// Block barrier that orders LDS only (the stencil waves exchange their rows through LDS;
// a full barrier would also wait for the next plane's global loads in flight).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <bool LP>
__global__ __launch_bounds__(256) void stream_collide_kernel(BatchArgs B) {
    constexpr int R = kRows;
    int pi, local;
    if (!locate(B, KT_SC, blockIdx.x, pi, local)) return;
    const StepArgs a = args_of(B, pi);   // by value: no reloads after stores
    const int bx = local % a.tiles_x;
    const int by = (local / a.tiles_x) % a.tiles_y;
    const int g = local / (a.tiles_x * a.tiles_y);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nx = a.nx, ny = a.ny;
    const int64_t P = a.P, C = a.C;
    const int x = bx * kStripX + lane - 1;
    const int ybase = by * kTileY + wave * R;
    const int q0 = g * a.qchunk;
    const int q1 = min(a.Q, q0 + a.qchunk);
    const bool xok = x >= 0 && x < nx;
    const bool outl = xok && lane >= 1 && lane <= 62;

    float aa[R], bs[R], gs[R], ss[R], isov[R], fix[R], mx[R];
    double phacc[R];
    bool in[R];
    uint32_t off_ld[R], off_st[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int y = ybase + r;
        const bool yok = y < ny;
        const uint32_t c = (uint32_t)(y * nx + x);
        in[r] = outl && yok;
        off_ld[r] = (xok && yok) ? 4u * c : kOOB;
        off_st[r] = in[r] ? 4u * c : kOOB;
        aa[r] = bs[r] = gs[r] = ss[r] = isov[r] = fix[r] = 0.f;
        mx[r] = 0.f;
        phacc[r] = 0.0;
        if (in[r]) {
            const float4 cf = gp(a.coef)[c];
            aa[r] = cf.x;
            bs[r] = cf.y;
            gs[r] = cf.z;
            ss[r] = cf.w;
            isov[r] = gp(a.iso)[c];
            if (LP) fix[r] = gp(a.fix)[c];
        }
    }
    const uint32_t off_hlo =
        (xok && ybase >= 1 && ybase - 1 < ny) ? 4u * (uint32_t)((ybase - 1) * nx + x) : kOOB;
    const uint32_t off_hhi = (xok && ybase + R < ny) ? 4u * (uint32_t)((ybase + R) * nx + x) : kOOB;
    const bool edge = bx == 0 || bx == a.tiles_x - 1 || by == 0 || by == a.tiles_y - 1;
    double defect = 0.0, outflow = 0.0;

    struct Plane {
        float v[R], y[R], hy;
    };
    auto load = [&](int q, int dir, Plane& pn) {
        const __amdgpu_buffer_rsrc_t rp = plane_rsrc(a.psi + (size_t)q * P, C);
        const __amdgpu_buffer_rsrc_t ry = plane_rsrc(a.Y + (size_t)q * P, C);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            pn.v[r] = load_plane(rp, off_ld[r]);
            pn.y[r] = load_plane(ry, off_ld[r]);
        }
        // only the block's outer halo rows come from memory (wave 0 the row below the
        // tile for eta > 0, wave 3 the row above it for eta < 0); the others are the
        // neighbouring waves' own rows, exchanged through LDS
        const uint32_t oh = ((dir & 4) && wave == 0) ? off_hlo : (((dir & 8) && wave == 3) ? off_hhi : kOOB);
        pn.hy = load_plane(rp, oh);
    };
    // xr[q & 1][row of the tile][lane]: the tile's 16 rows of plane q; hr[q & 1][wave]: the
    // halo row each wave loaded (only waves 0 and 3 load one; every wave stores its
    // slot so that no store depends on the wave index)
    __shared__ float xr[2][kTileY][64];
    __shared__ float hr[2][4][64];

    // Ordinate q updates from plane slot q & 1 while the next plane loads into the
    // other slot.  The slots are fixed per unrolled half and every load is issued
    // unconditionally (the last ordinate of the chunk is loaded again at the end), so
    // no slot is ever copied or merged across a branch, which would wait for the
    // loads in flight.
    const ASN_G QInfo* __restrict__ qtab = gp(a.qi);
    auto body = [&](int q, const QInfo& qc, const Plane& cur) {
        const __amdgpu_buffer_rsrc_t ro = plane_rsrc(a.psi_new + (size_t)q * P, C);
        float (*xq)[64] = xr[q & 1];
#pragma unroll
        for (int r = 0; r < R; ++r) xq[wave * R + r][lane] = cur.v[r];
        hr[q & 1][wave][lane] = cur.hy;
        lds_barrier();
        // the row below the wave's rows (eta > 0) or above them (eta < 0)
        const float* hsrc = (qc.dir & 4) ? (wave == 0 ? &hr[q & 1][0][0] : &xq[wave * R - 1][0])
                                         : (wave == 3 ? &hr[q & 1][3][0] : &xq[(wave + 1) * R][0]);
        const float hy = hsrc[lane];
        float colsum = 0.f;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float v = cur.v[r];
            float uy = 0.f;
            if (qc.dir & 4) uy = (r == 0) ? hy : cur.v[r - 1];
            else if (qc.dir & 8) uy = (r == R - 1) ? hy : cur.v[r + 1];
            float ux = 0.f;
            if (qc.dir & 1) ux = __shfl_up(v, 1, 64);
            else if (qc.dir & 2) ux = __shfl_down(v, 1, 64);
            const float col = gs[r] * ((cur.y[r] - fix[r]) - v) + bs[r] * (isov[r] - v);
            const float nv = v - qc.cx * (v - ux) - qc.cy * (v - uy) - aa[r] * v + col + ss[r];
            store_plane(nv, ro, off_st[r]);
            phacc[r] += qc.w * (double)nv;
            colsum += in[r] ? col : 0.f;
            if (LP) mx[r] = fmaxf(mx[r], in[r] ? fabsf(nv) : 0.f);
        }
        defect += qc.w * (double)colsum;
        if (edge) {
            // Mass leaving through the boundary this step: the donor flux of the
            // last cell before a boundary face, for the directions that exit there.
            float o = 0.f;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!in[r]) continue;
                const int y = ybase + r;
                if (((qc.dir & 1) && x == nx - 1) || ((qc.dir & 2) && x == 0)) o += qc.cx * cur.v[r];
                if (((qc.dir & 4) && y == ny - 1) || ((qc.dir & 8) && y == 0)) o += qc.cy * cur.v[r];
            }
            outflow += qc.w * (double)o;
        }
    };
    Plane pa, pb;
    QInfo qa = qtab[min(q0, a.Q - 1)], qb;
    load(min(q0, a.Q - 1), qa.dir, pa);
    for (int q = q0; q < q1; q += 2) {
        const int qn = min(q + 1, q1 - 1);
        qb = qtab[qn];
        load(qn, qb.dir, pb);
        body(q, qa, pa);
        if (q + 1 >= q1) break;
        const int qn2 = min(q + 2, q1 - 1);
        qa = qtab[qn2];
        load(qn2, qa.dir, pa);
        body(q + 1, qb, pb);
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (in[r]) gp(a.phi_part)[(size_t)g * P + (uint32_t)((ybase + r) * nx + x)] = phacc[r];
    if (LP) {
        // The updating lanes of one row (at most 62 cells) cover at most two scale blocks.
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = ybase + r;
            const int64_t c_first = (int64_t)y * nx + bx * kStripX;
            const int64_t b0 = c_first >> a.sb_log;
            const int64_t cb = ((int64_t)y * nx + x) >> a.sb_log;
            const unsigned bits = in[r] ? __float_as_uint(mx[r]) : 0u;
            const unsigned m0 = wave_max_u32(cb == b0 ? bits : 0u);
            const unsigned m1 = wave_max_u32(cb != b0 ? bits : 0u);
            if (lane == 0 && y < ny) {
                if (m0) atomicMax(&a.bmax_next[b0], m0);
                if (m1) atomicMax(&a.bmax_next[b0 + 1], m1);
            }
        }
    }
    double sums[2] = {defect, outflow};
    block_sum_256<2>(sums, gp(a.blk_part) + 2 * (size_t)local);
}

// ---------------------------------------------------------------------------
// 2'. Stream + collide over flat cell chunks (separate forward-Euler stencil).
//     Block (chunk bt, ordinate chunk g) updates cells b0 .. b0 + kFlatCells - 1 for
//     the ordinates of chunk g.  Per ordinate the plane segment [b0 - 1, b0 + L + 1)
//     plus the row below it (eta > 0) or above it (eta < 0) is staged in LDS (float4
//     loads from a 16-byte aligned start, so every row segment is read as whole
//     128-byte lines; cells outside the planes read as 0 through the buffer bounds),
//     the x- and y-upwind values are read from there with ghost masks at the domain
//     boundary, and the next ordinate's segment is fetched meanwhile into the other
//     register slot.  Thread t updates cells b0 + t + 512 j, j = 0..3: a wave's 64
//     lanes read 64 consecutive LDS words (no bank conflicts) and store 256 contiguous
//     bytes.  Same arithmetic and partials as stream_collide_kernel.
// ---------------------------------------------------------------------------
template <bool LP>
__global__ __launch_bounds__(kFlatThreads) void stream_collide_flat_kernel(BatchArgs B) {
    constexpr int T = kFlatThreads, L = kFlatCells, NR = kFlatRounds, J = L / T;
    int pi, local;
    // consecutive chunks on one XCD: the rows a chunk stages beyond its own cells are
    // its neighbours' cells, read at about the same time through the same L2
    if (!locate(B, KT_SC, xcd_remap(blockIdx.x, gridDim.x), pi, local)) return;
    const StepArgs a = args_of(B, pi);   // by value: no reloads after stores
    const int tiles = a.tiles_x;
    const int bt = local % tiles, g = local / tiles;
    const int tid = threadIdx.x, lane = tid & 63;
    const int nx = a.nx, ny = a.ny;
    const int C = (int)a.C, Pi = (int)a.P;
    const int b0 = bt * L;
    const int q0 = g * a.qchunk;
    const int q1 = min(a.Q, q0 + a.qchunk);

    // the thread's cells b0 + tid + T j
    float aa[J], bs[J], gs[J], ss[J], isov[J], fix[J], mx[J];
    uint32_t off[J];   // byte offset of the cell in a plane, out of range beyond the pitch
    double phacc[J];
    int e_in = 0;      // 4 bits per cell: boundary faces as the bits of the direction code
    int live = 0;      // bit j: cell j is a grid cell (not padding)
    int wedge = 0;     // bit j: some lane of the wave holds a boundary cell j (uniform)
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int c = b0 + tid + T * j;
        const bool in = c < C;
        const int y = c / nx, x = c - y * nx;
        float4 cf = make_float4(0.f, 0.f, 0.f, 0.f);
        if (in) cf = gp(a.coef)[c];
        aa[j] = cf.x;
        bs[j] = cf.y;
        gs[j] = cf.z;
        ss[j] = cf.w;
        isov[j] = in ? gp(a.iso)[c] : 0.f;
        fix[j] = (LP && in) ? gp(a.fix)[c] : 0.f;
        mx[j] = 0.f;
        phacc[j] = 0.0;
        off[j] = c < Pi ? 4u * (uint32_t)c : kOOB;
        // bit0 x = 0, bit1 x = nx - 1, bit2 y = 0, bit3 y = ny - 1: the upwind
        // neighbour of direction d is a ghost where d & e != 0
        const int e = (x == 0 ? 1 : 0) | (x == nx - 1 ? 2 : 0) | (y == 0 ? 4 : 0) |
                      (y == ny - 1 ? 8 : 0);
        e_in |= e << (4 * j);
        live |= in ? 1 << j : 0;
        wedge |= __ballot(in && e != 0) ? 1 << j : 0;
    }
    double defect = 0.0, outflow = 0.0;

    // staged segment start (16-byte aligned, may be negative)
    auto seg_start = [&](int dir) { return (dir & 4) ? ((b0 - nx - 1) & ~3) : ((b0 - 1) & ~3); };
    struct Plane {
        float4 r[NR];
        float y[J];
    };
    auto load = [&](int q, int dir, Plane& pn) {
        // bounds at the pitch (cells C .. P - 1 hold zeros), so a float4 never straddles
        const __amdgpu_buffer_rsrc_t rp = plane_rsrc(a.psi + (size_t)q * a.P, a.P);
        const __amdgpu_buffer_rsrc_t ry = plane_rsrc(a.Y + (size_t)q * a.P, a.P);
        const int st = seg_start(dir);
        const int seg_len = L + nx + 8;   // floats the update reads (rounds past it are not fetched)
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int i = 4 * (tid + T * r);
            const int c = st + i;
            const uint32_t o = (c >= 0 && i < seg_len) ? 4u * (uint32_t)c : kOOB;
            pn.r[r] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rp, o, 0, 0));
        }
#pragma unroll
        for (int j = 0; j < J; ++j) pn.y[j] = load_plane_nt(ry, off[j]);
    };
    __shared__ float4 seg[2][NR * T];
    const ASN_G QInfo* __restrict__ qtab = gp(a.qi);
    // stage: the plane's segment into LDS buffer q & 1 (consumes the slot's segment)
    auto stage = [&](int q, const Plane& cur) {
        float4* sq = seg[q & 1];
#pragma unroll
        for (int r = 0; r < NR; ++r) sq[tid + T * r] = cur.r[r];
    };
    // compute: the update of plane q from LDS buffer q & 1 and the slot's Y values
    auto compute = [&](int q, const QInfo& qc, const Plane& cur) {
        lds_barrier();
        const int d = qc.dir;
        const float* sf = reinterpret_cast<const float*>(seg[q & 1]) + (b0 - seg_start(d) + tid);
        const __amdgpu_buffer_rsrc_t ro = plane_rsrc(a.psi_new + (size_t)q * a.P, a.P);
        const int ysh = (d & 4) ? -nx : nx;   // y-upwind cell (cy = 0 when d & 12 = 0)
        const int xsh = (d & 1) ? -1 : 1;     // x-upwind cell (cx = 0 when d & 3 = 0)
        const int dout = ((d & 5) << 1) | ((d & 10) >> 1);   // outflow faces of d
        float colsum = 0.f, o = 0.f;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const float* pc = sf + T * j;
            const int e = (e_in >> (4 * j)) & 15;
            const bool in = (live >> j) & 1;
            const float v = pc[0];
            const float ux = (d & e & 3) ? 0.f : pc[xsh];
            const float uy = (d & e & 12) ? 0.f : pc[ysh];
            const float col = gs[j] * ((cur.y[j] - fix[j]) - v) + bs[j] * (isov[j] - v);
            const float r = v - qc.cx * (v - ux) - qc.cy * (v - uy) - aa[j] * v + col + ss[j];
            const float nv = in ? r : 0.f;   // padding cells stay zero
            store_plane_nt(nv, ro, off[j]);
            phacc[j] += qc.w * (double)nv;
            colsum += in ? col : 0.f;
            if ((wedge >> j) & 1) {   // only waves holding a boundary cell j
                const int go = dout & e;
                o += in ? ((go & 3) ? qc.cx * v : 0.f) + ((go & 12) ? qc.cy * v : 0.f) : 0.f;
            }
            if (LP) mx[j] = fmaxf(mx[j], fabsf(nv));
        }
        defect += qc.w * (double)colsum;
        outflow += qc.w * (double)o;
    };
    // two plane slots used alternately, loads unconditional (as in stream + collide).
    // Loads and stores share one counter, so the wait for a slot also waits for loads
    // issued after it: more slots or planes per wait did not help (measured).
    const int ql = max(q1 - 1, 0);
    Plane pa, pb;
    QInfo qa = qtab[min(q0, ql)], qb;
    load(min(q0, ql), qa.dir, pa);
    for (int q = q0; q < q1; q += 2) {
        const int qn = min(q + 1, ql);
        qb = qtab[qn];
        load(qn, qb.dir, pb);
        stage(q, pa);
        compute(q, qa, pa);
        if (q + 1 >= q1) break;
        const int qn2 = min(q + 2, ql);
        qa = qtab[qn2];
        load(qn2, qa.dir, pa);
        stage(q + 1, pb);
        compute(q + 1, qb, pb);
    }
#pragma unroll
    for (int j = 0; j < J; ++j)
        if ((live >> j) & 1) gp(a.phi_part)[(size_t)g * a.P + b0 + tid + T * j] = phacc[j];
    if (LP) {
        // a wave's 64 cells j lie in one scale block of the next operand
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const unsigned m = wave_max_u32(__float_as_uint(mx[j]));
            const int cw = b0 + (tid & ~63) + T * j;
            if (lane == 0 && m && cw < Pi) atomicMax(&a.bmax_next[cw >> a.sb_log], m);
        }
    }
    double sums[2] = {defect, outflow};
    block_sum_waves<T / 64, 2>(sums, gp(a.blk_part) + 2 * (size_t)local);
}

// ---------------------------------------------------------------------------
// 2b. Heun stage with limited second-order upwind fluxes (paper Section 3.1).
//     Per ordinate and axis a cell's slope is minmod(psi_i - psi_{i-1},
//     psi_{i+1} - psi_i); a face carries the value reconstructed on its upwind
//     side, psi_i + s_i / 2 or psi_{i+1} - s_{i+1} / 2, and cells outside the
//     grid read 0 (vacuum, also for their slopes).  Same block shape as
//     stream_collide_kernel, with a strip of 60 columns: lane l holds column
//     x0 + l - 2, lanes 2..61 update, and each wave reads two halo rows on each side.
//     Runs for grids wider than the flat-chunk form takes (muscl_flat_kernel).
//       STAGE 1: out = psi + dt R(psi)                 (psi^n  -> psi^1)
//       STAGE 2: out = (old + psi + dt R(psi)) / 2     (psi^1, old = psi^n)
//     In stage 2 the output buffer holds psi^n: every lane reads its own cell
//     of it before overwriting that cell, and no other lane reads it.
// ---------------------------------------------------------------------------
// minmod(a, b) is the median of a, b and 0: the operand of smaller magnitude when the
// signs agree, else 0 (one v_med3_f32).
__device__ __forceinline__ float minmod(float a, float b) {
    return __builtin_amdgcn_fmed3f(a, b, 0.f);
}

template <bool LP, int STAGE>
__global__ __launch_bounds__(256) void muscl_kernel(BatchArgs B) {
    constexpr int R = kRows;
    int pi, local;
    if (!locate(B, KT_SC, blockIdx.x, pi, local)) return;
    const StepArgs a = args_of(B, pi);   // by value: no reloads after stores
    const int bx = local % a.tiles_x;
    const int by = (local / a.tiles_x) % a.tiles_y;
    const int g = local / (a.tiles_x * a.tiles_y);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nx = a.nx, ny = a.ny;
    const int64_t P = a.P, C = a.C;
    const int x = bx * kStripXM + lane - 2;
    const int ybase = by * kTileY + wave * R;
    const int q0 = g * a.qchunk;
    const int q1 = min(a.Q, q0 + a.qchunk);
    const bool xok = x >= 0 && x < nx;
    const bool outl = xok && lane >= 2 && lane <= 61;

    float aa[R], bs[R], gs[R], ss[R], isov[R], fix[R], mx[R];
    double phacc[R];
    bool in[R];
    uint32_t off_ld[R], off_st[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int y = ybase + r;
        const bool yok = y < ny;
        const uint32_t c = (uint32_t)(y * nx + x);
        in[r] = outl && yok;
        off_ld[r] = (xok && yok) ? 4u * c : kOOB;
        off_st[r] = in[r] ? 4u * c : kOOB;
        aa[r] = bs[r] = gs[r] = ss[r] = isov[r] = fix[r] = 0.f;
        mx[r] = 0.f;
        phacc[r] = 0.0;
        if (in[r]) {
            const float4 cf = gp(a.coef)[c];
            aa[r] = cf.x;
            bs[r] = cf.y;
            gs[r] = cf.z;
            ss[r] = cf.w;
            isov[r] = gp(a.iso)[c];
            if (LP) fix[r] = gp(a.fix)[c];
        }
    }
    // halo rows ybase - 2, ybase - 1, ybase + R, ybase + R + 1
    uint32_t off_h[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int yy = k < 2 ? ybase - 2 + k : ybase + R + (k - 2);
        off_h[k] = (xok && yy >= 0 && yy < ny) ? 4u * (uint32_t)(yy * nx + x) : kOOB;
    }
    const bool edge = bx == 0 || bx == a.tiles_x - 1 || by == 0 || by == a.tiles_y - 1;
    double defect = 0.0, outflow = 0.0;

    struct Plane {
        float v[R], y[R], h[4], o[R];
    };
    auto load = [&](int q, int dir, Plane& pn) {
        const __amdgpu_buffer_rsrc_t rp = plane_rsrc(a.psi + (size_t)q * P, C);
        const __amdgpu_buffer_rsrc_t ry = plane_rsrc(a.Y + (size_t)q * P, C);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            pn.v[r] = load_plane(rp, off_ld[r]);
            pn.y[r] = load_plane(ry, off_ld[r]);
        }
        // eta > 0 takes two rows below and one above, eta < 0 the mirror image; only
        // the block's outer halo rows come from memory (wave 0 below the tile, wave 3
        // above it), the others are the neighbouring waves' own rows, through LDS
        pn.h[0] = load_plane(rp, ((dir & 4) && wave == 0) ? off_h[0] : kOOB);
        pn.h[1] = load_plane(rp, ((dir & 12) && wave == 0) ? off_h[1] : kOOB);
        pn.h[2] = load_plane(rp, ((dir & 12) && wave == 3) ? off_h[2] : kOOB);
        pn.h[3] = load_plane(rp, ((dir & 8) && wave == 3) ? off_h[3] : kOOB);
        if (STAGE == 2) {
            const __amdgpu_buffer_rsrc_t ro = plane_rsrc(a.psi_new + (size_t)q * P, C);
#pragma unroll
            for (int r = 0; r < R; ++r) pn.o[r] = load_plane(ro, off_st[r]);
        }
    };

    // Two plane slots used alternately, loads unconditional (as in stream + collide).
    const ASN_G QInfo* __restrict__ qtab = gp(a.qi);
    // xr[q & 1][row of the tile][lane]: the tile's 16 rows of plane q; hr[q & 1][wave][k]:
    // the halo rows each wave loaded (only waves 0 and 3 load any; every wave stores its
    // slots so that no store depends on the wave index)
    __shared__ float xr[2][kTileY][64];
    __shared__ float hr[2][4][4][64];
    auto body = [&](int q, const QInfo& qc, const Plane& cur) {
        const __amdgpu_buffer_rsrc_t ro = plane_rsrc(a.psi_new + (size_t)q * P, C);
        float (*xq)[64] = xr[q & 1];
#pragma unroll
        for (int r = 0; r < R; ++r) xq[wave * R + r][lane] = cur.v[r];
#pragma unroll
        for (int k = 0; k < 4; ++k) hr[q & 1][wave][k][lane] = cur.h[k];
        lds_barrier();
        // column e[k] = row ybase - 2 + k: two rows below the wave's rows (the tile's
        // outer halo for wave 0), its own rows, two rows above (outer halo for wave 3)
        const float* lo = wave == 0 ? &hr[q & 1][0][0][0] : &xq[wave * R - 2][0];
        const float* hi = wave == 3 ? &hr[q & 1][3][2][0] : &xq[(wave + 1) * R][0];
        float e[R + 4];
        e[0] = lo[lane];
        e[1] = lo[64 + lane];
#pragma unroll
        for (int r = 0; r < R; ++r) e[r + 2] = cur.v[r];
        e[R + 2] = hi[lane];
        e[R + 3] = hi[64 + lane];
        // upwind face values along y: fy[k] = value on the face above row k - 2
        // (eta > 0, k = 1..R+1 used) or below row k - 2 (eta < 0, k = 2..R+2 used)
        float fy[R + 4];
#pragma unroll
        for (int k = 1; k < R + 3; ++k) {
            const float sl = minmod(e[k] - e[k - 1], e[k + 1] - e[k]);
            fy[k] = (qc.dir & 4) ? e[k] + 0.5f * sl : e[k] - 0.5f * sl;
        }
        float colsum = 0.f, o = 0.f;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float v = cur.v[r];
            const float vl = __shfl_up(v, 1, 64);
            const float vr = __shfl_down(v, 1, 64);
            const float sx = minmod(v - vl, vr - v);
            float dfx = 0.f, fout_x = 0.f;
            if (qc.dir & 1) {
                const float f = v + 0.5f * sx;
                dfx = f - __shfl_up(f, 1, 64);
                fout_x = f;
            } else if (qc.dir & 2) {
                const float gl = v - 0.5f * sx;
                dfx = gl - __shfl_down(gl, 1, 64);
                fout_x = gl;
            }
            float dfy = 0.f, fout_y = 0.f;
            if (qc.dir & 4) {
                dfy = fy[r + 2] - fy[r + 1];
                fout_y = fy[r + 2];
            } else if (qc.dir & 8) {
                dfy = fy[r + 2] - fy[r + 3];
                fout_y = fy[r + 2];
            }
            const float col = gs[r] * ((cur.y[r] - fix[r]) - v) + bs[r] * (isov[r] - v);
            const float nv = v - qc.cx * dfx - qc.cy * dfy - aa[r] * v + col + ss[r];
            const float res = STAGE == 2 ? 0.5f * (cur.o[r] + nv) : nv;
            store_plane(res, ro, off_st[r]);
            phacc[r] += qc.w * (double)res;
            colsum += in[r] ? col : 0.f;
            if (LP) mx[r] = fmaxf(mx[r], in[r] ? fabsf(res) : 0.f);
            if (edge && in[r]) {
                // particles leaving through a boundary face: the reconstructed
                // value on the face of the last cell, for directions that exit there
                const int y = ybase + r;
                if (((qc.dir & 1) && x == nx - 1) || ((qc.dir & 2) && x == 0)) o += qc.cx * fout_x;
                if (((qc.dir & 4) && y == ny - 1) || ((qc.dir & 8) && y == 0)) o += qc.cy * fout_y;
            }
        }
        defect += qc.w * (double)colsum;
        outflow += qc.w * (double)o;
    };
    Plane pa, pb;
    QInfo qa = qtab[min(q0, a.Q - 1)], qb;
    load(min(q0, a.Q - 1), qa.dir, pa);
    for (int q = q0; q < q1; q += 2) {
        const int qn = min(q + 1, q1 - 1);
        qb = qtab[qn];
        load(qn, qb.dir, pb);
        body(q, qa, pa);
        if (q + 1 >= q1) break;
        const int qn2 = min(q + 2, q1 - 1);
        qa = qtab[qn2];
        load(qn2, qa.dir, pa);
        body(q + 1, qb, pb);
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (in[r]) gp(a.phi_part)[(size_t)g * P + (uint32_t)((ybase + r) * nx + x)] = phacc[r];
    if (LP) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = ybase + r;
            const int64_t c_first = (int64_t)y * nx + bx * kStripXM;
            const int64_t b0 = c_first >> a.sb_log;
            const int64_t cb = ((int64_t)y * nx + x) >> a.sb_log;
            const unsigned bits = in[r] ? __float_as_uint(mx[r]) : 0u;
            const unsigned m0 = wave_max_u32(cb == b0 ? bits : 0u);
            const unsigned m1 = wave_max_u32(cb != b0 ? bits : 0u);
            if (lane == 0 && y < ny) {
                if (m0) atomicMax(&a.bmax_next[b0], m0);
                if (m1) atomicMax(&a.bmax_next[b0 + 1], m1);
            }
        }
    }
    double sums[2] = {defect, outflow};
    block_sum_256<2>(sums, gp(a.blk_part) + 2 * (size_t)local);
}

// Per-cell particle correction of the reduced-precision Y: the w-weighted sum of
// Y over all ordinates (from the per-tile partials, fixed order) minus Phi, over W.
__global__ __launch_bounds__(256) void particle_fix_kernel(BatchArgs B) {
    int pi, local;
    if (!locate(B, KT_FIX, blockIdx.x, pi, local)) return;
    const StepArgs a = args_of(B, pi);   // by value: no reloads after stores
    const int64_t c = (int64_t)local * 256 + threadIdx.x;
    if (c >= a.C) return;
    double m = -gp(a.phi64)[c];
    const int nparts = a.Qp / kGemmBM;
    const ASN_G double* yp = gp(a.ypart);
    for (int t = 0; t < nparts; ++t) m += yp[(size_t)t * a.P + c];
    gp(a.fix)[c] = (float)(m / a.W);
}

// ---------------------------------------------------------------------------
// 2c. Heun pass over flat cell chunks: the MUSCL update of muscl_kernel (same
//     arithmetic) in the flat-chunk form of stream_collide_flat_kernel.  The staged
//     segment holds the chunk with two cells of x context and the two rows below and
//     one above it (eta > 0) or the mirror image (eta < 0).  Cells beyond the grid's
//     rows read as zero; x ghosts (two per side) are masked from the cell's x.  Thread
//     t updates cells b0 + t + 512 j, j = 0..3, so that the 64 lanes of a wave read
//     64 consecutive LDS words (no bank conflicts) and store 256 contiguous bytes.
// ---------------------------------------------------------------------------
template <bool LP, int STAGE>
__global__ __launch_bounds__(kFlatThreads) void muscl_flat_kernel(BatchArgs B) {
    constexpr int T = kFlatThreads, L = kFlatCells, NR = kFlatRounds, J = L / T;
    int pi, local;
    // consecutive chunks on one XCD: the rows a chunk stages beyond its own cells are
    // its neighbours' cells, read at about the same time through the same L2
    if (!locate(B, KT_SC, xcd_remap(blockIdx.x, gridDim.x), pi, local)) return;
    const StepArgs a = args_of(B, pi);   // by value: no reloads after stores
    const int tiles = a.tiles_x;
    const int bt = local % tiles, g = local / tiles;
    const int tid = threadIdx.x, lane = tid & 63;
    const int nx = a.nx, ny = a.ny;
    const int C = (int)a.C, Pi = (int)a.P;
    const int b0 = bt * L;
    const int q0 = g * a.qchunk;
    const int q1 = min(a.Q, q0 + a.qchunk);

    float aa[J], bs[J], gs[J], ss[J], isov[J], fix[J], mx[J];
    int xk[J];
    uint32_t off[J];   // byte offset of the cell in a plane, out of range beyond the pitch
    double phacc[J];
    int live = 0;      // bit j: cell j is a grid cell (not padding)
    unsigned ex = 0;   // 4 bits per cell: the direction bits that leave the grid there
    int wexit = 0;     // bit j: some lane of the wave holds a boundary cell j (uniform)
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int c = b0 + tid + T * j;
        const bool in = c < C;
        const int y = c / nx, x = c - y * nx;
        float4 cf = make_float4(0.f, 0.f, 0.f, 0.f);
        if (in) cf = gp(a.coef)[c];
        aa[j] = cf.x;
        bs[j] = cf.y;
        gs[j] = cf.z;
        ss[j] = cf.w;
        isov[j] = in ? gp(a.iso)[c] : 0.f;
        fix[j] = (LP && in) ? gp(a.fix)[c] : 0.f;
        mx[j] = 0.f;
        phacc[j] = 0.0;
        xk[j] = x;
        off[j] = c < Pi ? 4u * (uint32_t)c : kOOB;
        live |= in ? 1 << j : 0;
        // +x leaves at x = nx - 1, -x at x = 0, +y at y = ny - 1, -y at y = 0
        const unsigned e = in ? (unsigned)(x == nx - 1) | (unsigned)(x == 0) << 1 |
                                    (unsigned)(y == ny - 1) << 2 | (unsigned)(y == 0) << 3
                              : 0u;
        ex |= e << (4 * j);
        wexit |= __ballot(e != 0) ? 1 << j : 0;
    }
    double defect = 0.0, outflow = 0.0;

    // staged segment start (16-byte aligned, may be negative)
    auto seg_start = [&](int dir) {
        return (dir & 4) ? ((b0 - 2 * nx - 2) & ~3) : ((dir & 8) ? ((b0 - nx - 2) & ~3) : ((b0 - 2) & ~3));
    };
    struct Plane {
        float4 r[NR];
        float y[J], o[J];
    };
    auto load = [&](int q, int dir, Plane& pn) {
        // bounds at the pitch (cells C .. P - 1 hold zeros), so a float4 never straddles
        const __amdgpu_buffer_rsrc_t rp = plane_rsrc(a.psi + (size_t)q * a.P, a.P);
        const __amdgpu_buffer_rsrc_t ry = plane_rsrc(a.Y + (size_t)q * a.P, a.P);
        const int st = seg_start(dir);
        const int seg_len = L + 3 * nx + 8;   // floats the update reads
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int i = 4 * (tid + T * r);
            const int c = st + i;
            const uint32_t o = (c >= 0 && i < seg_len) ? 4u * (uint32_t)c : kOOB;
            pn.r[r] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rp, o, 0, 0));
        }
#pragma unroll
        for (int j = 0; j < J; ++j) pn.y[j] = load_plane(ry, off[j]);
        if (STAGE == 2) {   // the old level, stored where the result goes
            const __amdgpu_buffer_rsrc_t ro = plane_rsrc(a.psi_new + (size_t)q * a.P, a.P);
#pragma unroll
            for (int j = 0; j < J; ++j) pn.o[j] = load_plane(ro, off[j]);
        } else {
#pragma unroll
            for (int j = 0; j < J; ++j) pn.o[j] = 0.f;
        }
    };
    __shared__ float4 seg[2][NR * T];
    const ASN_G QInfo* __restrict__ qtab = gp(a.qi);
    auto body = [&](int q, const QInfo& qc, const Plane& cur) {
        float4* sq = seg[q & 1];
#pragma unroll
        for (int r = 0; r < NR; ++r) sq[tid + T * r] = cur.r[r];
        lds_barrier();
        const int d = qc.dir;
        const float* sf = reinterpret_cast<const float*>(sq) + (b0 - seg_start(d) + tid);
        const __amdgpu_buffer_rsrc_t ro = plane_rsrc(a.psi_new + (size_t)q * a.P, a.P);
        float colsum = 0.f, o = 0.f;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const float* pc = sf + T * j;
            const int x = xk[j];
            const float v = pc[0];
            // x neighbours, zero ghosts outside the row
            const float vm1 = x >= 1 ? pc[-1] : 0.f;
            const float vp1 = x <= nx - 2 ? pc[1] : 0.f;
            const float sx = minmod(v - vm1, vp1 - v);
            float dfx = 0.f, fout_x = 0.f;
            if (d & 1) {
                const float vm2 = x >= 2 ? pc[-2] : 0.f;
                const float f = v + 0.5f * sx;
                const float fl = vm1 + 0.5f * minmod(vm1 - vm2, v - vm1);
                dfx = f - fl;
                fout_x = f;
            } else if (d & 2) {
                const float vp2 = x <= nx - 3 ? pc[2] : 0.f;
                const float gl = v - 0.5f * sx;
                const float gr = vp1 - 0.5f * minmod(vp1 - v, vp2 - vp1);
                dfx = gl - gr;
                fout_x = gl;
            }
            // y neighbours (rows beyond the grid read as zero)
            float dfy = 0.f, fout_y = 0.f;
            if (d & 4) {
                const float ym2 = pc[-2 * nx], ym1 = pc[-nx], yp1 = pc[nx];
                const float f = v + 0.5f * minmod(v - ym1, yp1 - v);
                const float fb = ym1 + 0.5f * minmod(ym1 - ym2, v - ym1);
                dfy = f - fb;
                fout_y = f;
            } else if (d & 8) {
                const float ym1 = pc[-nx], yp1 = pc[nx], yp2 = pc[2 * nx];
                const float gb = v - 0.5f * minmod(v - ym1, yp1 - v);
                const float ga = yp1 - 0.5f * minmod(yp1 - v, yp2 - yp1);
                dfy = gb - ga;
                fout_y = gb;
            }
            const bool in = (live >> j) & 1;
            const float col = gs[j] * ((cur.y[j] - fix[j]) - v) + bs[j] * (isov[j] - v);
            const float nv = v - qc.cx * dfx - qc.cy * dfy - aa[j] * v + col + ss[j];
            const float res = STAGE == 2 ? 0.5f * (cur.o[j] + nv) : nv;
            const float rv = in ? res : 0.f;   // padding cells stay zero
            store_plane(rv, ro, off[j]);
            phacc[j] += qc.w * (double)rv;
            colsum += in ? col : 0.f;
            if (LP) mx[j] = fmaxf(mx[j], fabsf(rv));
            if ((wexit >> j) & 1) {
                // particles leaving through a boundary face: the reconstructed value on
                // the face of the last cell, for directions that exit there
                const unsigned e = (ex >> (4 * j)) & (unsigned)d;
                if (e & 3u) o += qc.cx * fout_x;
                if (e & 12u) o += qc.cy * fout_y;
            }
        }
        defect += qc.w * (double)colsum;
        outflow += qc.w * (double)o;
    };
    // two plane slots used alternately, loads unconditional (as in stream + collide)
    Plane pa, pb;
    QInfo qa = qtab[min(q0, a.Q - 1)], qb;
    load(min(q0, a.Q - 1), qa.dir, pa);
    for (int q = q0; q < q1; q += 2) {
        const int qn = min(q + 1, q1 - 1);
        qb = qtab[qn];
        load(qn, qb.dir, pb);
        body(q, qa, pa);
        if (q + 1 >= q1) break;
        const int qn2 = min(q + 2, q1 - 1);
        qa = qtab[qn2];
        load(qn2, qa.dir, pa);
        body(q + 1, qb, pb);
    }
#pragma unroll
    for (int j = 0; j < J; ++j)
        if ((live >> j) & 1) gp(a.phi_part)[(size_t)g * a.P + b0 + tid + T * j] = phacc[j];
    if (LP) {
        // a wave's 64 cells j lie in one scale block of the next operand
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const unsigned m = wave_max_u32(__float_as_uint(mx[j]));
            const int cw = b0 + (tid & ~63) + T * j;
            if (lane == 0 && m && cw < Pi) atomicMax(&a.bmax_next[cw >> a.sb_log], m);
        }
    }
    double sums[2] = {defect, outflow};
    block_sum_waves<T / 64, 2>(sums, gp(a.blk_part) + 2 * (size_t)local);
}

// ---------------------------------------------------------------------------
// 3. Finalize: Phi = sum of the G partials (fixed order), Phi/W, mass partials.
// ---------------------------------------------------------------------------
// sum over g < G of p[g P + c], added in the order g = 0, 1, ...; the loads of eight
// partials are issued together (one memory round trip per eight, not per partial)
__device__ __forceinline__ double sum_partials(const ASN_G double* p, int G, int64_t P,
                                               int64_t c) {
    double s = 0.0;
    for (int g0 = 0; g0 < G; g0 += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(size_t)min(g0 + u, G - 1) * P + c];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (g0 + u < G) s += v[u];
    }
    return s;
}

__global__ __launch_bounds__(256) void finalize_kernel(BatchArgs B, int init) {
    int pi, local;
    if (!locate(B, KT_FIN, blockIdx.x, pi, local)) return;
    const StepArgs a = args_of(B, pi);   // by value: no reloads after stores
    const int G = init ? 1 : a.G;
    ASN_G unsigned* bmax_zero = init ? nullptr : gp(a.bmax_cur);
    const int64_t c = (int64_t)local * 256 + threadIdx.x;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    if (c < a.C) {
        const float4 cf = gp(a.coef)[c];
        const bool lp_fused = a.dtype != 0 && a.fused;
        const double phi_old = lp_fused && !init ? gp(a.phi64)[c] : 0.0;
        double phi = sum_partials(gp(a.phi_part), G, a.P, c);
        double corr = 0.0;   // W delta: particles of the pending correction (fused BF16 / FP16)
        if (lp_fused) {
            if (init) {
                gp(a.delta)[c] = 0.f;
            } else {
                // the particle correction of this step's reduced-precision Y: every
                // ordinate of the cell gets delta = -dt sigma_as (sum_q w_q Y^ - Phi^n) / W
                const double ys = sum_partials(gp(a.ypart), G, a.P, c);
                const float d = (float)(-(double)cf.z * (ys - phi_old) / a.W);
                gp(a.delta)[c] = d;
                corr = a.W * (double)d;
            }
        }
        // iso holds Phi^ / W of the stored state; phi64 the true Phi
        gp(a.iso)[c] = (float)(phi / a.W);
        phi += corr;
        gp(a.phi64)[c] = phi;
        s[0] = phi;
        s[1] = (double)cf.x * phi;
        s[2] = (double)cf.w;
        s[3] = corr;
    }
    if (bmax_zero != nullptr && c < scale_blocks(a.P, a.sb_log)) bmax_zero[c] = 0u;
    block_sum_256<4>(s, gp(a.fin_part) + 4 * (size_t)local);
}

// The stored state of a fused reduced-precision problem plus its pending per-cell
// correction becomes the plain state: psi[q][c] += delta[c], delta = 0, iso = Phi / W.
__global__ void materialize_kernel(StepArgs a, float* psi) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (c >= a.C || q >= a.Q) return;
    psi[(size_t)q * a.P + c] += a.delta[c];
}

__global__ void materialize_done_kernel(StepArgs a) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.C) return;
    a.delta[c] = 0.f;
    a.iso[c] = (float)(a.phi64[c] / a.W);
}

// ---------------------------------------------------------------------------
// 4. Budget: fold block partials into the record (one block, fixed order).
// ---------------------------------------------------------------------------
//    BUD_STEP    Euler step: M^{n+1} against M^n - A^n - O + S + D.
//    BUD_STAGE1  Heun, first pass: checks the intermediate level M^1 against
//                M^n + its full increment, and keeps half of that increment.
//    BUD_STAGE2  Heun, second pass: M^{n+1} against M^n + half of each pass's
//                increment (the new level is the mean of psi^n and psi^1 +
//                dt R(psi^1)).
//    BUD_INIT    after set_state: M^0.
// One block of 1024 threads per problem.  Each thread folds a strided share of the
// partials, the loads of both kinds issued together, four of each at a time (one
// round trip per four partials instead of per partial), then the block folds the
// threads in a fixed order.  Thread 0 reads the record while the partials arrive and
// writes it back whole.
constexpr int kBudgetThreads = 1024;
__global__ __launch_bounds__(kBudgetThreads) void budget_kernel(BatchArgs B, int mode) {
    int pi, local;
    if (!locate(B, KT_BUDGET, blockIdx.x, pi, local)) return;
    const StepArgs a = args_of(B, pi);   // by value: no reloads after stores
    const bool init = mode == BUD_INIT;
    ASN_G double* rec = gp(a.rec);
    double r[REC_LEN];
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < REC_LEN; ++k) r[k] = rec[k];
    const int n_fin = a.fin_blocks;
    const int n_blk = init ? 0 : a.tiles_x * a.tiles_y * a.G;
    double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const ASN_G double4* fp = reinterpret_cast<const ASN_G double4*>(gp(a.fin_part));
    const ASN_G double2* bp = reinterpret_cast<const ASN_G double2*>(gp(a.blk_part));
    constexpr int T = kBudgetThreads, U = 4;
    for (int i0 = threadIdx.x; i0 < max(n_fin, n_blk); i0 += T * U) {
        double4 v[U];
        double2 w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * T;
            v[u] = fp[min(i, n_fin - 1)];
            w[u] = double2{0.0, 0.0};
            if (n_blk > 0) w[u] = bp[min(i, n_blk - 1)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * T;
            if (i < n_fin) {
                s[0] += v[u].x;
                s[1] += v[u].y;
                s[2] += v[u].z;
                s[5] += v[u].w;
            }
            if (i < n_blk) {
                s[3] += w[u].x;
                s[4] += w[u].y;
            }
        }
    }
    __shared__ double tot[6];
    block_sum_waves<T / 64, 6>(s, tot);
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (mode == BUD_STEP || mode == BUD_STAGE2) gp(B.steps_left)[pi] -= 1;
    const double m_next = a.area * tot[0];
    const double abs_next = a.area * tot[1];
    auto store = [&]() {
#pragma unroll
        for (int k = 0; k < REC_LEN; ++k) rec[k] = r[k];
    };
    if (init) {
#pragma unroll
        for (int k = 0; k < REC_LEN; ++k) r[k] = 0.0;
        r[REC_MASS] = m_next;
        r[REC_MASS0] = m_next;
        r[REC_ABS_NEXT] = abs_next;
        r[REC_SRC_STEP] = a.area * a.W * tot[2];
        store();
        return;
    }
    // collision defect: the stencil's increments plus the pending correction's particles
    const double def = a.area * (tot[3] + tot[5]);
    const double out = a.area * tot[4];
    const double ref = fmax(r[REC_MASS0], r[REC_MASS]);
    auto residual = [&](double got, double pred) {
        const double rel = ref > 0.0 ? fabs(got - pred) / ref : fabs(got - pred);
        r[REC_RES] = fmax(r[REC_RES], rel);
    };
    if (mode == BUD_STEP) {
        residual(m_next, r[REC_MASS] - r[REC_ABS_NEXT] - out + r[REC_SRC_STEP] + def);
        r[REC_ABS] += r[REC_ABS_NEXT];
        r[REC_OUT] += out;
        r[REC_SRC] += r[REC_SRC_STEP];
        r[REC_DEF] += def;
        r[REC_STEPS] += 1.0;
        r[REC_MASS] = m_next;
        r[REC_ABS_NEXT] = abs_next;
        store();
        return;
    }
    // Heun passes: each contributes half of its increment to the step
    const double abs_in = mode == BUD_STAGE1 ? r[REC_ABS_NEXT] : r[REC_ABS_STAGE];
    const double inc = -abs_in - out + r[REC_SRC_STEP] + def;
    r[REC_ABS] += 0.5 * abs_in;
    r[REC_OUT] += 0.5 * out;
    r[REC_SRC] += 0.5 * r[REC_SRC_STEP];
    r[REC_DEF] += 0.5 * def;
    if (mode == BUD_STAGE1) {
        residual(m_next, r[REC_MASS] + inc);
        r[REC_HALF] = 0.5 * inc;
        r[REC_ABS_STAGE] = abs_next;
    } else {
        residual(m_next, r[REC_MASS] + r[REC_HALF] + 0.5 * inc);
        r[REC_STEPS] += 1.0;
        r[REC_MASS] = m_next;
        r[REC_ABS_NEXT] = abs_next;
    }
    store();
}

// ---------------------------------------------------------------------------
// Moments of a freshly set state: Phi partial (G = 1) and block max |psi|.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void moments_kernel(StepArgs a) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= a.C) return;
    double phi = 0.0;
    float mx = 0.f;
    for (int q = 0; q < a.Q; ++q) {
        const float v = a.psi[(size_t)q * a.P + c];
        phi += a.qi[q].w * (double)v;
        mx = fmaxf(mx, fabsf(v));
    }
    a.phi_part[c] = phi;
    atomicMax(&a.bmax_cur[c >> a.sb_log], __float_as_uint(mx));
}

__global__ void fill_u32_kernel(unsigned* p, int64_t n, unsigned v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void broadcast_kernel(float* psi, const float* cell, int Q, int64_t C, int64_t P) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (c < P && q < Q) psi[(size_t)q * P + c] = (c < C) ? cell[c] : 0.f;
}

// ---------------------------------------------------------------------------
// 5. Banded forward-Euler step for product ordinate sets (FP32).
//    The set is invariant under rotations by 2 pi / n_az about the polar axis, so
//    Y_(i,k) = sum_j sum_delta c_ij(delta) psi_(j, k + delta): per output level a
//    short circular convolution along the azimuth with each of the levels within
//    `reach`.  Block = kBandCells consecutive cells (flat index) x every ordinate,
//    walking the levels in order.  Ring slot l % (2 reach + 2) holds level l of the
//    block's cells (and the cell before and after them); while output level i is
//    computed, level i + reach + 1 is written into the slot level i - reach - 1 left
//    and level i + reach + 2 is loaded into registers, so one LDS barrier per level
//    suffices and each cell-ordinate of psi^n is read from memory once by its own
//    block (the y-upwind values are read again by the block below or above).  Level
//    i's coefficients sit in one of two LDS buffers (written a level ahead); its pair
//    codes, decoded on the host (band_device_code), come with its descriptor, a scalar
//    load made a level ahead.  A lane's outputs of a level are kBandO consecutive azimuths of one cell.
//    Narrow pairs (coupling azimuths at most kBandNarrow apart) are unrolled per width
//    with their LDS rows at compile-time offsets (the slot carries wrapped copies of
//    the rows at either end); wide pairs go in steps of four offsets from the wrapped
//    start row.  The epilogue is the donor-cell stream + collide update as one FMA
//    chain; the x-upwind value comes from the slot, the y-upwind value from memory
//    (loaded a level ahead).  The block writes each cell's complete Phi^{n+1} (one
//    partial, G = 1) and its defect and outflow partials, in a fixed order.
// ---------------------------------------------------------------------------
// The band tables are written by the host before any step and only read by the
// kernels: reached through the constant address space, their uniform loads are scalar
// (SMEM) loads, which do not wait behind the vector memory counter.
#if defined(__HIP_DEVICE_COMPILE__)
#define ASN_K __attribute__((address_space(4)))
#else
#define ASN_K
#endif
template <typename T>
__device__ __forceinline__ const ASN_K T* kp(const T* p) {
    return (const ASN_K T*)p;
}

// A narrow pair: offsets -S .. S.  row: the lane's column in the row of its first
// output azimuth; cf: the run's coefficients in LDS (16-byte aligned, the same words
// for every lane).
template <int S>
__device__ __forceinline__ void band_narrow(float (&acc)[kBandO], const float* row,
                                            const float* cf) {
    constexpr int O = kBandO, N = O + 2 * S, NC = (2 * S + 4) / 4;
    float in[N];
#pragma unroll
    for (int j = 0; j < N; ++j) in[j] = row[(j - S) * kBandStride];
    float k[4 * NC];
#pragma unroll
    for (int t = 0; t < NC; ++t) {
        const float4 v = reinterpret_cast<const float4*>(cf)[t];
        k[4 * t] = v.x;
        k[4 * t + 1] = v.y;
        k[4 * t + 2] = v.z;
        k[4 * t + 3] = v.w;
    }
#pragma unroll
    for (int d = 0; d <= 2 * S; ++d)
#pragma unroll
        for (int o = 0; o < O; ++o) acc[o] = fmaf(k[d], in[o + d], acc[o]);
}

// A wide pair: offsets lo .. lo + len - 1 in steps of four (coefficients past len are
// zero), from the slot row of azimuth a0 + lo wrapped into [0, A).  A step reads the
// rows m .. m + kBandO + 2 of its start m in [0, A) (the trailing copies cover those
// past A - 1); the start advances by four rows and wraps once it passes the last
// azimuth.  slot: the lane's column in row 0 of the slot.
template <int A>
__device__ __forceinline__ void band_wide(float (&acc)[kBandO], const float* slot, int a0, int lo,
                                          int len, const float* cf) {
    constexpr int O = kBandO;
    const int m0 = a0 + lo;   // >= 1 - A / 2 - ... > -A
    const float* r = slot + (m0 < 0 ? m0 + A + kBandLead : m0 + kBandLead) * kBandStride;
    const float* const rend = slot + (A + kBandLead) * kBandStride;
    const float4* k4 = reinterpret_cast<const float4*>(cf);
    for (int j0 = 0; j0 < len; j0 += 4) {
        float in[O + 3];
#pragma unroll
        for (int u = 0; u < O + 3; ++u) in[u] = r[u * kBandStride];
        const float4 k = *k4++;
        const float kk[4] = {k.x, k.y, k.z, k.w};
#pragma unroll
        for (int d = 0; d < 4; ++d)
#pragma unroll
            for (int o = 0; o < O; ++o) acc[o] = fmaf(kk[d], in[o + d], acc[o]);
        r += 4 * kBandStride;
        r = r >= rend ? r - A * kBandStride : r;
    }
}

template <int A, bool YNT>
__global__ __launch_bounds__(8 * A) void banded_euler_kernel(BatchArgs B) {
    constexpr int O = kBandO, NW = A / (2 * O), ROWS = kBandLead + A + kBandTrail;
    constexpr int SLOT = ROWS * kBandStride;
    extern __shared__ float ring[];
    int pi, local;
    if (!locate(B, KT_SC, xcd_remap(blockIdx.x, gridDim.x), pi, local)) return;
    const StepArgs a = args_of(B, pi);   // by value: no reloads after stores
    const int tid = threadIdx.x, wave = tid >> 6, h = (tid >> 5) & 1, c = tid & 31;
    const int a0 = (2 * wave + h) * O;
    const int nx = a.nx, ny = a.ny, L = a.n_lev, R = a.reach, NS = 2 * R + 2;
    const int C = (int)a.C, CM = a.bcmax;
    const int64_t P = a.P;
    const int c0 = local * kBandCells, cell = c0 + c;
    const bool in = cell < C;
    float* stage = ring + NS * SLOT;   // two buffers of CM coefficients
    // then two (cx, cy) tables of the level's ordinates (8-byte aligned)
    float2* cxys = reinterpret_cast<float2*>(stage + 2 * ((CM + 1) & ~1));
    const ASN_G QInfo* __restrict__ qtab = gp(a.qi);
    const ASN_K QInfo* qk = kp(a.qi);
    const ASN_K uint4* ldesc = kp(a.band);
    const ASN_K int2* lrange = kp(a.brange);
    const ASN_G float* __restrict__ bcoef = gp(a.bcoef);

    float4 cf = make_float4(0.f, 0.f, 0.f, 0.f);
    float isov = 0.f;
    if (in) {
        cf = gp(a.coef)[cell];
        isov = gp(a.iso)[cell];
    }
    const int y = cell / nx, x = cell - y * nx;
    const int e = in ? ((x == 0 ? 1 : 0) | (x == nx - 1 ? 2 : 0) | (y == 0 ? 4 : 0) |
                        (y == ny - 1 ? 8 : 0))
                     : 0;
    const bool wedge = __ballot(e != 0) != 0;   // some lane of the wave is on the boundary
    // Memory is reached through one buffer descriptor per level (uniform; the two
    // halves of a wave hold different azimuths) and a per-lane byte offset within the
    // level, (a0 + o) P + cell floats; offsets at or beyond the level read 0.
    const uint32_t lvl_bytes = (uint32_t)(A * P * 4);
    const uint32_t pb = (uint32_t)(P * 4);   // bytes of an azimuth plane
    // the lane's cell in its first azimuth plane (plane o: + o pb)
    const uint32_t off0 = 4u * (uint32_t)(a0 * P) + 4u * (uint32_t)cell;
    // its y-upwind cell; kOOB (reads 0, the vacuum ghost) where that lies outside the grid
    uint32_t yoff[O];
    // per output azimuth (the direction is the same on every level): the x-upwind value
    // is the left neighbour (tl), the right one (tr) or a ghost (neither); ox / oy: the
    // cell's x / y face is an outflow face
    bool tl[O], tr[O], ox[O], oy[O];
#pragma unroll
    for (int o = 0; o < O; ++o) {
        const int d = qtab[a0 + o].dir;
        const int yc = (d & 4) ? cell - nx : cell + nx;
        yoff[o] = (in && yc >= 0 && yc < C) ? off0 + (uint32_t)o * pb + 4u * (uint32_t)(yc - cell)
                                             : kOOB;
        const bool gx = !in || (d & e & 3) != 0;
        tl[o] = !gx && (d & 1);
        tr[o] = !gx && !(d & 1);
        const int go = (((d & 5) << 1) | ((d & 10) >> 1)) & e;   // outflow faces of d
        ox[o] = in && (go & 3);
        oy[o] = in && (go & 12);
    }

    const size_t lvl_floats = (size_t)A * (size_t)P;
    auto level_rsrc = [&](const float* base) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, (int)lvl_bytes,
                                                 kRsrcWord3);
    };

    // Ring fill: the lane's kBandO azimuths of level l, cell c.  Lanes 0 and 31 also
    // fetch the cell before / after the block (the other lanes' halo offsets lie
    // outside the level and read 0) into column 0 / 33 of the row; the other lanes
    // write theirs into a padding column.  The first kBandTrail and the last kBandLead
    // azimuths are also written to their wrapped copy (other rows: to themselves
    // again).  No branches.
    struct Fill {
        float v[O], lo[O];   // the cell, and the block's halo cell (lanes 0 and 31)
    };
    const int hcol = c == 0 ? 0 : (c == 31 ? 33 : 34);
    // the halo cell's offset in plane o (kOOB: reads 0)
    const bool hvalid = (c == 0 && c0 > 0) || c == 31;
    const uint32_t hdel = c == 0 ? (uint32_t)-4 : 4u;
    uint32_t hoff[O];
#pragma unroll
    for (int o = 0; o < O; ++o) hoff[o] = hvalid ? off0 + (uint32_t)o * pb + hdel : kOOB;
    // the lane's rows for azimuth a0 + o: own (rrow0 + o kBandStride), wrapped copies
    // after the last and before the first azimuth (at most one unless A < lead + trail)
    constexpr bool kTwoCopies = A < kBandLead + kBandTrail;
    const int rrow0 = (a0 + kBandLead) * kBandStride;
    // byte distance from the row of azimuth a0 + o to its (first) wrapped copy
    int cpy[O];
#pragma unroll
    for (int o = 0; o < O; ++o) {
        const int az = a0 + o;
        const int up = az < kBandTrail ? A * kBandStride : 0;
        const int dn = az >= A - kBandLead ? -A * kBandStride : 0;
        cpy[o] = 4 * (kTwoCopies ? up : (up != 0 ? up : dn));
    }
    auto fetch = [&](const float* base, Fill& f) {
        const __amdgpu_buffer_rsrc_t r = level_rsrc(base);
#pragma unroll
        for (int o = 0; o < O; ++o) {
            f.v[o] = load_plane(r, off0 + (uint32_t)o * pb);
            f.lo[o] = load_plane(r, hoff[o]);
        }
    };
    auto put = [&](int slot, const Fill& f) {
        float* s = ring + slot * SLOT;
#pragma unroll
        for (int o = 0; o < O; ++o) {
            const int az = a0 + o, rr = rrow0 + o * kBandStride;
            const int dn = az >= A - kBandLead ? rr - A * kBandStride : rr;
            float* pv = s + rr + c + 1;
            float* ph = s + rr + hcol;
            *pv = f.v[o];
            *ph = f.lo[o];
            *reinterpret_cast<float*>(reinterpret_cast<char*>(pv) + cpy[o]) = f.v[o];
            *reinterpret_cast<float*>(reinterpret_cast<char*>(ph) + cpy[o]) = f.lo[o];
            if constexpr (kTwoCopies) {
                s[dn + c + 1] = f.v[o];
                s[dn + hcol] = f.lo[o];
            }
        }
    };
    // a level's coefficients: thread t holds number t (the count is below the block
    // size: at most 2 reach + 1 runs of at most n_az), and threads 0 .. 2 n_az - 1 the
    // level's cx, cy (thread 2 m + k: component k of azimuth m)
    struct Coef {
        float k, c;
    };
    auto fetch_coef = [&](int l) {
        const int2 rg = lrange[l];
        Coef v;
        v.k = bcoef[rg.x + min(tid, rg.y - 1)];
        v.c = reinterpret_cast<const ASN_G float*>(qtab + l * A + min(tid >> 1, A - 1))[tid & 1];
        return v;
    };
    auto put_coef = [&](int l, const Coef& v) {
        if (tid < CM) stage[(l & 1) * CM + tid] = v.k;
        if (tid < 2 * A) reinterpret_cast<float*>(cxys + (l & 1) * A)[tid] = v.c;
    };
    // per level, loaded one level ahead (after the level's stores, so that the wait
    // for them in the next epilogue does not also wait for the prefetches, which are
    // issued later): the y-upwind values and the ordinates' constants (the weight w_q
    // of a product set depends on the level only: a scalar load)
    struct Ahead {
        float y[O];
        double w;
    };
    // base: the level's planes; q0: its first ordinate
    // The y-upwind row belongs to the block nx / kBandCells blocks away.  With YNT (rows
    // of kBandWideRowCells or more) that block runs about half a block's time apart (an
    // XCD holds 64 blocks) and its lines are no longer in the L2: they are read
    // non-temporally, so they do not push out lines that are (1024^2 x 2048: -0.8 %, with
    // the non-temporal stores -3.9 %; on narrower rows the L2 still serves them and the
    // same reads cost 2 to 3 %; measured).
    auto fetch_ahead = [&](const float* base, int q0, Ahead& ah) {
        const __amdgpu_buffer_rsrc_t r = level_rsrc(base);
#pragma unroll
        for (int o = 0; o < O; ++o)
            ah.y[o] = YNT ? load_plane_nt(r, yoff[o]) : load_plane(r, yoff[o]);
        ah.w = qk[q0].w;
    };

    {   // prologue: levels 0 .. reach into the ring, level 0's coefficients staged
        Fill f;
        for (int l = 0; l <= R && l < L; ++l) {
            fetch(a.psi + (uint32_t)l * lvl_floats, f);
            put(l, f);   // slot l
        }
        put_coef(0, fetch_coef(0));
    }
    // The values loaded a level ahead alternate between two register sets (the loop
    // body is written twice), and every load is unconditional (the last level again
    // near the end), so no loop-carried copy of a load in flight forces a wait.
    Coef cpre = fetch_coef(min(1, L - 1));
    Fill pre;
    // level cursors (uniform), advanced once per level and held at the last level:
    // pf the planes of the level fetched next, pa / qa those and the first ordinate of
    // the level whose constants are loaded next, po the output planes of level i
    const float* pf = a.psi + (uint32_t)min(R + 1, L - 1) * lvl_floats;
    fetch(pf, pre);
    pf += (R + 2 <= L - 1) ? lvl_floats : 0;
    const float* pa = a.psi;
    int qa = 0;
    float* po = a.psi_new;
    Ahead ahA, ahB;
    uint4 dA = ldesc[0], dB = ldesc[1];   // level 0's descriptor
    uint4 eA = dA, eB = dB;               // level 1's (set in the loop)
    fetch_ahead(pa, qa, ahA);
    const bool more_levels = L > 1;
    pa += more_levels ? lvl_floats : 0;
    qa += more_levels ? A : 0;
    lds_barrier();

    double phacc = 0.0, defect = 0.0, outflow = 0.0;
    // level i in ring slot si, level i + reach + 1 goes into slot sp: `pre` holds level
    // i + reach + 1 and is refilled with level i + reach + 2, `cpre` holds level i + 1's
    // coefficients and is refilled with level i + 2's; `d0`, `d1` / `ah` hold level i's
    // descriptor / constants and y-upwind values, `n0`, `n1` / `ah_next` receive level
    // i + 1's
    auto level = [&](int i, int si, int sp, const uint4& d0, const uint4& d1, uint4& n0,
                     uint4& n1, const Ahead& ah, Ahead& ah_next) {
        // into the slot level i - reach - 1 held and the buffer level i - 1's coefficients
        // held (their last readers passed the barrier)
        if (i + R + 1 < L) put(sp, pre);
        put_coef(i + 1, cpre);
        cpre = fetch_coef(min(i + 2, L - 1));
        fetch(pf, pre);
        pf += (i + R + 3 <= L - 1) ? lvl_floats : 0;
        // contraction, one pair of levels at a time
        const float* cbuf = stage + (i & 1) * CM;
        float acc[O];
#pragma unroll
        for (int o = 0; o < O; ++o) acc[o] = 0.f;
        const int n_pairs = (int)d0.x;
        // pair codes in the kernel's form (band_device_code), loaded with the level's
        // descriptor a level ahead and shifted through scalar registers (no scalar load
        // in flight in the loop, so the waits for a pair's LDS rows can be partial)
        uint32_t c0 = d0.y, c1 = d0.z, c2 = d0.w, c3 = d1.x, c4 = d1.y, c5 = d1.z, c6 = d1.w;
        for (int p = 0; p < n_pairs; ++p) {
            const uint32_t code = c0;
            c0 = c1;
            c1 = c2;
            c2 = c3;
            c3 = c4;
            c4 = c5;
            c5 = c6;
            const uint32_t w = code >> 24;
            const float* slot =
                reinterpret_cast<const float*>(reinterpret_cast<const char*>(ring) + (code & 0x1FFFFu)) +
                c + 1;
            const float* cfp = cbuf + 4 * ((code >> 17) & 127u);
            if (w <= (uint32_t)kBandNarrow) {
                const float* row = slot + (a0 + kBandLead) * kBandStride;
                switch (w) {
                    case 0: band_narrow<0>(acc, row, cfp); break;
                    case 1: band_narrow<1>(acc, row, cfp); break;
                    case 2: band_narrow<2>(acc, row, cfp); break;
                    case 3: band_narrow<3>(acc, row, cfp); break;
                    case 4: band_narrow<4>(acc, row, cfp); break;
                    case 5: band_narrow<5>(acc, row, cfp); break;
                    case 6: band_narrow<6>(acc, row, cfp); break;
                    case 7: band_narrow<7>(acc, row, cfp); break;
                    default: band_narrow<8>(acc, row, cfp); break;
                }
            } else {
                const bool whole = w == kBandRingTag;
                const int s = (int)w - (int)kBandWideTag;
                band_wide<A>(acc, slot, a0, whole ? 1 - A / 2 : -s, whole ? A : 2 * s + 1, cfp);
            }
        }
        // level i + 1's descriptor, after the contraction: a scalar load in flight there
        // would make every wait for LDS rows a full one
        n0 = ldesc[2 * min(i + 1, L - 1)];
        n1 = ldesc[2 * min(i + 1, L - 1) + 1];
        // stream + collide of the lane's outputs:
        //   psi' = psi + [cx (ux - psi) + cy (uy - psi) - aa psi + gs (Y - psi) + bs (iso - psi) + ss]
        // (aa = dt sigma_a, bs = dt sigma_s, gs = dt sigma_as, ss = dt q), the bracket
        // in one chain of FMAs; no coefficient of psi is folded into a per-cell constant,
        // whose rounding would bias every ordinate of the cell alike.  Phi takes each new
        // value in FP64; the collision term's sum over the outputs, gs sum (Y - psi) +
        // bs sum (iso - psi), is formed in FP32 (small terms) and added once per level.
        const float* own = ring + si * SLOT + (a0 + kBandLead) * kBandStride + c + 1;
        const float2* cxy = cxys + (i & 1) * A + a0;   // the outputs' (cx, cy)
        const __amdgpu_buffer_rsrc_t ro = level_rsrc(po);
        po += lvl_floats;
        // The cells and both x neighbours of every output read first (one LDS round
        // trip), or each output's as it is updated (the upwind one only): the first is
        // faster where a SIMD holds three waves of this kernel (n_az 32, 48), the second
        // at four (n_az 64; measured)
        constexpr bool kEarly = NW < 8;
        float vl[O], vv[O], vr[O];
        if constexpr (kEarly) {
#pragma unroll
            for (int o = 0; o < O; ++o) {
                const float* pc = own + o * kBandStride;
                vl[o] = pc[-1];
                vv[o] = pc[0];
                vr[o] = pc[1];
            }
        }
        float sd = 0.f;
#pragma unroll
        for (int o = 0; o < O; ++o) {
            const float* pc = own + o * kBandStride;
            if constexpr (!kEarly) vv[o] = pc[0];
            const float v = vv[o];
            const float ux = kEarly ? (tl[o] ? vl[o] : (tr[o] ? vr[o] : 0.f))
                                    : (tl[o] ? pc[-1] : (tr[o] ? pc[1] : 0.f));
            const float uy = ah.y[o];
            const float dy = acc[o] - v;
            float t = fmaf(cf.y, isov - v, cf.w);
            t = fmaf(cf.z, dy, t);
            t = fmaf(-cf.x, v, t);
            const float2 cc = cxy[o];
            t = fmaf(cc.y, uy - v, t);
            t = fmaf(cc.x, ux - v, t);
            // a padding cell (not in) has psi = 0, zero coefficients and zero upwind
            // values, so it stays zero
            const float nv = v + t;
            store_plane_nt(nv, ro, off0 + (uint32_t)o * pb);   // read next step, not from L2
            phacc += ah.w * (double)nv;
            sd += dy;
        }
        defect += ah.w * (double)(in ? cf.z * sd : 0.f);
        if (wedge) {
            float ob = 0.f;
#pragma unroll
            for (int o = 0; o < O; ++o)
                ob += (ox[o] ? cxy[o].x * vv[o] : 0.f) + (oy[o] ? cxy[o].y * vv[o] : 0.f);
            outflow += ah.w * (double)ob;
        }
        fetch_ahead(pa, qa, ah_next);
        const bool adv = i + 2 <= L - 1;
        pa += adv ? lvl_floats : 0;
        qa += adv ? A : 0;
        lds_barrier();
    };
    int si = 0, sp = R + 1;   // ring slots of levels i and i + reach + 1
    auto next_slot = [NS](int s) { return s + 1 == NS ? 0 : s + 1; };
    for (int i = 0; i < L; i += 2) {
        level(i, si, sp, dA, dB, eA, eB, ahA, ahB);
        si = next_slot(si);
        sp = next_slot(sp);
        if (i + 1 >= L) break;
        level(i + 1, si, sp, eA, eB, dA, dB, ahB, ahA);
        si = next_slot(si);
        sp = next_slot(sp);
    }

    // Phi^{n+1} of each cell: the 2 NW lane groups' partials in a fixed order
    double* red = reinterpret_cast<double*>(ring);
    red[(2 * wave + h) * kBandCells + c] = phacc;
    lds_barrier();
    if (tid < kBandCells && in) {
        double s = red[c];
#pragma unroll
        for (int g = 1; g < 2 * NW; ++g) s += red[g * kBandCells + c];
        gp(a.phi_part)[cell] = s;
    }
    // the physical scattering's part of the collision defect, sum_q w_q bs (iso - psi_q)
    // = bs (W iso - Phi), once per cell (Phi of psi^n in FP64)
    if (wave == 0 && h == 0 && in)
        defect += (double)cf.y * (a.W * (double)isov - gp(a.phi64)[cell]);
    double sums[2] = {defect, outflow};
    block_sum_waves<NW, 2>(sums, gp(a.blk_part) + 2 * (size_t)local);
}

// ---------------------------------------------------------------------------
// 6. Banded reduced-precision step (BF16 / FP16 operands, FP32 accumulate) on product
//    sets of 32, 48 or 64 azimuths.  As in the fused reduced-precision form the state is
//    stored without its pending per-cell particle correction delta (isotropic, so it
//    drops out of the rounded deviation), and only the anisotropic part is rounded:
//      x = T((psi^ - iso^) 2^(E - e_b))  (BF16: hi + lo),
//      Y^ - iso^ = 2^(e_b - E) sum_j T(C_ij) x_j + r_q (psi^ - iso^),
//    T(C_ij) the circulant block of level pair (i, j) of the stored K.  Block =
//    kBandLpCells cells x every ordinate; wave (m-tile mt, n-tile nt) owns azimuths
//    16 mt .. + 15 of cells 16 nt .. + 15, lane l the four azimuths 16 mt + 4 (l / 16) ..
//    of cell 16 nt + l % 16, which is where MFMA 16x16x32 leaves them.  Per level pair
//    and k-step of 32 azimuths one MFMA per operand term: A is the block's 16 x 32 slice
//    at the wave's azimuth offset (host-built, staged in LDS a level ahead), B eight
//    consecutive azimuths of one cell of the partner level from a ring of quantised
//    levels ([8-azimuth chunk][cell], 16-byte reads).  The ring is filled from registers
//    loaded a level before; the unrounded values of the lane's own cell wait in registers
//    (reach + 1 levels) for the level's update, which runs one level behind the products
//    and is interleaved with them; x neighbours come from the adjacent lanes (DPP) or, at
//    the edges of a 16-cell tile, from a small ring the neighbouring waves (or the block's
//    halo loads) fill at the same time.  Outputs as the fused form:
//    psi^{n+1} without its correction, per cell Phi^ and sum_q w_q Y^, budget partials,
//    block maxima of the next operand scale.
// ---------------------------------------------------------------------------
// (lanes at the row's edge get 0; the kernel takes their value from the edge ring)
__device__ __forceinline__ float dpp_from_left(float v) {   // lane l gets lane l - 1 (row of 16)
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x111, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_from_right(float v) {  // lane l gets lane l + 1 (row of 16)
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x101, 0xF, 0xF, true));
}

template <int A, int DT, int R>
__global__ __launch_bounds__(band_lp_threads(A)) void banded_lp_kernel(BatchArgs B) {
    constexpr int MT = A / 16, NT = kBandLpCells / 16, KS = band_lp_ksteps(A), TERMS = DT == 1 ? 2 : 1;
    constexpr int NW = MT * NT, T = NW * 64;
    constexpr int KC = 4 * KS;                // 16-byte chunks of 8 azimuths a cell holds
    constexpr int NS = 2 * R + 2, NE = R + 3, NP = 2 * R + 1;
    constexpr int XSLOT = band_lp_slot(A);    // elements per ring slot and term:
                                              // [chunk][cell][8 azimuths]
    constexpr int FR = NP * MT * 64;          // uint4 of A operands (NP pair slots)
    constexpr int FRX = FR + A / 2;           // and the (cx, cy) table: uint4 per buffer
    constexpr int FSL = (2 * kBandLpMaxReach + 1) * MT * 64;   // uint4 of a level's slots
    constexpr int CPT = (FRX + T - 1) / T;    // uint4 staged per thread
    extern __shared__ __attribute__((aligned(16))) char lds_raw[];
    uint16_t* xr = reinterpret_cast<uint16_t*>(lds_raw);
    uint4* fr = reinterpret_cast<uint4*>(lds_raw + (size_t)NS * TERMS * XSLOT * 2);
    float* edge = reinterpret_cast<float*>(lds_raw + (size_t)NS * TERMS * XSLOT * 2 + (size_t)2 * FRX * 16);
    int pi, local;
    if (!locate(B, KT_SC, xcd_remap(blockIdx.x, gridDim.x), pi, local)) return;
    const StepArgs a = args_of(B, pi);   // by value: no reloads after stores
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int mt = wave % MT, nt = wave / MT;
    const int g = lane >> 4, cl = lane & 15;
    const int a0 = 16 * mt + 4 * g;      // the lane's first azimuth
    const int cc = 16 * nt + cl;         // its cell within the block
    const int nx = a.nx, ny = a.ny, L = a.n_lev, RE = a.reach;
    const int C = (int)a.C;
    const int64_t P = a.P;
    const int cell = local * kBandLpCells + cc;
    const bool in = cell < C;
    const ASN_G QInfo* __restrict__ qtab = gp(a.qi);
    const ASN_K QInfo* qk = kp(a.qi);
    const ASN_K uint4* ldesc = kp(a.band);
    const ASN_G uint4* __restrict__ frag = gp(a.bfrag);
    const ASN_K float* rdk = kp(a.rdef);   // r_q, the same for every ordinate of a level

    float4 cf = make_float4(0.f, 0.f, 0.f, 0.f);
    float ihv = 0.f, dv = 0.f;   // iso^ = Phi^ / W and the pending correction of the cell
    if (in) {
        cf = gp(a.coef)[cell];
        ihv = gp(a.iso)[cell];
        dv = gp(a.delta)[cell];
    }
    float s_in, s_out;   // the cell's operand scale 2^(E - e_b) and its inverse
    {
        const float bm = in ? __uint_as_float(gp(a.bmax_cur)[cell >> a.sb_log]) : 0.f;
        int e = 0;
        if (bm > 0.f) (void)frexpf(bm, &e);
        e = max(e, -100);
        s_in = ldexpf(1.f, kScaleExp - e);
        s_out = ldexpf(1.f, e - kScaleExp);
    }
    const float ivs = ihv * s_in;
    const int y = cell / nx, x = cell - y * nx;
    const int e = in ? ((x == 0 ? 1 : 0) | (x == nx - 1 ? 2 : 0) | (y == 0 ? 4 : 0) |
                        (y == ny - 1 ? 8 : 0))
                     : 0;
    const bool wedge = __ballot(e != 0) != 0;
    const uint32_t lvl_bytes = (uint32_t)(A * P * 4), pb = (uint32_t)(P * 4);
    const uint32_t off0 = 4u * (uint32_t)(a0 * P) + 4u * (uint32_t)cell;
    // the lane's four azimuths lie in one quadrant (n_az / 4 is a multiple of 4): one
    // y-upwind cell; its offsets yoff + o pb (from kOOB they stay past every plane: a
    // level holds under 2^31 bytes, and 3 pb more stays below 2^32)
    uint32_t yoff;
    float ydl;   // pending correction of the y-upwind cell
    bool tl[4], tr[4], ox[4], oy[4];
    {
        const int d = qtab[a0].dir;
        const int yc = (d & 4) ? cell - nx : cell + nx;
        const bool yv = in && yc >= 0 && yc < C;
        ydl = yv ? gp(a.delta)[yc] : 0.f;
        yoff = yv ? off0 + 4u * (uint32_t)(yc - cell) : kOOB;
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const int d = qtab[a0 + o].dir;
        const bool gx = !in || (d & e & 3) != 0;
        tl[o] = !gx && (d & 1);
        tr[o] = !gx && !(d & 1);
        const int go = (((d & 5) << 1) | ((d & 10) >> 1)) & e;   // outflow faces of d
        ox[o] = in && (go & 3);
        oy[o] = in && (go & 12);
    }
    // the block's halo cells, one value a lane: in tile 0 lanes 0 .. 3 of each row of 16
    // read azimuth a0 + cl of the cell before the block, in the last tile lanes 12 .. 15
    // azimuth a0 + cl - 12 of the cell after it (the other lanes' halo offsets read 0)
    const bool hlo = nt == 0 && cl < 4, hhi = nt == NT - 1 && cl >= 12;
    const int hcell = hlo ? local * kBandLpCells - 1 : local * kBandLpCells + kBandLpCells;
    const int haz = a0 + (hlo ? cl : cl - 12);
    const bool hvalid = (hlo || hhi) && hcell >= 0 && hcell < (int)P;
    const float hdl = (hvalid && hcell < C) ? gp(a.delta)[hcell] : 0.f;
    const uint32_t hoff = hvalid ? 4u * (uint32_t)(haz * P) + 4u * (uint32_t)hcell : kOOB;
    const int hslot = hlo ? haz : (NT + NT - 1) * A + haz;   // its place in an edge slot
    const size_t lvl_floats = (size_t)A * (size_t)P;
    auto level_rsrc = [&](const float* base) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, (int)lvl_bytes, kRsrcWord3);
    };

    struct Fill {
        float v[4], h;
    };
    auto fetch = [&](int l, Fill& f) {
        const __amdgpu_buffer_rsrc_t r = level_rsrc(a.psi + (size_t)l * lvl_floats);
#pragma unroll
        for (int o = 0; o < 4; ++o) f.v[o] = load_plane(r, off0 + (uint32_t)o * pb);
        f.h = load_plane(r, hoff);
    };
    // the lane's four azimuths of level l into the ring (rounded operand terms) and the
    // tile-edge values (true state psi^ + delta) its neighbours need
    auto put = [&](int l, const Fill& f) {
        uint16_t* xs = xr + (size_t)(l % NS) * TERMS * XSLOT + ((a0 >> 3) * kBandLpCells + cc) * 8 + (a0 & 7);
        float xv[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) xv[o] = __builtin_fmaf(f.v[o], s_in, -ivs);
        uint2 pk;
        pk.x = pack2<DT>(xv[0], xv[1]);
        pk.y = pack2<DT>(xv[2], xv[3]);
        *reinterpret_cast<uint2*>(xs) = pk;
        if constexpr (DT == 1) {
            uint2 pl;
            pl.x = bf16_residual2(pk.x, xv[0], xv[1]);
            pl.y = bf16_residual2(pk.y, xv[2], xv[3]);
            *reinterpret_cast<uint2*>(xs + XSLOT) = pl;
        }
        float* es = edge + (size_t)(l % NE) * 2 * NT * A;
        if (cl == 15 && nt < NT - 1) {   // the left neighbour of the next tile
            float* d = es + (nt + 1) * A + a0;
#pragma unroll
            for (int o = 0; o < 4; ++o) d[o] = f.v[o] + dv;
        }
        if (cl == 0 && nt > 0) {         // the right neighbour of the previous tile
            float* d = es + (NT + nt - 1) * A + a0;
#pragma unroll
            for (int o = 0; o < 4; ++o) d[o] = f.v[o] + dv;
        }
        if (hlo || hhi) es[hslot] = f.h + hdl;   // the block's halo
    };
    // block l of the operand table into buffer l & 1 (thread t moves uint4 t and t + T):
    // level l's A operands (2 kBandLpMaxReach + 1 pair slots, the coupled pairs first; the
    // kernel runs the first NP, those past a problem's pairs hold zero operands), then the
    // (cx, cy) of level l - 1's ordinates, read by the update that runs one level behind.
    // Block n_lev holds the last level's (cx, cy).
    static_assert(CPT <= 2, "at most two staged uint4 per thread");
    auto src_of = [&](int x) { return x < FR ? x : FSL + (x - FR); };
    auto fetch_frag = [&](int l, uint4& f0, uint4& f1) {
        const ASN_G uint4* src = frag + ldesc[2 * l].y;
        f0 = src[src_of(FRX >= T ? tid : min(tid, FRX - 1))];
        if constexpr (CPT > 1) f1 = src[src_of(min(tid + T, FRX - 1))];
    };
    auto put_frag = [&](int l, const uint4& f0, const uint4& f1) {
        uint4* dst = fr + (size_t)(l & 1) * FRX;
        if (FRX >= T || tid < FRX) dst[tid] = f0;
        if constexpr (CPT > 1) if (tid + T < FRX) dst[tid + T] = f1;
    };
    // the next update's inputs: the lane's own four values (from the register queue), the
    // y-upwind values and the level's r_q and weight (its (cx, cy) come from LDS)
    struct Ahead {
        float v[4], y[4];
        float rq;
        double w;
    };
    auto fetch_ahead = [&](int l, Ahead& ah) {
        const __amdgpu_buffer_rsrc_t r = level_rsrc(a.psi + (size_t)l * lvl_floats);
        const int q0 = l * A;
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            ah.y[o] = load_plane(r, yoff + (uint32_t)o * pb);
        }
        ah.rq = rdk[q0];
        ah.w = qk[q0].w;
    };

    // n_az not a multiple of 32: the last k-step reads azimuths past n_az, which the ring
    // holds at zero (the A operands' wrapped values there multiply zeros)
    if constexpr (A % 32 != 0) {
        uint4* z = reinterpret_cast<uint4*>(xr);
        constexpr int NZ = NS * TERMS * XSLOT * 2 / 16;
        for (int t = tid; t < NZ; t += T) z[t] = make_uint4(0u, 0u, 0u, 0u);
        lds_barrier();
    }
    // The level loop runs one level behind in its update: pass i contracts level i and
    // updates level i - 1 with the products of the pass before, two independent streams
    // (LDS reads and MFMA; VALU, DPP and stores) interleaved in one schedule.  The edge
    // ring is reach + 3 levels deep: a level's edges stay until its lagging update has
    // read them.
    // the lane's own unrounded values of the levels in the ring ahead of the update
    // (levels i + 1 .. i + R + 1 at the end of pass i)
    float fifo[R + 1][4];
    {   // prologue: levels 0 .. R into the ring and the queue, level 0's operands
        Fill f;
#pragma unroll
        for (int l = 0; l <= R; ++l) {
            fetch(min(l, L - 1), f);
            if (l < L) put(l, f);
#pragma unroll
            for (int o = 0; o < 4; ++o) fifo[l][o] = f.v[o];
        }
        uint4 g0, g1;
        fetch_frag(0, g0, g1);
        put_frag(0, g0, g1);
    }
    Fill pre;
    fetch(min(R + 1, L - 1), pre);
    uint4 fp0, fp1;
    fetch_frag(1, fp0, fp1);
    Ahead ah;
    lds_barrier();

    double phacc = 0.0, ypacc = 0.0, defect = 0.0, outflow = 0.0;
    float mx = 0.f;
    const int mtk0 = ((0 - mt) % MT + MT) % MT;   // fragment of k-step 0: offset (32 kt - 16 mt) mod A
    // B operand of k-step kt: chunk g + 4 kt of the lane's cell (16 lanes of a row read
    // 256 contiguous bytes)
    const uint16_t* xl = xr + (g * kBandLpCells + cc) * 8;
    static_assert(KC * kBandLpCells * 8 == XSLOT, "ring slot layout");
    static_assert(A * 256 <= NS * TERMS * XSLOT * 2, "the final partials fit in the ring");
    // level i's products: every pair slot, k-steps of 32 azimuths, operand terms
    struct Ops {
        uint4 a[KS], b[KS];
        const uint16_t* xs;
    };
    struct Pass {
        uint32_t kcodes;
        int sb;
        const uint4* fl;
    };
    auto pass_of = [&](int i) {
        Pass ps;
        ps.kcodes = ldesc[2 * i].z;
        ps.fl = fr + (size_t)(i & 1) * FRX + lane;
        // ring slot of level i - RE (k = 0); a pair's partner i - RE + k sits k slots on
        ps.sb = ((i - RE) % NS + NS) % NS;
        return ps;
    };
    // a pair's A operands and its first operand term; the second term (BF16) is read
    // into the same registers after the first term's products
    auto load_pair = [&](const Pass& ps, int p, Ops& op) {
        int sl = ps.sb + (int)((ps.kcodes >> (4 * p)) & 15u);
        sl = sl >= NS ? sl - NS : sl;
        op.xs = xl + (size_t)sl * TERMS * XSLOT;
#pragma unroll
        for (int kt = 0; kt < KS; ++kt) op.a[kt] = ps.fl[(p * MT + (mtk0 + 2 * kt) % MT) * 64];
#pragma unroll
        for (int kt = 0; kt < KS; ++kt)
            op.b[kt] = *reinterpret_cast<const uint4*>(op.xs + 4 * kBandLpCells * 8 * kt);
    };
    auto load_term = [&](int t, Ops& op) {
#pragma unroll
        for (int kt = 0; kt < KS; ++kt)
            op.b[kt] = *reinterpret_cast<const uint4*>(op.xs + t * XSLOT + 4 * kBandLpCells * 8 * kt);
    };
    auto mul_term = [&](const Ops& op, f32x4& acc) {
#pragma unroll
        for (int kt = 0; kt < KS; ++kt) acc = mfma_lp<DT>(op.a[kt], op.b[kt], acc);
    };
    auto mul_pair = [&](Ops& op, f32x4& acc) {   // (no overlap with other work)
        mul_term(op, acc);
#pragma unroll
        for (int t = 1; t < TERMS; ++t) {
            load_term(t, op);
            mul_term(op, acc);
        }
    };
    // the update of the lane's four outputs of level j (as the fused reduced-precision form):
    //   v = psi^ + delta, dev = psi^ - iso^, Y^ - iso^ = s_out acc + r_q dev
    //   col = gs ((iso^ + Y^ - iso^) - psi^) + bs (iso^ - psi^)
    //   new = v - cx (v - ux) - cy (v - uy) - aa v + col + ss
    // (the look-ahead values hold level j)
    struct Upd {
        __amdgpu_buffer_rsrc_t ro;
        const float* es;   // the level's edge slot at the lane's tile and azimuths
        const float2* cxy;   // the level's (cx, cy) at the lane's azimuths
        float colsum, yas;
        double ph;
    };
    auto upd_begin = [&](int j, Upd& u) {
        u.es = edge + (size_t)(j % NE) * 2 * NT * A + nt * A + a0;
        u.cxy = reinterpret_cast<const float2*>(fr + (size_t)((j + 1) & 1) * FRX + FR) + a0;
        u.ro = level_rsrc(a.psi_new + (size_t)j * lvl_floats);
        u.colsum = 0.f;
        u.yas = 0.f;
        u.ph = 0.0;
    };
    auto upd_out = [&](int o, const f32x4& acc, Upd& u) {
        const float vh = ah.v[o];
        const float v = vh + dv;
        // the row shifts run in every lane (a lane whose neighbour is inactive would read
        // 0), then the row's edge lanes (0 and 15) take the edge ring's value
        const float dl = dpp_from_left(v), dr = dpp_from_right(v);
        const float left = cl == 0 ? u.es[o] : dl;
        const float right = cl == 15 ? u.es[NT * A + o] : dr;
        const float ux = tl[o] ? left : (tr[o] ? right : 0.f);
        const float uy = ah.y[o] + ydl;
        const float dev = vh - ihv;
        const float ya = s_out * acc[o] + ah.rq * dev;
        const float col = cf.z * ((ihv + ya) - vh) + cf.y * (ihv - vh);
        // a padding cell (not in) has psi^ = delta = iso^ = 0, zero coefficients, zero
        // operands and ghosts: its update is 0 without a select
        const float2 c = u.cxy[o];
        const float nv = v - c.x * (v - ux) - c.y * (v - uy) - cf.x * v + col + cf.w;
        // a wave writes half of each 128-byte line, a sibling wave the other half: the L2
        // joins them (non-temporal stores wrote 1.4x the bytes)
        store_plane(nv, u.ro, off0 + (uint32_t)o * pb);
        u.ph += (double)nv;
        u.yas += ya;
        u.colsum += col;
        mx = fmaxf(mx, fabsf(nv));
    };
    auto upd_end = [&](const Upd& u) {
        phacc += ah.w * u.ph;
        // sum over the four outputs of Y^ = iso^ + delta + (Y^ - iso^); the deviations,
        // small against iso^, summed in FP32
        ypacc += ah.w * ((in ? 4.0 * (double)(ihv + dv) : 0.0) + (double)u.yas);
        defect += ah.w * (double)u.colsum;
    };
    // the outflow of the level just updated (the look-ahead values still hold it)
    auto outflow_of = [&](const Upd& u) {
        if (wedge) {
            float ob = 0.f;
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const float v = ah.v[o] + dv;
                const float2 c = u.cxy[o];
                ob += (ox[o] ? c.x * v : 0.f) + (oy[o] ? c.y * v : 0.f);
            }
            outflow += ah.w * (double)ob;
        }
    };
    // the end of pass i: level i + R + 1 goes into the ring slot level i - R - 1 held and
    // the queue, level i leaves the queue for the next pass's update, loads for the next
    // passes
    auto advance = [&](int i) {
        if (i + R + 1 < L) put(i + R + 1, pre);
        fetch_ahead(i, ah);
#pragma unroll
        for (int o = 0; o < 4; ++o) ah.v[o] = fifo[0][o];
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int o = 0; o < 4; ++o) fifo[q][o] = fifo[q + 1][o];
#pragma unroll
        for (int o = 0; o < 4; ++o) fifo[R][o] = pre.v[o];
        fetch(min(i + R + 2, L - 1), pre);
        lds_barrier();
    };

    f32x4 accp = {0.f, 0.f, 0.f, 0.f};
    {   // pass 0: products only
        put_frag(1, fp0, fp1);
        fetch_frag(min(2, L), fp0, fp1);
        const Pass ps = pass_of(0);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            Ops op;
            load_pair(ps, p, op);
            mul_pair(op, accp);
        }
        advance(0);
    }
    for (int i = 1; i < L; ++i) {
        // block i + 1 of the operand table (its buffer's last readers passed the barrier)
        put_frag(i + 1, fp0, fp1);
        fetch_frag(min(i + 2, L), fp0, fp1);
        // pass i in chunks the scheduler may not merge: chunk p reads pair p's operands,
        // updates output p of level i - 1 while they arrive, then multiplies pair p (the
        // MFMAs run on while the next chunk issues)
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        const Pass ps = pass_of(i);
        Upd u;
        upd_begin(i - 1, u);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            __builtin_amdgcn_sched_barrier(0);
            Ops op;
            load_pair(ps, p, op);
            if (p < 4) upd_out(p, accp, u);
            mul_term(op, acc);
#pragma unroll
            for (int t = 1; t < TERMS; ++t) {
                load_term(t, op);
                mul_term(op, acc);
            }
        }
#pragma unroll
        for (int o = NP; o < 4; ++o) upd_out(o, accp, u);
        __builtin_amdgcn_sched_barrier(0);
        upd_end(u);
        accp = acc;
        outflow_of(u);
        advance(i);
    }
    {
        Upd u;
        upd_begin(L - 1, u);
#pragma unroll
        for (int o = 0; o < 4; ++o) upd_out(o, accp, u);
        upd_end(u);
        outflow_of(u);
    }

    // per cell Phi^ and sum_q w_q Y^: the (n_az / 4) lane groups' partials in a fixed order
    double* red = reinterpret_cast<double*>(lds_raw);
    red[(4 * mt + g) * kBandLpCells + cc] = phacc;
    red[(A / 4 + 4 * mt + g) * kBandLpCells + cc] = ypacc;
    lds_barrier();
    if (tid < kBandLpCells) {
        const int c = local * kBandLpCells + tid;
        if (c < C) {
            double s = red[tid], sy = red[(A / 4) * kBandLpCells + tid];
#pragma unroll
            for (int k = 1; k < A / 4; ++k) {
                s += red[k * kBandLpCells + tid];
                sy += red[(A / 4 + k) * kBandLpCells + tid];
            }
            gp(a.phi_part)[c] = s;
            gp(a.ypart)[c] = sy;
        }
    }
    // block max |psi^{n+1}| of the next operand scale: the block's cells lie in one block
    const unsigned mbits = wave_max_u32(__float_as_uint(mx));
    if (lane == 0 && mbits) atomicMax(&a.bmax_next[(local * kBandLpCells) >> a.sb_log], mbits);
    double sums[2] = {defect, outflow};
    block_sum_waves<NW, 2>(sums, gp(a.blk_part) + 2 * (size_t)local);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline unsigned div_up(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

void blocks_per_kind(const StepArgs& a, int out[KT_COUNT]) {
    const bool banded = a.band != nullptr;
    out[KT_GEMM] = banded ? 0 : (a.Qp / kGemmBM) * (int)(a.P / kGemmBN);
    out[KT_FIX] = (a.dtype != 0 && !a.fused) ? a.fin_blocks : 0;
    out[KT_SC] = (a.fused && !banded) ? 0 : a.tiles_x * a.tiles_y * a.G;
    out[KT_FIN] = a.fin_blocks;
    out[KT_BUDGET] = 1;
}

template <int A>
static void launch_banded_az(const BatchArgs& b, int blocks, size_t lds, hipStream_t s, bool wide) {
    if (wide) banded_euler_kernel<A, true><<<blocks, 8 * A, lds, s>>>(b);
    else banded_euler_kernel<A, false><<<blocks, 8 * A, lds, s>>>(b);
}

static hipError_t launch_banded(const BatchArgs& b, int blocks, int az, size_t lds, hipStream_t s,
                                bool wide) {
    switch (az) {
        case 8: launch_banded_az<8>(b, blocks, lds, s, wide); break;
        case 16: launch_banded_az<16>(b, blocks, lds, s, wide); break;
        case 24: launch_banded_az<24>(b, blocks, lds, s, wide); break;
        case 32: launch_banded_az<32>(b, blocks, lds, s, wide); break;
        case 40: launch_banded_az<40>(b, blocks, lds, s, wide); break;
        case 48: launch_banded_az<48>(b, blocks, lds, s, wide); break;
        case 56: launch_banded_az<56>(b, blocks, lds, s, wide); break;
        case 64: launch_banded_az<64>(b, blocks, lds, s, wide); break;
        default: return hipErrorInvalidValue;
    }
    return hipSuccess;
}

template <int A, int DT, int R>
static void launch_banded_lp_r(const BatchArgs& b, int blocks, size_t lds, hipStream_t s) {
    banded_lp_kernel<A, DT, R><<<blocks, band_lp_threads(A), lds, s>>>(b);
}
template <int A, int DT>
static hipError_t launch_banded_lp_a(const BatchArgs& b, int blocks, size_t lds, hipStream_t s,
                                     int reach) {
    switch (reach) {
        case 0: launch_banded_lp_r<A, DT, 0>(b, blocks, lds, s); break;
        case 1: launch_banded_lp_r<A, DT, 1>(b, blocks, lds, s); break;
        case 2: launch_banded_lp_r<A, DT, 2>(b, blocks, lds, s); break;
        case 3: launch_banded_lp_r<A, DT, 3>(b, blocks, lds, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipSuccess;
}
static hipError_t launch_banded_lp(const BatchArgs& b, int blocks, int az, int dtype, size_t lds,
                                   hipStream_t s, int reach) {
    if (az == 32 && dtype == 1) return launch_banded_lp_a<32, 1>(b, blocks, lds, s, reach);
    if (az == 32 && dtype == 2) return launch_banded_lp_a<32, 2>(b, blocks, lds, s, reach);
    if (az == 48 && dtype == 1) return launch_banded_lp_a<48, 1>(b, blocks, lds, s, reach);
    if (az == 48 && dtype == 2) return launch_banded_lp_a<48, 2>(b, blocks, lds, s, reach);
    if (az == 64 && dtype == 1) return launch_banded_lp_a<64, 1>(b, blocks, lds, s, reach);
    if (az == 64 && dtype == 2) return launch_banded_lp_a<64, 2>(b, blocks, lds, s, reach);
    return hipErrorInvalidValue;
}
template <int A, int DT, int R>
static hipError_t prepare_banded_lp_r(size_t lds) {
    return hipFuncSetAttribute((const void*)banded_lp_kernel<A, DT, R>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}
template <int A, int DT>
static hipError_t prepare_banded_lp_a(int reach, size_t lds) {
    switch (reach) {
        case 0: return prepare_banded_lp_r<A, DT, 0>(lds);
        case 1: return prepare_banded_lp_r<A, DT, 1>(lds);
        case 2: return prepare_banded_lp_r<A, DT, 2>(lds);
        case 3: return prepare_banded_lp_r<A, DT, 3>(lds);
        default: return hipErrorInvalidValue;
    }
}
hipError_t prepare_banded_lp(int band_az, int dtype, int reach, size_t band_lds) {
    if (band_az == 32 && dtype == 1) return prepare_banded_lp_a<32, 1>(reach, band_lds);
    if (band_az == 32 && dtype == 2) return prepare_banded_lp_a<32, 2>(reach, band_lds);
    if (band_az == 48 && dtype == 1) return prepare_banded_lp_a<48, 1>(reach, band_lds);
    if (band_az == 48 && dtype == 2) return prepare_banded_lp_a<48, 2>(reach, band_lds);
    if (band_az == 64 && dtype == 1) return prepare_banded_lp_a<64, 1>(reach, band_lds);
    if (band_az == 64 && dtype == 2) return prepare_banded_lp_a<64, 2>(reach, band_lds);
    return hipErrorInvalidValue;
}

template <int A>
static hipError_t prepare_banded_az(size_t lds) {
    const hipError_t e = hipFuncSetAttribute((const void*)banded_euler_kernel<A, false>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)banded_euler_kernel<A, true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t prepare_banded(int az, size_t lds) {
    switch (az) {
        case 8: return prepare_banded_az<8>(lds);
        case 16: return prepare_banded_az<16>(lds);
        case 24: return prepare_banded_az<24>(lds);
        case 32: return prepare_banded_az<32>(lds);
        case 40: return prepare_banded_az<40>(lds);
        case 48: return prepare_banded_az<48>(lds);
        case 56: return prepare_banded_az<56>(lds);
        case 64: return prepare_banded_az<64>(lds);
        default: return hipErrorInvalidValue;
    }
}

// Stencil kinds of a pass: 0 donor-cell strips, 1 / 2 Heun stages (strips), 3 donor-cell
// flat chunks, 4 / 5 Heun stages (flat chunks), kStencilBanded the banded step (its
// contraction and stencil are one kernel).
constexpr int kStencilBanded = 16;

// One pass: contraction, stencil, finalize, budget.
static hipError_t launch_pass(const BatchArgs& b, const int* grid, int dtype, int stencil,
                              int bud, hipStream_t s, hipEvent_t* ev, int band_az = 0,
                              size_t band_lds = 0, bool band_wide_rows = false,
                              int band_reach = 0) {
    hipError_t e = hipSuccess;
    auto mark = [&](int k) {
        if (ev && e == hipSuccess) e = hipEventRecord(ev[k], s);
    };
    if (stencil == kStencilBanded) {   // contraction and stencil in one kernel
        mark(0);
        e = dtype == 0 ? launch_banded(b, grid[KT_SC], band_az, band_lds, s, band_wide_rows)
                       : launch_banded_lp(b, grid[KT_SC], band_az, dtype, band_lds, s, band_reach);
        mark(1);
        mark(2);
        if (e == hipSuccess) finalize_kernel<<<grid[KT_FIN], 256, 0, s>>>(b, 0);
        mark(3);
        if (e == hipSuccess) budget_kernel<<<grid[KT_BUDGET], kBudgetThreads, 0, s>>>(b, BUD_STEP);
        mark(4);
        if (e != hipSuccess) return e;
        return hipGetLastError();
    }
    // a batch whose stencil grid is empty runs the stencil inside the contraction
    const bool fused = grid[KT_SC] == 0;
    mark(0);
    if (dtype == 0 && fused)
        gemm_f32_kernel<true><<<grid[KT_GEMM], 256, 0, s>>>(b);
    else if (dtype == 0)
        gemm_f32_kernel<false><<<grid[KT_GEMM], 256, 0, s>>>(b);
    else if (dtype == 1 && fused)
        gemm_lp_kernel<1, true><<<grid[KT_GEMM], 256, 0, s>>>(b);
    else if (dtype == 1)
        gemm_lp_kernel<1, false><<<grid[KT_GEMM], 256, 0, s>>>(b);
    else if (fused)
        gemm_lp_kernel<2, true><<<grid[KT_GEMM], 256, 0, s>>>(b);
    else
        gemm_lp_kernel<2, false><<<grid[KT_GEMM], 256, 0, s>>>(b);
    if (dtype != 0 && !fused) particle_fix_kernel<<<grid[KT_FIX], 256, 0, s>>>(b);
    mark(1);
    const bool lp = dtype != 0;
    if (!fused && stencil == 0) {
        if (lp) stream_collide_kernel<true><<<grid[KT_SC], 256, 0, s>>>(b);
        else stream_collide_kernel<false><<<grid[KT_SC], 256, 0, s>>>(b);
    } else if (!fused && stencil == 3) {
        if (lp) stream_collide_flat_kernel<true><<<grid[KT_SC], kFlatThreads, 0, s>>>(b);
        else stream_collide_flat_kernel<false><<<grid[KT_SC], kFlatThreads, 0, s>>>(b);
    } else if (!fused && stencil == 1) {
        if (lp) muscl_kernel<true, 1><<<grid[KT_SC], 256, 0, s>>>(b);
        else muscl_kernel<false, 1><<<grid[KT_SC], 256, 0, s>>>(b);
    } else if (!fused && stencil == 2) {
        if (lp) muscl_kernel<true, 2><<<grid[KT_SC], 256, 0, s>>>(b);
        else muscl_kernel<false, 2><<<grid[KT_SC], 256, 0, s>>>(b);
    } else if (!fused && stencil == 4) {
        if (lp) muscl_flat_kernel<true, 1><<<grid[KT_SC], kFlatThreads, 0, s>>>(b);
        else muscl_flat_kernel<false, 1><<<grid[KT_SC], kFlatThreads, 0, s>>>(b);
    } else if (!fused && stencil == 5) {
        if (lp) muscl_flat_kernel<true, 2><<<grid[KT_SC], kFlatThreads, 0, s>>>(b);
        else muscl_flat_kernel<false, 2><<<grid[KT_SC], kFlatThreads, 0, s>>>(b);
    }
    mark(2);
    finalize_kernel<<<grid[KT_FIN], 256, 0, s>>>(b, 0);
    mark(3);
    budget_kernel<<<grid[KT_BUDGET], kBudgetThreads, 0, s>>>(b, bud);
    mark(4);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_step(const BatchArgs& b, const int* grid, int dtype, int scheme, hipStream_t s,
                       hipEvent_t* ev, int band_az, size_t band_lds, bool band_wide_rows,
                       int band_reach) {
    if (scheme == SCHEME_EULER_BANDED)
        return launch_pass(b, grid, dtype, kStencilBanded, BUD_STEP, s, ev, band_az, band_lds,
                           band_wide_rows, band_reach);
    if (scheme != SCHEME_HEUN && scheme != SCHEME_HEUN_FLAT)
        return launch_pass(b, grid, dtype, scheme == SCHEME_EULER_FLAT ? 3 : 0, BUD_STEP, s, ev);
    const int st = scheme == SCHEME_HEUN_FLAT ? 4 : 1;   // stencil of the first pass
    BatchArgs b1 = b;
    b1.s_par = 0;
    hipError_t e = launch_pass(b1, grid, dtype, st, BUD_STAGE1, s, ev);
    if (e != hipSuccess) return e;
    b1.s_par = 1;
    return launch_pass(b1, grid, dtype, st + 1, BUD_STAGE2, s, ev ? ev + 5 : nullptr);
}

__global__ void arm_kernel(int* steps_left, int* base, int n, ArmArgs v) {
    const int i = threadIdx.x;
    if (i < n) {
        steps_left[i] = v.limit[i];
        base[i] = v.cur[i];
    }
}

hipError_t launch_arm(int* steps_left, int* base, int n, const ArmArgs& v, hipStream_t s) {
    if (n < 1 || n > kMaxArm) return hipErrorInvalidValue;
    arm_kernel<<<1, kMaxArm, 0, s>>>(steps_left, base, n, v);
    return hipGetLastError();
}

hipError_t launch_init(const StepArgs& a, const BatchArgs& one, hipStream_t s) {
    const int64_t nb = scale_blocks(a.P, a.sb_log);
    fill_u32_kernel<<<div_up(nb, 256), 256, 0, s>>>(a.bmax_cur, nb, 0u);
    fill_u32_kernel<<<div_up(nb, 256), 256, 0, s>>>(a.bmax_next, nb, 0u);
    moments_kernel<<<div_up(a.C, 256), 256, 0, s>>>(a);
    finalize_kernel<<<a.fin_blocks, 256, 0, s>>>(one, 1);
    budget_kernel<<<1, kBudgetThreads, 0, s>>>(one, BUD_INIT);
    return hipGetLastError();
}

hipError_t launch_materialize(const StepArgs& a, hipStream_t s) {
    dim3 g(div_up(a.C, 256), a.Q);
    materialize_kernel<<<g, 256, 0, s>>>(a, const_cast<float*>(a.psi));
    materialize_done_kernel<<<div_up(a.C, 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_broadcast(float* psi, const float* cell, int Q, int64_t C, int64_t P,
                            hipStream_t s) {
    dim3 g(div_up(P, 256), Q);
    broadcast_kernel<<<g, 256, 0, s>>>(psi, cell, Q, C, P);
    return hipGetLastError();
}

}  // namespace asn
