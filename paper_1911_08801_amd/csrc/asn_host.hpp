// Host-side set-up of an as-S_N problem: quadrature, kernel matrix, time step
// and operand rounding.  Plain C++ (no HIP), FP64 throughout.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace asn {

// Gauss-Legendre nodes x[n] (ascending) and weights w[n] on [-1, 1].
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// Product set: mu = Gauss-Legendre nodes, phi_k = (k + 1/2) 2 pi / n_azim,
// ordinate q = i * n_azim + k; omega is [Q][3], weights sum to 4 pi.
void product_quadrature(int n_polar, int n_azim, std::vector<double>& omega,
                        std::vector<double>& w);

// Icosahedron set of the given order (>= 2): N = 10 (order - 1)^2 + 2 ordinates on
// the subdivided faces of a regular icosahedron with a vertex at (0, 0, 1); the
// weight of a node is the area of the spherical polygon through the centres of
// its surrounding triangles.  Sorted by decreasing z, then increasing azimuth.
void icosahedron_quadrature(int order, std::vector<double>& omega, std::vector<double>& w);

// Normalised artificial in-scattering matrix K[Q][Q] (row-major) from
// S_qp = exp(-((1 - Omega_q . Omega_p)/eps)^2).  mode 0: symmetric scaling
// (rows and w-weighted columns sum to one); mode 1: row normalisation.
// Returns false (with a message) if the scaling does not converge.
bool kernel_matrix(int Q, const double* omega, const double* w, double eps, int mode,
                   std::vector<double>& K, std::string& err);

// Banded form of K for a product set of `levels` polar levels times `azim` azimuths
// (ordinate q = i * azim + k).  The set is invariant under rotations by 2 pi / azim
// about the polar axis, so K[(i, k), (j, k')] depends on i, j and (k' - k) mod azim
// only: per pair of levels one run of coefficients c_ij(delta) over azimuth offsets,
// nonzero for |delta| <= s_ij (cyclic distance).  Pair k of level i is level
// j = i + k - reach, k = 0 .. 2 reach.  A run either is symmetric, delta = -s .. s
// (2 s + 1 < azim), or covers the whole ring, delta = 1 - azim/2 .. azim/2; the runs
// of a level are stored one after the other, each zero-padded to a multiple of 4, at
// coef[range[2 i] .. range[2 i] + range[2 i + 1]).  desc[8 i .. 8 i + 7] describes
// level i: desc[8 i] is the number n of coupled pairs, desc[8 i + 1 + p] (p < n) the
// code of pair p:
//   bits 0-5   s (azim / 2 for a whole ring)       bit 6  wide: whole ring or s > narrow_max
//   bit 7      whole ring                          bits 8-10  k
//   bits 11-17 the run's start within the level, in units of 4 coefficients.
// cmax is the largest coefficient count of a level; reach the largest |i - j| with a
// nonzero.
struct BandForm {
    int levels = 0, azim = 0, reach = 0, cmax = 0;
    std::vector<uint32_t> desc;
    std::vector<int32_t> range;
    std::vector<float> coef;
};
// From the FP32 values K32[Q][Q] (row-major); false when the stored values are not
// exactly of that form (every row of a level equal to the level's first row shifted),
// when reach exceeds max_reach (at most 3) or a level has more than 508 coefficients.
// Even azim up to 126.
bool band_form(int levels, int azim, const float* K32, int max_reach, int narrow_max,
               BandForm& out);
// The A operands of MFMA 16x16x32 for pair `pair` of level `level` of a banded form of
// the BF16 (dtype 1) or FP16 (dtype 2) K: the pair's circulant block C[a][a'] =
// c((a' - a) mod azim) sliced as 16 output x 32 input azimuths at the offsets 16 f,
// f = 0 .. azim / 16 - 1 (slice f: rows m, columns k hold c((16 f + k - m) mod azim)),
// each as 64 lanes x 8 values (lane l: row l % 16, columns 8 (l / 16) .. + 7), appended
// to `out` as operand bits.  azim 32, 48 or 64 (48: columns past the last azimuth meet
// zero operands in the kernel).
void band_lp_fragments(const BandForm& bf, int level, int pair, int dtype,
                       std::vector<uint16_t>& out);
// The run of a pair code: first offset and length.
inline void band_run(uint32_t code, int azim, int& lo, int& len) {
    const int s = (int)(code & 63u);
    const bool ring = (code & 128u) != 0;
    lo = ring ? 1 - azim / 2 : -s;
    len = ring ? azim : 2 * s + 1;
}

// dt = t_final / n with n = ceil(t_final / dt_max), dt_max = cfl / max(|xi|/dx + |eta|/dy).
void cfl_time_step(int Q, const double* omega, double dx, double dy, double cfl, double t_final,
                   double& dt, int64_t& n);

// Decay rate bound of a cell-to-cell sawtooth mode in a uniform region:
//   2 max_q (|xi_q|/dx + |eta_q|/dy) + max_c (sigma_a + sigma_s + 2 (1 - min_q K_qq) sigma_as).
// K is Q x Q row-major.  dt times this is the stability number.
double stability_rate(int Q, const double* omega, const double* K, double dx, double dy, int64_t C,
                      const float* sigma_a, const float* sigma_s, const float* sigma_as);
// The streaming rule with dt_max further limited to 2 cfl / srate.
void stiff_time_step(int Q, const double* omega, double dx, double dy, double srate, double cfl,
                     double t_final, double& dt, int64_t& n);

// Round a float to bfloat16 / IEEE half bits, round to nearest, ties to even.
uint16_t float_to_bf16_rne(float f);
uint16_t float_to_half_rne(float f);
float bf16_to_float(uint16_t h);
float half_to_float(uint16_t h);

}  // namespace asn
