// Implicit as-S_N time step (paper Section 3.4, Section 3.5, Algorithms 1-3):
// implicit Euler with second-order upwind fluxes, the artificial scattering moved
// into the sweep and resolved by source iteration, and GMRES on the scalar flux.
// FP64 on the device; the iteration control (stopping tests, the Hessenberg least
// squares of GMRES) runs on the host.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace asn {

struct ImplicitParams {
    int nx, ny, Q;
    int64_t C, P;            // cells, plane pitch
    double dx, dy, dt, W;
    double gmres_tol;        // relative residual of the scalar-flux system
    double source_tol;       // estimated error at which a source iteration stops
    bool source_relative;    // that error relative to the iterate's norm (else absolute)
    int gmres_restart;
};

class ImplicitSolver {
public:
    // omega [Q][3], w [Q], K [Q][Q] row-major (FP64, host); fields per cell (host).
    // Device memory comes from `base` (bytes() of it, 256-byte aligned).
    static size_t bytes(const ImplicitParams& p);
    bool init(const ImplicitParams& p, const double* omega, const double* w, const double* K,
              const float* sigma_s, const float* sigma_a, const float* sigma_as,
              const float* source, char* base, hipStream_t s, std::string& err);
    // psi FP32 [Q][P] on the device -> the FP64 state, its scalar flux and the budget start.
    bool set_state(const float* psi32, double* phi64_out, std::string& err);
    // The FP64 state -> FP32 [Q][P] on the device.
    bool get_state(float* psi32, std::string& err);
    // n implicit steps; phi64_out receives the scalar flux after each step.
    bool step(int64_t n, double* phi64_out, std::string& err);

    double budget[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // mass, mass0, abs, out, src, def, res, steps
    int64_t sweeps = 0, matvecs = 0;

private:
    ImplicitParams p_{};
    hipStream_t s_ = nullptr;
    double T_ = 0.0;                    // a-priori contraction bound of the source iteration
    double src_rate_ = 0.0;             // area W sum_c q_c (particles emitted per unit time)
    // device buffers
    double *psi_old_ = nullptr, *psi_a_ = nullptr, *psi_b_ = nullptr, *rhs_ = nullptr;
    double *K_ = nullptr, *wq_ = nullptr, *dq_ = nullptr, *dir_ = nullptr;
    float4* coef_ = nullptr;            // per cell {sigma_a, sigma_s, sigma_as, q}
    double* sig_ = nullptr;             // per cell sigma_a + sigma_s + sigma_as + 1/dt
    double *phi_ = nullptr, *vecs_ = nullptr, *part_ = nullptr;
    std::vector<double> hpart_;
    int nparts_ = 0;
    int* stat_ = nullptr;               // device: {stopping test met, its iteration}
    int hstat_[2] = {0, 0};

    double* vec(int i) const { return vecs_ + (size_t)i * p_.P; }
    // psi_out = L^-1 (sigma_as K psi_in + alpha sigma_s phi / W + beta (q + psi_old / dt))
    bool sweep_once(const double* psi_in, double* psi_out, const double* phi, double alpha,
                    double beta, std::string& err, const int* stop = nullptr);
    // Algorithm 1 from psi_old; returns the buffer holding the result (psi_a_ or psi_b_)
    double* source_iteration(const double* phi, double alpha, double beta, std::string& err,
                             bool& ok);
    bool moments(const double* psi, double* phi, std::string& err);
    bool dot(const double* a, const double* b, double& out, std::string& err);
    bool axpy(double* y, double alpha, const double* x, std::string& err);   // y += alpha x
    bool scale_copy(double* y, double alpha, const double* x, std::string& err);  // y = alpha x
    bool lhs(const double* v, double* out, std::string& err);   // Algorithm 2
    bool fold_budget(const double* psi_new, double mass_prev, std::string& err);
};

}  // namespace asn
