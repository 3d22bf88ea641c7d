// Test-particle tracking through an analytic wakefield and its adjoint.
#pragma once
#include <hip/hip_runtime.h>

namespace spinpic {

template <typename real>
struct TrackParams {
    real E0, kp;          // wake amplitude (m_e c omega0 / e), plasma wavenumber (omega0 / c)
    real dt, half_dt;     // time step and its half
    real r, a;            // Z / mu, anomaly
    real eps;             // r dt / 2
    int nsteps, K;        // steps, checkpoint interval
};

// state0 (real), final_state (double): component c of particle i at
// [c * n + i], 9 components x y z ux uy uz sx sy sz; ckpt holds
// ceil(nsteps / K) states in the kernels' representation.
template <typename real>
hipError_t launch_track_forward(const TrackParams<real>& P, long long n, const real* state0, real* ckpt,
                                double* final_state, double* acc, hipStream_t stream);

// scratch holds K states; grad receives dJ/d(state0) for J = c . mean final
// spin; gtheta_each (2 x n doubles, may be NULL) each particle's share of
// dJ/dE0 and dJ/dkp; acc[0..1] += their sums.
template <typename real>
hipError_t launch_track_backward(const TrackParams<real>& P, long long n, const real* state0, const real* ckpt,
                                 real* scratch, const double c[3], real* grad, double* gtheta_each,
                                 double* acc, hipStream_t stream);

}  // namespace spinpic
