// Test-particle spin tracking through an analytic wakefield and the adjoint
// of that map: the gradient of the final polarization (section 2 Eq. 4) with
// respect to the field amplitude E0, the plasma wavenumber kp and every
// particle's initial position, momentum and spin.
//
// Each step is the Boris push and the Cayley rotation of the Thomas-BMT
// equation (section 2 Eq. 1-3) of the PIC step, with the fields of a linear
// wake that moves at c along z, evaluated at the particle (xi = z - t):
//   E = (E0 kp x / 2 sin, E0 kp y / 2 sin, E0 cos),
//   B = (-E0 kp y / 4 sin, E0 kp x / 4 sin, 0),   sin, cos of kp xi.
// The particles are independent: one thread per particle runs the whole
// trajectory.  The forward pass keeps the state every K steps; the backward
// pass recomputes one K-step segment at a time into a scratch buffer and
// runs the adjoint of each step in reverse over it.  The adjoint of a step is
// written out by hand, operation by operation, in reverse order.
//
// State representation (what makes float32 work over thousands of steps):
// the longitudinal position is kept as xi = z - t, which stays small while z
// grows, and advanced by dt (beta_z - 1) written without cancellation; the
// momentum and the spin are kept as their change since t = 0, added up from
// the small per-step increments, while the initial values stay constant.  A
// float32 u_z ~ 20 would otherwise round away ~10 % of each 1e-5 kick.  The
// map is the same, so its adjoint is too.
#include "common.h"
#include "track.h"

namespace spinpic {

// Reciprocal for the tracking kernels: FP32 takes the hardware v_rcp_f32
// (about 1 ulp) without the Newton step of the PIC push.  The step keeps its
// state as small increments (above), so the FP32 gradients sit within 7e-5 to
// 4e-4 of the FP64 oracle's without it, and these kernels are bound by their
// arithmetic, which the refinement would only lengthen.
__device__ inline float trecip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double trecip(double x) { return 1.0 / x; }
// Square root of 1 + u.u (>= 1): FP32 takes the hardware v_sqrt_f32 (about
// 1 ulp) instead of the correctly rounded sequence (scaling for tiny
// arguments and two correction steps, some fifteen instructions), for the
// same reason as above.
__device__ inline float tsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double tsqrt(double x) { return sqrt(x); }

template <typename real>
struct V3 {
    real x, y, z;
};

template <typename real>
__device__ inline V3<real> v3(real a, real b, real c) {
    return V3<real>{a, b, c};
}
template <typename real>
__device__ inline V3<real> operator+(V3<real> a, V3<real> b) {
    return v3(a.x + b.x, a.y + b.y, a.z + b.z);
}
template <typename real>
__device__ inline V3<real> operator-(V3<real> a, V3<real> b) {
    return v3(a.x - b.x, a.y - b.y, a.z - b.z);
}
template <typename real>
__device__ inline V3<real> operator*(real k, V3<real> a) {
    return v3(k * a.x, k * a.y, k * a.z);
}
template <typename real>
__device__ inline real dot(V3<real> a, V3<real> b) {
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename real>
__device__ inline V3<real> cross(V3<real> a, V3<real> b) {
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// Sine and cosine of one angle.  FP32: the angle is reduced to r in
// [-pi, pi] by the nearest whole turn k (Cody and Waite's two-constant
// reduction: 2 pi = 6.28125 + 1.9353071795864769e-3, whose first part times
// k is exact for |k| < 2^16), and the hardware sine and cosine, which take
// their argument in turns, get r / (2 pi).
__device__ inline void sin_cos(float x, float* s, float* c) {
    const float k = rintf(x * 0.159154943f);
    float r = fmaf(-k, 6.28125f, x);
    r = fmaf(-k, 1.9353071795864769e-3f, r);
    const float turns = r * 0.159154943f;
    *s = __builtin_amdgcn_sinf(turns);
    *c = __builtin_amdgcn_cosf(turns);
}
__device__ inline void sin_cos(double x, double* s, double* c) { sincos(x, s, c); }

// Every intermediate of one step that its adjoint needs.
template <typename real>
struct StepVals {
    real xi, S, C, A;
    V3<real> E, B, um, tv, up1, up, un, bb, sp1, tau;
    real gm, ig, f, cB, cV, cE, bdB, fs, gn, ign;
};

// x = (x, y, xi); u and s the full momentum and spin
template <typename real>
__device__ inline void step_values(const TrackParams<real>& P, V3<real> x, V3<real> u, V3<real> s,
                                   StepVals<real>& v) {
    v.xi = x.z;
    const real ph = P.kp * v.xi;
    sin_cos(ph, &v.S, &v.C);
    v.A = P.E0 * P.kp * v.S;
    v.E = v3(real(0.5) * v.A * x.x, real(0.5) * v.A * x.y, P.E0 * v.C);
    v.B = v3(real(-0.25) * v.A * x.y, real(0.25) * v.A * x.x, real(0));
    // Boris: half kick, rotation by the Cayley map, half kick
    v.um = u + P.eps * v.E;
    v.gm = tsqrt(real(1) + dot(v.um, v.um));
    v.ig = trecip(v.gm);
    v.tv = (P.eps * v.ig) * v.B;
    v.f = real(2) * trecip(real(1) + dot(v.tv, v.tv));
    v.up1 = v.um + cross(v.um, v.tv);
    v.up = v.um + v.f * cross(v.up1, v.tv);
    v.un = v.up + P.eps * v.E;
    // Thomas-BMT precession vector at the Boris midpoint, Cayley rotation of s
    v.bb = (real(0.5) * v.ig) * (v.um + v.up);
    v.cB = P.a + v.ig;
    const real igp1 = trecip(v.gm + real(1));
    v.cV = P.a * v.gm * igp1;
    v.cE = P.a + igp1;
    v.bdB = dot(v.bb, v.B);
    const V3<real> Om = P.r * (v.cB * v.B - (v.cV * v.bdB) * v.bb - v.cE * cross(v.bb, v.E));
    v.tau = P.half_dt * Om;
    v.fs = real(2) * trecip(real(1) + dot(v.tau, v.tau));
    v.sp1 = s + cross(s, v.tau);
    // move
    v.gn = tsqrt(real(1) + dot(v.un, v.un));
    v.ign = trecip(v.gn);
}

// xi' - xi = dt (beta_z - 1), with beta_z - 1 = -(1 + ux^2 + uy^2) / (gamma (gamma + uz))
// for uz > 0 (no cancellation near beta_z = 1)
template <typename real>
__device__ inline real xi_rate(V3<real> un, real gn, real ign) {
    if (un.z > real(0)) return -(real(1) + un.x * un.x + un.y * un.y) * ign * trecip(gn + un.z);
    return un.z * ign - real(1);
}

// One step of the state (pos, du, ds): pos = (x, y, xi), u = u0 + du, s = s0 + ds.
template <typename real>
__device__ inline void forward_step(const TrackParams<real>& P, V3<real>& pos, V3<real>& du, V3<real>& ds,
                                    V3<real> u0, V3<real> s0) {
    StepVals<real> v;
    step_values(P, pos, u0 + du, s0 + ds, v);
    ds = ds + v.fs * cross(v.sp1, v.tau);
    du = du + (real(2) * P.eps) * v.E + v.f * cross(v.up1, v.tv);
    pos.x += P.dt * v.ign * v.un.x;
    pos.y += P.dt * v.ign * v.un.y;
    pos.z += P.dt * xi_rate(v.un, v.gn, v.ign);
}

// Adjoint of one step taken from position x = (x, y, xi), momentum u and spin
// s: on entry L* hold the derivative of the objective with respect to the
// state after the step, on exit with respect to the state before it (the
// xi component of Lx is the derivative with respect to xi, equal to that with
// respect to z at the same time); gE0 and gkp accumulate this step's share of
// the parameter derivatives.
template <typename real>
__device__ inline void adjoint_step(const TrackParams<real>& P, V3<real> x, V3<real> u, V3<real> s,
                                    V3<real>& Lx, V3<real>& Lu, V3<real>& Ls, double& gE0, double& gkp) {
    StepVals<real> v;
    step_values(P, x, u, s, v);
    const V3<real> Lxn = Lx, Lun = Lu, Lsn = Ls;
    // x' = x + dt ign un (xi' = xi + dt (ign un_z - 1)),  ign = 1 / sqrt(1 + un.un)
    const real Lign = P.dt * dot(v.un, Lxn);
    const real Lgn2 = real(-0.5) * v.ign * v.ign * v.ign * Lign;
    V3<real> LunT = Lun + (P.dt * v.ign) * Lxn + (real(2) * Lgn2) * v.un;
    // s' = s + fs (sp1 x tau),  sp1 = s + s x tau,  fs = 2 / (1 + tau.tau)
    const V3<real> fL = v.fs * Lsn;
    const real Lfs = dot(Lsn, cross(v.sp1, v.tau));
    const V3<real> Lsp1 = cross(v.tau, fL);
    V3<real> Ltau = cross(fL, v.sp1) + cross(Lsp1, s);
    Ls = Lsn + Lsp1 + cross(v.tau, Lsp1);
    Ltau = Ltau + (real(-1) * Lfs * v.fs * v.fs) * v.tau;
    // tau = dt/2 Om,  Om = r (cB B - cV (bb.B) bb - cE bb x E)
    const V3<real> LOm = P.half_dt * Ltau;
    const real Lobb = dot(LOm, v.bb);
    const real LcB = P.r * dot(LOm, v.B);
    const real LcV = -P.r * v.bdB * Lobb;
    const real Lbdb = -P.r * v.cV * Lobb;
    const real LcE = -P.r * dot(LOm, cross(v.bb, v.E));
    V3<real> LB = (P.r * v.cB) * LOm + Lbdb * v.bb;
    V3<real> Lbb = (-P.r * v.cV * v.bdB) * LOm + (-P.r * v.cE) * cross(v.E, LOm) + Lbdb * v.B;
    V3<real> LE = (-P.r * v.cE) * cross(LOm, v.bb);
    const real gp1 = v.gm + real(1);
    real Lig = LcB;
    const real igp1 = trecip(gp1);
    real Lgm = (LcV * P.a - LcE) * igp1 * igp1;
    // bb = ig (um + up) / 2
    V3<real> Lum = (real(0.5) * v.ig) * Lbb;
    V3<real> LupT = (real(0.5) * v.ig) * Lbb + LunT;
    Lig += real(0.5) * dot(v.um + v.up, Lbb);
    // un = up + eps E
    LE = LE + P.eps * LunT;
    // up = um + f (up1 x tv),  up1 = um + um x tv,  f = 2 / (1 + tv.tv)
    Lum = Lum + LupT;
    const V3<real> fLu = v.f * LupT;
    const real Lf = dot(LupT, cross(v.up1, v.tv));
    const V3<real> Lup1 = cross(v.tv, fLu);
    V3<real> Ltv = cross(fLu, v.up1) + cross(Lup1, v.um) + (real(-1) * Lf * v.f * v.f) * v.tv;
    Lum = Lum + Lup1 + cross(v.tv, Lup1);
    // tv = eps ig B
    Lig += P.eps * dot(v.B, Ltv);
    LB = LB + (P.eps * v.ig) * Ltv;
    // ig = 1 / gm,  gm = sqrt(1 + um.um)
    Lgm += -v.ig * v.ig * Lig;
    Lum = Lum + (Lgm * v.ig) * v.um;
    // um = u + eps E
    Lu = Lum;
    LE = LE + P.eps * Lum;
    // E, B from A = E0 kp sin(kp xi), cos(kp xi), x and y
    const real LA = real(0.5) * (x.x * LE.x + x.y * LE.y) + real(0.25) * (x.x * LB.y - x.y * LB.x);
    Lx = Lxn;
    Lx.x += real(0.5) * v.A * LE.x + real(0.25) * v.A * LB.y;
    Lx.y += real(0.5) * v.A * LE.y - real(0.25) * v.A * LB.x;
    const real LC = P.E0 * LE.z;
    const real LS = P.E0 * P.kp * LA;
    const real Lph = v.C * LS - v.S * LC;
    Lx.z += P.kp * Lph;
    gE0 += (double)(v.C * LE.z) + (double)(P.kp * v.S * LA);
    gkp += (double)(P.E0 * v.S * LA) + (double)(v.xi * Lph);
}

// SoA state arrays: component c of particle i at base[c * n + i].
template <typename real>
__device__ inline void load_state(const real* __restrict__ base, long long n, long long i, V3<real>& x,
                                  V3<real>& u, V3<real>& s) {
    x = v3(base[i], base[n + i], base[2 * n + i]);
    u = v3(base[3 * n + i], base[4 * n + i], base[5 * n + i]);
    s = v3(base[6 * n + i], base[7 * n + i], base[8 * n + i]);
}

template <typename real>
__device__ inline void store_state(real* __restrict__ base, long long n, long long i, V3<real> x, V3<real> u,
                                   V3<real> s) {
    base[i] = x.x;
    base[n + i] = x.y;
    base[2 * n + i] = x.z;
    base[3 * n + i] = u.x;
    base[4 * n + i] = u.y;
    base[5 * n + i] = u.z;
    base[6 * n + i] = s.x;
    base[7 * n + i] = s.y;
    base[8 * n + i] = s.z;
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    return v;
}

template <int NV>
__device__ inline void block_add(double (&v)[NV], double* acc) {
    __shared__ double part[kBlock / 64][NV];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum_d(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) part[wv][q] = v[q];
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) t += part[w][threadIdx.x];
        atomicAdd(acc + threadIdx.x, t);
    }
}

// Forward: state0 (9 x n: x y z ux uy uz sx sy sz at t = 0) -> final_state
// (9 x n doubles, the same at t = nsteps dt); ckpt[k] (9 x n) = the
// representation (x, y, xi, du, ds) before step k K; acc[0..2] += sum of the
// final spins.
template <typename real>
__global__ void __launch_bounds__(kBlock)
k_track_forward(TrackParams<real> P, long long n, const real* __restrict__ state0, real* __restrict__ ckpt,
                double* __restrict__ final_state, double* __restrict__ acc) {
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    double sum[3] = {0.0, 0.0, 0.0};
    if (i < n) {
        V3<real> pos, u0, s0;
        load_state(state0, n, i, pos, u0, s0);     // xi = z at t = 0
        V3<real> du = v3(real(0), real(0), real(0)), ds = du;
        for (int k = 0; k * P.K < P.nsteps; ++k) {
            store_state(ckpt + (long long)k * 9 * n, n, i, pos, du, ds);
            const int n1 = min(P.nsteps, (k + 1) * P.K);
            for (int m = k * P.K; m < n1; ++m) forward_step(P, pos, du, ds, u0, s0);
        }
        const double T = (double)P.nsteps * (double)P.dt;
        const double f[9] = {(double)pos.x, (double)pos.y, (double)pos.z + T,
                             (double)u0.x + (double)du.x, (double)u0.y + (double)du.y, (double)u0.z + (double)du.z,
                             (double)s0.x + (double)ds.x, (double)s0.y + (double)ds.y, (double)s0.z + (double)ds.z};
#pragma unroll
        for (int c = 0; c < 9; ++c) final_state[c * n + i] = f[c];
        sum[0] = f[6];
        sum[1] = f[7];
        sum[2] = f[8];
    }
    block_add<3>(sum, acc);
}

// Backward for J = c . (mean final spin): grad (9 x n) receives dJ/dx0,
// dJ/du0, dJ/ds0; gtheta_each (2 x n, may be NULL) each particle's share of
// dJ/dE0 and dJ/dkp, acc[0..1] their sums.  scratch holds K states (9 x n each).
template <typename real>
__global__ void __launch_bounds__(kBlock)
k_track_backward(TrackParams<real> P, long long n, const real* __restrict__ state0, const real* __restrict__ ckpt,
                 real* __restrict__ scratch, double cx, double cy, double cz, real* __restrict__ grad,
                 double* __restrict__ gtheta_each, double* __restrict__ acc) {
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    double g[2] = {0.0, 0.0};
    if (i < n) {
        const real inv_n = (real)(1.0 / (double)n);
        V3<real> x0, u0, s0;
        load_state(state0, n, i, x0, u0, s0);
        V3<real> Lx = v3(real(0), real(0), real(0)), Lu = Lx;
        V3<real> Ls = v3((real)cx * inv_n, (real)cy * inv_n, (real)cz * inv_n);
        const int nseg = (P.nsteps + P.K - 1) / P.K;
        for (int k = nseg - 1; k >= 0; --k) {
            const int n0 = k * P.K, n1 = min(P.nsteps, n0 + P.K);
            V3<real> pos, du, ds;
            load_state(ckpt + (long long)k * 9 * n, n, i, pos, du, ds);
            for (int m = n0; m < n1; ++m) {
                store_state(scratch + (long long)(m - n0) * 9 * n, n, i, pos, du, ds);
                forward_step(P, pos, du, ds, u0, s0);
            }
            for (int m = n1 - 1; m >= n0; --m) {
                load_state(scratch + (long long)(m - n0) * 9 * n, n, i, pos, du, ds);
                adjoint_step(P, pos, u0 + du, s0 + ds, Lx, Lu, Ls, g[0], g[1]);
            }
        }
        store_state(grad, n, i, Lx, Lu, Ls);
        if (gtheta_each) {
            gtheta_each[i] = g[0];
            gtheta_each[n + i] = g[1];
        }
    }
    block_add<2>(g, acc);
}

template <typename real>
hipError_t launch_track_forward(const TrackParams<real>& P, long long n, const real* state0, real* ckpt,
                                double* final_state, double* acc, hipStream_t stream) {
    const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_track_forward<real>), dim3(blocks), dim3(kBlock), 0, stream, P, n, state0, ckpt,
                       final_state, acc);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_track_backward(const TrackParams<real>& P, long long n, const real* state0, const real* ckpt,
                                 real* scratch, const double c[3], real* grad, double* gtheta_each,
                                 double* acc, hipStream_t stream) {
    const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_track_backward<real>), dim3(blocks), dim3(kBlock), 0, stream, P, n, state0, ckpt,
                       scratch, c[0], c[1], c[2], grad, gtheta_each, acc);
    return hipGetLastError();
}

template hipError_t launch_track_forward<float>(const TrackParams<float>&, long long, const float*, float*,
                                                double*, double*, hipStream_t);
template hipError_t launch_track_forward<double>(const TrackParams<double>&, long long, const double*,
                                                 double*, double*, double*, hipStream_t);
template hipError_t launch_track_backward<float>(const TrackParams<float>&, long long, const float*,
                                                 const float*, float*, const double*, float*, double*,
                                                 double*, hipStream_t);
template hipError_t launch_track_backward<double>(const TrackParams<double>&, long long, const double*,
                                                  const double*, double*, const double*, double*, double*,
                                                  double*, hipStream_t);

}  // namespace spinpic
