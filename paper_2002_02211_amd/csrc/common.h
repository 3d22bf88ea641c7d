// Device-side building blocks of the spin-resolved PIC step (gfx950).
//
// Particles live in a structure of arrays, grouped in segments by
// (tile, species).  A particle stores its cell as one packed int32 and its
// position inside the cell as offsets in [0, 1) per axis, so FP32 keeps full
// resolution anywhere in a large box.  Particles and the push use the type
// `real` (float or double); the grid fields E, B, J are always double, the
// type `freal` below: in FP32 the rounding of the large laser field would
// accumulate step after step in the field update.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace spinpic {

constexpr int kMaxSpecies = 4;
constexpr double kMeC2MeV = 0.51099895;   // electron rest energy, MeV
constexpr int kBlock = 256;   // threads per workgroup: 4 wave64

// ---------------------------------------------------------------- layout

template <typename real>
struct PArrays {
    int32_t* cell;    // packed cell index
    real* off[3];     // offset inside the cell along x, y, z (z unused in 2D)
    real* u[3];       // u = gamma * beta
    real* s[3];       // spin vector
    real* w;          // weight (density units)
    int32_t* id;      // row index in the initial state of its species
    int32_t* sp;      // species (leaver and overflow stores only)
};

template <typename real>
struct Fields {
    real* E[3];
    real* B[3];
    real* J[3];
    // Mur state of open x faces (NULL when periodic), 8 columns of ny nz
    // values: E_y, E_z ghosts beyond the high face, E_y, E_z of the last
    // column, B_y, B_z ghosts beyond the low face, B_y, B_z of the first
    // column, each at its last time level
    real* mur;
};

enum MurColumn { MUR_HI_GHOST = 0, MUR_HI_PREV = 2, MUR_LO_GHOST = 4, MUR_LO_PREV = 6, MUR_COLUMNS = 8 };

struct Geom {
    int ndim;
    int nsp;
    int n[3];       // cells per axis (n[2] = 1 in 2D)
    int T[3];       // tile edge per axis (T[2] = 1 in 2D)
    int nt[3];      // tiles per axis
    int ntiles;
    long long ncells;
    int open_x;     // x faces open (moving window): no wrap along x
};

// Cell word of a particle that left the box through an open x face: it is
// dropped by the leaver insertion and skipped everywhere else.
constexpr int32_t kDeadCell = -1;

template <typename real>
struct Consts {
    real dt;
    real dt_d[3];     // dt / d_a: displacement in cells per unit velocity
    real dt_d_lo[3];  // dt / d_a - dt_d[a] (0 in FP64): the rounding of dt_d, so that
                      // FP32 moves carry no systematic drift of one rounding per step
    real d_dt[3];     // d_a / dt: Esirkepov current scale
    real eps[kMaxSpecies];   // r dt / 2 with r = Z / mu
    real r[kMaxSpecies];
    real a[kMaxSpecies];
    real Z[kMaxSpecies];
    real cb[3];       // (dt / 2) / d_a  (B half step)
    real ce[3];       // dt / d_a        (E step)
    real mur_k;       // (c dt - dx) / (c dt + dx), Mur's coefficient at open x faces
    double fx_scale;  // deterministic mode: units per 1 of the fixed-point current (0: off)
};

struct Segs {
    int32_t* start;     // first slot of each (tile, species) segment
    int32_t* cap;       // slots reserved for it
    int32_t* count;     // particles it holds
    int dummy;          // first of 64 spare slots past the last segment; masked-off
                        // lanes store there so every lane issues the same stores
    int max_chunks;     // ceil(largest segment capacity / 64)
};

// Device counters (int32 unless noted), cleared at init.
enum {
    CTR_LEAVE0 = 0,   // leavers of even steps
    CTR_LEAVE1 = 1,   // leavers of odd steps
    CTR_STASH = 2,    // particles in the overflow store
    CTR_NONFINITE = 3,  // set to 1 by a push that produced a non-finite momentum or spin
    CTR_QUEUE = 8,    // next work item of the batched push: 8 per XCD queue,
                      // even steps at CTR_QUEUE, odd steps at CTR_QUEUE + 8
    CTR_NCTR = 24
};

// ---------------------------------------------------------------- fixed point
//
// The deterministic mode sums currents as 64-bit integers: a contribution v
// becomes rint(v * scale) (two's complement in an unsigned word, so that
// the hardware's unsigned atomic add does signed sums).  Integer sums do not
// depend on the order of the additions, so the result is the same on every
// run; scale is a power of two chosen so that no node's sum can pass 2^62.
template <typename acc_t>
inline constexpr bool kFixedAcc = std::is_same<acc_t, unsigned long long>::value;

__device__ inline unsigned long long to_fixed(double v, double scale) {
    return (unsigned long long)__double2ll_rn(v * scale);
}

// ---------------------------------------------------------------- cells

template <int DIM>
__host__ __device__ inline int32_t pack_cell(int cx, int cy, int cz) {
    if (DIM == 2) return cx | (cy << 16);
    return cx | (cy << 11) | (cz << 22);
}

template <int DIM>
__host__ __device__ inline void unpack_cell(int32_t c, int& cx, int& cy, int& cz) {
    if (DIM == 2) {
        cx = c & 0xFFFF;
        cy = (int)((uint32_t)c >> 16);
        cz = 0;
    } else {
        cx = c & 0x7FF;
        cy = (c >> 11) & 0x7FF;
        cz = (int)((uint32_t)c >> 22);
    }
}

__host__ __device__ inline int wrap_index(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// Element access through a uniform base pointer and a 32-bit byte offset:
// the compiler folds this into scalar-base + vector-offset loads and stores
// (one offset register shared by every array) instead of a 64-bit address
// per lane and array.  Slot counts are bounded so offsets fit in 32 bits.
// Both carry the non-temporal hint: the particle streams are read and
// written once per step, and keeping them from displacing the staged field
// and current guards that neighbouring tiles share in L2 made the c2 push
// 7 % faster (the hint on loads alone or stores alone made it slower).
template <typename T>
__device__ inline T ldo(const T* base, uint32_t byte_off) {
    return __builtin_nontemporal_load(reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off));
}
template <typename T>
__device__ inline void sto(T* base, uint32_t byte_off, T v) {
    __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off));
}

// ---------------------------------------------------------------- math

__device__ inline float fsqrt(float x) { return sqrtf(x); }
__device__ inline double fsqrt(double x) { return sqrt(x); }

// Reciprocal and reciprocal square root of arguments >= 1.  FP64 keeps the
// correctly rounded division and square root.  FP32 takes the hardware
// approximations v_rcp_f32 and v_rsq_f32 (about 1 ulp) and refines each by
// one Newton step (two fused multiply-adds), a fraction of the cost of IEEE
// division.  Unrefined, their error is biased: a particle that keeps about
// the same gamma gets the same error in 1/gamma every step, and over 100
// steps its position drifted by twice what float32 storage costs.
__device__ inline float recip(float x) {
    const float y = __builtin_amdgcn_rcpf(x);
    return fmaf(fmaf(-x, y, 1.0f), y, y);          // y (2 - x y)
}
__device__ inline double recip(double x) { return 1.0 / x; }
__device__ inline float rsqrt1(float x) {
    const float y = __builtin_amdgcn_rsqf(x);
    const float h = 0.5f * x * y;
    return fmaf(fmaf(-h, y, 0.5f), y, y);          // y (3/2 - x y^2 / 2)
}
__device__ inline double rsqrt1(double x) { return 1.0 / sqrt(x); }

template <typename real>
__device__ inline void cross(const real a[3], const real b[3], real out[3]) {
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

template <typename real>
__device__ inline real dot3(const real a[3], const real b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// ---------------------------------------------------------------- stencils
//
// Along one axis a particle sits in cell l at offset o.  A component stored
// at integer positions is interpolated from nodes l, l+1 with weight o on
// l+1; a component stored at half-integer positions (index i holds i + 1/2)
// from the two half points that straddle the particle.
template <typename real>
struct Stencil1 {
    int li;  real fi;    // integer-staggered: first node, weight of the second
    int lh;  real fh;    // half-staggered
};

template <typename real>
__device__ inline Stencil1<real> stencil1(int l, real o) {
    Stencil1<real> st;
    st.li = l;
    st.fi = o;
    const bool upper = o >= real(0.5);
    st.lh = upper ? l : l - 1;
    st.fh = upper ? o - real(0.5) : o + real(0.5);
    return st;
}

template <typename real>
__device__ inline real lerp(real a, real b, real f) { return a + f * (b - a); }

// Field source in the shared-memory tile: element (i, j, k) of a component
// is the value at local cell (i, j, k), for i in -1 .. T (guard included).
template <typename real, int DIM>
struct TileFields {
    const real* base;   // 6 components of G values each: Ex Ey Ez Bx By Bz
    int Gx, Gxy, G;
    __device__ inline const real* comp(int c, int i, int j, int k) const {
        return base + c * G + (DIM == 3 ? (k + 1) * Gxy : 0) + (j + 1) * Gx + (i + 1);
    }
    __device__ inline int sx() const { return 1; }
    __device__ inline int sy() const { return Gx; }
    __device__ inline int sz() const { return Gxy; }
};

// Interpolate component c whose per-axis stagger is (hx, hy, hz) (1 = half).
template <typename real, int DIM>
__device__ inline real interp(const TileFields<real, DIM>& F, int c,
                                   const Stencil1<real> st[3], int hx, int hy, int hz) {
    const int i = hx ? st[0].lh : st[0].li;
    const real fx = hx ? st[0].fh : st[0].fi;
    const int j = hy ? st[1].lh : st[1].li;
    const real fy = hy ? st[1].fh : st[1].fi;
    if (DIM == 2) {
        const real* q = F.comp(c, i, j, 0);
        const real lo = lerp(q[0], q[1], fx);
        const real hi = lerp(q[F.Gx], q[F.Gx + 1], fx);
        return lerp(lo, hi, fy);
    }
    const int k = hz ? st[2].lh : st[2].li;
    const real fz = hz ? st[2].fh : st[2].fi;
    const real* q = F.comp(c, i, j, k);
    const int Gx = F.Gx, Gxy = F.Gxy;
    const real a0 = lerp(lerp(q[0], q[1], fx), lerp(q[Gx], q[Gx + 1], fx), fy);
    const real a1 = lerp(lerp(q[Gxy], q[Gxy + 1], fx),
                         lerp(q[Gxy + Gx], q[Gxy + Gx + 1], fx), fy);
    return lerp(a0, a1, fz);
}

// Field source in global memory with periodic wrap (or zero beyond open x
// faces); cells are absolute.
template <typename freal, int DIM>
struct GlobalFields {
    const freal* c[6];
    int n[3];
    int open_x;
    __device__ inline freal at(int comp, int i, int j, int k) const {
        if (open_x && (i < 0 || i >= n[0])) return freal(0);
        i = wrap_index(i, n[0]);
        j = wrap_index(j, n[1]);
        k = DIM == 3 ? wrap_index(k, n[2]) : 0;
        return c[comp][((long long)k * n[1] + j) * n[0] + i];
    }
};

// Values are rounded to the push precision as they are read.
template <typename real, typename freal, int DIM>
__device__ inline real interp(const GlobalFields<freal, DIM>& F, int c,
                              const Stencil1<real> st[3], int hx, int hy, int hz) {
    const int i = hx ? st[0].lh : st[0].li;
    const real fx = hx ? st[0].fh : st[0].fi;
    const int j = hy ? st[1].lh : st[1].li;
    const real fy = hy ? st[1].fh : st[1].fi;
    auto at = [&](int ii, int jj, int kk) { return (real)F.at(c, ii, jj, kk); };
    if (DIM == 2) {
        const real lo = lerp(at(i, j, 0), at(i + 1, j, 0), fx);
        const real hi = lerp(at(i, j + 1, 0), at(i + 1, j + 1, 0), fx);
        return lerp(lo, hi, fy);
    }
    const int k = hz ? st[2].lh : st[2].li;
    const real fz = hz ? st[2].fh : st[2].fi;
    const real a0 = lerp(lerp(at(i, j, k), at(i + 1, j, k), fx),
                         lerp(at(i, j + 1, k), at(i + 1, j + 1, k), fx), fy);
    const real a1 = lerp(lerp(at(i, j, k + 1), at(i + 1, j, k + 1), fx),
                         lerp(at(i, j + 1, k + 1), at(i + 1, j + 1, k + 1), fx), fy);
    return lerp(a0, a1, fz);
}

// E and B at the particle; the stagger arguments (x, y, z) follow the Yee
// cell: E_a is half-staggered along a, B_a along the two other axes.
template <typename real, class Src>
__device__ inline void gather_all(const Src& F, const Stencil1<real> st[3], real E[3], real B[3]) {
    E[0] = interp(F, 0, st, 1, 0, 0);
    E[1] = interp(F, 1, st, 0, 1, 0);
    E[2] = interp(F, 2, st, 0, 0, 1);
    B[0] = interp(F, 3, st, 0, 1, 1);
    B[1] = interp(F, 4, st, 1, 0, 1);
    B[2] = interp(F, 5, st, 1, 1, 0);
}

// ---------------------------------------------------------------- push
//
// Boris push and Thomas-BMT rotation of one particle.  On entry u = u^(n-1/2),
// s = s^(n-1/2); on exit u^(n+1/2), s^(n+1/2).
//
// Boris: u- = u + eps E, t = eps B / gamma-, u' = u- + u- x t,
//        u+ = u- + 2/(1+t.t) u' x t, u^(n+1/2) = u+ + eps E, eps = r dt/2.
// Spin (section 2 Eq. 1-3 with q/(mc) -> r, v/c -> beta): with gamma = gamma-
// and beta = (u- + u+)/(2 gamma-),
//   Omega = r [(a + 1/gamma) B - a gamma/(gamma+1) (beta.B) beta
//              - (a + 1/(1+gamma)) beta x E],
// and ds/dt = -Omega x s = s x Omega is advanced by the same rotation with
// tau = Omega dt/2 in place of t.
template <typename real>
__device__ inline void boris_tbmt(real u[3], real s[3], const real E[3], const real B[3],
                                  real eps, real r, real a, real half_dt) {
    real kick[3], um[3], t[3], rot[3], tmp[3], uprime[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        kick[q] = eps * E[q];
        um[q] = u[q] + kick[q];
    }
    const real g2 = real(1) + dot3(um, um);
    const real igm = rsqrt1(g2);
    const real gm = g2 * igm;
    const real ke = eps * igm;
    t[0] = ke * B[0];
    t[1] = ke * B[1];
    t[2] = ke * B[2];
    cross(um, t, tmp);
    uprime[0] = um[0] + tmp[0];
    uprime[1] = um[1] + tmp[1];
    uprime[2] = um[2] + tmp[2];
    const real sfac = real(2) * recip(real(1) + dot3(t, t));
    cross(uprime, t, tmp);
    // rot = u+ - u-, the magnetic rotation's change of u
    rot[0] = sfac * tmp[0];
    rot[1] = sfac * tmp[1];
    rot[2] = sfac * tmp[2];

    // Thomas-BMT precession vector at gamma-, beta = (u- + u+)/(2 gamma-)
    // = (u- + rot/2)/gamma-
    real beta[3], bxe[3], Om[3], tau[3], sprime[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) beta[q] = (um[q] + real(0.5) * rot[q]) * igm;
    const real igp1 = recip(gm + real(1));
    const real Omega_B = a + igm;
    const real Omega_v = a * gm * igp1;
    const real Omega_E = a + igp1;
    const real bB = dot3(beta, B);
    cross(beta, E, bxe);
    const real kv = Omega_v * bB;
    Om[0] = r * (Omega_B * B[0] - kv * beta[0] - Omega_E * bxe[0]);
    Om[1] = r * (Omega_B * B[1] - kv * beta[1] - Omega_E * bxe[1]);
    Om[2] = r * (Omega_B * B[2] - kv * beta[2] - Omega_E * bxe[2]);
    tau[0] = half_dt * Om[0];
    tau[1] = half_dt * Om[1];
    tau[2] = half_dt * Om[2];
    cross(s, tau, tmp);
    sprime[0] = s[0] + tmp[0];
    sprime[1] = s[1] + tmp[1];
    sprime[2] = s[2] + tmp[2];
    const real sf = real(2) * recip(real(1) + dot3(tau, tau));
    cross(sprime, tau, tmp);
    s[0] = s[0] + sf * tmp[0];
    s[1] = s[1] + sf * tmp[1];
    s[2] = s[2] + sf * tmp[2];

    // u^(n+1/2) = u+ + eps E = u + (2 eps E + rot): the step's change is
    // summed at its own scale and added to u once, so that u (large for a
    // relativistic particle) takes one rounding per step instead of three
#pragma unroll
    for (int q = 0; q < 3; ++q) u[q] = u[q] + ((kick[q] + kick[q]) + rot[q]);
}

// Displacement in cells along axis a for velocity v: v dt / d_a with the
// step constant in two parts (exact in FP64, where the low part is 0).
template <typename real>
__device__ inline real displacement(real v, const Consts<real>& k, int a) {
    return fma(v, k.dt_d[a], v * k.dt_d_lo[a]);
}

// Advance one offset by disp cells (|disp| < 1); returns the cell change
// (-1, 0, +1) and leaves the new offset in [0, 1).  If an offset just below
// a cell edge rounds up to 1, the particle is placed at the edge of the
// next cell instead.  Written with selects, not branches: the lanes of a
// wavefront take different cases, and branches made every lane walk all
// of them with exec-mask juggling around each.
template <typename real>
__device__ inline int advance_offset(real& o, real disp) {
    const real x = o + disp;
    const bool up = x >= real(1);
    const bool dn = x < real(0);
    const real y = up ? x - real(1) : (dn ? x + real(1) : x);
    const int dc = up ? 1 : (dn ? -1 : 0);
    // x in (-ulp, 0) wraps to x + 1, which can round to 1
    const bool tie = dn && y >= real(1);
    o = tie ? real(0) : y;
    return tie ? 0 : dc;
}

// CIC shape factors before and after the move on the three nodes b, b+1, b+2
// with b = min(old cell, new cell).  Returns b relative to the old cell
// (0 or -1).  Selects, as above.
template <typename real>
__device__ inline int shape_pair(real o0, real o1, int dc, real S0[3], real S1[3]) {
    const bool neg = dc < 0, pos = dc > 0;
    const real a0 = real(1) - o0, a1 = real(1) - o1;
    S0[0] = neg ? real(0) : a0;
    S0[1] = neg ? a0 : o0;
    S0[2] = neg ? o0 : real(0);
    S1[0] = pos ? real(0) : a1;
    S1[1] = pos ? a1 : o1;
    S1[2] = pos ? o1 : real(0);
    return neg ? -1 : 0;
}

// Esirkepov current of one particle.  sink(c, i, j, k, v) adds v to J_c at
// stencil node (i, j, k) relative to the base node b (the lower of the old
// and new cell along each axis).  With q_a = -Z w d_a/dt, J_a at b + i + 1/2
// along a is q_a times the running sum of W_a over the nodes up to i, so that
// (rho^(n+1) - rho^n)/dt + div J = 0 on every node.  With DS = S1 - S0:
//   2D: W_x = DSx (S0y + DSy/2), W_y = (S0x + DSx/2) DSy, and
//       J_z = Z w v_z [S0x S0y + (DSx S0y + S0x DSy)/2 + DSx DSy/3];
//   3D: W_x = DSx (S0y S0z + DSy S0z/2 + S0y DSz/2 + DSy DSz/3), cyclic.
// The running sum up to node 1 is written as -W at node 2 (the sum over all
// three nodes vanishes), so that along an axis the particle does not cross
// every entry on node 2 is exactly zero.  The eight (2D) or twelve (3D)
// entries that can be nonzero without a crossing are added for every lane;
// the others only by lanes that changed cell.  In 3D a particle that changed
// cell along one axis e only has eight more nonzero entries: J_e one node
// further along e (4), and J_f, J_g on node 2 along e (2 each; f, g the other
// axes).  With a sink that takes linear offsets (Sink::kStrided) such lanes
// add just these eight, the axis picked per lane; lanes that crossed two or
// three axes add all 42.  (The same in 2D, five entries instead of 13, made
// the memory-bound 2D push slower.)
template <typename real, int DIM, class Sink>
__device__ inline void esirkepov(const real S0[3][3], const real S1[3][3], const int dc[3],
                                 const real q[3], real qz2d, Sink& sink) {
    real DS[3][3], h[3][3], gq[3][3], C[3][2];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            DS[a][k] = S1[a][k] - S0[a][k];
            h[a][k] = S0[a][k] + real(0.5) * DS[a][k];               // S0 + DS/2
            gq[a][k] = real(0.5) * S0[a][k] + (real(1) / real(3)) * DS[a][k];  // S0/2 + DS/3
        }
        C[a][0] = DS[a][0];
        C[a][1] = -DS[a][2];
    }
    bool crossed = false;
#pragma unroll
    for (int a = 0; a < DIM; ++a) crossed = crossed || dc[a] != 0;
    if (DIM == 2) {
        // J_x(k, l) = qx C_x[k] h_y[l];  J_y(k, l) = qy h_x[k] C_y[l];
        // J_z(k, l) = qz (S0x[k] h_y[l] + DSx[k] g_y[l])
        const real ax = q[0] * C[0][0], ay = q[1] * C[1][0];
        sink.add(0, 0, 0, 0, ax * h[1][0]);
        sink.add(0, 0, 1, 0, ax * h[1][1]);
        sink.add(1, 0, 0, 0, ay * h[0][0]);
        sink.add(1, 1, 0, 0, ay * h[0][1]);
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int l = 0; l < 2; ++l)
                sink.add(2, k, l, 0, qz2d * (S0[0][k] * h[1][l] + DS[0][k] * gq[1][l]));
        if (crossed) {
            sink.add_nz(0, 0, 2, 0, ax * h[1][2]);
            const real bx = q[0] * C[0][1];
#pragma unroll
            for (int l = 0; l < 3; ++l) sink.add_nz(0, 1, l, 0, bx * h[1][l]);
            sink.add_nz(1, 2, 0, 0, ay * h[0][2]);
            const real by = q[1] * C[1][1];
#pragma unroll
            for (int k = 0; k < 3; ++k) sink.add_nz(1, k, 1, 0, by * h[0][k]);
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int l = 0; l < 3; ++l)
                    if (k == 2 || l == 2)
                        sink.add_nz(2, k, l, 0, qz2d * (S0[0][k] * h[1][l] + DS[0][k] * gq[1][l]));
        }
        return;
    }
    // 3D: J_a(k, jb, jc) = q_a C_a[k] T_a(jb, jc) with the transverse factor
    // T_a(jb, jc) = S0b[jb] h_c[jc] + DSb[jb] g_c[jc], b, c the axes after a
    // in cyclic order
    real T[3][2][2], qa0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int b = (a + 1) % 3;
        const int c = (a + 2) % 3;
        qa0[a] = q[a] * C[a][0];
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int jc = 0; jc < 2; ++jc) {
                int idx[3];
                idx[a] = 0;
                idx[b] = jb;
                idx[c] = jc;
                T[a][jb][jc] = S0[b][jb] * h[c][jc] + DS[b][jb] * gq[c][jc];
                sink.add(a, idx[0], idx[1], idx[2], qa0[a] * T[a][jb][jc]);
            }
    }
    if (!crossed) return;
    bool all42 = true;
    if constexpr (Sink::kStrided) {
        const int nx = (dc[0] != 0) + (dc[1] != 0) + (dc[2] != 0);
        all42 = nx > 1;
        if (nx == 1) {
            // the crossed axis e, and f = e + 1, g = e + 2 (cyclic): pk picks
            // the value belonging to e from the ones for e = 0, 1, 2
            const bool x0 = dc[0] != 0, x1 = dc[1] != 0;
            auto pk = [&](auto v0, auto v1, auto v2) { return x0 ? v0 : (x1 ? v1 : v2); };
            const real qe1 = pk(q[0] * C[0][1], q[1] * C[1][1], q[2] * C[2][1]);
            const real qf0 = pk(qa0[1], qa0[2], qa0[0]);
            const real qg0 = pk(qa0[2], qa0[0], qa0[1]);
            const real S0e = pk(S0[0][2], S0[1][2], S0[2][2]), DSe = pk(DS[0][2], DS[1][2], DS[2][2]);
            const real he = pk(h[0][2], h[1][2], h[2][2]), gqe = pk(gq[0][2], gq[1][2], gq[2][2]);
            const int Se = pk(sink.stride(0), sink.stride(1), sink.stride(2));
            const int Sf = pk(sink.stride(1), sink.stride(2), sink.stride(0));
            const int Sg = pk(sink.stride(2), sink.stride(0), sink.stride(1));
            const int ce = pk(sink.comp(0), sink.comp(1), sink.comp(2)) + Se;
            const int cf = pk(sink.comp(1), sink.comp(2), sink.comp(0)) + 2 * Se;
            const int cg = pk(sink.comp(2), sink.comp(0), sink.comp(1)) + 2 * Se;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                // J_e one node further along e: the core's T_e times C_e[1]
#pragma unroll
                for (int jc = 0; jc < 2; ++jc)
                    sink.add_off(ce + j * Sf + jc * Sg, qe1 * pk(T[0][j][jc], T[1][j][jc], T[2][j][jc]));
                // J_f (b = g, c = e) at node j along g, 2 along e
                const real S0g = pk(S0[2][j], S0[0][j], S0[1][j]), DSg = pk(DS[2][j], DS[0][j], DS[1][j]);
                sink.add_off(cf + j * Sg, qf0 * (S0g * he + DSg * gqe));
                // J_g (b = e, c = f) at node 2 along e, j along f
                const real hf = pk(h[1][j], h[2][j], h[0][j]), gqf = pk(gq[1][j], gq[2][j], gq[0][j]);
                sink.add_off(cg + j * Sf, qg0 * (S0e * hf + DSe * gqf));
            }
        }
    }
    if (all42) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int b = (a + 1) % 3;
            const int c = (a + 2) % 3;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const real qa = q[a] * C[a][k];
#pragma unroll
                for (int jb = 0; jb < 3; ++jb)
#pragma unroll
                    for (int jc = 0; jc < 3; ++jc) {
                        if (k == 0 && jb < 2 && jc < 2) continue;
                        int idx[3];
                        idx[a] = k;
                        idx[b] = jb;
                        idx[c] = jc;
                        sink.add_nz(a, idx[0], idx[1], idx[2],
                                    qa * (S0[b][jb] * h[c][jc] + DS[b][jb] * gq[c][jc]));
                    }
            }
        }
    }
}

}  // namespace spinpic
