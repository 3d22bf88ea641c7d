// Grid kernels: the Yee FDTD update and the FP64 diagnostics (section 2
// Eq. 4 polarization, energies, charge density and div E - rho).
#include "common.h"
#include "kernels.h"

namespace spinpic {

// The current buffer of the previous step, no longer needed, is zeroed by
// the Yee step for the next step's deposit (when jclear is non-NULL).
struct JClear {
    void* c[3];
};

// ---------------------------------------------------------------- Yee step

// The Yee step in one pass: B' = B - (dt/2) curl E, E_out = E + dt (curl B'
// - J), B_out = B' - (dt/2) curl E_out.  B_x sits at (i, j+1/2, k+1/2), B_y
// at (i+1/2, j, k+1/2), B_z at (i+1/2, j+1/2, k) and E_a half a cell along
// a, so curl E takes forward and curl B backward differences, with periodic
// wrap along y and z, and along x unless its faces are open (Mur ghosts,
// below).  In 2D every d/dz is zero.  The step reads E, B and J once and
// writes E_out and B_out once (the input arrays are not written: other
// workgroups still read them as guard cells).
//
// A workgroup owns an in-plane block of cells (x, plus y in 3D) and a run of
// M planes along the marching axis (y in 2D, z in 3D).  It walks the planes
// p = m0 - 1 .. m0 + M keeping two planes of E, B' and E_out in shared
// memory: at plane p it loads E(p + 1), computes B'(p) (which needs E(p) and
// E(p + 1)), then E_out(p) (which needs B'(p) and B'(p - 1)), then B_out(p -
// 1) (which needs E_out(p - 1) and E_out(p)).  Differences inside a plane
// reach one cell: E is held on the block widened by 1 below and 2 above, B'
// by 1 on both sides, E_out by 1 above.
template <int DIM>
struct YeeBlock;
// 2D: 253 columns, so that the E tile with its guards is one row of 256
// cells, one per thread.  3D: 32 x 8 cells (an E tile of 35 x 11) on 512
// threads: against 32 x 4 on 256 threads it fetches a third fewer guard
// cells again (the 3D field update of c3 1.21 -> 1.10 ms).
template <>
struct YeeBlock<2> {
    static constexpr int RX = 253, RY = 1, M = 8, threads = 256;
};
template <>
struct YeeBlock<3> {
    static constexpr int RX = 32, RY = 8, M = 16, threads = 512;
};

template <int DIM>
struct YeeDims {
    static constexpr int RX = YeeBlock<DIM>::RX, RY = YeeBlock<DIM>::RY;
    static constexpr int EX = RX + 3, EY = DIM == 3 ? RY + 3 : 1;   // E: origin (-1, -1)
    static constexpr int BX = RX + 2, BY = DIM == 3 ? RY + 2 : 1;   // B': origin (-1, -1)
    static constexpr int FX = RX + 1, FY = DIM == 3 ? RY + 1 : 1;   // E_out: origin (0, 0)
    static constexpr int NE = EX * EY, NB = BX * BY, NF = FX * FY;
};

// Shared memory for the old Mur state of a block's rows and planes.
template <typename real, int DIM>
constexpr size_t yee_mur_lds_bytes() {
    return (size_t)MUR_COLUMNS * (YeeBlock<DIM>::M + 2) * (DIM == 3 ? YeeBlock<DIM>::RY + 2 : 1) * sizeof(real);
}

// Blocks of one grid: in-plane blocks across, runs of planes down.
template <int DIM>
__host__ __device__ inline int yee_tiles_u(const Geom& g) { return (g.n[0] + YeeBlock<DIM>::RX - 1) / YeeBlock<DIM>::RX; }
template <int DIM>
__host__ __device__ inline int yee_tiles(const Geom& g) {
    return yee_tiles_u<DIM>(g) * (DIM == 3 ? (g.n[1] + YeeBlock<DIM>::RY - 1) / YeeBlock<DIM>::RY : 1);
}
template <int DIM>
__host__ __device__ inline int yee_chunks(const Geom& g) {
    return ((DIM == 3 ? g.n[2] : g.n[1]) + YeeBlock<DIM>::M - 1) / YeeBlock<DIM>::M;
}

// Block b (0 <= b < yee_tiles * yee_chunks) of one grid's fused Yee step.
// Consecutive b walk the in-plane blocks of one run of planes before the
// next run.  Every thread of the workgroup must call it.
template <typename real, int DIM>
__device__ __attribute__((always_inline)) void yee_fused_block(const Geom& g, const Consts<real>& k,
                                                               const Fields<real>& f, const Fields<real>& out,
                                                               const JClear& jclear, int b) {
    using D = YeeDims<DIM>;
    constexpr int RX = D::RX, RY = D::RY, M = YeeBlock<DIM>::M;
    static_assert(D::NE <= YeeBlock<DIM>::threads, "one E cell per thread");
    __shared__ real sE[2][3][D::NE];
    __shared__ real sB[2][3][D::NB];
    __shared__ real sF[2][3][D::NF];

    const int tiles_u = yee_tiles_u<DIM>(g);
    const int ntile = yee_tiles<DIM>(g);
    const int chunk = b / ntile;
    const int tile = b - chunk * ntile;
    const int x0 = (tile % tiles_u) * RX;
    const int y0 = DIM == 3 ? (tile / tiles_u) * RY : 0;
    const int nx = g.n[0], ny = g.n[1];
    const int nw = DIM == 3 ? g.n[2] : g.n[1];        // planes along the marching axis
    const long long pstride = DIM == 3 ? (long long)nx * ny : nx;
    const int m0 = chunk * M;
    const int mend = min(m0 + M, nw);
    const int t = threadIdx.x;

    // Thread t holds cell t of each of the E, B' and E_out tiles and of the
    // block; its in-plane offsets are fixed (periodic wrap).
    auto inplane = [&](int u, int v) -> long long {
        const int x = wrap_index(x0 + u, nx);
        if (DIM == 3) return (long long)wrap_index(y0 + v, ny) * nx + x;
        return x;
    };
    auto plane = [&](int w) -> long long { return (long long)wrap_index(w, nw) * pstride; };
    const bool hasE = t < D::NE, hasB = t < D::NB, hasF = t < D::NF;
    // threads without a cell load cell 0 of the tile (every lane loads, so
    // the loads in flight are counted the same on every path)
    const int te = hasE ? t : 0, tb = hasB ? t : 0, tf = hasF ? t : 0;
    const long long offE = inplane(te % D::EX - 1, te / D::EX - 1);
    const long long offB = inplane(tb % D::BX - 1, tb / D::BX - 1);
    const int fu = tf % D::FX, fv = tf / D::FX;
    const long long offF = inplane(fu, fv);
    const bool ownF = hasF && fu < RX && fv < RY && x0 + fu < nx && (DIM == 2 || y0 + fv < ny);
    const int ou = t % RX, ov = t / RX;
    const bool ownO = t < RX * RY && x0 + ou < nx && (DIM == 2 || y0 + ov < ny);
    const long long offO = inplane(ou, ov);

    // Open x faces (Mur): the B' cells of the last column take E_y, E_z one
    // cell beyond from the high ghosts as they stand; the E_out cells of the
    // first column take B'_y, B'_z one cell below from the low ghosts
    // advanced to this step, and the B_out cells of the last column E_out
    // from the high ghosts advanced to this step.  The state is read from
    // f.mur and the advanced state written to out.mur, each row by the one
    // thread that owns its face cell: ghost(new) = inside(old) + k
    // (inside(new) - ghost(old)).  Blocks that also compute a neighbour's
    // face cells (a run's guard planes) advance the ghosts themselves from
    // the old state, which no block overwrites.
    const bool open = g.open_x != 0;
    const long long nrow = (long long)ny * (DIM == 3 ? g.n[2] : 1);
    auto mrow = [&](int w, int v) -> long long {
        if (DIM == 3) return (long long)wrap_index(w, nw) * ny + wrap_index(y0 + v, ny);
        return wrap_index(w, nw);
    };
    const bool hiB = open && hasB && x0 - 1 + t % D::BX == nx - 1;
    const bool loF = open && hasF && x0 + fu == 0;
    const bool hiO = open && ownO && x0 + ou == nx - 1;
    // the old state of the block's rows (planes m0 - 1 .. m0 + M, in-plane
    // rows y0 - 1 .. y0 + RY in 3D) is staged in shared memory first, so
    // that no global load of it sits in the plane loop
    // (dynamic shared memory, launched with its size only for open faces)
    constexpr int MY = DIM == 3 ? RY + 2 : 1;
    extern __shared__ __align__(16) unsigned char yee_dyn[];
    real* sMur = reinterpret_cast<real*>(yee_dyn);
    auto mur_old = [&](int col, int w, int v) -> real {
        return sMur[(col * (M + 2) + w - (m0 - 1)) * MY + (DIM == 3 ? v + 1 : 0)];
    };
    if (open) {
        for (int idx = t; idx < MUR_COLUMNS * (M + 2) * MY; idx += YeeBlock<DIM>::threads) {
            const int col = idx / ((M + 2) * MY), rem = idx - col * (M + 2) * MY;
            const int pl = rem / MY, yr = rem - pl * MY;
            sMur[idx] = f.mur[col * nrow + mrow(m0 - 1 + pl, yr - (DIM == 3 ? 1 : 0))];
        }
        __syncthreads();
    }

    // Inputs of plane p (E(p + 1), B(p), J(p)) are loaded two planes ahead
    // into one of two register sets, used by turns (the plane loop below is
    // unrolled, so each set keeps its registers).
    struct PlaneIn {
        real E[3], B[3], J[3];
    };
    // each part is loaded again as soon as its last value has been used, so
    // the new values can take the old ones' registers
    auto load_E = [&](PlaneIn& q, int p) {
        const long long c = plane(p + 1) + offE;
#pragma unroll
        for (int a = 0; a < 3; ++a) q.E[a] = f.E[a][c];
    };
    auto load_B = [&](PlaneIn& q, int p) {
        const long long c = plane(p) + offB;
#pragma unroll
        for (int a = 0; a < 3; ++a) q.B[a] = f.B[a][c];
    };
    auto load_J = [&](PlaneIn& q, int p) {
        const long long c = plane(p) + offF;
#pragma unroll
        for (int a = 0; a < 3; ++a) q.J[a] = f.J[a][c];
    };

    auto step = [&](int p, PlaneIn& q) {
        const int s0 = (p + 2) & 1, s1 = (p + 3) & 1, sm = (p + 1) & 1;   // planes p, p + 1, p - 1
        // (loads run past the run's end too, so every path has the same
        // loads in flight)
        if (hasE) {
#pragma unroll
            for (int a = 0; a < 3; ++a) sE[s1][a][t] = q.E[a];
        }
        load_E(q, p + 2);
        __syncthreads();
        // B'(p) on the block widened by 1.  Each phase takes the values one
        // cell beyond an open face as arguments.
        if (hasB) {
            const int e = (t / D::BX) * D::EX + t % D::BX;   // same cell in the E tile
            auto bprime = [&](real eyp, real ezp) {          // E_y, E_z one cell along +x
                const real ex = sE[s0][0][e], ey = sE[s0][1][e], ez = sE[s0][2][e];
                real ezy, exy;                               // +y
                if (DIM == 3) {
                    ezy = sE[s0][2][e + D::EX];
                    exy = sE[s0][0][e + D::EX];
                } else {
                    ezy = sE[s1][2][e];
                    exy = sE[s1][0][e];
                }
                real cx = k.cb[1] * (ezy - ez);
                real cy = -k.cb[0] * (ezp - ez);
                const real cz = k.cb[0] * (eyp - ey) - k.cb[1] * (exy - ex);
                if (DIM == 3) {
                    cx -= k.cb[2] * (sE[s1][1][e] - ey);
                    cy += k.cb[2] * (sE[s1][0][e] - ex);
                }
                sB[s0][0][t] = q.B[0] - cx;
                sB[s0][1][t] = q.B[1] - cy;
                sB[s0][2][t] = q.B[2] - cz;
            };
            if (hiB) {
                const int v = t / D::BX - 1;
                bprime(mur_old(MUR_HI_GHOST, p, v), mur_old(MUR_HI_GHOST + 1, p, v));
            } else {
                bprime(sE[s0][1][e + 1], sE[s0][2][e + 1]);
            }
        }
        load_B(q, p + 2);
        __syncthreads();
        if (p >= m0) {
            // E_out(p) on the block widened by 1 above
            if (hasF) {
                const int r = fv + (DIM == 3 ? 1 : 0);
                const int bb = r * D::BX + fu + 1;   // same cell in the B' tile
                const int e = r * D::EX + fu + 1;    // and in the E tile
                auto eout = [&](real bym, real bzm) {   // B'_y, B'_z one cell along -x
                    const real bx = sB[s0][0][bb], by = sB[s0][1][bb], bz = sB[s0][2][bb];
                    real bzy, bxy;                      // -y
                    if (DIM == 3) {
                        bzy = sB[s0][2][bb - D::BX];
                        bxy = sB[s0][0][bb - D::BX];
                    } else {
                        bzy = sB[sm][2][bb];
                        bxy = sB[sm][0][bb];
                    }
                    real cx = k.ce[1] * (bz - bzy);
                    real cy = -k.ce[0] * (bz - bzm);
                    const real cz = k.ce[0] * (by - bym) - k.ce[1] * (bx - bxy);
                    if (DIM == 3) {
                        cx -= k.ce[2] * (by - sB[sm][1][bb]);
                        cy += k.ce[2] * (bx - sB[sm][0][bb]);
                    }
                    const real e0 = sE[s0][0][e] + (cx - k.dt * q.J[0]);
                    const real e1 = sE[s0][1][e] + (cy - k.dt * q.J[1]);
                    const real e2 = sE[s0][2][e] + (cz - k.dt * q.J[2]);
                    sF[s0][0][t] = e0;
                    sF[s0][1][t] = e1;
                    sF[s0][2][t] = e2;
                    if (ownF && p < mend) {
                        const long long c = plane(p) + offF;
                        out.E[0][c] = e0;
                        out.E[1][c] = e1;
                        out.E[2][c] = e2;
                        if (jclear.c[0]) {
                            static_cast<real*>(jclear.c[0])[c] = real(0);
                            static_cast<real*>(jclear.c[1])[c] = real(0);
                            static_cast<real*>(jclear.c[2])[c] = real(0);
                        }
                    }
                };
                if (loF) {
                    const long long mr = mrow(p, fv);
                    const real by = sB[s0][1][bb], bz = sB[s0][2][bb];
                    const real gy = mur_old(MUR_LO_GHOST, p, fv), gz = mur_old(MUR_LO_GHOST + 1, p, fv);
                    const real py = mur_old(MUR_LO_PREV, p, fv), pz = mur_old(MUR_LO_PREV + 1, p, fv);
                    const real bym = py + k.mur_k * (by - gy);
                    const real bzm = pz + k.mur_k * (bz - gz);
                    if (ownF && p < mend) {
                        out.mur[MUR_LO_GHOST * nrow + mr] = bym;
                        out.mur[(MUR_LO_GHOST + 1) * nrow + mr] = bzm;
                        out.mur[MUR_LO_PREV * nrow + mr] = by;
                        out.mur[(MUR_LO_PREV + 1) * nrow + mr] = bz;
                    }
                    eout(bym, bzm);
                } else {
                    eout(sB[s0][1][bb - 1], sB[s0][2][bb - 1]);
                }
            }
            __syncthreads();
        }
        load_J(q, p + 2);
        if (p > m0 && p <= mend && ownO) {
            // B_out(p - 1) on the block
            const int fi = ov * D::FX + ou;                                  // E_out tile
            const int bb = (ov + (DIM == 3 ? 1 : 0)) * D::BX + ou + 1;       // B' tile
            auto bout = [&](real eyp, real ezp) {   // E_out y, z one cell along +x
                const real ex = sF[sm][0][fi], ey = sF[sm][1][fi], ez = sF[sm][2][fi];
                real ezy, exy;                      // +y
                if (DIM == 3) {
                    ezy = sF[sm][2][fi + D::FX];
                    exy = sF[sm][0][fi + D::FX];
                } else {
                    ezy = sF[s0][2][fi];
                    exy = sF[s0][0][fi];
                }
                real cx = k.cb[1] * (ezy - ez);
                real cy = -k.cb[0] * (ezp - ez);
                const real cz = k.cb[0] * (eyp - ey) - k.cb[1] * (exy - ex);
                if (DIM == 3) {
                    cx -= k.cb[2] * (sF[s0][1][fi] - ey);
                    cy += k.cb[2] * (sF[s0][0][fi] - ex);
                }
                const long long c = plane(p - 1) + offO;
                out.B[0][c] = sB[sm][0][bb] - cx;
                out.B[1][c] = sB[sm][1][bb] - cy;
                out.B[2][c] = sB[sm][2][bb] - cz;
            };
            if (hiO) {
                const long long mr = mrow(p - 1, ov);
                const real ey = sF[sm][1][fi], ez = sF[sm][2][fi];
                const real gy = mur_old(MUR_HI_GHOST, p - 1, ov), gz = mur_old(MUR_HI_GHOST + 1, p - 1, ov);
                const real py = mur_old(MUR_HI_PREV, p - 1, ov), pz = mur_old(MUR_HI_PREV + 1, p - 1, ov);
                const real eyp = py + k.mur_k * (ey - gy);
                const real ezp = pz + k.mur_k * (ez - gz);
                out.mur[MUR_HI_GHOST * nrow + mr] = eyp;
                out.mur[(MUR_HI_GHOST + 1) * nrow + mr] = ezp;
                out.mur[MUR_HI_PREV * nrow + mr] = ey;
                out.mur[(MUR_HI_PREV + 1) * nrow + mr] = ez;
                bout(eyp, ezp);
            } else {
                bout(sF[sm][1][fi + 1], sF[sm][2][fi + 1]);
            }
        }
    };

    if (hasE) {
        const long long c = plane(m0 - 1) + offE;
#pragma unroll
        for (int a = 0; a < 3; ++a) sE[(m0 + 1) & 1][a][t] = f.E[a][c];
    }
    PlaneIn qa, qb;
    load_E(qa, m0 - 1);
    load_B(qa, m0 - 1);
    load_J(qa, m0 - 1);
    load_E(qb, m0);
    load_B(qb, m0);
    load_J(qb, m0);
    // planes m0 - 1 .. m0 + M, a fixed count, fully unrolled: no loop
    // header at which the loads in flight would have to be waited for.  A
    // run cut short by the end of the grid computes its last planes on
    // wrapped data and writes nothing there.
    static_assert(M % 2 == 0, "an even number of steps");
#pragma unroll
    for (int i = 0; i < (M + 2) / 2; ++i) {
        step(m0 - 1 + 2 * i, qa);
        step(m0 + 2 * i, qb);
    }
}

// In 2D consecutive block numbers go to one XCD (workgroups are dealt
// round-robin over the 8 XCDs), so the blocks that run side by side are
// in-plane neighbours whose guard cells meet in that XCD's L2.
template <typename real, int DIM>
__global__ void __launch_bounds__(YeeBlock<DIM>::threads)
k_yee_fused(Geom g, Consts<real> k, Fields<real> f, Fields<real> out, JClear jclear) {
    const int nblk = yee_tiles<DIM>(g) * yee_chunks<DIM>(g);
    const int per = (nblk + 7) >> 3;
    // 3D: blocks in launch order (one band across the XCDs measured faster
    // than a contiguous range per XCD: c3 1.11 -> 1.03 ms; 2D the reverse)
    const int b = DIM == 3 ? (int)blockIdx.x : (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (b >= nblk) return;
    yee_fused_block<real, DIM>(g, k, f, out, jclear, b);
}

// Moving window: dst = src moved S cells towards -x, zero in the last S columns.
template <typename freal>
__global__ void __launch_bounds__(kBlock)
k_shift_x(Geom g, const freal* __restrict__ src, freal* __restrict__ dst, int S) {
    const int nx = g.n[0];
    for (long long c = blockIdx.x * (long long)kBlock + threadIdx.x; c < g.ncells;
         c += (long long)gridDim.x * kBlock) {
        const int i = (int)(c % nx);
        dst[c] = i < nx - S ? src[c + S] : freal(0);
    }
}

template <typename freal>
hipError_t launch_shift_x(const Geom& g, const freal* src, freal* dst, int S, hipStream_t stream) {
    long long blocks = (g.ncells + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL((k_shift_x<freal>), dim3((unsigned)blocks), dim3(kBlock), 0, stream, g, src, dst, S);
    return hipGetLastError();
}
template hipError_t launch_shift_x<double>(const Geom&, const double*, double*, int, hipStream_t);

// Batches of 2D runs: run blockIdx.z, its cells at its offset.
template <typename real>
__device__ inline Fields<freal> offset_fields(const Fields<freal>& f, long long off) {
    Fields<freal> r;
    r.mur = f.mur;   // runs of a batch are periodic: never read
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        r.E[c] = f.E[c] + off;
        r.B[c] = f.B[c] + off;
        r.J[c] = f.J[c] + off;
    }
    return r;
}

// The fused Yee step of every run of a batch: one flat list of the runs'
// blocks (yee_blocks(g) from runs[r].yee_blk_base on; blk_run[b] = r).
template <typename real>
__global__ void __launch_bounds__(kBlock)
k_yee_fused_batch(const RunDesc<real>* __restrict__ runs, const int32_t* __restrict__ blk_run, int nblk,
                  Fields<freal> f, Fields<freal> out, JClear jclear) {
    static_assert(YeeBlock<2>::threads == kBlock, "batched 2D Yee blocks are launched with kBlock threads");
    const int per = (nblk + 7) >> 3;
    const int b = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (b >= nblk) return;
    const int run = blk_run[b];
    const RunDesc<real>& rd = runs[run];
    JClear jc = jclear;
    if (jc.c[0])
        for (int a = 0; a < 3; ++a) jc.c[a] = static_cast<freal*>(jc.c[a]) + rd.cell_off;
    yee_fused_block<freal, 2>(rd.g, rd.kf, offset_fields<real>(f, rd.cell_off), offset_fields<real>(out, rd.cell_off),
                              jc, b - rd.yee_blk_base);
}

// ---------------------------------------------------------------- reductions

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off));
    return v;
}

// Sums NV values over the workgroup and adds them to acc[0 .. NV-1].
template <int NV>
__device__ inline void block_sum_add(double (&v)[NV], double* acc) {
    __shared__ double part[kBlock / 64][NV];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) part[wv][q] = v[q];
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) t += part[w][threadIdx.x];
        if (t != 0.0) atomicAdd(acc + threadIdx.x, t);
    }
}


template <typename real, int DIM>
__device__ inline void reduce_one(int mode, const PArrays<real>& p, long long i, int sp,
                                  const Geom& g, const ReduceArgs& ra, double (&v)[4],
                                  double* rho) {
    const double ux = p.u[0][i], uy = p.u[1][i], uz = p.u[2][i];
    const double gamma = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
    if (mode == RED_POLARIZATION) {
        if (ra.species >= 0 && sp != ra.species) return;
        const double ek = ra.mu[sp] * (gamma - 1.0) * kMeC2MeV;
        if (ek >= ra.emin && ek < ra.emax) {
            v[0] += (double)p.s[0][i];
            v[1] += (double)p.s[1][i];
            v[2] += (double)p.s[2][i];
            v[3] += 1.0;
        }
    } else if (mode == RED_KINETIC) {
        v[sp] += ra.mu[sp] * (gamma - 1.0) * (double)p.w[i];
    } else {
        if (ra.species >= 0 && sp != ra.species) return;
        int c[3];
        unpack_cell<DIM>(p.cell[i], c[0], c[1], c[2]);
        const double q = ra.Z[sp] * (double)p.w[i];
        double o[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < DIM; ++a) o[a] = (double)p.off[a][i];
        for (int corner = 0; corner < (1 << DIM); ++corner) {
            double wgt = q;
            int idx[3] = {0, 0, 0};
            bool inside = true;
            for (int a = 0; a < DIM; ++a) {
                const int up = (corner >> a) & 1;
                wgt *= up ? o[a] : 1.0 - o[a];
                idx[a] = c[a] + up;
                if (idx[a] >= g.n[a]) {
                    idx[a] -= g.n[a];
                    if (a == 0 && g.open_x) inside = false;   // beyond an open x face
                }
            }
            if (inside) atomicAdd(rho + ((long long)idx[2] * g.n[1] + idx[1]) * g.n[0] + idx[0], wgt);
        }
    }
}

// Blocks [0, nseg) take one segment each; the remaining blocks stride over
// the overflow store.
template <typename real, int DIM>
__global__ void __launch_bounds__(kBlock)
k_reduce_particles(int mode, Geom g, PArrays<real> p, Segs seg, PArrays<real> st,
                   const int32_t* __restrict__ ctr, ReduceArgs ra, double* acc, double* rho,
                   int nseg) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if ((int)blockIdx.x < nseg) {
        const int sid = blockIdx.x;
        const int sp = sid % g.nsp;
        const long long start = seg.start[sid];
        const int n = seg.count[sid];
        for (int i = threadIdx.x; i < n; i += kBlock) reduce_one<real, DIM>(mode, p, start + i, sp, g, ra, v, rho);
    } else {
        const int n = ctr[CTR_STASH];
        const int b = blockIdx.x - nseg, nb = gridDim.x - nseg;
        for (int i = b * kBlock + threadIdx.x; i < n; i += nb * kBlock) {
            if (st.cell[i] == kDeadCell) continue;   // left the box
            const int tag = st.sp[i];   // run * kMaxSpecies + species
            if (tag / kMaxSpecies != ra.run) continue;
            reduce_one<real, DIM>(mode, st, i, tag % kMaxSpecies, g, ra, v, rho);
        }
    }
    if (mode != RED_RHO) block_sum_add<4>(v, acc + (blockIdx.x % kRedSlots) * kRedStride);
}

// Charge density of the tile particles (RED_RHO): one workgroup per
// segment adds its particles' CIC weights into a shared-memory node tile
// (nodes org .. org + T along each axis), then adds the non-zero nodes to rho
// (periodic wrap; beyond an open x face dropped).  One global add per node
// and segment instead of 2^DIM per particle.
template <typename real, int DIM>
__global__ void __launch_bounds__(kBlock)
k_rho_tiles(Geom g, PArrays<real> p, Segs seg, ReduceArgs ra, double* rho) {
    extern __shared__ double rl[];
    const int sid = blockIdx.x;
    const int sp = sid % g.nsp;
    if (ra.species >= 0 && sp != ra.species) return;
    const int n = seg.count[sid];
    if (n == 0) return;
    const int t = sid / g.nsp;
    const int org[3] = {(t % g.nt[0]) * g.T[0], ((t / g.nt[0]) % g.nt[1]) * g.T[1],
                        DIM == 3 ? (t / (g.nt[0] * g.nt[1])) * g.T[2] : 0};
    const int Nx = g.T[0] + 1, Ny = g.T[1] + 1, Nz = DIM == 3 ? g.T[2] + 1 : 1;
    const int N = Nx * Ny * Nz;
    for (int k = threadIdx.x; k < N; k += kBlock) rl[k] = 0.0;
    __syncthreads();
    const long long start = seg.start[sid];
    const double Z = ra.Z[sp];
    for (int i = threadIdx.x; i < n; i += kBlock) {
        int c[3];
        unpack_cell<DIM>(p.cell[start + i], c[0], c[1], c[2]);
        const double q = Z * (double)p.w[start + i];
        double o[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < DIM; ++a) o[a] = (double)p.off[a][start + i];
        const int base = ((DIM == 3 ? c[2] - org[2] : 0) * Ny + (c[1] - org[1])) * Nx + (c[0] - org[0]);
#pragma unroll
        for (int corner = 0; corner < (1 << DIM); ++corner) {
            double wgt = q;
            int off = 0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const int up = (corner >> a) & 1;
                wgt *= up ? o[a] : 1.0 - o[a];
                off += up ? (a == 0 ? 1 : (a == 1 ? Nx : Nx * Ny)) : 0;
            }
            atomicAdd(&rl[base + off], wgt);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < N; k += kBlock) {
        const double v = rl[k];
        if (v == 0.0) continue;
        int ix = org[0] + k % Nx;
        int iy = org[1] + (k / Nx) % Ny;
        int iz = DIM == 3 ? org[2] + k / (Nx * Ny) : 0;
        if (ix >= g.n[0]) {
            if (g.open_x) continue;   // beyond an open x face
            ix -= g.n[0];
        }
        if (iy >= g.n[1]) iy -= g.n[1];
        if (DIM == 3 && iz >= g.n[2]) iz -= g.n[2];
        atomicAdd(rho + ((long long)iz * g.n[1] + iy) * g.n[0] + ix, v);
    }
}

// ---- deterministic mode

// A spin component s (|s| <= 1) as two integers: s = (hi + lo 2^-31) 2^-31,
// hi = floor(s 2^31), lo = rint((s 2^31 - hi) 2^31), exact to 2^-62.  Sums of
// the integers are exact, so they do not depend on the order of the adds.
__device__ inline void split31(double s, long long& hi, long long& lo) {
    const double x = s * 2147483648.0;
    const double h = floor(x);
    hi = (long long)h;
    lo = __double2ll_rn((x - h) * 2147483648.0);
}

__device__ inline long long wave_sum_ll(long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    return v;
}

// Section 2 Eq. 4 in the deterministic mode: over the selected particles
// acc[k] += hi(s_k), acc[3 + k] += lo(s_k) (k = 0..2), acc[6] += 1, all as
// 64-bit integers; the selection is the one of RED_POLARIZATION.
template <typename real, int DIM>
__global__ void __launch_bounds__(kBlock)
k_polarization_fixed(Geom g, PArrays<real> p, Segs seg, PArrays<real> st, const int32_t* __restrict__ ctr,
                     ReduceArgs ra, unsigned long long* acc, int nseg) {
    long long v[7] = {0, 0, 0, 0, 0, 0, 0};
    auto one = [&](const PArrays<real>& A, long long i, int sp) {
        if (ra.species >= 0 && sp != ra.species) return;
        const double ux = A.u[0][i], uy = A.u[1][i], uz = A.u[2][i];
        const double gamma = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
        const double ek = ra.mu[sp] * (gamma - 1.0) * kMeC2MeV;
        if (!(ek >= ra.emin && ek < ra.emax)) return;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            long long h, l;
            split31((double)A.s[k][i], h, l);
            v[k] += h;
            v[3 + k] += l;
        }
        v[6] += 1;
    };
    if ((int)blockIdx.x < nseg) {
        const int sid = blockIdx.x;
        const int sp = sid % g.nsp;
        const long long start = seg.start[sid];
        const int n = seg.count[sid];
        for (int i = threadIdx.x; i < n; i += kBlock) one(p, start + i, sp);
    } else {
        const int n = ctr[CTR_STASH];
        const int b = blockIdx.x - nseg, nb = gridDim.x - nseg;
        for (int i = b * kBlock + threadIdx.x; i < n; i += nb * kBlock) {
            if (st.cell[i] == kDeadCell) continue;
            const int tag = st.sp[i];
            if (tag / kMaxSpecies != ra.run) continue;
            one(st, i, tag % kMaxSpecies);
        }
    }
    __shared__ long long part[kBlock / 64][7];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 7; ++q) v[q] = wave_sum_ll(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 7; ++q) part[wv][q] = v[q];
    __syncthreads();
    if (threadIdx.x < 7) {
        long long t = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) t += part[w][threadIdx.x];
        if (t != 0) atomicAdd(acc + threadIdx.x, (unsigned long long)t);
    }
}

// The deterministic mode's current: each J word holds a fixed-point integer
// (units of 1/scale) during the push; here it becomes its FP64 value, in place.
__global__ void __launch_bounds__(kBlock)
k_fixed_to_double(double* __restrict__ J0, double* __restrict__ J1, double* __restrict__ J2, long long n,
                  double inv_scale) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
        J0[i] = (double)__double_as_longlong(J0[i]) * inv_scale;
        J1[i] = (double)__double_as_longlong(J1[i]) * inv_scale;
        J2[i] = (double)__double_as_longlong(J2[i]) * inv_scale;
    }
}

hipError_t launch_fixed_to_double(double* const J[3], long long n, double inv_scale, hipStream_t stream) {
    long long blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fixed_to_double, dim3((unsigned)blocks), dim3(kBlock), 0, stream, J[0], J[1], J[2], n,
                       inv_scale);
    return hipGetLastError();
}

template <typename real, int DIM>
hipError_t launch_polarization_fixed(const Geom& g, const PArrays<real>& p, const Segs& seg, const PArrays<real>& st,
                                     const int32_t* ctr, const ReduceArgs& ra, unsigned long long* acc,
                                     hipStream_t stream) {
    const int nseg = g.ntiles * g.nsp;
    hipLaunchKernelGGL((k_polarization_fixed<real, DIM>), dim3(nseg + 64), dim3(kBlock), 0, stream, g, p, seg, st,
                       ctr, ra, acc, nseg);
    return hipGetLastError();
}

// Bin of v among n equal bins over [lo, hi), or -1 outside.  The energy and
// bin arithmetic is written out without contraction into fused multiply-adds,
// so that bin decisions are reproducible from the particle values alone.
__device__ inline int bin_of(double v, double lo, double hi, int n) {
#pragma clang fp contract(off)
    if (!(v >= lo && v < hi)) return -1;
    const double b = floor((v - lo) / (hi - lo) * (double)n);
    return b >= (double)(n - 1) ? n - 1 : (int)b;
}

__device__ inline double kinetic_mev(double ux, double uy, double uz, double mu) {
#pragma clang fp contract(off)
    const double u2 = (ux * ux + uy * uy) + uz * uz;
    return mu * (sqrt(1.0 + u2) - 1.0) * kMeC2MeV;
}

template <typename real, int DIM>
__device__ inline void bin_one(const PArrays<real>& p, long long i, int sp, const BinArgs& ba,
                               double* hist, double* out) {
    if (ba.mode == BIN_SPECTRUM) {
        const int b = bin_of(kinetic_mev((double)p.u[0][i], (double)p.u[1][i], (double)p.u[2][i], ba.mu[sp]),
                             ba.lo, ba.hi, ba.nbins);
        if (b < 0) return;
        atomicAdd(hist + b, 1.0);
        atomicAdd(hist + ba.nbins + b, (double)p.w[i]);
#pragma unroll
        for (int k = 0; k < 3; ++k) atomicAdd(hist + 2 * ba.nbins + 3 * b + k, (double)p.s[k][i]);
    } else {
        int c[3];
        unpack_cell<DIM>(p.cell[i], c[0], c[1], c[2]);
        double x;
        {
#pragma clang fp contract(off)
            x = ((double)c[ba.axis] + (double)p.off[ba.axis][i]) * ba.d[ba.axis];
        }
        const int bx = bin_of(x, ba.lo, ba.hi, ba.nbins);
        if (bx < 0) return;
        double pm;
        {
#pragma clang fp contract(off)
            pm = ba.mu[sp] * (double)p.u[ba.comp][i];
        }
        const int bp = bin_of(pm, ba.plo, ba.phi, ba.np);
        if (bp < 0) return;
        atomicAdd(out + (long long)bx * ba.np + bp, (double)p.w[i]);
    }
}

// Workgroups stride over the tile segments, then over the overflow store.
// The spectrum is summed in shared memory per workgroup and added to out
// once; the phase-space histogram goes to out directly.
template <typename real, int DIM>
__global__ void __launch_bounds__(kBlock)
k_bin_particles(Geom g, PArrays<real> p, Segs seg, PArrays<real> st, const int32_t* __restrict__ ctr,
                BinArgs ba, double* out) {
    extern __shared__ double hist[];
    const bool spectrum = ba.mode == BIN_SPECTRUM;
    const int nh = 5 * ba.nbins;
    if (spectrum) {
        for (int b = threadIdx.x; b < nh; b += kBlock) hist[b] = 0.0;
        __syncthreads();
    }
    const int nseg = g.ntiles * g.nsp;
    for (int sid = blockIdx.x; sid < nseg; sid += gridDim.x) {
        const int sp = sid % g.nsp;
        if (ba.species >= 0 && sp != ba.species) continue;
        const long long start = seg.start[sid];
        const int n = seg.count[sid];
        for (int i = threadIdx.x; i < n; i += kBlock) bin_one<real, DIM>(p, start + i, sp, ba, hist, out);
    }
    const int nst = ctr[CTR_STASH];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < nst; i += gridDim.x * kBlock) {
        if (st.cell[i] == kDeadCell) continue;   // left the box
        const int sp = st.sp[i];
        if (ba.species >= 0 && sp != ba.species) continue;
        bin_one<real, DIM>(st, i, sp, ba, hist, out);
    }
    if (spectrum) {
        __syncthreads();
        for (int b = threadIdx.x; b < nh; b += kBlock)
            if (hist[b] != 0.0) atomicAdd(out + b, hist[b]);
    }
}

template <typename real>
__global__ void __launch_bounds__(kBlock)
k_field_energy(long long ncells, Fields<real> f, double* acc) {
    double v[1] = {0.0};
    for (long long c = blockIdx.x * (long long)kBlock + threadIdx.x; c < ncells;
         c += (long long)gridDim.x * kBlock) {
        double e = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double x = f.E[a][c], y = f.B[a][c];
            e += x * x + y * y;
        }
        v[0] += 0.5 * e;
    }
    block_sum_add<1>(v, acc);
}

// div E at node (i, j, k) with backward differences, minus rho, in FP64.
template <typename real, int DIM>
__global__ void __launch_bounds__(kBlock)
k_div_residual(Geom g, Vec3d inv_d, Fields<real> f, const double* rho, const double* ref,
               double* ref_out, double* blockmax) {
    const int nx = g.n[0], ny = g.n[1];
    const long long nxy = (long long)nx * ny;
    double m = 0.0;
    for (long long c = blockIdx.x * (long long)kBlock + threadIdx.x; c < g.ncells;
         c += (long long)gridDim.x * kBlock) {
        const long long kz = c / nxy;
        const long long rem = c - kz * nxy;
        const int j = (int)(rem / nx);
        const int i = (int)(rem - (long long)j * nx);
        const long long im = i == 0 ? c + nx - 1 : c - 1;
        const long long jm = j == 0 ? c + (long long)(ny - 1) * nx : c - nx;
        const double exm = (g.open_x && i == 0) ? 0.0 : (double)f.E[0][im];   // zero beyond an open face
        double div = ((double)f.E[0][c] - exm) * inv_d.v[0]
                   + ((double)f.E[1][c] - (double)f.E[1][jm]) * inv_d.v[1];
        if (DIM == 3) {
            const long long km = kz == 0 ? c + (g.n[2] - 1) * nxy : c - nxy;
            div += ((double)f.E[2][c] - (double)f.E[2][km]) * inv_d.v[2];
        }
        const double res = div - rho[c];
        if (ref_out) ref_out[c] = res;
        else m = fmax(m, fabs(res - ref[c]));
    }
    __shared__ double part[kBlock / 64];
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t = fmax(t, part[w]);
        blockmax[blockIdx.x] = t;
    }
}

template <typename real>
__global__ void __launch_bounds__(kBlock)
k_nonfinite(const real* data, long long n, int32_t* flag) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        if (!isfinite(data[i])) flag[0] = 1;
}

// ---------------------------------------------------------------- launchers

// Mur state of open x faces from the current fields: every ghost and
// previous value starts as the first (low face) or last (high face) column.
template <typename real, int DIM>
__global__ void __launch_bounds__(kBlock)
k_mur_reset(Geom g, Fields<real> f) {
    const long long nrow = (long long)g.n[1] * (DIM == 3 ? g.n[2] : 1);
    for (long long row = blockIdx.x * (long long)kBlock + threadIdx.x; row < nrow;
         row += (long long)gridDim.x * kBlock) {
        const long long first = row * g.n[0], last = first + g.n[0] - 1;
        for (int c = 0; c < 2; ++c) {
            const real e = f.E[1 + c][last], b = f.B[1 + c][first];
            f.mur[(MUR_HI_GHOST + c) * nrow + row] = e;
            f.mur[(MUR_HI_PREV + c) * nrow + row] = e;
            f.mur[(MUR_LO_GHOST + c) * nrow + row] = b;
            f.mur[(MUR_LO_PREV + c) * nrow + row] = b;
        }
    }
}

template <typename real, int DIM>
hipError_t launch_mur_reset(const Geom& g, const Fields<real>& f, hipStream_t stream) {
    const long long nrow = (long long)g.n[1] * (DIM == 3 ? g.n[2] : 1);
    const long long blocks = std::min<long long>((nrow + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL((k_mur_reset<real, DIM>), dim3((unsigned)blocks), dim3(kBlock), 0, stream, g, f);
    return hipGetLastError();
}

template <typename real, int DIM>
hipError_t launch_yee_fused(const Geom& g, const Consts<real>& k, const Fields<real>& f, const Fields<real>& out,
                            real* const* jclear, hipStream_t stream) {
    if (g.open_x && (!f.mur || !out.mur || f.mur == out.mur)) return hipErrorInvalidValue;
    JClear jc{{nullptr, nullptr, nullptr}};
    if (jclear)
        for (int a = 0; a < 3; ++a) jc.c[a] = jclear[a];
    const long long nblk = (long long)yee_tiles<DIM>(g) * yee_chunks<DIM>(g);
    const long long grid = (nblk + 7) / 8 * 8;
    const size_t mur_lds = g.open_x ? yee_mur_lds_bytes<real, DIM>() : 0;
    hipLaunchKernelGGL((k_yee_fused<real, DIM>), dim3((unsigned)grid), dim3(YeeBlock<DIM>::threads), mur_lds, stream, g, k, f, out,
                       jc);
    return hipGetLastError();
}

int yee_blocks(int nx, int ny) {
    Geom g{};
    g.n[0] = nx;
    g.n[1] = ny;
    g.n[2] = 1;
    return yee_tiles<2>(g) * yee_chunks<2>(g);
}

template <typename real, int DIM>
hipError_t launch_reduce_particles(int mode, const Geom& g, const PArrays<real>& p,
                                   const Segs& seg, const PArrays<real>& st, const int32_t* ctr,
                                   const ReduceArgs& ra, double* acc, double* rho,
                                   hipStream_t stream) {
    const int nseg = g.ntiles * g.nsp;
    if (mode == RED_RHO) {
        // tile particles through shared-memory node tiles, then the overflow store
        const size_t lds = (size_t)(g.T[0] + 1) * (g.T[1] + 1) * (DIM == 3 ? g.T[2] + 1 : 1) * sizeof(double);
        hipLaunchKernelGGL((k_rho_tiles<real, DIM>), dim3(nseg), dim3(kBlock), lds, stream, g, p, seg, ra, rho);
        hipLaunchKernelGGL((k_reduce_particles<real, DIM>), dim3(64), dim3(kBlock), 0, stream,
                           mode, g, p, seg, st, ctr, ra, acc, rho, 0);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_reduce_particles<real, DIM>), dim3(nseg + 64), dim3(kBlock), 0, stream,
                       mode, g, p, seg, st, ctr, ra, acc, rho, nseg);
    return hipGetLastError();
}

template <typename real, int DIM>
hipError_t launch_bin_particles(const Geom& g, const PArrays<real>& p, const Segs& seg,
                                const PArrays<real>& st, const int32_t* ctr, const BinArgs& ba,
                                double* out, hipStream_t stream) {
    const int nseg = g.ntiles * g.nsp;
    const int blocks = nseg < 1024 ? (nseg > 0 ? nseg : 1) : 1024;
    const size_t lds = ba.mode == BIN_SPECTRUM ? (size_t)5 * ba.nbins * sizeof(double) : 0;
    hipLaunchKernelGGL((k_bin_particles<real, DIM>), dim3(blocks), dim3(kBlock), lds, stream, g, p,
                       seg, st, ctr, ba, out);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_yee_fused_batch(const RunDesc<real>* runs, const int32_t* blk_run, int nblocks,
                                  const Fields<freal>& f, const Fields<freal>& out, freal* const* jclear,
                                  hipStream_t stream) {
    JClear jc{{nullptr, nullptr, nullptr}};
    if (jclear)
        for (int a = 0; a < 3; ++a) jc.c[a] = jclear[a];
    const long long grid = ((long long)nblocks + 7) / 8 * 8;
    hipLaunchKernelGGL((k_yee_fused_batch<real>), dim3((unsigned)grid), dim3(kBlock), 0, stream, runs, blk_run,
                       nblocks, f, out, jc);
    return hipGetLastError();
}

template hipError_t launch_yee_fused_batch<float>(const RunDesc<float>*, const int32_t*, int, const Fields<freal>&,
                                                  const Fields<freal>&, freal* const*, hipStream_t);
template hipError_t launch_yee_fused_batch<double>(const RunDesc<double>*, const int32_t*, int, const Fields<freal>&,
                                                   const Fields<freal>&, freal* const*, hipStream_t);

template <typename real>
hipError_t launch_field_energy(const Geom& g, const Fields<real>& f, double* acc,
                               hipStream_t stream) {
    long long blocks = (g.ncells + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_field_energy<real>), dim3((unsigned)blocks), dim3(kBlock), 0, stream,
                       g.ncells, f, acc);
    return hipGetLastError();
}

template <typename real, int DIM>
hipError_t launch_div_residual(const Geom& g, const Vec3d& inv_d, const Fields<real>& f,
                               const double* rho, const double* ref, double* ref_out,
                               double* blockmax, int blocks, hipStream_t stream) {
    hipLaunchKernelGGL((k_div_residual<real, DIM>), dim3(blocks), dim3(kBlock), 0, stream, g,
                       inv_d, f, rho, ref, ref_out, blockmax);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_nonfinite(const real* data, long long n, int32_t* flag, hipStream_t stream) {
    long long blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((k_nonfinite<real>), dim3((unsigned)blocks), dim3(kBlock), 0, stream, data,
                       n, flag);
    return hipGetLastError();
}

// out[0 .. n) = 0 by a plain kernel (no memset node, so that the clear
// stays correct when a caller captures the launches in a graph).
__global__ void __launch_bounds__(kBlock) k_fill_zero(double* __restrict__ out, long long n) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        out[i] = 0.0;
}

hipError_t launch_fill_zero(double* out, long long n, hipStream_t stream) {
    long long blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(kBlock), 0, stream, out, n);
    return hipGetLastError();
}

#define SPINPIC_INST_GRID(DIM)                                                                 \
    template hipError_t launch_yee_fused<double, DIM>(const Geom&, const Consts<double>&,     \
        const Fields<double>&, const Fields<double>&, double* const*, hipStream_t);             \
    template hipError_t launch_mur_reset<double, DIM>(const Geom&, const Fields<double>&,     \
                                                      hipStream_t);                            \
    template hipError_t launch_div_residual<double, DIM>(const Geom&, const Vec3d&,           \
        const Fields<double>&, const double*, const double*, double*, double*, int, hipStream_t);

#define SPINPIC_INST_PART(real, DIM)                                                           \
    template hipError_t launch_reduce_particles<real, DIM>(int, const Geom&,                  \
        const PArrays<real>&, const Segs&, const PArrays<real>&, const int32_t*,               \
        const ReduceArgs&, double*, double*, hipStream_t);                                      \
    template hipError_t launch_bin_particles<real, DIM>(const Geom&, const PArrays<real>&,     \
        const Segs&, const PArrays<real>&, const int32_t*, const BinArgs&, double*, hipStream_t); \
    template hipError_t launch_polarization_fixed<real, DIM>(const Geom&, const PArrays<real>&, \
        const Segs&, const PArrays<real>&, const int32_t*, const ReduceArgs&, unsigned long long*, hipStream_t);

SPINPIC_INST_GRID(2)
SPINPIC_INST_GRID(3)
SPINPIC_INST_PART(float, 2)
SPINPIC_INST_PART(float, 3)
SPINPIC_INST_PART(double, 2)
SPINPIC_INST_PART(double, 3)

template hipError_t launch_field_energy<double>(const Geom&, const Fields<double>&, double*,
                                                hipStream_t);
template hipError_t launch_nonfinite<float>(const float*, long long, int32_t*, hipStream_t);
template hipError_t launch_nonfinite<double>(const double*, long long, int32_t*, hipStream_t);

}  // namespace spinpic
