// Particle kernels: fused gather + Boris + Thomas-BMT + move + Esirkepov
// deposit per tile, the overflow-store push, and the per-step rebinning
// (compaction of vacated slots and insertion of tile leavers).
#include "common.h"
#include "kernels.h"

namespace spinpic {

// Current sink into the shared-memory J tile.  Node l of the tile (local
// index, -1 .. T+1) is shared-memory coordinate l + 1.  With acc_t a 64-bit
// unsigned word (the deterministic mode) every contribution is added as the
// fixed-point integer to_fixed(v, fscale).
template <typename acc_t, int DIM>
struct TileJ {
    acc_t* base;
    int Hx, Hxy, H;
    int o;   // offset of the stencil's base node
    double fscale;
    static constexpr bool kStrided = true;
    __device__ inline int stride(int a) const { return a == 0 ? 1 : (a == 1 ? Hx : Hxy); }
    __device__ inline int comp(int c) const { return c * H; }
    // v to J at offset off (comp(c) plus node offsets) from the base node
    template <typename real>
    __device__ inline void add_off(int off, real v) const {
        acc_t* q = base + o + off;
        if constexpr (kFixedAcc<acc_t>) atomicAdd(q, to_fixed((double)v, fscale));
        else atomicAdd(q, (acc_t)v);
    }
    template <typename real>
    __device__ inline void add(int c, int i, int j, int k, real v) const {
        add_off(c * H + (DIM == 3 ? k * Hxy : 0) + j * Hx + i, v);
    }
    // The entries the stencil reaches only when the particle changed cell:
    // added without testing for zero (in the tile, a branch per entry cost
    // more than an add of zero: c3 push 5.04 -> 4.94 ms, c2 unchanged).
    template <typename real>
    __device__ inline void add_nz(int c, int i, int j, int k, real v) const {
        add(c, i, j, k, v);
    }
};

// Current sink straight into global J with periodic wrap (current beyond
// open x faces is dropped).  fscale != 0: the deterministic mode, J holds
// fixed-point integers during the push (see to_fixed).
template <typename freal, int DIM>
struct GlobalJ {
    static constexpr bool kStrided = false;
    freal* J[3];
    int n[3];
    int b[3];  // absolute base node
    int open_x;
    double fscale;
    template <typename real>
    __device__ inline void add_nz(int c, int i, int j, int k, real v) const {
        if (v != real(0)) add(c, i, j, k, v);
    }
    template <typename real>
    __device__ inline void add(int c, int i, int j, int k, real v) const {
        if (open_x && (b[0] + i < 0 || b[0] + i >= n[0])) return;
        const int ix = wrap_index(b[0] + i, n[0]);
        const int iy = wrap_index(b[1] + j, n[1]);
        const int iz = DIM == 3 ? wrap_index(b[2] + k, n[2]) : 0;
        freal* q = J[c] + ((long long)iz * n[1] + iy) * n[0] + ix;
        if (fscale != 0.0) atomicAdd(reinterpret_cast<unsigned long long*>(q), to_fixed((double)v, fscale));
        else atomicAdd(q, (freal)v);
    }
};

// Per-step Eq. 4 record: a pushed particle's contribution, if selected.
template <typename real>
__device__ inline void rec_accumulate(const RecArgs& rec, int sp, const real u[3], const real s[3],
                                      double (&racc)[4]) {
    if (rec.species >= 0 && sp != rec.species) return;
    if (rec.window) {
        const double ux = u[0], uy = u[1], uz = u[2];
        const double gamma = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
        const double ek = rec.mu[sp] * (gamma - 1.0) * kMeC2MeV;
        if (!(ek >= rec.emin && ek < rec.emax)) return;
    }
    racc[0] += (double)s[0];
    racc[1] += (double)s[1];
    racc[2] += (double)s[2];
    racc[3] += 1.0;
}

// The workgroup's record sums added into its slot.  Every thread calls it.
__device__ inline void rec_add_block(double (&racc)[4], double* slot) {
    __shared__ double part[kBlock / 64][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double v = racc[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
        if (lane == 0) part[wv][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) t += part[w][threadIdx.x];
        if (t != 0.0) atomicAdd(slot + threadIdx.x, t);
    }
}

constexpr int kPairCap = 256;   // compaction pairs per round
constexpr int kStageRows = 4;   // field rows a thread loads before storing them

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) & ~size_t(15); }

template <typename real, typename acc_t>
size_t tile_lds_bytes(const Geom& g, int max_chunks) {
    const int Gz = g.ndim == 3 ? g.T[2] + 2 : 1;
    const int Hz = g.ndim == 3 ? g.T[2] + 3 : 1;
    const size_t G = (size_t)(g.T[0] + 2) * (g.T[1] + 2) * Gz;
    const size_t H = (size_t)(g.T[0] + 3) * (g.T[1] + 3) * Hz;
    return align16(6 * G * sizeof(real)) + align16(3 * H * sizeof(acc_t)) +
           align16((size_t)(max_chunks + 4) * sizeof(unsigned long long)) +
           align16((size_t)(max_chunks + 4) * sizeof(int)) + (size_t)kPairCap * sizeof(int);
}

// Wrap an index that is at most a few periods outside [0, n).
__device__ inline int wrap_near(int i, int n) {
    while (i < 0) i += n;
    while (i >= n) i -= n;
    return i;
}

// Copy particle i of one store to slot j of another (or the same) store.
// Every value is loaded before the first store, so the loads go out
// together instead of one round trip per array.
template <typename real>
__device__ inline void copy_particle(const PArrays<real>& from, long long i, const PArrays<real>& to,
                                     long long j, int ndim) {
    const int32_t cell = from.cell[i], id = from.id[i];
    real o[3], u[3], s[3];
    for (int a = 0; a < 3; ++a) o[a] = a < ndim ? from.off[a][i] : real(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u[a] = from.u[a][i];
        s[a] = from.s[a][i];
    }
    const real w = from.w[i];
    to.cell[j] = cell;
    for (int a = 0; a < ndim; ++a) to.off[a][j] = o[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        to.u[a][j] = u[a];
        to.s[a][j] = s[a];
    }
    to.w[j] = w;
    to.id[j] = id;
}

// One workgroup per tile.  The tile's E and B, with one guard cell on each
// side, are staged in shared memory (rounded to the push precision); every
// particle of every species in the tile gathers from there, is pushed and
// moved, and deposits its Esirkepov current into a shared-memory J tile
// (tile + 1 guard node below, 2 above), which is added to global J once at
// the end.  Particles that stay in the tile are written back in place; those
// that leave are appended to the leaver store, and the tile closes the holes
// they leave before it finishes.
// One tile: every particle of every species.  g, k and f are those of the
// run the tile belongs to; its segments are sid_base + t nsp + sp, and its
// leavers carry inst_tag + sp in the leaver store's species word.  Every
// thread of the workgroup must call it.
// In a z-march (3D, see k_push_march), consecutive tiles of one column share
// guard planes: fz0 = 2 when the first two field planes (local z = -1, 0)
// were carried over from the previous tile and only the others are staged
// (0: stage all); jz0 = 3 when the first three current planes hold the
// previous tile's carried sums and only the others start at zero; jkeep = 3
// when the last three current planes (local z = T-1 .. T+1) are kept in
// shared memory for the next tile instead of being added to global J.
// With REC, the pushed particles of the tile are also summed into the
// step's Eq. 4 record (rec).
template <typename real, typename acc_t, int DIM, bool REC = false>
__device__ __attribute__((always_inline)) void push_tile(const Geom& g, const Consts<real>& k, const PArrays<real>& p, const Segs& seg,
                          const PArrays<real>& lv, int32_t* __restrict__ ctr, int slot, const Fields<freal>& f,
                          int deposit, int t, int sid_base, int inst_tag, int fz0 = 0, int jz0 = 0,
                          int jkeep = 0, const RecArgs& rec = RecArgs{}) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_nleave, s_lbase;
    int tc[3];
    tc[0] = t % g.nt[0];
    tc[1] = (t / g.nt[0]) % g.nt[1];
    tc[2] = t / (g.nt[0] * g.nt[1]);
    int org[3], ext[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        org[a] = tc[a] * g.T[a];
        ext[a] = min(g.T[a], g.n[a] - org[a]);
    }

    const int Gx = g.T[0] + 2, Gy = g.T[1] + 2, Gz = DIM == 3 ? g.T[2] + 2 : 1;
    const int Gxy = Gx * Gy, G = Gxy * Gz;
    const int Hx = g.T[0] + 3, Hy = g.T[1] + 3, Hz = DIM == 3 ? g.T[2] + 3 : 1;
    const int Hxy = Hx * Hy, H = Hxy * Hz;
    real* F = reinterpret_cast<real*>(smem);
    acc_t* Jl = reinterpret_cast<acc_t*>(smem + align16((size_t)6 * G * sizeof(real)));
    // one ballot of leavers per 64-particle chunk of the current segment,
    // their exclusive prefix counts, and the source slots of one round of
    // compaction
    const size_t lm_off = align16((size_t)6 * G * sizeof(real)) + align16((size_t)3 * H * sizeof(acc_t));
    unsigned long long* leavemask = reinterpret_cast<unsigned long long*>(smem + lm_off);
    int* lprefix = reinterpret_cast<int*>(smem + lm_off + align16((size_t)(seg.max_chunks + 4) * 8));
    int* srcpos = reinterpret_cast<int*>(smem + lm_off + align16((size_t)(seg.max_chunks + 4) * 8) +
                                         align16((size_t)(seg.max_chunks + 4) * 4));

    // Software pipeline: the next particle of this thread is loaded while
    // the current one is pushed.  Every lane issues the same loads and
    // stores in every iteration (clamped load index, masked-off lanes
    // storing into the spare slots), so the wait for the prefetched data
    // does not also wait for this iteration's stores to complete.
    int cell_n = 0;
    real o_n[3] = {real(0), real(0), real(0)}, u_n[3] = {real(0), real(0), real(0)},
         s_n[3] = {real(0), real(0), real(0)}, w_n = real(0);
    auto load = [&](int start, int i) {
        const uint32_t bi = (uint32_t)(start + i) * 4u;
        const uint32_t br = (uint32_t)(start + i) * (uint32_t)sizeof(real);
        cell_n = ldo(p.cell, bi);
#pragma unroll
        for (int a = 0; a < DIM; ++a) o_n[a] = ldo(p.off[a], br);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            u_n[a] = ldo(p.u[a], br);
            s_n[a] = ldo(p.s[a], br);
        }
        w_n = ldo(p.w, br);
    };

    // stage E and B: each thread owns one x position of several (y, z) rows
    // and issues the loads of up to kStageRows rows before writing any
    {
        const int rpp = kBlock / Gx;              // rows per pass
        const int r0 = threadIdx.x / Gx;
        const int gx = threadIdx.x - r0 * Gx;
        const long long ix = wrap_near(org[0] - 1 + gx, g.n[0]);
        // beyond an open x face the fields are zero
        const bool xin = !g.open_x || (org[0] - 1 + gx >= 0 && org[0] - 1 + gx < g.n[0]);
        const int rows = Gy * Gz;
        if (r0 < rpp) {
            for (int rb = fz0 * Gy + r0; rb < rows; rb += kStageRows * rpp) {
                freal v[kStageRows][6];
#pragma unroll
                for (int q = 0; q < kStageRows; ++q) {
                    const int row = rb + q * rpp;
                    if (row < rows) {
                        const int gz = row / Gy, gy = row - gz * Gy;
                        const long long iz = DIM == 3 ? wrap_near(org[2] - 1 + gz, g.n[2]) : 0;
                        const long long iy = wrap_near(org[1] - 1 + gy, g.n[1]);
                        const long long gi = (iz * g.n[1] + iy) * g.n[0] + ix;
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            v[q][c] = xin ? f.E[c][gi] : freal(0);
                            v[q][3 + c] = xin ? f.B[c][gi] : freal(0);
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < kStageRows; ++q) {
                    const int row = rb + q * rpp;
                    if (row < rows) {
                        const int li = row * Gx + gx;
#pragma unroll
                        for (int c = 0; c < 6; ++c) F[c * G + li] = (real)v[q][c];
                    }
                }
            }
        }
    }
    if (deposit) {
        if (jz0 == 0) {
            for (int idx = threadIdx.x; idx < 3 * H; idx += kBlock) Jl[idx] = acc_t(0);
        } else {
            const int per = H - jz0 * Hxy;   // per component, from plane jz0 on
            for (int idx = threadIdx.x; idx < 3 * per; idx += kBlock) {
                const int c = idx / per;
                Jl[c * H + jz0 * Hxy + (idx - c * per)] = acc_t(0);
            }
        }
    }
    __syncthreads();

    const TileFields<real, DIM> TF{F, Gx, Gxy, G};
    const int lane = threadIdx.x & 63;
    const real half_dt = real(0.5) * k.dt;

    const int wave = threadIdx.x >> 6;
    double racc[4] = {0.0, 0.0, 0.0, 0.0};
    const uint32_t dummy_i = (uint32_t)(seg.dummy + lane) * 4u;
    const uint32_t dummy_r = (uint32_t)(seg.dummy + lane) * (uint32_t)sizeof(real);

    for (int sp = 0; sp < g.nsp; ++sp) {
        const int sid = sid_base + t * g.nsp + sp;
        const int start = __builtin_amdgcn_readfirstlane(seg.start[sid]);
        const int n = __builtin_amdgcn_readfirstlane(seg.count[sid]);
        const real eps = k.eps[sp], r = k.r[sp], an = k.a[sp], Z = k.Z[sp];
        if (n > 0) load(start, min((int)threadIdx.x, n - 1));

        for (int base = 0; base < n; base += kBlock) {
            const int i = base + threadIdx.x;
            const bool active = i < n;
            const int cell0 = cell_n;
            real o[3], u[3], s[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                o[a] = o_n[a];
                u[a] = u_n[a];
                s[a] = s_n[a];
            }
            const real wgt = w_n;
            if (base + kBlock < n) load(start, min(i + kBlock, n - 1));

            bool leave = false, bad = false, gone = false;
            int newcell = cell0;
            if (active) {
                int c[3];
                unpack_cell<DIM>(cell0, c[0], c[1], c[2]);
                int l[3] = {c[0] - org[0], c[1] - org[1], DIM == 3 ? c[2] - org[2] : 0};
                Stencil1<real> st[3];
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    st[a] = a < DIM ? stencil1(l[a], o[a]) : Stencil1<real>{0, real(0), 0, real(0)};
                real E[3], B[3];
                gather_all(TF, st, E, B);
                boris_tbmt(u, s, E, B, eps, r, an, half_dt);
                // non-finite probe: a NaN or infinity anywhere in u or s
                // makes this sum non-finite
                bad = !__builtin_isfinite(dot3(u, u) + dot3(s, s));

                const real ig = rsqrt1(real(1) + dot3(u, u));
                real o0[3];
                int dc[3] = {0, 0, 0};
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    o0[a] = o[a];
                    dc[a] = advance_offset(o[a], displacement(u[a] * ig, k, a));
                }
                if (deposit) {
                    real S0[3][3], S1[3][3], q[3];
                    int b[3] = {0, 0, 0};
#pragma unroll
                    for (int a = 0; a < DIM; ++a) {
                        b[a] = l[a] + shape_pair(o0[a], o[a], dc[a], S0[a], S1[a]);
                        q[a] = -Z * wgt * k.d_dt[a];
                    }
                    TileJ<acc_t, DIM> sink{Jl, Hx, Hxy, H,
                                           (DIM == 3 ? (b[2] + 1) * Hxy : 0) + (b[1] + 1) * Hx + (b[0] + 1),
                                           k.fx_scale};
                    esirkepov<real, DIM>(S0, S1, dc, q, Z * wgt * u[2] * ig, sink);
                }
                if (dc[0] | dc[1] | dc[2]) {
                    int nc[3];
                    // through an open x face the particle leaves the box: a
                    // leaver whose cell word marks it dead
                    const bool dead = g.open_x && (c[0] + dc[0] < 0 || c[0] + dc[0] >= g.n[0]);
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        nc[a] = c[a];
                        if (a < DIM) {
                            const int nl = l[a] + dc[a];
                            // along an axis with one tile the wrap comes back in
                            leave = leave || (g.nt[a] > 1 && (nl < 0 || nl >= ext[a]));
                            nc[a] = c[a] + dc[a];
                            if (nc[a] < 0) nc[a] += g.n[a];
                            if (nc[a] >= g.n[a]) nc[a] -= g.n[a];
                        }
                    }
                    newcell = dead ? kDeadCell : pack_cell<DIM>(nc[0], nc[1], nc[2]);
                    leave = leave || dead;
                    gone = dead;
                }
                // a particle that left the box is not in the step's ensemble
                if constexpr (REC) {
                    if (!gone) rec_accumulate(rec, sp, u, s, racc);
                }
            }

            // Every particle, leaver or not, is written back to its own slot
            // (a leaver's slot becomes a hole that the tail fills later); the
            // cell word only where it changed.
            const uint32_t bi = active ? (uint32_t)(start + i) * 4u : dummy_i;
            const uint32_t br = active ? (uint32_t)(start + i) * (uint32_t)sizeof(real) : dummy_r;
            sto(p.cell, newcell != cell0 ? bi : dummy_i, newcell);
#pragma unroll
            for (int a = 0; a < DIM; ++a) sto(p.off[a], br, o[a]);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                sto(p.u[a], br, u[a]);
                sto(p.s[a], br, s[a]);
            }
            const unsigned long long m = __ballot(leave);
            const unsigned long long nf = __ballot(bad);
            if (lane == 0) {
                leavemask[(base >> 6) + wave] = m;
                if (nf) ctr[CTR_NONFINITE] = 1;
            }
        }
        __syncthreads();

        // Leavers and compaction, from the per-chunk leaver ballots in shared
        // memory.  Exclusive prefix counts of the ballots give every leaver
        // its rank in the leaver store (one global reservation per segment),
        // and every slot a leaver vacated below the segment's new end n - L
        // the particle that fills it: the one of equal rank among those still
        // present in the tail [n - L, n).
        const int nchunks = (n + 63) >> 6;
        if (wave == 0) {
            int carry = 0;
            for (int c0 = 0; c0 <= nchunks; c0 += 64) {
                const int c = c0 + lane;
                unsigned long long m = 0ull;
                if (c < nchunks) m = leavemask[c];
                else if (c == nchunks) leavemask[c] = 0ull;   // read when counting up to slot n
                const int v = __popcll(m);
                int x = v;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const int y = __shfl_up(x, off);
                    if (lane >= off) x += y;
                }
                if (c <= nchunks) lprefix[c] = carry + x - v;
                carry += __shfl(x, 63);
            }
            if (lane == 0) {
                s_nleave = carry;
                s_lbase = carry > 0 ? atomicAdd(&ctr[slot], carry) : 0;
            }
        }
        __syncthreads();
        const int L = s_nleave;
        if (L > 0) {
            const int lbase = s_lbase;
            const int nn = n - L;
            // leavers among slots [0, x), 0 <= x <= n
            auto leavers_below = [&](int x) {
                const int c = x >> 6;
                return lprefix[c] + __popcll(leavemask[c] & ((1ull << (x & 63)) - 1ull));
            };
            const int pairs = leavers_below(nn);
            // slot of the leaver of rank q (0 <= q < L): the last chunk whose
            // exclusive prefix count is at most q, then the (q - prefix)-th
            // set bit of its ballot
            auto leaver_slot = [&](int q) {
                int lo = 0, hi = nchunks - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (lprefix[mid] <= q) lo = mid;
                    else hi = mid - 1;
                }
                unsigned long long m = leavemask[lo];
                for (int k = q - lprefix[lo]; k > 0; --k) m &= m - 1ull;
                return (lo << 6) + __builtin_ctzll(m);
            };
            for (int r0 = 0; r0 == 0 || r0 < pairs; r0 += kPairCap) {
                for (int q = threadIdx.x; q < L; q += kBlock) {
                    const int pos = nn + q;
                    if (!((leavemask[pos >> 6] >> (pos & 63)) & 1ull)) {
                        const int rank = q - (leavers_below(pos) - pairs);
                        if (rank >= r0 && rank < r0 + kPairCap) srcpos[rank - r0] = pos;
                    }
                }
                __syncthreads();
                // one thread per leaver: its copy to the leaver store and, if
                // its slot lies below the new end n - L (rank < pairs), the
                // copy of the tail particle that fills it; all leavers of
                // the segment are handled at once instead of chunk by chunk
                for (int q = threadIdx.x; q < L; q += kBlock) {
                    const bool out = r0 == 0;
                    const bool fill = q >= r0 && q < pairs && q < r0 + kPairCap;
                    if (!out && !fill) continue;
                    const int h = leaver_slot(q);
                    // the leaver is read before its slot is refilled (same thread)
                    if (out) {
                        copy_particle(p, (long long)start + h, lv, (long long)lbase + q, DIM);
                        lv.sp[lbase + q] = inst_tag + sp;
                    }
                    if (fill) copy_particle(p, (long long)start + srcpos[q - r0], p, (long long)start + h, DIM);
                }
                __syncthreads();
            }
        }
        if (threadIdx.x == 0) seg.count[sid] = n - L;
        __syncthreads();
    }
    if constexpr (REC) rec_add_block(racc, rec.acc + (blockIdx.x % kRecSlots) * kRecStride);

    if (deposit) {
        __syncthreads();
        const int rpp = kBlock / Hx;
        const int r0 = threadIdx.x / Hx;
        const int hx = threadIdx.x - r0 * Hx;
        const long long ix = wrap_near(org[0] - 1 + hx, g.n[0]);
        // current beyond an open x face is dropped
        const bool xin = !g.open_x || (org[0] - 1 + hx >= 0 && org[0] - 1 + hx < g.n[0]);
        if (r0 < rpp && xin) {
            for (int hz = 0; hz < Hz - jkeep; ++hz) {
                const long long iz = DIM == 3 ? wrap_near(org[2] - 1 + hz, g.n[2]) : 0;
                for (int hy = r0; hy < Hy; hy += rpp) {
                    const long long iy = wrap_near(org[1] - 1 + hy, g.n[1]);
                    const long long gi = (iz * g.n[1] + iy) * g.n[0] + ix;
                    const int li = hz * Hxy + hy * Hx + hx;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const acc_t v = Jl[c * H + li];
                        if (v != acc_t(0)) {
                            if constexpr (kFixedAcc<acc_t>)
                                atomicAdd(reinterpret_cast<unsigned long long*>(f.J[c] + gi), v);
                            else
                                atomicAdd(f.J[c] + gi, (freal)v);
                        }
                    }
                }
            }
        }
    }
}

template <typename real, typename acc_t, int DIM, bool REC>
__global__ void __launch_bounds__(kBlock)
k_push_tiles(Geom g, Consts<real> k, PArrays<real> p, Segs seg, PArrays<real> lv,
             int32_t* __restrict__ ctr, int slot, Fields<freal> f, int deposit, RecArgs rec) {
    // the other step's leaver counter is free again: clear it for the next step
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr[slot ^ 1] = 0;
    // tiles in launch order: workgroups are dealt round-robin over the 8
    // XCDs, so the tiles running at any time form one contiguous band of
    // the grid (its guard cells shared through the last-level cache);
    // giving each XCD a contiguous range of its own measured slower
    const int t = (int)blockIdx.x;
    if (t >= g.ntiles) return;
    push_tile<real, acc_t, DIM, REC>(g, k, p, seg, lv, ctr, slot, f, deposit, t, 0, 0, 0, 0, 0, rec);
}

// The push that also keeps the Eq. 4 record: the same kernel, held to two
// waves per SIMD (256 registers at most).  The FP64 3D one took 264 without
// the cap, one wave per SIMD, which doubled its time; the others stay below
// it.  A kernel of its own, so that the cap leaves the code of the push
// without the record as it is.
template <typename real, typename acc_t, int DIM>
__global__ void __launch_bounds__(kBlock, 2)
k_push_tiles_rec(Geom g, Consts<real> k, PArrays<real> p, Segs seg, PArrays<real> lv,
                 int32_t* __restrict__ ctr, int slot, Fields<freal> f, int deposit, RecArgs rec) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr[slot ^ 1] = 0;
    const int t = (int)blockIdx.x;
    if (t >= g.ntiles) return;
    push_tile<real, acc_t, DIM, true>(g, k, p, seg, lv, ctr, slot, f, deposit, t, 0, 0, 0, 0, 0, rec);
}

// 3D push marching along z (an alternative to k_push_tiles that moves fewer
// guard bytes; measured no faster on c3, see the engine's kMarchRun):
// workgroup w takes a run of up to R tiles of one
// (x, y) tile column, z tile rz R .. rz R + R - 1, and pushes them in order.
// Between two tiles of a run the field planes at local z = T-1, T (the next
// tile's guard planes -1, 0) stay in shared memory, and the current planes
// at local z = T-1 .. T+1 (the next tile's -1 .. 1) carry their sums over
// instead of being added to global J; the next tile then stages T new field
// planes instead of T + 2 and the run adds T current planes per tile to
// global J instead of T + 3.  Needs T[2] >= 3 (the carried planes and their
// destinations do not overlap).  Runs are numbered x fastest, then y, then
// z; with xcd_major the runs of XCD x (workgroups x, x + 8, ...) are one
// contiguous range of that order, else they go in launch order.
template <typename real, typename acc_t>
__global__ void __launch_bounds__(kBlock)
k_push_march(Geom g, Consts<real> k, PArrays<real> p, Segs seg, PArrays<real> lv, int32_t* __restrict__ ctr,
             int slot, Fields<freal> f, int deposit, int R, int nruns, int xcd_major) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr[slot ^ 1] = 0;
    int item = (int)blockIdx.x;
    if (xcd_major) {
        const int per = (nruns + 7) >> 3;
        item = (item & 7) * per + (item >> 3);
    }
    if (item >= nruns) return;
    const int tx = item % g.nt[0];
    const int ty = (item / g.nt[0]) % g.nt[1];
    const int rz = item / (g.nt[0] * g.nt[1]);
    const int z0 = rz * R, z1 = min(g.nt[2], z0 + R);
    const int T2 = g.T[2];
    const int Gx = g.T[0] + 2, Gy = g.T[1] + 2, Gz = T2 + 2;
    const int Gxy = Gx * Gy, G = Gxy * Gz;
    const int Hx = g.T[0] + 3, Hy = g.T[1] + 3, Hz = T2 + 3;
    const int Hxy = Hx * Hy, H = Hxy * Hz;
    real* F = reinterpret_cast<real*>(smem);
    acc_t* Jl = reinterpret_cast<acc_t*>(smem + align16((size_t)6 * G * sizeof(real)));
    for (int tz = z0; tz < z1; ++tz) {
        const bool first = tz == z0, last = tz == z1 - 1;
        if (!first) {
            // carry: field planes T, T + 1 -> 0, 1; current planes T .. T + 2 -> 0 .. 2
            for (int idx = threadIdx.x; idx < 6 * 2 * Gxy; idx += kBlock) {
                const int c = idx / (2 * Gxy), r = idx - c * 2 * Gxy;
                F[c * G + r] = F[c * G + T2 * Gxy + r];
            }
            if (deposit)
                for (int idx = threadIdx.x; idx < 3 * 3 * Hxy; idx += kBlock) {
                    const int c = idx / (3 * Hxy), r = idx - c * 3 * Hxy;
                    Jl[c * H + r] = Jl[c * H + T2 * Hxy + r];
                }
            __syncthreads();
        }
        const int t = tx + g.nt[0] * (ty + g.nt[1] * tz);
        push_tile<real, acc_t, 3>(g, k, p, seg, lv, ctr, slot, f, deposit, t, 0, 0, first ? 0 : 2, first ? 0 : 3,
                                  last ? 0 : 3);
        __syncthreads();   // the carried planes are read by the next tile's setup
    }
}

// Particles in the overflow store (tiles that ran out of slots): the same
// step, gathering from and depositing into global memory directly.
// One particle of the overflow store (species sp): gather from and deposit
// into the global fields of its run.
// Returns true when the pushed momentum or spin is not finite.
template <typename real, int DIM, bool REC = false>
__device__ inline bool push_stash_one(const Geom& g, const Consts<real>& k, const PArrays<real>& st, int i,
                                      int sp, const Fields<freal>& f, int deposit,
                                      const RecArgs& rec = RecArgs{}, double* racc = nullptr) {
    const int32_t cell = st.cell[i];
    if (cell == kDeadCell) return false;   // left the box earlier
    GlobalFields<freal, DIM> GF;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        GF.c[c] = f.E[c];
        GF.c[3 + c] = f.B[c];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) GF.n[a] = g.n[a];
    GF.open_x = g.open_x;
    const real half_dt = real(0.5) * k.dt;
    int c[3];
    unpack_cell<DIM>(cell, c[0], c[1], c[2]);
    real o[3] = {real(0), real(0), real(0)}, u[3], s[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) o[a] = st.off[a][i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u[a] = st.u[a][i];
        s[a] = st.s[a][i];
    }
    const real wgt = st.w[i];
    Stencil1<real> stc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        stc[a] = a < DIM ? stencil1(c[a], o[a]) : Stencil1<real>{0, real(0), 0, real(0)};
    real E[3], B[3];
    gather_all(GF, stc, E, B);
    boris_tbmt(u, s, E, B, k.eps[sp], k.r[sp], k.a[sp], half_dt);
    // the same arithmetic as the tile push, so that a particle gets the same
    // result whichever of the two pushes it
    const real ig = rsqrt1(real(1) + dot3(u, u));
    real o0[3];
    int dc[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        o0[a] = o[a];
        dc[a] = advance_offset(o[a], displacement(u[a] * ig, k, a));
    }
    if (deposit) {
        real S0[3][3], S1[3][3], q[3];
        GlobalJ<freal, DIM> sink;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            sink.J[a] = f.J[a];
            sink.n[a] = g.n[a];
            sink.b[a] = 0;
        }
        sink.open_x = g.open_x;
        sink.fscale = k.fx_scale;
        const real Z = k.Z[sp];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            sink.b[a] = c[a] + shape_pair(o0[a], o[a], dc[a], S0[a], S1[a]);
            q[a] = -Z * wgt * k.d_dt[a];
        }
        esirkepov<real, DIM>(S0, S1, dc, q, Z * wgt * u[2] * ig, sink);
    }
    int nc[3];
    const bool dead = g.open_x && (c[0] + dc[0] < 0 || c[0] + dc[0] >= g.n[0]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        nc[a] = c[a] + dc[a];
        if (a < DIM) {
            if (nc[a] < 0) nc[a] += g.n[a];
            if (nc[a] >= g.n[a]) nc[a] -= g.n[a];
        }
    }
    st.cell[i] = dead ? kDeadCell : pack_cell<DIM>(nc[0], nc[1], nc[2]);
    if constexpr (REC) {
        if (!dead) rec_accumulate(rec, sp, u, s, *reinterpret_cast<double(*)[4]>(racc));
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) st.off[a][i] = o[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        st.u[a][i] = u[a];
        st.s[a][i] = s[a];
    }
    return !__builtin_isfinite(dot3(u, u) + dot3(s, s));
}

template <typename real, int DIM, bool REC>
__global__ void __launch_bounds__(kBlock)
k_push_stash(Geom g, Consts<real> k, PArrays<real> st, int32_t* __restrict__ ctr,
             Fields<freal> f, int deposit, RecArgs rec) {
    const int n = ctr[CTR_STASH];
    bool bad = false;
    double racc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        bad = push_stash_one<real, DIM, REC>(g, k, st, i, st.sp[i], f, deposit, rec, racc) || bad;
    if (bad) ctr[CTR_NONFINITE] = 1;
    if constexpr (REC) rec_add_block(racc, rec.acc + (blockIdx.x % kRecSlots) * kRecStride);
}

// Positions for the active lanes of a wavefront that each add 1 to
// counter[key]: one atomic add per distinct key among them (the leavers of
// a wavefront mostly come from one tile and go to a few neighbours), each
// lane's position being the group's old count plus its rank in the group.
// Every lane of the wavefront must call it.
__device__ inline int wave_reserve(int32_t* counter, int key, bool active) {
    const int lane = threadIdx.x & 63;
    unsigned long long pending = __ballot(active);
    int pos = 0;
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int lkey = __shfl(key, leader);
        const unsigned long long grp = __ballot(active && key == lkey) & pending;
        int base = 0;
        if (lane == leader) base = atomicAdd(&counter[lkey], __popcll(grp));
        base = __shfl(base, leader);
        if ((grp >> lane) & 1ull) pos = base + __popcll(grp & ((1ull << lane) - 1ull));
        pending &= ~grp;
    }
    return pos;
}

// Every leaver takes a slot at the end of its new segment, or a slot in the
// overflow store when the segment is full.
template <typename real, int DIM>
__global__ void __launch_bounds__(kBlock)
k_insert(Geom g, PArrays<real> p, Segs seg, PArrays<real> lv, PArrays<real> st,
         int32_t* __restrict__ ctr, int slot, unsigned long long* __restrict__ moved) {
    const int L = ctr[slot];
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(moved, (unsigned long long)L);
    for (int q0 = blockIdx.x * kBlock; q0 < L; q0 += gridDim.x * kBlock) {
        const int q = q0 + threadIdx.x;
        int32_t cell = kDeadCell;
        int sp = 0, sid = 0;
        if (q < L) {
            cell = lv.cell[q];
            sp = lv.sp[q];
        }
        const bool live = cell != kDeadCell;   // a dead leaver left the box: dropped
        if (live) {
            int c[3];
            unpack_cell<DIM>(cell, c[0], c[1], c[2]);
            const int tile =
                c[0] / g.T[0] + g.nt[0] * (c[1] / g.T[1] + (DIM == 3 ? g.nt[1] * (c[2] / g.T[2]) : 0));
            sid = tile * g.nsp + sp;
        }
        const int pos = wave_reserve(seg.count, sid, live);
        if (!live) continue;
        if (pos < seg.cap[sid]) {
            copy_particle(lv, q, p, (long long)seg.start[sid] + pos, DIM);
        } else {
            atomicSub(&seg.count[sid], 1);
            const int j = atomicAdd(&ctr[CTR_STASH], 1);
            copy_particle(lv, q, st, j, DIM);
            st.sp[j] = sp;
        }
    }
}

// Re-layout after a capacity change: segment sid moves from old_start to
// new_start (one workgroup per segment).
template <typename real>
__global__ void __launch_bounds__(kBlock)
k_repack_segments(PArrays<real> from, PArrays<real> to, const int32_t* __restrict__ old_start,
                  const int32_t* __restrict__ new_start, const int32_t* __restrict__ count,
                  int ndim) {
    const int sid = blockIdx.x;
    const long long a = old_start[sid], b = new_start[sid];
    const int n = count[sid];
    for (int i = threadIdx.x; i < n; i += kBlock) copy_particle(from, a + i, to, b + i, ndim);
}

// ---------------------------------------------------------------- batches

template <typename real>
__device__ inline Fields<freal> run_fields(const Fields<freal>& f, long long off) {
    Fields<freal> r;
    r.mur = nullptr;   // runs of a batch are periodic
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        r.E[c] = f.E[c] + off;
        r.B[c] = f.B[c] + off;
        r.J[c] = f.J[c] + off;
    }
    return r;
}

// Persistent push over the tiles of every run.  The work list holds each
// run's tiles in row-major order, cut into 8 contiguous chunks of about
// equal cost, one per XCD: workgroup b runs on XCD b mod 8 (workgroups are
// dealt round-robin over the XCDs) and takes the next tile of its XCD's
// chunk from a counter, so neighbouring tiles, which share guard cells,
// are worked on by one L2; when its chunk is used up it takes tiles from
// the other chunks in turn.  The other step parity's counters are cleared
// for the next step.
template <typename real, typename acc_t>
__global__ void __launch_bounds__(kBlock)
k_push_tiles_batch(const RunDesc<real>* __restrict__ runs, const TileRef* __restrict__ order, XcdQueues q,
                   PArrays<real> p, Segs seg, PArrays<real> lv, int32_t* __restrict__ ctr, int slot,
                   Fields<freal> f, int deposit, unsigned long long* __restrict__ run_ns) {
    __shared__ int s_item;
    if (blockIdx.x == 0 && threadIdx.x < 8) {
        if (threadIdx.x == 0) ctr[slot ^ 1] = 0;
        ctr[CTR_QUEUE + 8 * (slot ^ 1) + threadIdx.x] = 0;
    }
    int32_t* const queue = ctr + CTR_QUEUE + 8 * slot;
    int x = blockIdx.x & 7, tried = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            int item = -1;
            while (tried < 8) {
                const int k = atomicAdd(&queue[x], 1);
                if (k < q.start[x + 1] - q.start[x]) {
                    item = q.start[x] + k;
                    break;
                }
                ++tried;
                x = (x + 1) & 7;
            }
            s_item = item;
        }
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item < 0) break;
        const TileRef tr = order[item];
        // the run's geometry and constants are read in place: a local copy
        // of the constants, indexed by species, would live in scratch memory
        const RunDesc<real>& rd = runs[tr.run];
        const Fields<freal> fr = run_fields<real>(f, rd.cell_off);
        const unsigned long long t0 = run_ns ? wall_clock64() : 0ull;
        push_tile<real, acc_t, 2>(rd.g, rd.k, p, seg, lv, ctr, slot, fr, deposit, tr.t, rd.sid_base,
                                  tr.run * kMaxSpecies);
        __syncthreads();   // shared memory is restaged for the next tile
        if (run_ns && threadIdx.x == 0) atomicAdd(run_ns + tr.run, (wall_clock64() - t0) * 10ull);
    }
}

template <typename real>
__global__ void __launch_bounds__(kBlock)
k_push_stash_batch(const RunDesc<real>* __restrict__ runs, PArrays<real> st, int32_t* __restrict__ ctr,
                   Fields<freal> f, int deposit) {
    const int n = ctr[CTR_STASH];
    bool bad = false;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const int tag = st.sp[i];
        const int run = tag / kMaxSpecies;
        bad = push_stash_one<real, 2>(runs[run].g, runs[run].k, st, i, tag - run * kMaxSpecies,
                                      run_fields<real>(f, runs[run].cell_off), deposit) || bad;
    }
    if (bad) ctr[CTR_NONFINITE] = 1;
}

// The batch's leavers (the list [0, ctr[slot]) of the leaver store): each
// takes a slot at the end of its new segment in its own run, or a slot in
// the overflow store when that segment is full.
template <typename real>
__global__ void __launch_bounds__(kBlock)
k_insert_batch(const RunDesc<real>* __restrict__ runs, PArrays<real> p, Segs seg, PArrays<real> lv,
               PArrays<real> st, int32_t* __restrict__ ctr, int slot, unsigned long long* __restrict__ moved) {
    const int L = ctr[slot];
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(moved, (unsigned long long)L);
    for (int q0 = blockIdx.x * kBlock; q0 < L; q0 += gridDim.x * kBlock) {
        const int q = q0 + threadIdx.x;
        const bool live = q < L;
        int tag = 0, sid = 0;
        if (live) {
            tag = lv.sp[q];
            const int run = tag / kMaxSpecies;
            const int sp = tag - run * kMaxSpecies;
            const Geom& g = runs[run].g;
            int c[3];
            unpack_cell<2>(lv.cell[q], c[0], c[1], c[2]);
            const int tile = c[0] / g.T[0] + g.nt[0] * (c[1] / g.T[1]);
            sid = runs[run].sid_base + tile * g.nsp + sp;
        }
        const int pos = wave_reserve(seg.count, sid, live);
        if (!live) continue;
        if (pos < seg.cap[sid]) {
            copy_particle(lv, q, p, (long long)seg.start[sid] + pos, 2);
        } else {
            atomicSub(&seg.count[sid], 1);
            const int j = atomicAdd(&ctr[CTR_STASH], 1);
            copy_particle(lv, q, st, j, 2);
            st.sp[j] = tag;
        }
    }
}

// ---------------------------------------------------------------- moving window

// After the segment table has been rotated by whole tile columns, every
// particle of a kept segment moves S cells down in x (one workgroup per
// segment; the segments that left the box have count 0).
template <typename real, int DIM>
__global__ void __launch_bounds__(kBlock)
k_shift_cells(PArrays<real> p, Segs seg, int S) {
    const int sid = blockIdx.x;
    const long long start = seg.start[sid];
    const int n = seg.count[sid];
    for (int i = threadIdx.x; i < n; i += kBlock) {
        int c[3];
        unpack_cell<DIM>(p.cell[start + i], c[0], c[1], c[2]);
        p.cell[start + i] = pack_cell<DIM>(c[0] - S, c[1], c[2]);
    }
}

__global__ void __launch_bounds__(kBlock)
k_rotate_segments(Geom g, Segs from, Segs to, int k) {
    const int nseg = g.ntiles * g.nsp;
    for (int d = blockIdx.x * kBlock + threadIdx.x; d < nseg; d += gridDim.x * kBlock) {
        const int t = d / g.nsp, sp = d - t * g.nsp;
        const int tx = t % g.nt[0];
        const bool kept = tx < g.nt[0] - k;
        const int src = (t - tx + (kept ? tx + k : tx - (g.nt[0] - k))) * g.nsp + sp;
        to.start[d] = from.start[src];
        to.cap[d] = from.cap[src];
        to.count[d] = kept ? from.count[src] : 0;
    }
}

hipError_t launch_rotate_segments(const Geom& g, const Segs& from, const Segs& to, int k, hipStream_t stream) {
    const int nseg = g.ntiles * g.nsp;
    const int blocks = std::min((nseg + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_rotate_segments, dim3(blocks), dim3(kBlock), 0, stream, g, from, to, k);
    return hipGetLastError();
}

template <typename real, int DIM>
__global__ void __launch_bounds__(kBlock)
k_shift_stash(PArrays<real> st, const int32_t* __restrict__ ctr, int S) {
    const int n = ctr[CTR_STASH];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const int32_t cell = st.cell[i];
        if (cell == kDeadCell) continue;
        int c[3];
        unpack_cell<DIM>(cell, c[0], c[1], c[2]);
        st.cell[i] = c[0] < S ? kDeadCell : pack_cell<DIM>(c[0] - S, c[1], c[2]);
    }
}

template <typename real, int DIM>
hipError_t launch_shift_stash(const PArrays<real>& st, const int32_t* ctr, int S, hipStream_t stream) {
    hipLaunchKernelGGL((k_shift_stash<real, DIM>), dim3(256), dim3(kBlock), 0, stream, st, ctr, S);
    return hipGetLastError();
}

// Cold plasma in the last S columns: thread idx is particle q of column col,
// row (cy, cz), species sp, with idx = (((sp nz + cz) ny + cy) S + col) ppc + q.
// A cell whose centre sees no density (lab frame) gets no particles.  Each
// particle takes the next slot of its tile's segment, or one in the overflow
// store when the segment is full.
template <typename real, int DIM>
__global__ void __launch_bounds__(kBlock)
k_inject(Geom g, PArrays<real> p, Segs seg, PArrays<real> st, int32_t* __restrict__ ctr, InjectArgs a) {
#pragma clang fp contract(off)
    const int nz = DIM == 3 ? g.n[2] : 1;
    const long long per_sp = (long long)nz * g.n[1] * a.S * a.ppc;
    const long long total = per_sp * g.nsp;
    for (long long idx = blockIdx.x * (long long)kBlock + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * kBlock) {
        const int sp = (int)(idx / per_sp);
        const long long in_sp = idx - sp * per_sp;
        long long r = in_sp;
        const int q = (int)(r % a.ppc);
        r /= a.ppc;
        const int col = (int)(r % a.S);
        r /= a.S;
        const int cy = (int)(r % g.n[1]);
        const int cz = (int)(r / g.n[1]);
        const int cx = g.n[0] - a.S + col;
        const double x = ((double)cx + 0.5 + (double)a.origin) * a.dx;
        double dens;
        if (a.ramp_len > 0.0) {
            double v = (x - a.ramp_start) / a.ramp_len;
            v = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
            dens = a.n0 * v;
        } else {
            dens = x >= a.ramp_start ? a.n0 : 0.0;
        }
        if (!(dens > 0.0)) continue;
        const real off = (real)(((double)q + 0.5) / (double)a.ppc);
        const int tile = cx / g.T[0] + g.nt[0] * (cy / g.T[1] + (DIM == 3 ? g.nt[1] * (cz / g.T[2]) : 0));
        const int sid = tile * g.nsp + sp;
        const int pos = atomicAdd(&seg.count[sid], 1);
        const PArrays<real>* to = &p;
        long long j;
        if (pos < seg.cap[sid]) {
            j = (long long)seg.start[sid] + pos;
        } else {
            atomicSub(&seg.count[sid], 1);
            j = atomicAdd(&ctr[CTR_STASH], 1);
            to = &st;
            st.sp[j] = sp;
        }
        to->cell[j] = pack_cell<DIM>(cx, cy, cz);
        for (int d = 0; d < DIM; ++d) to->off[d][j] = off;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            to->u[d][j] = real(0);
            to->s[d][j] = (real)a.s0[d];
        }
        to->w[j] = (real)(dens / (double)a.ppc);
        to->id[j] = a.next_id[sp] + (int32_t)in_sp;
    }
}

// ---------------------------------------------------------------- launchers

template <typename real, int DIM>
hipError_t launch_shift_cells(const PArrays<real>& p, const Segs& seg, int S, int nseg, hipStream_t stream) {
    hipLaunchKernelGGL((k_shift_cells<real, DIM>), dim3(nseg), dim3(kBlock), 0, stream, p, seg, S);
    return hipGetLastError();
}

template <typename real, int DIM>
hipError_t launch_inject(const Geom& g, const PArrays<real>& p, const Segs& seg, const PArrays<real>& st,
                         int32_t* ctr, const InjectArgs& a, hipStream_t stream) {
    const long long total = (long long)(DIM == 3 ? g.n[2] : 1) * g.n[1] * a.S * a.ppc * g.nsp;
    if (total <= 0) return hipSuccess;
    const long long blocks = std::min<long long>((total + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL((k_inject<real, DIM>), dim3((unsigned)blocks), dim3(kBlock), 0, stream, g, p, seg, st,
                       ctr, a);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_repack_segments(const PArrays<real>& from, const PArrays<real>& to,
                                  const int32_t* old_start, const int32_t* new_start,
                                  const int32_t* count, int nseg, int ndim, hipStream_t stream) {
    hipLaunchKernelGGL((k_repack_segments<real>), dim3(nseg), dim3(kBlock), 0, stream, from, to,
                       old_start, new_start, count, ndim);
    return hipGetLastError();
}

template <typename real, typename acc_t, int DIM>
hipError_t launch_push_tiles(const Geom& g, const Consts<real>& k, const PArrays<real>& p,
                             const Segs& seg, const PArrays<real>& lv, int32_t* ctr, int slot,
                             const Fields<freal>& f, int deposit, const RecArgs& rec, hipStream_t stream) {
    const size_t lds = tile_lds_bytes<real, acc_t>(g, seg.max_chunks);
    const int grid = ((g.ntiles + 7) >> 3) * 8;
    if constexpr (!kFixedAcc<acc_t>) {
        if (rec.acc) {
            hipLaunchKernelGGL((k_push_tiles_rec<real, acc_t, DIM>), dim3(grid), dim3(kBlock), lds, stream,
                               g, k, p, seg, lv, ctr, slot, f, deposit, rec);
            return hipGetLastError();
        }
    } else {
        if (rec.acc) return hipErrorInvalidValue;   // the record is not kept in the deterministic mode
    }
    hipLaunchKernelGGL((k_push_tiles<real, acc_t, DIM, false>), dim3(grid), dim3(kBlock), lds, stream,
                       g, k, p, seg, lv, ctr, slot, f, deposit, rec);
    return hipGetLastError();
}

template <typename real, typename acc_t>
hipError_t launch_push_march(const Geom& g, const Consts<real>& k, const PArrays<real>& p, const Segs& seg,
                             const PArrays<real>& lv, int32_t* ctr, int slot, const Fields<freal>& f, int deposit,
                             int R, int xcd_major, hipStream_t stream) {
    if (g.ndim != 3 || g.T[2] < 3 || R < 1) return hipErrorInvalidValue;
    const size_t lds = tile_lds_bytes<real, acc_t>(g, seg.max_chunks);
    const int nruns = g.nt[0] * g.nt[1] * ((g.nt[2] + R - 1) / R);
    const int grid = ((nruns + 7) >> 3) * 8;
    hipLaunchKernelGGL((k_push_march<real, acc_t>), dim3(grid), dim3(kBlock), lds, stream, g, k, p, seg, lv, ctr,
                       slot, f, deposit, R, nruns, xcd_major);
    return hipGetLastError();
}

template <typename real, int DIM>
hipError_t launch_push_stash(const Geom& g, const Consts<real>& k, const PArrays<real>& st,
                             int32_t* ctr, const Fields<freal>& f, int deposit, const RecArgs& rec,
                             int blocks, hipStream_t stream) {
    if (rec.acc)
        hipLaunchKernelGGL((k_push_stash<real, DIM, true>), dim3(blocks), dim3(kBlock), 0, stream,
                           g, k, st, ctr, f, deposit, rec);
    else
        hipLaunchKernelGGL((k_push_stash<real, DIM, false>), dim3(blocks), dim3(kBlock), 0, stream,
                           g, k, st, ctr, f, deposit, rec);
    return hipGetLastError();
}

template <typename real, int DIM>
hipError_t launch_insert(const Geom& g, const PArrays<real>& p, const Segs& seg,
                         const PArrays<real>& lv, const PArrays<real>& st, int32_t* ctr, int slot,
                         unsigned long long* moved, int blocks, hipStream_t stream) {
    hipLaunchKernelGGL((k_insert<real, DIM>), dim3(blocks), dim3(kBlock), 0, stream,
                       g, p, seg, lv, st, ctr, slot, moved);
    return hipGetLastError();
}

template <typename real, typename acc_t>
hipError_t launch_push_tiles_batch(const RunDesc<real>* runs, const TileRef* order, const XcdQueues& q, int blocks,
                                   size_t lds, const PArrays<real>& p, const Segs& seg, const PArrays<real>& lv,
                                   int32_t* ctr, int slot, const Fields<freal>& f, int deposit,
                                   unsigned long long* run_ns, hipStream_t stream) {
    hipLaunchKernelGGL((k_push_tiles_batch<real, acc_t>), dim3(blocks), dim3(kBlock), lds, stream, runs, order,
                       q, p, seg, lv, ctr, slot, f, deposit, run_ns);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_push_stash_batch(const RunDesc<real>* runs, const PArrays<real>& st, int32_t* ctr,
                                   const Fields<freal>& f, int deposit, int blocks, hipStream_t stream) {
    hipLaunchKernelGGL((k_push_stash_batch<real>), dim3(blocks), dim3(kBlock), 0, stream, runs, st, ctr, f,
                       deposit);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_insert_batch(const RunDesc<real>* runs, const PArrays<real>& p, const Segs& seg,
                               const PArrays<real>& lv, const PArrays<real>& st, int32_t* ctr, int slot,
                               unsigned long long* moved, int blocks, hipStream_t stream) {
    hipLaunchKernelGGL((k_insert_batch<real>), dim3(blocks), dim3(kBlock), 0, stream, runs, p, seg, lv, st, ctr,
                       slot, moved);
    return hipGetLastError();
}

#define SPINPIC_WINDOW_INST(real, DIM)                                                                        \
    template hipError_t launch_shift_cells<real, DIM>(const PArrays<real>&, const Segs&, int, int, hipStream_t); \
    template hipError_t launch_shift_stash<real, DIM>(const PArrays<real>&, const int32_t*, int, hipStream_t); \
    template hipError_t launch_inject<real, DIM>(const Geom&, const PArrays<real>&, const Segs&,               \
                                                 const PArrays<real>&, int32_t*, const InjectArgs&, hipStream_t);
SPINPIC_WINDOW_INST(float, 2)
SPINPIC_WINDOW_INST(float, 3)
SPINPIC_WINDOW_INST(double, 2)
SPINPIC_WINDOW_INST(double, 3)
#undef SPINPIC_WINDOW_INST

template hipError_t launch_push_tiles_batch<float, double>(const RunDesc<float>*, const TileRef*, const XcdQueues&, int,
    size_t, const PArrays<float>&, const Segs&, const PArrays<float>&, int32_t*, int, const Fields<freal>&, int,
    unsigned long long*, hipStream_t);
template hipError_t launch_push_tiles_batch<float, float>(const RunDesc<float>*, const TileRef*, const XcdQueues&, int,
    size_t, const PArrays<float>&, const Segs&, const PArrays<float>&, int32_t*, int, const Fields<freal>&, int,
    unsigned long long*, hipStream_t);
template hipError_t launch_push_tiles_batch<double, double>(const RunDesc<double>*, const TileRef*, const XcdQueues&, int,
    size_t, const PArrays<double>&, const Segs&, const PArrays<double>&, int32_t*, int, const Fields<freal>&,
    int, unsigned long long*, hipStream_t);
template hipError_t launch_push_stash_batch<float>(const RunDesc<float>*, const PArrays<float>&, int32_t*,
    const Fields<freal>&, int, int, hipStream_t);
template hipError_t launch_push_stash_batch<double>(const RunDesc<double>*, const PArrays<double>&,
    int32_t*, const Fields<freal>&, int, int, hipStream_t);
template hipError_t launch_insert_batch<float>(const RunDesc<float>*, const PArrays<float>&, const Segs&,
    const PArrays<float>&, const PArrays<float>&, int32_t*, int, unsigned long long*, int, hipStream_t);
template hipError_t launch_insert_batch<double>(const RunDesc<double>*, const PArrays<double>&, const Segs&,
    const PArrays<double>&, const PArrays<double>&, int32_t*, int, unsigned long long*, int, hipStream_t);

template <typename real, typename acc_t>
int push_batch_blocks_per_cu(size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_push_tiles_batch<real, acc_t>, kBlock, lds) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}
template int push_batch_blocks_per_cu<float, double>(size_t);
template int push_batch_blocks_per_cu<float, float>(size_t);
template int push_batch_blocks_per_cu<double, double>(size_t);

#define SPINPIC_INST_PUSH(real, acc, DIM)                                                       \
    template hipError_t launch_push_tiles<real, acc, DIM>(const Geom&, const Consts<real>&,    \
        const PArrays<real>&, const Segs&, const PArrays<real>&, int32_t*, int,                \
        const Fields<freal>&, int, const RecArgs&, hipStream_t);

SPINPIC_INST_PUSH(float, float, 2)
SPINPIC_INST_PUSH(float, float, 3)
SPINPIC_INST_PUSH(float, double, 2)
SPINPIC_INST_PUSH(float, double, 3)
SPINPIC_INST_PUSH(double, double, 2)
SPINPIC_INST_PUSH(double, double, 3)
#define SPINPIC_INST_MARCH(real, acc)                                                           \
    template hipError_t launch_push_march<real, acc>(const Geom&, const Consts<real>&,          \
        const PArrays<real>&, const Segs&, const PArrays<real>&, int32_t*, int,                \
        const Fields<freal>&, int, int, int, hipStream_t);
SPINPIC_INST_MARCH(float, float)
SPINPIC_INST_MARCH(float, double)
SPINPIC_INST_MARCH(double, double)
SPINPIC_INST_MARCH(float, unsigned long long)
SPINPIC_INST_MARCH(double, unsigned long long)
#undef SPINPIC_INST_MARCH
// deterministic mode: fixed-point current sums
SPINPIC_INST_PUSH(float, unsigned long long, 2)
SPINPIC_INST_PUSH(float, unsigned long long, 3)
SPINPIC_INST_PUSH(double, unsigned long long, 2)
SPINPIC_INST_PUSH(double, unsigned long long, 3)
template size_t tile_lds_bytes<float, float>(const Geom&, int);
template size_t tile_lds_bytes<float, unsigned long long>(const Geom&, int);
template size_t tile_lds_bytes<double, unsigned long long>(const Geom&, int);
template size_t tile_lds_bytes<float, double>(const Geom&, int);
template size_t tile_lds_bytes<double, double>(const Geom&, int);

#define SPINPIC_INST_REST(real, DIM)                                                            \
    template hipError_t launch_push_stash<real, DIM>(const Geom&, const Consts<real>&,         \
        const PArrays<real>&, int32_t*, const Fields<freal>&, int, const RecArgs&, int,         \
        hipStream_t);                                                                          \
    template hipError_t launch_insert<real, DIM>(const Geom&, const PArrays<real>&,            \
        const Segs&, const PArrays<real>&, const PArrays<real>&, int32_t*, int,                 \
        unsigned long long*, int, hipStream_t);

SPINPIC_INST_REST(float, 2)
SPINPIC_INST_REST(float, 3)
SPINPIC_INST_REST(double, 2)
SPINPIC_INST_REST(double, 3)

template hipError_t launch_repack_segments<float>(const PArrays<float>&, const PArrays<float>&,
    const int32_t*, const int32_t*, const int32_t*, int, int, hipStream_t);
template hipError_t launch_repack_segments<double>(const PArrays<double>&, const PArrays<double>&,
    const int32_t*, const int32_t*, const int32_t*, int, int, hipStream_t);
}  // namespace spinpic
