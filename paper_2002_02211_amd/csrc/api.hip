// Host runtime and C ABI of libspinpic: configuration checks, the tile-sorted
// upload of the initial state, the per-step launch sequence, the lazy repack
// of overflowing tiles, and the read-back calls.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/spinpic.h"
#include "common.h"
#include "kernels.h"

using namespace spinpic;

// The bins of pic_spectrum_noalloc (count, weight sum and three spin sums per
// bin, at most PIC_MAX_SPECTRUM_BINS bins: 40 KiB), one copy on every GPU the
// library runs on, held until the process ends.  In host code this name is a
// host-side stand-in, not a device address: host code uses only the address
// that hipGetSymbolAddress returns for the device (scratch_address below).
static __device__ __align__(256) double scratch[5 * PIC_MAX_SPECTRUM_BINS];

namespace {

thread_local std::string g_init_error;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_addr[kMaxDevices] = {};

struct Status {
    int code = PIC_OK;
    std::string msg;
};

Status fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    Status s;
    s.code = code;
    s.msg = buf;
    return s;
}

#define HIP_OR_FAIL(expr)                                                                  \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess) return fail(PIC_EHIP, "%s: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

// Device address of `scratch` on device dev, which must be the current
// device: looked up once per device (at the first pic_init on it) and kept.
Status scratch_address(int dev, double** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(PIC_EINVAL, "device %d outside 0..%d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PIC_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_addr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_addr[dev];
    return Status{};
}

// Overflow policy.  Every kStashCheck steps the step loop waits for its
// stream, so that the pinned copy of the overflow count is current (the host
// can otherwise run many steps ahead of the GPU), and folds the overflow
// store back into the tiles when it holds more than npart / kStashFrac
// particles, or any at all on a kStashPeriod boundary: overflow particles are
// pushed from global memory at a fraction of the tile push's rate.  While the
// store holds more than a quarter of that, the next check comes after
// kStashCheckSoon steps instead (a laser-compressed plasma can fill it by
// several times the threshold within 16 steps); checks stay on multiples of
// their interval, so every kStashPeriod boundary is one.
constexpr int kStashCheck = 16;
constexpr int kStashCheckSoon = 4;
constexpr int kStashPeriod = 64;
constexpr long long kStashFrac = 512;
constexpr int kStashBlocks = 1024;
// A segment that overflowed is usually in a region still being compressed
// (a laser's ponderomotive front): the repack gives it kGrowSlack times the
// slack and keeps room it was given while the count stays within that.
constexpr double kGrowSlack = 3.0;

// ---------------------------------------------------------------- config

struct Resolved {
    pic_config cfg;
    int ndim;
    int n[3];
    int T[3];
    int nt[3];
    double slack;
    int use_acc64;
    int det;         // PIC_FLAG_DETERMINISTIC: fixed-point current and polarization sums
    int cell_rows;   // PIC_FLAG_CELL_ROWS: initial rows in cell form
};

template <typename real, typename acc_t>
size_t lds_need(const int T[3], int ndim) {
    Geom g{};
    g.ndim = ndim;
    for (int a = 0; a < 3; ++a) g.T[a] = T[a];
    return tile_lds_bytes<real, acc_t>(g, 0);
}

Status resolve_config(const pic_config* cfg, const pic_state* init, Resolved& R) {
    if (!cfg) return fail(PIC_EINVAL, "cfg is NULL");
    R.cfg = *cfg;
    const pic_config& c = *cfg;
    if (c.ndim != 2 && c.ndim != 3) return fail(PIC_EINVAL, "ndim must be 2 or 3 (got %d)", c.ndim);
    R.ndim = c.ndim;
    const int maxn2[3] = {65535, 65535, 1};
    const int maxn3[3] = {2047, 2047, 1023};
    for (int a = 0; a < 3; ++a) {
        if (a >= c.ndim) {
            R.n[a] = 1;
            continue;
        }
        const int lim = c.ndim == 2 ? maxn2[a] : maxn3[a];
        if (c.n[a] < 1 || c.n[a] > lim)
            return fail(PIC_EINVAL, "n[%d] = %d outside 1..%d", a, c.n[a], lim);
        if (!(c.d[a] > 0.0) || !std::isfinite(c.d[a]))
            return fail(PIC_EINVAL, "d[%d] must be positive and finite", a);
        R.n[a] = c.n[a];
    }
    if (!(c.dt > 0.0) || !std::isfinite(c.dt)) return fail(PIC_EINVAL, "dt must be positive and finite");
    double cour = 0.0;
    for (int a = 0; a < c.ndim; ++a) cour += 1.0 / (c.d[a] * c.d[a]);
    cour = c.dt * std::sqrt(cour);
    if (!(cour < 1.0)) return fail(PIC_ECFL, "Courant number %.6f >= 1", cour);
    if (c.precision != PIC_FP64 && c.precision != PIC_FP32_MIXED)
        return fail(PIC_EINVAL, "unknown precision %d", c.precision);
    if (c.nspecies < 1 || c.nspecies > PIC_MAX_SPECIES)
        return fail(PIC_EINVAL, "nspecies must be 1..%d (got %d)", PIC_MAX_SPECIES, c.nspecies);
    for (int s = 0; s < c.nspecies; ++s) {
        const pic_species& sp = c.sp[s];
        if (!(sp.mu > 0.0) || !std::isfinite(sp.mu) || !std::isfinite(sp.Z) || !std::isfinite(sp.a))
            return fail(PIC_EINVAL, "species %d: mass must be positive, Z and a finite", s);
    }
    if (c.flags & ~(PIC_FLAG_TEST_PARTICLE | PIC_FLAG_DETERMINISTIC | PIC_FLAG_CELL_ROWS))
        return fail(PIC_EINVAL, "unknown flags 0x%x", c.flags);
    R.det = (c.flags & PIC_FLAG_DETERMINISTIC) ? 1 : 0;
    R.cell_rows = (c.flags & PIC_FLAG_CELL_ROWS) ? 1 : 0;
    if (c.deposit_acc < PIC_ACC_DEFAULT || c.deposit_acc > PIC_ACC_FP64)
        return fail(PIC_EINVAL, "unknown deposit_acc %d", c.deposit_acc);
    // FP64 shared-memory sums are the default: besides their precision, the
    // LDS FP64 atomic add runs the deposit about twice as fast as the FP32 one
    // on gfx950 (measured on the c2 workload)
    R.use_acc64 = c.precision == PIC_FP64 || c.deposit_acc != PIC_ACC_FP32;
    if (c.slack < 0.0 || !std::isfinite(c.slack)) return fail(PIC_EINVAL, "slack must be >= 0");
    // default slack: 25 %; 100 % for 3D FP64, whose 6 x 6 x 6 tiles hold half
    // as many particles per segment as the FP32 ones, so that compression by
    // a laser fills them sooner (c3 FP64 with 25 %: steps 10-60 took 112 ms
    // each with the push at 10.5 ms, the overflow store's push from global
    // memory taking the rest)
    R.slack = c.slack > 0.0 ? c.slack : (c.ndim == 3 && c.precision == PIC_FP64 ? 1.0 : 0.25);
    for (int a = 0; a < 3; ++a) {
        if (a >= c.ndim) {
            R.T[a] = 1;
            R.nt[a] = 1;
            continue;
        }
        int t = c.tile[a];
        // defaults measured on gfx950: 16 x 16 in 2D; in 3D tiles of 12 x 6 x 6
        // (FP32 particles) or 6 x 6 x 6 (FP64) fit three workgroups per CU
        // in shared memory
        if (t == 0) t = c.ndim == 2 ? 16 : (c.precision == PIC_FP64 ? 6 : (a == 0 ? 12 : 6));
        if (t < 1 || t > 64) return fail(PIC_EINVAL, "tile[%d] = %d outside 1..64", a, c.tile[a]);
        t = std::min(t, R.n[a]);
        R.T[a] = t;
        R.nt[a] = (R.n[a] + t - 1) / t;
    }
    size_t lds;
    if (c.precision == PIC_FP64) lds = lds_need<double, double>(R.T, c.ndim);
    else if (R.use_acc64) lds = lds_need<float, double>(R.T, c.ndim);
    else lds = lds_need<float, float>(R.T, c.ndim);
    if (lds > 64 * 1024)
        return fail(PIC_EINVAL, "tile %dx%dx%d needs %zu bytes of shared memory (max 65536)", R.T[0],
                    R.T[1], R.T[2], lds);
    const long long ntiles = (long long)R.nt[0] * R.nt[1] * R.nt[2];
    if (ntiles * c.nspecies > (1LL << 30)) return fail(PIC_EINVAL, "too many tiles");
    if (init) {
        long long total = 0;
        for (int s = 0; s < c.nspecies; ++s) {
            if (init->count[s] < 0) return fail(PIC_EINVAL, "species %d: negative count", s);
            if (init->count[s] > 0 && !init->particles[s])
                return fail(PIC_EINVAL, "species %d: particles pointer is NULL", s);
            total += init->count[s];
        }
        if (total > (1LL << 30)) return fail(PIC_EINVAL, "more than 2^30 particles");
    }
    return Status{};
}

// ---------------------------------------------------------------- engine

constexpr int kTimers = 4;   // push+deposit, overflow push, insertion, field update

struct Timer {
    bool on = false;
    unsigned mask = 0;   // kernel classes recorded (bit k: class k)
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> rec;
    size_t used = 0;
};

// HIP events around each kernel class on a stream: start/stop pairs recorded
// while on, summed per class by timer_read.  The events are created ahead,
// at enable (creating them between launches would delay the launches that
// follow a wait).
constexpr size_t kTimerPool = 1024;

void timer_grow(Timer& tm, size_t want) {
    while (tm.pool.size() < want) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        tm.pool.push_back(e);
    }
}

void timer_start(Timer& tm, hipStream_t stream, int k) {
    if (!tm.on || !((tm.mask >> k) & 1u)) return;
    if (tm.used + 2 > tm.pool.size()) timer_grow(tm, 2 * tm.pool.size() + 2);
    if (tm.used + 2 > tm.pool.size()) return;
    hipEvent_t a = tm.pool[tm.used++];
    hipEvent_t b = tm.pool[tm.used++];
    (void)hipEventRecord(a, stream);
    tm.rec.push_back({k, {a, b}});
}

void timer_stop(Timer& tm, hipStream_t stream, int k) {
    if (!tm.on || tm.rec.empty() || tm.rec.back().first != k) return;
    (void)hipEventRecord(tm.rec.back().second.second, stream);
}

Status timer_enable(Timer& tm, hipStream_t stream, int enable) {
    if (enable < 0 || enable > 2) return fail(PIC_EINVAL, "timing mode %d is not 0, 1 or 2", enable);
    HIP_OR_FAIL(hipStreamSynchronize(stream));
    tm.on = enable != 0;
    tm.mask = enable == 2 ? 1u : (1u << kTimers) - 1u;
    tm.rec.clear();
    tm.used = 0;
    if (tm.on) timer_grow(tm, kTimerPool);
    return Status{};
}

Status timer_read(Timer& tm, hipStream_t stream, double* ms, int64_t* launches, int cap) {
    if (cap < kTimers) return fail(PIC_EINVAL, "timing_read needs cap >= %d", kTimers);
    HIP_OR_FAIL(hipStreamSynchronize(stream));
    double t[kTimers] = {0, 0, 0, 0};
    int64_t c[kTimers] = {0, 0, 0, 0};
    for (auto& r : tm.rec) {
        float e = 0.f;
        HIP_OR_FAIL(hipEventElapsedTime(&e, r.second.first, r.second.second));
        t[r.first] += e;
        c[r.first]++;
    }
    for (int i = 0; i < kTimers; ++i) {
        if (ms) ms[i] = t[i];
        if (launches) launches[i] = c[i];
    }
    return Status{};
}

void timer_free(Timer& tm) {
    for (auto& e : tm.pool) (void)hipEventDestroy(e);
    tm.pool.clear();
    tm.rec.clear();
    tm.used = 0;
}

class EngineBase {
public:
    virtual ~EngineBase() {}
    virtual Status init(const Resolved& R, const pic_state* st) = 0;
    virtual Status step(int n) = 0;
    virtual Status polarization(int species, double emin, double emax, double P[3], int64_t* N) = 0;
    virtual Status record(int species, double emin, double emax, int capacity) = 0;
    virtual Status record_read(double* P, int64_t* N, int cap, int* n_out) = 0;
    virtual Status fields(uint32_t mask, double* out, size_t cap) = 0;
    virtual Status particles(int species, double* out, size_t cap, int64_t* n, bool cells = false) = 0;
    virtual Status poison(int species) = 0;
    virtual Status spectrum(int species, double emin, double emax, int nbins, double* count,
                            double* weight, double* spin) = 0;
    virtual Status spectrum_noalloc(int species, double emin, double emax, int nbins, double* count,
                                    double* weight, double* spin) = 0;
    virtual Status phase_space(int species, int axis, double xmin, double xmax, int nx, int comp,
                               double pmin, double pmax, int np, double* out) = 0;
    virtual Status density(int species, double* out, size_t cap) = 0;
    virtual Status energy(double* out, int cap) = 0;
    virtual Status stats(int64_t* out, int cap) = 0;
    virtual Status timing(int enable) = 0;
    virtual Status timing_read(double* ms, int64_t* launches, int cap) = 0;
    virtual Status window(const pic_window_config* w) = 0;
    virtual void release() = 0;
};

template <typename real, int DIM>
class Engine : public EngineBase {
public:
    Engine(const pic_allocator* alloc, hipStream_t stream) : stream_(stream) {
        if (alloc && alloc->alloc && alloc->free) {
            alloc_ = *alloc;
            has_alloc_ = true;
        }
    }
    ~Engine() override { release(); }

    Status init(const Resolved& R, const pic_state* st) override;
    Status step(int n) override;
    Status polarization(int species, double emin, double emax, double P[3], int64_t* N) override;
    Status record(int species, double emin, double emax, int capacity) override;
    Status record_read(double* P, int64_t* N, int cap, int* n_out) override;
    Status fields(uint32_t mask, double* out, size_t cap) override;
    Status particles(int species, double* out, size_t cap, int64_t* n, bool cells = false) override;
    Status poison(int species) override;
    Status spectrum(int species, double emin, double emax, int nbins, double* count, double* weight,
                    double* spin) override;
    Status spectrum_noalloc(int species, double emin, double emax, int nbins, double* count, double* weight,
                            double* spin) override;
    Status phase_space(int species, int axis, double xmin, double xmax, int nx, int comp, double pmin,
                       double pmax, int np, double* out) override;
    Status density(int species, double* out, size_t cap) override;
    Status energy(double* out, int cap) override;
    Status stats(int64_t* out, int cap) override;
    Status timing(int enable) override;
    Status timing_read(double* ms, int64_t* launches, int cap) override;
    Status window(const pic_window_config* w) override;
    void release() override;

private:
    Status window_shift();
    Status live_counts(long long out[kMaxSpecies]);
    Status stored_count(long long* n);
    Status grow_stores(long long need);
    // device memory
    void* dalloc(size_t bytes) {
        if (bytes == 0) bytes = 256;
        void* p = nullptr;
        if (has_alloc_) p = alloc_.alloc(alloc_.user, bytes);
        else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
        if (p) live_.push_back(p);
        return p;
    }
    void dfree(void* p) {
        if (!p) return;
        auto it = std::find(live_.begin(), live_.end(), p);
        if (it != live_.end()) live_.erase(it);
        if (has_alloc_) alloc_.free(alloc_.user, p);
        else (void)hipFree(p);
    }
    Status alloc_store(PArrays<real>& a, long long cap, bool with_species);
    void free_store(PArrays<real>& a);
    Status repack();
    Status check_lds() {
        // the deterministic mode's 64-bit integer sums take the room of FP64 ones
        const size_t lds = (use_acc64_ || det_) ? tile_lds_bytes<real, double>(g_, seg_.max_chunks)
                                                : tile_lds_bytes<real, real>(g_, seg_.max_chunks);
        if (lds > 64 * 1024)
            return fail(PIC_ECAPACITY, "a tile segment of %d slots needs %zu bytes of shared memory "
                        "(max 65536); use smaller tiles", seg_.max_chunks * 64, lds);
        return Status{};
    }
    Status reduce(int mode, const ReduceArgs& ra, double* host_acc);
    Status nonfinite_flag(bool* set);
    Status spectrum_args(int species, double emin, double emax, int nbins, const double* count,
                         const double* weight, const double* spin, BinArgs& ba);
    Status compute_rho();
    Status residual_max(double* out);
    void tstart(int k);
    void tstop(int k);
    Status sync() {
        HIP_OR_FAIL(hipStreamSynchronize(stream_));
        return Status{};
    }

    pic_allocator alloc_{};
    bool has_alloc_ = false;
    hipStream_t stream_;
    std::vector<void*> live_;

    Resolved R_{};
    Geom g_{};
    Consts<real> k_{};
    int deposit_ = 1;
    int use_acc64_ = 0;
    int det_ = 0;                  // deterministic mode
    int march_R_ = 1;              // 3D: tiles per z-run of the marching push (1: one tile per workgroup)
    int march_xcd_ = 0;            // 3D marching push: contiguous range of runs per XCD
    double fx_inv_ = 0.0;          // 1 / the fixed-point current's scale
    int nseg_ = 0;
    long long cap_total_ = 0;
    long long store_slots_ = 0;   // slots allocated in p_ (at least cap_total_ + kSpareSlots)
    long long npart_ = 0;
    long long count_sp_[kMaxSpecies] = {0, 0, 0, 0};
    double d_[3] = {1, 1, 1};
    int64_t nstep_ = 0;
    int64_t check_at_ = kStashCheck;   // step of the next overflow check
    int64_t repacks_ = 0;

    PArrays<real> p_{}, lv_{}, st_{};
    Segs seg_{};
    Fields<freal> f_{};
    Consts<freal> kf_{};          // field-update constants in the field type
    int32_t* ctr_ = nullptr;
    unsigned long long* moved_ = nullptr;
    int32_t* h_ctr_ = nullptr;     // pinned mirror of the counters
    double* acc_ = nullptr;        // reduction accumulators
    double* rho_ = nullptr;
    double* ref_ = nullptr;        // div E - rho at init
    double* blockmax_ = nullptr;
    int resid_blocks_ = 0;
    int32_t* nf_flag_ = nullptr;
    int dev_ = 0;                  // the device current at init
    double* spec_buf_ = nullptr;   // this device's static spectrum buffer (scratch)
    freal* jbuf_[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    // the fused Yee step writes the new E and B here; the pointers are then
    // swapped with f_'s
    freal* enext_[3] = {nullptr, nullptr, nullptr};
    freal* bnext_[3] = {nullptr, nullptr, nullptr};
    freal* mur_next_ = nullptr;   // spare Mur state (open x faces)
    int jcur_ = 0;                 // buffer holding the last step's current
    long long store_cap_ = 0;      // slots of the leaver and overflow stores
    // moving window
    bool win_on_ = false;
    pic_window_config win_{};
    int64_t win_step0_ = 0;        // nstep_ at pic_window
    long long shifts_ = 0;
    long long next_id_[kMaxSpecies] = {0, 0, 0, 0};
    freal* scratch_ = nullptr;     // one field array, for the shifts
    Segs seg_tmp_{};               // a second segment table, for the shifts
    long long npart_bound_ = 0;    // stored entries at the last count + injected since
    // per-step Eq. 4 record (pic_polarization_record)
    bool rec_on_ = false;
    RecArgs rec_{};                // selection; acc set per step
    double* rec_buf_ = nullptr;    // rec_cap_ steps x kRecSlots x kRecStride sums
    int rec_cap_ = 0;
    int rec_n_ = 0;                // steps recorded since the last read
    Timer timer_;
};

template <typename real, int DIM>
Status Engine<real, DIM>::alloc_store(PArrays<real>& a, long long cap, bool with_species) {
    a = PArrays<real>{};
    const size_t n = (size_t)std::max(cap, 1LL);
    a.cell = (int32_t*)dalloc(n * sizeof(int32_t));
    for (int d = 0; d < DIM; ++d) a.off[d] = (real*)dalloc(n * sizeof(real));
    for (int d = 0; d < 3; ++d) {
        a.u[d] = (real*)dalloc(n * sizeof(real));
        a.s[d] = (real*)dalloc(n * sizeof(real));
    }
    a.w = (real*)dalloc(n * sizeof(real));
    a.id = (int32_t*)dalloc(n * sizeof(int32_t));
    if (with_species) a.sp = (int32_t*)dalloc(n * sizeof(int32_t));
    bool ok = a.cell && a.w && a.id && (!with_species || a.sp);
    for (int d = 0; d < DIM; ++d) ok = ok && a.off[d];
    for (int d = 0; d < 3; ++d) ok = ok && a.u[d] && a.s[d];
    if (!ok) return fail(PIC_ENOMEM, "device allocation of a particle store (%lld slots) failed", cap);
    return Status{};
}

template <typename real, int DIM>
void Engine<real, DIM>::free_store(PArrays<real>& a) {
    dfree(a.cell);
    for (int d = 0; d < 3; ++d) {
        dfree(a.off[d]);
        dfree(a.u[d]);
        dfree(a.s[d]);
    }
    dfree(a.w);
    dfree(a.id);
    dfree(a.sp);
    a = PArrays<real>{};
}

template <typename real, int DIM>
void Engine<real, DIM>::release() {
    if (stream_ != nullptr || !live_.empty()) (void)hipStreamSynchronize(stream_);
    timer_free(timer_);
    std::vector<void*> all = live_;
    for (void* p : all) dfree(p);
    live_.clear();
    if (h_ctr_) (void)hipHostFree(h_ctr_);
    h_ctr_ = nullptr;
}

static long long round_up(long long v, long long m) { return (v + m - 1) / m * m; }

// Slots of the particle store: the kernels address a slot's FP64 values
// with a 32-bit byte offset, so 2^29 slots at most.
constexpr long long kMaxSlots = (1LL << 29) - 64;
constexpr long long kSpareSlots = 64;   // write targets of masked-off lanes

// Slots to allocate for the store a repack builds, `need` of them used: the
// current store's size while that suffices, else a quarter more than needed.
// The repack fills the new store from the old one and only then frees it, so
// with a caching allocator (torch's) the block the previous repack freed
// serves this one; sizes that grew a little at every repack would each take
// a new block and leave all the older ones cached.
static long long store_alloc_slots(long long need, long long current) {
    if (need <= current) return current;
    return std::min(need + need / 4, kMaxSlots + kSpareSlots);
}

static long long seg_capacity(long long count, double slack) {
    return round_up((long long)std::ceil(count * (1.0 + slack)) + 32, 32);
}

// Tiles per z-run of the 3D marching push; 1 runs the single-tile push.
// Measured on c3 (12 x 6 x 6 tiles, counters over 24 launches): runs of 8
// tiles fetch 13.8 GB per launch instead of 15.5 (per-XCD ranges of runs:
// 10.1 GB) yet take 5.24 ms instead of 5.05 (5.95 ms): the 3D push is held
// by its instruction stream and shared-memory conflicts, not by its HBM
// traffic, so the single-tile push stays the default.
constexpr int kMarchRun = 1;


// The step of the next overflow check after one at nstep that found nstash
// particles in the overflow store (none left if it repacked).
static long long next_check(long long nstep, long long nstash, long long npart) {
    const long long every = nstash > std::max(256LL, npart / (4 * kStashFrac)) ? kStashCheckSoon : kStashCheck;
    return (nstep / every + 1) * every;
}

static bool repack_due(long long nstep, long long nstash, long long npart) {
    if (nstash <= 0) return false;
    return nstep % kStashPeriod == 0 || nstash > std::max(1024LL, npart / kStashFrac);
}

// capmax: the largest segment the tile's shared memory holds; a count above
// it fails the shared-memory check after the repack.
static long long regrow_capacity(long long want, long long oldcap, double slack, long long capmax) {
    const long long grown = seg_capacity(want, kGrowSlack * slack);
    long long cp = want > oldcap ? grown : std::max(seg_capacity(want, slack), std::min(oldcap, grown));
    if (cp > capmax) cp = std::max(capmax, round_up(want, 32));
    return cp;
}

// Largest segment capacity (whole 64-slot chunks) for which lds(max_chunks)
// stays within the 64 KiB a workgroup may allocate.
template <typename F>
static long long max_segment_slots(F lds) {
    int lo = 0, hi = 1 << 22;
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        if (lds(mid) <= 64 * 1024) lo = mid;
        else hi = mid - 1;
    }
    return (long long)lo * 64;
}

template <typename real, int DIM>
Status Engine<real, DIM>::init(const Resolved& R, const pic_state* st) {
    R_ = R;
    const pic_config& c = R.cfg;
    g_.ndim = DIM;
    g_.nsp = c.nspecies;
    for (int a = 0; a < 3; ++a) {
        g_.n[a] = R.n[a];
        g_.T[a] = R.T[a];
        g_.nt[a] = R.nt[a];
        d_[a] = a < DIM ? c.d[a] : 1.0;
    }
    g_.ntiles = g_.nt[0] * g_.nt[1] * g_.nt[2];
    g_.ncells = (long long)g_.n[0] * g_.n[1] * g_.n[2];
    nseg_ = g_.ntiles * g_.nsp;
    deposit_ = (c.flags & PIC_FLAG_TEST_PARTICLE) ? 0 : 1;
    use_acc64_ = R.use_acc64;
    det_ = R.det;
    // 3D: the push may march along z over runs of tiles (kMarchRun, or
    // SPINPIC_PUSH_RUN for measurements; 1 = one tile per workgroup); it
    // needs tiles of at least 3 cells along z
    march_R_ = 1;
    if (DIM == 3 && g_.T[2] >= 3) {
        march_R_ = kMarchRun;
        if (const char* e = std::getenv("SPINPIC_PUSH_RUN")) march_R_ = std::max(1, std::atoi(e));
        if (const char* e = std::getenv("SPINPIC_PUSH_XCD")) march_xcd_ = std::atoi(e) != 0;
    }
    const int cols = R.cell_rows ? PIC_PARTICLE_CELL_COLS : PIC_PARTICLE_IN_COLS;
    const int cu = R.cell_rows ? 6 : 3;   // column of ux (then s, then w)

    const double dt = c.dt;
    k_.dt = (real)dt;
    kf_.dt = dt;
    for (int a = 0; a < 3; ++a) {
        k_.dt_d[a] = (real)(dt / d_[a]);
        k_.dt_d_lo[a] = (real)(dt / d_[a] - (double)k_.dt_d[a]);
        k_.d_dt[a] = (real)(d_[a] / dt);
        kf_.cb[a] = 0.5 * dt / d_[a];
        kf_.ce[a] = dt / d_[a];
    }
    kf_.mur_k = (dt - d_[0]) / (dt + d_[0]);
    for (int s = 0; s < kMaxSpecies; ++s) {
        const bool on = s < c.nspecies;
        const double r = on ? c.sp[s].Z / c.sp[s].mu : 0.0;
        k_.r[s] = (real)r;
        k_.eps[s] = (real)(0.5 * r * dt);
        k_.a[s] = on ? (real)c.sp[s].a : real(0);
        k_.Z[s] = on ? (real)c.sp[s].Z : real(0);
    }

    // ---- bin the initial particles by (tile, species) on the host
    std::vector<long long> count(nseg_, 0);
    npart_ = 0;
    for (int s = 0; s < c.nspecies; ++s) {
        count_sp_[s] = st ? st->count[s] : 0;
        npart_ += count_sp_[s];
    }
    struct Placed {
        int cell[3];
        double off[3];
    };
    auto place = [&](const double* row, Placed& pl) -> bool {
        for (int a = 0; a < 3; ++a) {
            pl.cell[a] = 0;
            pl.off[a] = 0.0;
        }
        if (R.cell_rows) {
            // cell index and offset as stored; an offset that rounds to 1 in
            // the storage precision moves to the next cell (as in the push)
            for (int a = 0; a < DIM; ++a) {
                const double cf = row[a], off = row[3 + a];
                if (!(cf >= 0.0 && cf < (double)g_.n[a] && cf == std::floor(cf))) return false;
                if (!(off >= 0.0 && off < 1.0)) return false;
                int ci = (int)cf;
                double o = off;
                if ((real)o >= real(1)) {
                    o = 0.0;
                    ci = (ci + 1) % g_.n[a];
                }
                pl.cell[a] = ci;
                pl.off[a] = o;
            }
            return true;
        }
        for (int a = 0; a < DIM; ++a) {
            const double xi = row[a] / d_[a];
            if (!std::isfinite(xi)) return false;
            const double fl = std::floor(xi);
            double off = xi - fl;
            long long ci = (long long)fl % g_.n[a];
            if (ci < 0) ci += g_.n[a];
            if ((real)off >= real(1)) {   // rounds up to the next cell edge
                off = 0.0;
                ci = (ci + 1) % g_.n[a];
            }
            pl.cell[a] = (int)ci;
            pl.off[a] = off;
        }
        return true;
    };
    auto tile_of = [&](const Placed& pl) {
        return pl.cell[0] / g_.T[0] + g_.nt[0] * (pl.cell[1] / g_.T[1] + g_.nt[1] * (pl.cell[2] / g_.T[2]));
    };
    // Within a segment the particles are interleaved across cells: first one
    // particle of every cell, then a second one, and so on.  The lanes of a
    // wavefront then sit in different cells, so their current deposits hit
    // different shared-memory words instead of serializing on one.
    const int tile_cells = g_.T[0] * g_.T[1] * g_.T[2];
    double zw_sum = 0.0;   // sum of |Z w|: no node's current can exceed it
    // |s|^2 must be 1: to 1e-6 in FP64; in FP32 to 1e-4, since float32 spins
    // rotated over thousands of steps (a restart's input) drift by more than
    // 1e-6 from unit length
    const double s2_tol = std::is_same<real, float>::value ? 1e-4 : 1e-6;
    std::vector<int32_t> segof((size_t)npart_);
    std::vector<uint32_t> key((size_t)npart_);
    {
        std::vector<int32_t> cellrank((size_t)c.nspecies * g_.ncells, 0);
        long long q = 0;
        for (int s = 0; s < c.nspecies; ++s) {
            const double* P = st ? st->particles[s] : nullptr;
            const double Zs = std::fabs(c.sp[s].Z);
            for (long long i = 0; i < count_sp_[s]; ++i, ++q) {
                const double* row = P + i * cols;
                for (int col = 0; col < cols; ++col)
                    if (!std::isfinite(row[col]))
                        return fail(PIC_EINVAL, "species %d particle %lld: non-finite input", s, i);
                const double* sv = row + cu + 3;
                const double s2 = sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2];
                if (std::fabs(s2 - 1.0) > s2_tol)
                    return fail(PIC_EINVAL, "species %d particle %lld: |s| = %.9f, must be 1", s, i,
                                std::sqrt(s2));
                zw_sum += Zs * std::fabs((double)(real)row[cu + 6]);
                Placed pl;
                if (!place(row, pl))
                    return fail(PIC_EINVAL, "species %d particle %lld: cell outside 0..n-1 or offset outside [0, 1)",
                                s, i);
                const int sid = tile_of(pl) * c.nspecies + s;
                segof[q] = sid;
                count[sid]++;
                const long long gcell = ((long long)pl.cell[2] * g_.n[1] + pl.cell[1]) * g_.n[0] + pl.cell[0];
                const long long rank = cellrank[(size_t)s * g_.ncells + gcell]++;
                const int lc = (pl.cell[0] % g_.T[0]) +
                               g_.T[0] * ((pl.cell[1] % g_.T[1]) + g_.T[1] * (pl.cell[2] % g_.T[2]));
                const unsigned long long k64 = (unsigned long long)rank * tile_cells + lc;
                if (k64 > 0xFFFFFFFFull) return fail(PIC_EINVAL, "more than 2^32 particle ranks in a tile");
                key[q] = (uint32_t)k64;
            }
        }
    }
    // Deterministic mode: fixed-point unit 2^-S with the largest S for which
    // zw_sum, a bound on every node's current, stays below 2^61 units
    k_.fx_scale = 0.0;
    fx_inv_ = 0.0;
    if (det_) {
        int e = 0;
        if (zw_sum > 0.0) (void)std::frexp(zw_sum, &e);   // zw_sum < 2^e
        const int S = 61 - e;
        k_.fx_scale = std::ldexp(1.0, S);
        fx_inv_ = std::ldexp(1.0, -S);
    }
    std::vector<int32_t> h_start(nseg_), h_cap(nseg_), h_count(nseg_);
    cap_total_ = 0;
    for (int s = 0; s < nseg_; ++s) {
        const long long cp = seg_capacity(count[s], R.slack);
        h_start[s] = (int32_t)cap_total_;
        h_cap[s] = (int32_t)cp;
        h_count[s] = (int32_t)count[s];
        cap_total_ += cp;
        if (cap_total_ > kMaxSlots) return fail(PIC_ECAPACITY, "particle capacity exceeds 2^29 slots");
    }

    seg_.dummy = (int)cap_total_;
    {
        long long maxcap = 0;
        for (int sg = 0; sg < nseg_; ++sg) maxcap = std::max<long long>(maxcap, h_cap[sg]);
        seg_.max_chunks = (int)((maxcap + 63) / 64);
        Status L = check_lds();
        if (L.code) return L;
    }

    // ---- device allocations (and this device's static spectrum buffer)
    HIP_OR_FAIL(hipGetDevice(&dev_));
    {
        Status A = scratch_address(dev_, &spec_buf_);
        if (A.code) return A;
    }
    store_slots_ = cap_total_ + kSpareSlots;
    Status S = alloc_store(p_, store_slots_, false);
    if (S.code) return S;
    store_cap_ = std::max(npart_, 1LL);
    S = alloc_store(lv_, store_cap_, true);
    if (S.code) return S;
    S = alloc_store(st_, store_cap_, true);
    if (S.code) return S;
    for (int s = 0; s < c.nspecies; ++s) next_id_[s] = count_sp_[s];
    seg_.start = (int32_t*)dalloc(nseg_ * sizeof(int32_t));
    seg_.cap = (int32_t*)dalloc(nseg_ * sizeof(int32_t));
    seg_.count = (int32_t*)dalloc(nseg_ * sizeof(int32_t));
    for (int a = 0; a < 3; ++a) {
        f_.E[a] = (freal*)dalloc(g_.ncells * sizeof(freal));
        f_.B[a] = (freal*)dalloc(g_.ncells * sizeof(freal));
        for (int b = 0; b < 2; ++b) jbuf_[b][a] = (freal*)dalloc(g_.ncells * sizeof(freal));
        f_.J[a] = jbuf_[0][a];
        if (deposit_) {
            enext_[a] = (freal*)dalloc(g_.ncells * sizeof(freal));
            bnext_[a] = (freal*)dalloc(g_.ncells * sizeof(freal));
        }
    }
    ctr_ = (int32_t*)dalloc(CTR_NCTR * sizeof(int32_t));
    moved_ = (unsigned long long*)dalloc(sizeof(unsigned long long));
    acc_ = (double*)dalloc(kRedSlots * kRedStride * sizeof(double));
    rho_ = (double*)dalloc(g_.ncells * sizeof(double));
    ref_ = (double*)dalloc(g_.ncells * sizeof(double));
    resid_blocks_ = (int)std::min<long long>(4096, (g_.ncells + kBlock - 1) / kBlock);
    blockmax_ = (double*)dalloc(resid_blocks_ * sizeof(double));
    nf_flag_ = (int32_t*)dalloc(sizeof(int32_t));
    bool ok = seg_.start && seg_.cap && seg_.count && ctr_ && moved_ && acc_ && rho_ && ref_ &&
              blockmax_ && nf_flag_;
    for (int a = 0; a < 3; ++a)
        ok = ok && f_.E[a] && f_.B[a] && jbuf_[0][a] && jbuf_[1][a] && (!deposit_ || (enext_[a] && bnext_[a]));
    if (!ok) return fail(PIC_ENOMEM, "device allocation failed");
    HIP_OR_FAIL(hipHostMalloc((void**)&h_ctr_, CTR_NCTR * sizeof(int32_t), hipHostMallocDefault));
    std::memset(h_ctr_, 0, CTR_NCTR * sizeof(int32_t));

    // ---- upload particles in segment order
    {
        const size_t C = (size_t)cap_total_;
        std::vector<int32_t> hcell(C, 0), hid(C, 0);
        std::vector<real> hoff[3], hu[3], hs[3], hw(C, real(0));
        for (int a = 0; a < 3; ++a) {
            if (a < DIM) hoff[a].assign(C, real(0));
            hu[a].assign(C, real(0));
            hs[a].assign(C, real(0));
        }
        // particles of each segment in key order
        std::vector<uint32_t> perm((size_t)npart_);
        {
            std::vector<long long> fill(nseg_, 0);
            std::vector<long long> first(nseg_ + 1, 0);
            for (int sg = 0; sg < nseg_; ++sg) first[sg + 1] = first[sg] + count[sg];
            for (long long q = 0; q < npart_; ++q) perm[first[segof[q]] + fill[segof[q]]++] = (uint32_t)q;
            for (int sg = 0; sg < nseg_; ++sg)
                std::sort(perm.begin() + first[sg], perm.begin() + first[sg + 1],
                          [&](uint32_t a, uint32_t b) { return key[a] < key[b]; });
            for (int sg = 0; sg < nseg_; ++sg) fill[sg] = 0;
            std::vector<long long> spbase(c.nspecies + 1, 0);
            for (int s = 0; s < c.nspecies; ++s) spbase[s + 1] = spbase[s] + count_sp_[s];
            for (int sg = 0; sg < nseg_; ++sg) {
                const int s = sg % c.nspecies;
                const double* P = st ? st->particles[s] : nullptr;
                for (long long m = first[sg]; m < first[sg + 1]; ++m) {
                    const long long q = perm[m];
                    const long long i = q - spbase[s];
                    const double* row = P + i * cols;
                    Placed pl;
                    place(row, pl);
                    const long long slot = h_start[sg] + fill[sg]++;
                    hcell[slot] = pack_cell<DIM>(pl.cell[0], pl.cell[1], pl.cell[2]);
                    for (int a = 0; a < DIM; ++a) hoff[a][slot] = (real)pl.off[a];
                    for (int a = 0; a < 3; ++a) {
                        hu[a][slot] = (real)row[cu + a];
                        hs[a][slot] = (real)row[cu + 3 + a];
                    }
                    hw[slot] = (real)row[cu + 6];
                    hid[slot] = (int32_t)i;
                }
            }
        }
        HIP_OR_FAIL(hipMemcpyAsync(p_.cell, hcell.data(), C * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
        HIP_OR_FAIL(hipMemcpyAsync(p_.id, hid.data(), C * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
        HIP_OR_FAIL(hipMemcpyAsync(p_.w, hw.data(), C * sizeof(real), hipMemcpyHostToDevice, stream_));
        for (int a = 0; a < 3; ++a) {
            if (a < DIM)
                HIP_OR_FAIL(hipMemcpyAsync(p_.off[a], hoff[a].data(), C * sizeof(real), hipMemcpyHostToDevice, stream_));
            HIP_OR_FAIL(hipMemcpyAsync(p_.u[a], hu[a].data(), C * sizeof(real), hipMemcpyHostToDevice, stream_));
            HIP_OR_FAIL(hipMemcpyAsync(p_.s[a], hs[a].data(), C * sizeof(real), hipMemcpyHostToDevice, stream_));
        }
        HIP_OR_FAIL(hipStreamSynchronize(stream_));
    }
    HIP_OR_FAIL(hipMemcpyAsync(seg_.start, h_start.data(), nseg_ * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
    HIP_OR_FAIL(hipMemcpyAsync(seg_.cap, h_cap.data(), nseg_ * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
    HIP_OR_FAIL(hipMemcpyAsync(seg_.count, h_count.data(), nseg_ * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
    HIP_OR_FAIL(hipMemsetAsync(ctr_, 0, CTR_NCTR * sizeof(int32_t), stream_));
    HIP_OR_FAIL(hipMemsetAsync(moved_, 0, sizeof(unsigned long long), stream_));

    // ---- fields
    {
        const size_t N = (size_t)g_.ncells;
        for (int comp = 0; comp < 6; ++comp) {
            freal* dst = comp < 3 ? f_.E[comp] : f_.B[comp - 3];
            if (st && st->fields) {
                const double* src = st->fields + comp * N;
                for (size_t i = 0; i < N; ++i)
                    if (!std::isfinite(src[i])) return fail(PIC_EINVAL, "field component %d: non-finite value", comp);
                HIP_OR_FAIL(hipMemcpyAsync(dst, src, N * sizeof(freal), hipMemcpyHostToDevice, stream_));
                HIP_OR_FAIL(hipStreamSynchronize(stream_));
            } else {
                HIP_OR_FAIL(hipMemsetAsync(dst, 0, N * sizeof(freal), stream_));
            }
        }
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 3; ++a) HIP_OR_FAIL(hipMemsetAsync(jbuf_[b][a], 0, N * sizeof(freal), stream_));
    }

    // ---- reference residual div E - rho at t = 0
    S = compute_rho();
    if (S.code) return S;
    Vec3d inv;
    for (int a = 0; a < 3; ++a) inv.v[a] = 1.0 / d_[a];
    HIP_OR_FAIL((launch_div_residual<freal, DIM>(g_, inv, f_, rho_, ref_, ref_, blockmax_, resid_blocks_, stream_)));
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    return Status{};
}

template <typename real, int DIM>
void Engine<real, DIM>::tstart(int k) {
    timer_start(timer_, stream_, k);
}

template <typename real, int DIM>
void Engine<real, DIM>::tstop(int k) {
    timer_stop(timer_, stream_, k);
}

template <typename real, int DIM>
Status Engine<real, DIM>::step(int nsteps) {
    for (int it = 0; it < nsteps; ++it) {
        if (rec_on_ && rec_n_ >= rec_cap_)
            return fail(PIC_ECAPACITY, "the polarization record is full (%d steps): read it with "
                        "pic_polarization_history", rec_cap_);
        if (nstep_ > 0 && nstep_ == check_at_) {
            HIP_OR_FAIL(hipStreamSynchronize(stream_));
            if (h_ctr_[CTR_NONFINITE])
                return fail(PIC_ENONFINITE, "a push produced a non-finite momentum or spin before step %lld",
                            (long long)nstep_);
            long long left = h_ctr_[CTR_STASH];
            if (repack_due(nstep_, left, npart_)) {
                Status S = repack();
                if (S.code) return S;
                left = 0;
            }
            check_at_ = next_check(nstep_, left, npart_);
        }
        const int slot = (int)(nstep_ & 1);
        // the step's slot of the Eq. 4 record, if one is kept
        RecArgs rec = rec_;
        rec.acc = rec_on_ ? rec_buf_ + (size_t)rec_n_ * kRecSlots * kRecStride : nullptr;
        // this step deposits into the zeroed buffer; the field update zeroes
        // the previous step's buffer behind it
        const int jnext = jcur_ ^ 1;
        for (int a = 0; a < 3; ++a) f_.J[a] = jbuf_[jnext][a];
        tstart(0);
        if (march_R_ > 1 && !rec_on_) {
            if (det_)
                HIP_OR_FAIL((launch_push_march<real, unsigned long long>(g_, k_, p_, seg_, lv_, ctr_, slot, f_, deposit_,
                                                                         march_R_, march_xcd_, stream_)));
            else if (use_acc64_)
                HIP_OR_FAIL((launch_push_march<real, double>(g_, k_, p_, seg_, lv_, ctr_, slot, f_, deposit_, march_R_,
                                                             march_xcd_, stream_)));
            else
                HIP_OR_FAIL((launch_push_march<real, real>(g_, k_, p_, seg_, lv_, ctr_, slot, f_, deposit_, march_R_,
                                                           march_xcd_, stream_)));
        } else if (det_) {
            HIP_OR_FAIL((launch_push_tiles<real, unsigned long long, DIM>(g_, k_, p_, seg_, lv_, ctr_, slot, f_, deposit_,
                                                                          rec, stream_)));
        } else if (use_acc64_) {
            HIP_OR_FAIL((launch_push_tiles<real, double, DIM>(g_, k_, p_, seg_, lv_, ctr_, slot, f_, deposit_, rec,
                                                              stream_)));
        } else {
            HIP_OR_FAIL((launch_push_tiles<real, real, DIM>(g_, k_, p_, seg_, lv_, ctr_, slot, f_, deposit_, rec,
                                                            stream_)));
        }
        tstop(0);
        tstart(1);
        HIP_OR_FAIL((launch_push_stash<real, DIM>(g_, k_, st_, ctr_, f_, deposit_, rec, kStashBlocks, stream_)));
        // the deterministic mode's fixed-point current becomes FP64 for the field update
        if (det_ && deposit_) HIP_OR_FAIL(launch_fixed_to_double(f_.J, g_.ncells, fx_inv_, stream_));
        tstop(1);
        tstart(2);
        HIP_OR_FAIL((launch_insert<real, DIM>(g_, p_, seg_, lv_, st_, ctr_, slot, moved_, 1024, stream_)));
        tstop(2);
        if (deposit_) {
            tstart(3);
            // one fused pass into the spare arrays (and, with open x faces,
            // the advanced Mur state into the spare state)
            Fields<freal> nf = f_;
            for (int a = 0; a < 3; ++a) {
                nf.E[a] = enext_[a];
                nf.B[a] = bnext_[a];
            }
            nf.mur = mur_next_;
            HIP_OR_FAIL((launch_yee_fused<freal, DIM>(g_, kf_, f_, nf, jbuf_[jcur_], stream_)));
            for (int a = 0; a < 3; ++a) {
                std::swap(f_.E[a], enext_[a]);
                std::swap(f_.B[a], bnext_[a]);
            }
            if (g_.open_x) std::swap(f_.mur, mur_next_);
            tstop(3);
        }
        // the overflow count for the next check (read only there: a copy
        // every step would cost a transfer and two launch gaps per step)
        if (nstep_ + 1 == check_at_)
            HIP_OR_FAIL(hipMemcpyAsync(h_ctr_ + CTR_STASH, ctr_ + CTR_STASH, 2 * sizeof(int32_t),
                                       hipMemcpyDeviceToHost, stream_));
        if (deposit_) jcur_ = jnext;
        for (int a = 0; a < 3; ++a) f_.J[a] = jbuf_[jcur_][a];
        ++nstep_;
        if (rec_on_) ++rec_n_;
        if (win_on_) {
            // the window has moved (n - n0) speed dt; shift once per whole
            // shift_cells cells of that (evaluated as written, in FP64)
            const int S = win_.shift_cells;
            while ((double)(nstep_ - win_step0_) * win_.speed * R_.cfg.dt >= (double)((shifts_ + 1) * S) * d_[0]) {
                Status Sx = window_shift();
                if (Sx.code) return Sx;
            }
        }
    }
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::repack() {
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    int32_t nst = 0;
    HIP_OR_FAIL(hipMemcpy(&nst, ctr_ + CTR_STASH, sizeof(int32_t), hipMemcpyDeviceToHost));
    h_ctr_[CTR_STASH] = nst;
    if (nst == 0) return Status{};
    const long long capmax = max_segment_slots([&](int mc) {
        return use_acc64_ ? tile_lds_bytes<real, double>(g_, mc) : tile_lds_bytes<real, real>(g_, mc);
    });
    std::vector<int32_t> cnt(nseg_), old_start(nseg_), old_cap(nseg_);
    HIP_OR_FAIL(hipMemcpy(cnt.data(), seg_.count, nseg_ * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_OR_FAIL(hipMemcpy(old_start.data(), seg_.start, nseg_ * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_OR_FAIL(hipMemcpy(old_cap.data(), seg_.cap, nseg_ * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int32_t> scell(nst), ssp(nst);
    HIP_OR_FAIL(hipMemcpy(scell.data(), st_.cell, nst * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_OR_FAIL(hipMemcpy(ssp.data(), st_.sp, nst * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<long long> want(cnt.begin(), cnt.end());
    for (int i = 0; i < nst; ++i) {
        if (scell[i] == kDeadCell) continue;   // left the box: dropped by the insertion below
        int c[3];
        unpack_cell<DIM>(scell[i], c[0], c[1], c[2]);
        const int tile = c[0] / g_.T[0] + g_.nt[0] * (c[1] / g_.T[1] + g_.nt[1] * (c[2] / g_.T[2]));
        want[tile * g_.nsp + ssp[i]]++;
    }
    std::vector<int32_t> nstart(nseg_), ncap(nseg_);
    long long total = 0;
    for (int s = 0; s < nseg_; ++s) {
        const long long cp = regrow_capacity(want[s], old_cap[s], R_.slack, capmax);
        nstart[s] = (int32_t)total;
        ncap[s] = (int32_t)cp;
        total += cp;
        if (total > kMaxSlots) return fail(PIC_ECAPACITY, "particle capacity exceeds 2^29 slots");
    }
    {
        long long maxcap = 0;
        for (int sg = 0; sg < nseg_; ++sg) maxcap = std::max<long long>(maxcap, ncap[sg]);
        const int saved = seg_.max_chunks;
        seg_.max_chunks = (int)((maxcap + 63) / 64);
        Status L = check_lds();
        seg_.max_chunks = saved;
        if (L.code) return L;
    }
    PArrays<real> np{};
    const long long slots = store_alloc_slots(total + kSpareSlots, store_slots_);
    Status S = alloc_store(np, slots, false);
    if (S.code) return S;
    int32_t* d_nstart = (int32_t*)dalloc(nseg_ * sizeof(int32_t));
    if (!d_nstart) return fail(PIC_ENOMEM, "repack allocation failed");
    HIP_OR_FAIL(hipMemcpyAsync(d_nstart, nstart.data(), nseg_ * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
    HIP_OR_FAIL((launch_repack_segments<real>(p_, np, seg_.start, d_nstart, seg_.count, nseg_, DIM, stream_)));
    HIP_OR_FAIL(hipMemcpyAsync(seg_.start, nstart.data(), nseg_ * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
    HIP_OR_FAIL(hipMemcpyAsync(seg_.cap, ncap.data(), nseg_ * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
    // move the overflow particles into their tiles: the insertion kernel run
    // over the overflow store, which now always finds room
    HIP_OR_FAIL((launch_insert<real, DIM>(g_, np, seg_, st_, st_, ctr_, CTR_STASH, moved_, 256, stream_)));
    HIP_OR_FAIL(hipMemsetAsync(ctr_ + CTR_STASH, 0, sizeof(int32_t), stream_));
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    free_store(p_);
    dfree(d_nstart);
    p_ = np;
    store_slots_ = slots;
    cap_total_ = total;
    seg_.dummy = (int)total;
    {
        long long maxcap = 0;
        for (int sg = 0; sg < nseg_; ++sg) maxcap = std::max<long long>(maxcap, ncap[sg]);
        seg_.max_chunks = (int)((maxcap + 63) / 64);
    }
    h_ctr_[CTR_STASH] = 0;
    repacks_++;
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::reduce(int mode, const ReduceArgs& ra, double* host_acc) {
    double h[kRedSlots * kRedStride];
    HIP_OR_FAIL(hipMemsetAsync(acc_, 0, sizeof h, stream_));
    HIP_OR_FAIL((launch_reduce_particles<real, DIM>(mode, g_, p_, seg_, st_, ctr_, ra, acc_, rho_, stream_)));
    HIP_OR_FAIL(hipMemcpyAsync(h, acc_, sizeof h, hipMemcpyDeviceToHost, stream_));
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    for (int q = 0; q < kRedStride; ++q) {
        host_acc[q] = 0.0;
        for (int s = 0; s < kRedSlots; ++s) host_acc[q] += h[s * kRedStride + q];
    }
    return Status{};
}

// The push kernels' non-finite flag, read now (waits for the stream).
template <typename real, int DIM>
Status Engine<real, DIM>::nonfinite_flag(bool* set) {
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    HIP_OR_FAIL(hipMemcpy(h_ctr_ + CTR_NONFINITE, ctr_ + CTR_NONFINITE, sizeof(int32_t), hipMemcpyDeviceToHost));
    *set = h_ctr_[CTR_NONFINITE] != 0;
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::compute_rho() {
    ReduceArgs ra{};
    ra.species = -1;
    for (int s = 0; s < kMaxSpecies; ++s) {
        ra.mu[s] = s < g_.nsp ? R_.cfg.sp[s].mu : 1.0;
        ra.Z[s] = s < g_.nsp ? R_.cfg.sp[s].Z : 0.0;
    }
    HIP_OR_FAIL(hipMemsetAsync(rho_, 0, g_.ncells * sizeof(double), stream_));
    HIP_OR_FAIL((launch_reduce_particles<real, DIM>(RED_RHO, g_, p_, seg_, st_, ctr_, ra, acc_, rho_, stream_)));
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::polarization(int species, double emin, double emax, double P[3], int64_t* N) {
    if (species < -1 || species >= g_.nsp) return fail(PIC_EINVAL, "species %d out of range", species);
    if (std::isnan(emin) || std::isnan(emax)) return fail(PIC_EINVAL, "energy window is NaN");
    ReduceArgs ra{};
    ra.species = species;
    ra.emin = emin;
    ra.emax = emax;
    for (int s = 0; s < kMaxSpecies; ++s) {
        ra.mu[s] = s < g_.nsp ? R_.cfg.sp[s].mu : 1.0;
        ra.Z[s] = s < g_.nsp ? R_.cfg.sp[s].Z : 0.0;
    }
    bool bad = false;
    Status S = nonfinite_flag(&bad);
    if (S.code) return S;
    if (bad) return fail(PIC_ENONFINITE, "a push produced a non-finite momentum or spin");
    if (det_) {
        // integer sums of the two 31-bit parts of every spin component
        unsigned long long acc[8];
        HIP_OR_FAIL(hipMemsetAsync(acc_, 0, 8 * sizeof(double), stream_));
        HIP_OR_FAIL((launch_polarization_fixed<real, DIM>(g_, p_, seg_, st_, ctr_, ra,
                                                          reinterpret_cast<unsigned long long*>(acc_), stream_)));
        HIP_OR_FAIL(hipMemcpyAsync(acc, acc_, 8 * sizeof(double), hipMemcpyDeviceToHost, stream_));
        HIP_OR_FAIL(hipStreamSynchronize(stream_));
        const long long n = (long long)acc[6];
        *N = n;
        for (int a = 0; a < 3; ++a) {
            const double sum = ((double)(long long)acc[a] + (double)(long long)acc[3 + a] * 0x1p-31) * 0x1p-31;
            P[a] = n > 0 ? sum / (double)n : 0.0;
        }
    } else {
        double acc[8];
        S = reduce(RED_POLARIZATION, ra, acc);
        if (S.code) return S;
        const double n = acc[3];
        *N = (int64_t)std::llround(n);
        for (int a = 0; a < 3; ++a) P[a] = n > 0 ? acc[a] / n : 0.0;
    }
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(P[a])) return fail(PIC_ENONFINITE, "polarization is not finite");
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::record(int species, double emin, double emax, int capacity) {
    if (species < -1 || species >= g_.nsp) return fail(PIC_EINVAL, "species %d out of range", species);
    if (std::isnan(emin) || std::isnan(emax)) return fail(PIC_EINVAL, "energy window is NaN");
    if (capacity < 0 || capacity > PIC_MAX_RECORD_STEPS)
        return fail(PIC_EINVAL, "capacity %d outside 0..%d", capacity, PIC_MAX_RECORD_STEPS);
    if (det_ && capacity > 0) return fail(PIC_EINVAL, "no per-step polarization record in the deterministic mode");
    // steps already enqueued may still add into the old record
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    dfree(rec_buf_);
    rec_buf_ = nullptr;
    rec_on_ = false;
    rec_cap_ = rec_n_ = 0;
    if (capacity == 0) return Status{};
    const long long nval = (long long)capacity * kRecSlots * kRecStride;
    rec_buf_ = (double*)dalloc((size_t)nval * sizeof(double));
    if (!rec_buf_) return fail(PIC_ENOMEM, "polarization record of %d steps: out of device memory", capacity);
    HIP_OR_FAIL(launch_fill_zero(rec_buf_, nval, stream_));
    rec_ = RecArgs{};
    rec_.species = species;
    rec_.window = !(emin == -HUGE_VAL && emax == HUGE_VAL);
    rec_.emin = emin;
    rec_.emax = emax;
    for (int s = 0; s < kMaxSpecies; ++s) rec_.mu[s] = s < g_.nsp ? R_.cfg.sp[s].mu : 1.0;
    rec_cap_ = capacity;
    rec_on_ = true;
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::record_read(double* P, int64_t* N, int cap, int* n_out) {
    *n_out = 0;
    if (!rec_on_ || rec_n_ == 0) return Status{};
    if (!P || !N) return fail(PIC_EINVAL, "output arrays must not be NULL");
    if (cap < rec_n_) return fail(PIC_EINVAL, "cap %d is less than the %d steps recorded", cap, rec_n_);
    bool bad = false;
    Status S = nonfinite_flag(&bad);
    if (S.code) return S;
    if (bad) return fail(PIC_ENONFINITE, "a push produced a non-finite momentum or spin");
    const long long nval = (long long)rec_n_ * kRecSlots * kRecStride;
    std::vector<double> h((size_t)nval);
    HIP_OR_FAIL(hipMemcpyAsync(h.data(), rec_buf_, nval * sizeof(double), hipMemcpyDeviceToHost, stream_));
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    for (int k = 0; k < rec_n_; ++k) {
        double sum[kRecStride] = {0.0, 0.0, 0.0, 0.0};
        for (int sl = 0; sl < kRecSlots; ++sl)
            for (int q = 0; q < kRecStride; ++q) sum[q] += h[((size_t)k * kRecSlots + sl) * kRecStride + q];
        const double n = sum[3];
        N[k] = (int64_t)std::llround(n);
        for (int a = 0; a < 3; ++a) {
            P[3 * k + a] = n > 0 ? sum[a] / n : 0.0;
            if (!std::isfinite(P[3 * k + a])) return fail(PIC_ENONFINITE, "recorded polarization is not finite");
        }
    }
    HIP_OR_FAIL(launch_fill_zero(rec_buf_, nval, stream_));
    *n_out = rec_n_;
    rec_n_ = 0;
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::spectrum_args(int species, double emin, double emax, int nbins, const double* count,
                                        const double* weight, const double* spin, BinArgs& ba) {
    if (species < -1 || species >= g_.nsp) return fail(PIC_EINVAL, "species %d out of range", species);
    if (nbins < 1 || nbins > PIC_MAX_SPECTRUM_BINS)
        return fail(PIC_EINVAL, "nbins = %d outside 1..%d", nbins, PIC_MAX_SPECTRUM_BINS);
    if (!std::isfinite(emin) || !std::isfinite(emax) || !(emin < emax))
        return fail(PIC_EINVAL, "energy range must be finite with emin < emax");
    if (!count || !weight || !spin) return fail(PIC_EINVAL, "output arrays must not be NULL");
    ba = BinArgs{};
    ba.mode = BIN_SPECTRUM;
    ba.species = species;
    ba.lo = emin;
    ba.hi = emax;
    ba.nbins = nbins;
    for (int sp = 0; sp < kMaxSpecies; ++sp) ba.mu[sp] = sp < g_.nsp ? R_.cfg.sp[sp].mu : 1.0;
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::spectrum(int species, double emin, double emax, int nbins, double* count,
                                   double* weight, double* spin) {
    BinArgs ba;
    Status A = spectrum_args(species, emin, emax, nbins, count, weight, spin, ba);
    if (A.code) return A;
    const size_t nh = (size_t)5 * nbins;
    double* d = (double*)dalloc(nh * sizeof(double));
    if (!d) return fail(PIC_ENOMEM, "spectrum buffer allocation failed");
    std::vector<double> h(nh);
    hipError_t e = hipMemsetAsync(d, 0, nh * sizeof(double), stream_);
    if (e == hipSuccess) e = launch_bin_particles<real, DIM>(g_, p_, seg_, st_, ctr_, ba, d, stream_);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, nh * sizeof(double), hipMemcpyDeviceToHost, stream_);
    if (e == hipSuccess) e = hipStreamSynchronize(stream_);
    dfree(d);
    if (e != hipSuccess) return fail(PIC_EHIP, "spectrum: %s", hipGetErrorString(e));
    for (int b = 0; b < nbins; ++b) {
        count[b] = h[b];
        weight[b] = h[nbins + b];
    }
    for (int q = 0; q < 3 * nbins; ++q) spin[q] = h[2 * (size_t)nbins + q];
    return Status{};
}

// The same bins summed in the library's static device buffer of this GPU
// (spec_buf_, 5 * PIC_MAX_SPECTRUM_BINS doubles) and copied straight into the
// caller's arrays: no device or host allocation.  The buffer is cleared by a
// kernel first; calls that overlap on one GPU would share it.
template <typename real, int DIM>
Status Engine<real, DIM>::spectrum_noalloc(int species, double emin, double emax, int nbins, double* count,
                                           double* weight, double* spin) {
    BinArgs ba;
    Status A = spectrum_args(species, emin, emax, nbins, count, weight, spin, ba);
    if (A.code) return A;
    if (!spec_buf_) return fail(PIC_ESTATE, "the static spectrum buffer of device %d was not found", dev_);
    const size_t nb = (size_t)nbins * sizeof(double);
    hipError_t e = launch_fill_zero(spec_buf_, 5LL * nbins, stream_);
    if (e == hipSuccess) e = launch_bin_particles<real, DIM>(g_, p_, seg_, st_, ctr_, ba, spec_buf_, stream_);
    if (e == hipSuccess) e = hipMemcpyAsync(count, spec_buf_, nb, hipMemcpyDeviceToHost, stream_);
    if (e == hipSuccess) e = hipMemcpyAsync(weight, spec_buf_ + nbins, nb, hipMemcpyDeviceToHost, stream_);
    if (e == hipSuccess) e = hipMemcpyAsync(spin, spec_buf_ + 2 * (size_t)nbins, 3 * nb, hipMemcpyDeviceToHost, stream_);
    if (e == hipSuccess) e = hipStreamSynchronize(stream_);
    if (e != hipSuccess) return fail(PIC_EHIP, "spectrum (static buffer): %s", hipGetErrorString(e));
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::phase_space(int species, int axis, double xmin, double xmax, int nx, int comp,
                                      double pmin, double pmax, int np, double* out) {
    if (species < 0 || species >= g_.nsp) return fail(PIC_EINVAL, "species %d out of range", species);
    if (axis < 0 || axis >= DIM) return fail(PIC_EINVAL, "axis %d outside 0..%d", axis, DIM - 1);
    if (comp < 0 || comp > 2) return fail(PIC_EINVAL, "momentum component %d outside 0..2", comp);
    if (nx < 1 || np < 1 || (long long)nx * np > (1LL << 26))
        return fail(PIC_EINVAL, "bins %d x %d: need >= 1 each and at most 2^26 in all", nx, np);
    if (!std::isfinite(xmin) || !std::isfinite(xmax) || !(xmin < xmax) || !std::isfinite(pmin) ||
        !std::isfinite(pmax) || !(pmin < pmax))
        return fail(PIC_EINVAL, "ranges must be finite with min < max");
    if (!out) return fail(PIC_EINVAL, "out must not be NULL");
    BinArgs ba{};
    ba.mode = BIN_PHASE;
    ba.species = species;
    ba.lo = xmin;
    ba.hi = xmax;
    ba.nbins = nx;
    ba.axis = axis;
    ba.comp = comp;
    ba.plo = pmin;
    ba.phi = pmax;
    ba.np = np;
    for (int a = 0; a < 3; ++a) ba.d[a] = d_[a];
    for (int sp = 0; sp < kMaxSpecies; ++sp) ba.mu[sp] = sp < g_.nsp ? R_.cfg.sp[sp].mu : 1.0;
    const size_t nh = (size_t)nx * np;
    double* d = (double*)dalloc(nh * sizeof(double));
    if (!d) return fail(PIC_ENOMEM, "phase-space buffer allocation failed");
    hipError_t e = hipMemsetAsync(d, 0, nh * sizeof(double), stream_);
    if (e == hipSuccess) e = launch_bin_particles<real, DIM>(g_, p_, seg_, st_, ctr_, ba, d, stream_);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d, nh * sizeof(double), hipMemcpyDeviceToHost, stream_);
    if (e == hipSuccess) e = hipStreamSynchronize(stream_);
    dfree(d);
    if (e != hipSuccess) return fail(PIC_EHIP, "phase space: %s", hipGetErrorString(e));
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::density(int species, double* out, size_t cap) {
    if (species < 0 || species >= g_.nsp) return fail(PIC_EINVAL, "species %d out of range", species);
    if (!out) return fail(PIC_EINVAL, "out must not be NULL");
    if (cap < (size_t)g_.ncells) return fail(PIC_EINVAL, "cap too small: need %lld doubles", g_.ncells);
    ReduceArgs ra{};
    ra.species = species;
    for (int sp = 0; sp < kMaxSpecies; ++sp) {
        ra.mu[sp] = sp < g_.nsp ? R_.cfg.sp[sp].mu : 1.0;
        ra.Z[sp] = sp == species ? 1.0 : 0.0;
    }
    double* d = (double*)dalloc((size_t)g_.ncells * sizeof(double));
    if (!d) return fail(PIC_ENOMEM, "density buffer allocation failed");
    hipError_t e = hipMemsetAsync(d, 0, (size_t)g_.ncells * sizeof(double), stream_);
    if (e == hipSuccess)
        e = launch_reduce_particles<real, DIM>(RED_RHO, g_, p_, seg_, st_, ctr_, ra, acc_, d, stream_);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d, (size_t)g_.ncells * sizeof(double), hipMemcpyDeviceToHost, stream_);
    if (e == hipSuccess) e = hipStreamSynchronize(stream_);
    dfree(d);
    if (e != hipSuccess) return fail(PIC_EHIP, "density: %s", hipGetErrorString(e));
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::fields(uint32_t mask, double* out, size_t cap) {
    if (mask & ~0x3FFu) return fail(PIC_EINVAL, "unknown field mask bits 0x%x", mask);
    const size_t N = (size_t)g_.ncells;
    int nc = 0;
    for (int b = 0; b < 10; ++b) nc += (mask >> b) & 1;
    if (!out && nc) return fail(PIC_EINVAL, "host_out is NULL");
    if (cap < (size_t)nc * N) return fail(PIC_EINVAL, "cap %zu < %zu", cap, (size_t)nc * N);
    if (mask & PIC_RHO) {
        Status S = compute_rho();
        if (S.code) return S;
    }
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    size_t o = 0;
    for (int b = 0; b < 10; ++b) {
        if (!((mask >> b) & 1)) continue;
        const freal* src = b == 9 ? rho_ : (b < 3 ? f_.E[b] : (b < 6 ? f_.B[b - 3] : f_.J[b - 6]));
        HIP_OR_FAIL(hipMemcpy(out + o, src, N * sizeof(freal), hipMemcpyDeviceToHost));
        o += N;
    }
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::particles(int species, double* out, size_t cap, int64_t* n_out, bool cells) {
    if (species < 0 || species >= g_.nsp) return fail(PIC_EINVAL, "species %d out of range", species);
    long long per[kMaxSpecies];
    Status L = live_counts(per);
    if (L.code) return L;
    const long long n = per[species];
    if (n_out) *n_out = n;
    // rows: id, position (x y z, or cell index and offset per axis), u, s, w
    const int ncol = cells ? PIC_PARTICLE_CELL_OUT_COLS : PIC_PARTICLE_OUT_COLS;
    const int cu = cells ? 7 : 4;
    if (cap < (size_t)n * ncol) return fail(PIC_EINVAL, "cap too small for %lld particles", n);
    if (n > 0 && !out) return fail(PIC_EINVAL, "host_out is NULL");
    // Without a moving window the ids are 0 .. n-1 and row i is particle i;
    // with one, the rows are gathered first and sorted by id.
    const bool by_index = !win_on_;
    std::vector<double> rows;
    std::vector<long long> ids;
    if (!by_index) {
        rows.resize((size_t)n * ncol);
        ids.reserve((size_t)n);
    }
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    std::vector<int32_t> start(nseg_), count(nseg_);
    HIP_OR_FAIL(hipMemcpy(start.data(), seg_.start, nseg_ * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_OR_FAIL(hipMemcpy(count.data(), seg_.count, nseg_ * sizeof(int32_t), hipMemcpyDeviceToHost));
    int32_t nst = 0;
    HIP_OR_FAIL(hipMemcpy(&nst, ctr_ + CTR_STASH, sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<char> seen((size_t)n, 0);
    // read one store into host vectors and emit the rows of this species
    auto emit = [&](const PArrays<real>& A, long long len, const std::vector<std::pair<long long, long long>>& ranges,
                    bool stash) -> Status {
        if (len == 0) return Status{};
        std::vector<int32_t> cell(len), id(len), sp;
        std::vector<real> off[3], u[3], s[3], w(len);
        HIP_OR_FAIL(hipMemcpy(cell.data(), A.cell, len * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIP_OR_FAIL(hipMemcpy(id.data(), A.id, len * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIP_OR_FAIL(hipMemcpy(w.data(), A.w, len * sizeof(real), hipMemcpyDeviceToHost));
        if (stash) {
            sp.resize(len);
            HIP_OR_FAIL(hipMemcpy(sp.data(), A.sp, len * sizeof(int32_t), hipMemcpyDeviceToHost));
        }
        for (int a = 0; a < 3; ++a) {
            if (a < DIM) {
                off[a].resize(len);
                HIP_OR_FAIL(hipMemcpy(off[a].data(), A.off[a], len * sizeof(real), hipMemcpyDeviceToHost));
            }
            u[a].resize(len);
            s[a].resize(len);
            HIP_OR_FAIL(hipMemcpy(u[a].data(), A.u[a], len * sizeof(real), hipMemcpyDeviceToHost));
            HIP_OR_FAIL(hipMemcpy(s[a].data(), A.s[a], len * sizeof(real), hipMemcpyDeviceToHost));
        }
        for (const auto& r : ranges)
            for (long long q = r.first; q < r.second; ++q) {
                if (stash && (sp[q] != species || cell[q] == kDeadCell)) continue;
                const long long i = id[q];
                double* row;
                if (by_index) {
                    if (i < 0 || i >= n || seen[i]) return fail(PIC_ESTATE, "particle bookkeeping is corrupt (id %lld)", i);
                    seen[i] = 1;
                    row = out + i * ncol;
                } else {
                    if ((long long)ids.size() >= n) return fail(PIC_ESTATE, "particle bookkeeping is corrupt (count)");
                    row = rows.data() + ids.size() * ncol;
                    ids.push_back(i);
                }
                int c[3];
                unpack_cell<DIM>(cell[q], c[0], c[1], c[2]);
                row[0] = (double)i;
                if (cells) {
                    for (int a = 0; a < 3; ++a) {
                        row[1 + a] = a < DIM ? (double)c[a] : 0.0;
                        row[4 + a] = a < DIM ? (double)off[a][q] : 0.0;
                    }
                } else {
                    for (int a = 0; a < 3; ++a) row[1 + a] = a < DIM ? ((double)c[a] + (double)off[a][q]) * d_[a] : 0.0;
                }
                for (int a = 0; a < 3; ++a) {
                    row[cu + a] = (double)u[a][q];
                    row[cu + 3 + a] = (double)s[a][q];
                }
                row[cu + 6] = (double)w[q];
            }
        return Status{};
    };
    std::vector<std::pair<long long, long long>> ranges;
    for (int t = 0; t < g_.ntiles; ++t) {
        const int sid = t * g_.nsp + species;
        ranges.push_back({start[sid], (long long)start[sid] + count[sid]});
    }
    Status S = emit(p_, cap_total_, ranges, false);
    if (S.code) return S;
    S = emit(st_, nst, {{0, (long long)nst}}, true);
    if (S.code) return S;
    if (by_index) {
        for (long long i = 0; i < n; ++i)
            if (!seen[i]) return fail(PIC_ESTATE, "particle %lld of species %d is missing", i, species);
        return Status{};
    }
    if ((long long)ids.size() != n) return fail(PIC_ESTATE, "particle bookkeeping is corrupt (count)");
    std::vector<long long> order((size_t)n);
    for (long long q = 0; q < n; ++q) order[q] = q;
    std::sort(order.begin(), order.end(), [&](long long a, long long b) { return ids[a] < ids[b]; });
    for (long long q = 0; q < n; ++q) {
        if (q > 0 && ids[order[q]] == ids[order[q - 1]])
            return fail(PIC_ESTATE, "particle id %lld appears twice", ids[order[q]]);
        std::memcpy(out + q * ncol, rows.data() + order[q] * ncol, ncol * sizeof(double));
    }
    return Status{};
}

// Test hook: a NaN into u_x of the first particle of the first tile that
// holds one of this species.
template <typename real, int DIM>
Status Engine<real, DIM>::poison(int species) {
    if (species < 0 || species >= g_.nsp) return fail(PIC_EINVAL, "species %d out of range", species);
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    std::vector<int32_t> start(nseg_), count(nseg_);
    HIP_OR_FAIL(hipMemcpy(start.data(), seg_.start, nseg_ * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_OR_FAIL(hipMemcpy(count.data(), seg_.count, nseg_ * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int t = 0; t < g_.ntiles; ++t) {
        const int sid = t * g_.nsp + species;
        if (count[sid] > 0) {
            const real nan = std::numeric_limits<real>::quiet_NaN();
            HIP_OR_FAIL(hipMemcpy(p_.u[0] + start[sid], &nan, sizeof(real), hipMemcpyHostToDevice));
            return Status{};
        }
    }
    return fail(PIC_EINVAL, "species %d has no particle in a tile", species);
}

template <typename real, int DIM>
Status Engine<real, DIM>::residual_max(double* out) {
    Status S = compute_rho();
    if (S.code) return S;
    Vec3d inv;
    for (int a = 0; a < 3; ++a) inv.v[a] = 1.0 / d_[a];
    HIP_OR_FAIL((launch_div_residual<freal, DIM>(g_, inv, f_, rho_, ref_, nullptr, blockmax_, resid_blocks_, stream_)));
    std::vector<double> h(resid_blocks_);
    HIP_OR_FAIL(hipMemcpyAsync(h.data(), blockmax_, resid_blocks_ * sizeof(double), hipMemcpyDeviceToHost, stream_));
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    double m = 0.0;
    for (double v : h) m = std::max(m, v);
    *out = m;
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::energy(double* out, int cap) {
    if (!out || cap < g_.nsp + 2) return fail(PIC_EINVAL, "energy needs cap >= %d", g_.nsp + 2);
    double V = 1.0;
    for (int a = 0; a < DIM; ++a) V *= d_[a];
    ReduceArgs ra{};
    ra.species = -1;
    for (int s = 0; s < kMaxSpecies; ++s) {
        ra.mu[s] = s < g_.nsp ? R_.cfg.sp[s].mu : 1.0;
        ra.Z[s] = s < g_.nsp ? R_.cfg.sp[s].Z : 0.0;
    }
    double acc[8];
    Status S = reduce(RED_KINETIC, ra, acc);
    if (S.code) return S;
    for (int s = 0; s < g_.nsp; ++s) out[s] = acc[s] * V;
    HIP_OR_FAIL(hipMemsetAsync(acc_, 0, 8 * sizeof(double), stream_));
    HIP_OR_FAIL((launch_field_energy<freal>(g_, f_, acc_, stream_)));
    HIP_OR_FAIL(hipMemcpyAsync(acc, acc_, sizeof(double), hipMemcpyDeviceToHost, stream_));
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    out[g_.nsp] = acc[0] * V;
    S = residual_max(&out[g_.nsp + 1]);
    if (S.code) return S;
    for (int i = 0; i < g_.nsp + 2; ++i)
        if (!std::isfinite(out[i])) return fail(PIC_ENONFINITE, "energy diagnostic %d is not finite", i);
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::stats(int64_t* out, int cap) {
    if (!out || cap < 5) return fail(PIC_EINVAL, "stats needs cap >= 5");
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    unsigned long long moved = 0;
    int32_t nst = 0;
    HIP_OR_FAIL(hipMemcpy(&moved, moved_, sizeof moved, hipMemcpyDeviceToHost));
    HIP_OR_FAIL(hipMemcpy(&nst, ctr_ + CTR_STASH, sizeof nst, hipMemcpyDeviceToHost));
    long long per[kMaxSpecies];
    Status S = live_counts(per);
    if (S.code) return S;
    long long total = 0;
    for (int s = 0; s < g_.nsp; ++s) total += per[s];
    out[0] = nstep_;
    out[1] = (int64_t)moved;
    out[2] = nst;
    out[3] = repacks_;
    out[4] = total;
    for (int a = 0; a < 3 && 5 + a < cap; ++a) out[5 + a] = g_.T[a];
    for (int s = 0; s < kMaxSpecies && 8 + s < cap; ++s) out[8 + s] = per[s];
    if (cap > 12) out[12] = shifts_;
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::live_counts(long long out[kMaxSpecies]) {
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    for (int s = 0; s < kMaxSpecies; ++s) out[s] = 0;
    std::vector<int32_t> cnt(nseg_);
    HIP_OR_FAIL(hipMemcpy(cnt.data(), seg_.count, nseg_ * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int sg = 0; sg < nseg_; ++sg) out[sg % g_.nsp] += cnt[sg];
    int32_t nst = 0;
    HIP_OR_FAIL(hipMemcpy(&nst, ctr_ + CTR_STASH, sizeof nst, hipMemcpyDeviceToHost));
    if (nst > 0) {
        std::vector<int32_t> cell(nst), sp(nst);
        HIP_OR_FAIL(hipMemcpy(cell.data(), st_.cell, nst * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIP_OR_FAIL(hipMemcpy(sp.data(), st_.sp, nst * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int i = 0; i < nst; ++i)
            if (cell[i] != kDeadCell) out[sp[i]]++;
    }
    return Status{};
}

// Entries of the segments and of the overflow store, dead overflow entries
// included.  Until the next repack the overflow store can gain at most one
// entry per particle now in a segment and per particle injected later, so
// this number plus the later injections bounds the size of both stores.
template <typename real, int DIM>
Status Engine<real, DIM>::stored_count(long long* n) {
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    std::vector<int32_t> cnt(nseg_);
    HIP_OR_FAIL(hipMemcpy(cnt.data(), seg_.count, nseg_ * sizeof(int32_t), hipMemcpyDeviceToHost));
    int32_t nst = 0;
    HIP_OR_FAIL(hipMemcpy(&nst, ctr_ + CTR_STASH, sizeof nst, hipMemcpyDeviceToHost));
    *n = nst;
    for (int sg = 0; sg < nseg_; ++sg) *n += cnt[sg];
    return Status{};
}

// The leaver and overflow stores must hold every particle of the box (all
// may leave their tile in one step); injection can raise that number.  Both
// are empty between steps, so they are replaced without copying.
template <typename real, int DIM>
Status Engine<real, DIM>::grow_stores(long long need) {
    if (need <= store_cap_) return Status{};
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    int32_t nst = 0;
    HIP_OR_FAIL(hipMemcpy(&nst, ctr_ + CTR_STASH, sizeof nst, hipMemcpyDeviceToHost));
    if (nst != 0) return fail(PIC_ESTATE, "overflow store not empty when growing it");
    const long long cap = need + need / 4;
    free_store(lv_);
    free_store(st_);
    Status S = alloc_store(lv_, cap, true);
    if (S.code) return S;
    S = alloc_store(st_, cap, true);
    if (S.code) return S;
    store_cap_ = cap;
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::window(const pic_window_config* w) {
    if (!w) return fail(PIC_EINVAL, "window config is NULL");
    if (det_) return fail(PIC_EINVAL, "the moving window is not available in the deterministic mode");
    if (!(w->speed >= 0.0) || !std::isfinite(w->speed)) return fail(PIC_EINVAL, "window speed must be >= 0");
    if (w->shift_cells < 1 || w->shift_cells >= g_.n[0] || w->shift_cells % g_.T[0] != 0)
        return fail(PIC_EINVAL, "shift_cells = %d must be a multiple of the tile's x edge %d and below n[0] = %d",
                    w->shift_cells, g_.T[0], g_.n[0]);
    if (w->ppc < 0 || w->ppc > 256) return fail(PIC_EINVAL, "ppc = %d outside 0 .. 256", w->ppc);
    if (!(w->n0 >= 0.0) || !std::isfinite(w->n0) || !(w->ramp_len >= 0.0) || !std::isfinite(w->ramp_len) ||
        !std::isfinite(w->ramp_start))
        return fail(PIC_EINVAL, "n0 and ramp_len must be finite and >= 0, ramp_start finite");
    if (w->ppc > 0) {
        const double s2 = w->s0[0] * w->s0[0] + w->s0[1] * w->s0[1] + w->s0[2] * w->s0[2];
        if (!(std::fabs(s2 - 1.0) <= 1e-6)) return fail(PIC_EINVAL, "|s0| must be 1");
    }
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    if (!scratch_) {
        scratch_ = (freal*)dalloc(g_.ncells * sizeof(freal));
        f_.mur = (freal*)dalloc((size_t)MUR_COLUMNS * g_.n[1] * g_.n[2] * sizeof(freal));
        mur_next_ = (freal*)dalloc((size_t)MUR_COLUMNS * g_.n[1] * g_.n[2] * sizeof(freal));
        seg_tmp_.start = (int32_t*)dalloc((size_t)nseg_ * sizeof(int32_t));
        seg_tmp_.cap = (int32_t*)dalloc((size_t)nseg_ * sizeof(int32_t));
        seg_tmp_.count = (int32_t*)dalloc((size_t)nseg_ * sizeof(int32_t));
        if (!scratch_ || !f_.mur || !mur_next_ || !seg_tmp_.start || !seg_tmp_.cap || !seg_tmp_.count)
            return fail(PIC_ENOMEM, "device allocation failed");
    }
    {
        Status L = stored_count(&npart_bound_);
        if (L.code) return L;
    }
    win_ = *w;
    win_on_ = true;
    win_step0_ = nstep_;
    shifts_ = 0;
    g_.open_x = 1;
    HIP_OR_FAIL((launch_mur_reset<freal, DIM>(g_, f_, stream_)));
    // div E - rho reference with the open faces
    Status S = compute_rho();
    if (S.code) return S;
    Vec3d inv;
    for (int a = 0; a < 3; ++a) inv.v[a] = 1.0 / d_[a];
    HIP_OR_FAIL((launch_div_residual<freal, DIM>(g_, inv, f_, rho_, ref_, ref_, blockmax_, resid_blocks_, stream_)));
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    return Status{};
}

// One shift of the moving window by S = shift_cells cells (a whole number k
// of tile columns): every field array moves S cells towards -x, the segment
// table rotates by k tile columns (the first k columns' segments, whose
// particles leave the box, become the last k columns' with count 0), the
// kept particles and the overflow store's move S cells down in x, and cold
// plasma is injected into the last S columns.  All of it is queued on the
// stream without a wait, unless the particle stores have to grow.
template <typename real, int DIM>
Status Engine<real, DIM>::window_shift() {
    const int S = win_.shift_cells;
    const int k = S / g_.T[0];
    const int nz = DIM == 3 ? g_.n[2] : 1;
    const long long per_sp = (long long)nz * g_.n[1] * S * win_.ppc;
    // The leaver and overflow stores must not run out: npart_bound_ (the
    // stored entries at the last count plus the particles injected since)
    // bounds what they can receive.  It counts no removals; it is recounted
    // (a wait and a read of the counts) only when the stores would otherwise
    // have to grow, and growing them needs an empty overflow store.
    if (win_.ppc > 0 && npart_bound_ + per_sp * g_.nsp > store_cap_) {
        Status St = stored_count(&npart_bound_);
        if (St.code) return St;
        if (npart_bound_ + per_sp * g_.nsp > store_cap_) {
            St = repack();
            if (St.code) return St;
            St = stored_count(&npart_bound_);
            if (St.code) return St;
            St = grow_stores(npart_bound_ + per_sp * g_.nsp);
            if (St.code) return St;
        }
    }
    // fields and the last step's current
    freal** arrs[9] = {&f_.E[0], &f_.E[1], &f_.E[2], &f_.B[0], &f_.B[1], &f_.B[2],
                       &jbuf_[jcur_][0], &jbuf_[jcur_][1], &jbuf_[jcur_][2]};
    for (freal** a : arrs) {
        HIP_OR_FAIL((launch_shift_x<freal>(g_, *a, scratch_, S, stream_)));
        std::swap(*a, scratch_);
    }
    for (int a = 0; a < 3; ++a) f_.J[a] = jbuf_[jcur_][a];
    HIP_OR_FAIL((launch_mur_reset<freal, DIM>(g_, f_, stream_)));
    // segment table
    HIP_OR_FAIL(launch_rotate_segments(g_, seg_, seg_tmp_, k, stream_));
    std::swap(seg_.start, seg_tmp_.start);
    std::swap(seg_.cap, seg_tmp_.cap);
    std::swap(seg_.count, seg_tmp_.count);
    HIP_OR_FAIL((launch_shift_cells<real, DIM>(p_, seg_, S, nseg_, stream_)));
    HIP_OR_FAIL((launch_shift_stash<real, DIM>(st_, ctr_, S, stream_)));
    shifts_++;
    if (win_.ppc > 0) {
        npart_bound_ += per_sp * g_.nsp;
        InjectArgs a{};
        a.S = S;
        a.ppc = win_.ppc;
        a.origin = shifts_ * S;
        a.dx = d_[0];
        a.n0 = win_.n0;
        a.ramp_start = win_.ramp_start;
        a.ramp_len = win_.ramp_len;
        for (int c = 0; c < 3; ++c) a.s0[c] = win_.s0[c];
        for (int sp = 0; sp < g_.nsp; ++sp) {
            if (next_id_[sp] + per_sp > (1LL << 31) - 1)
                return fail(PIC_ECAPACITY, "particle ids of species %d would pass 2^31", sp);
            a.next_id[sp] = (int32_t)next_id_[sp];
            next_id_[sp] += per_sp;
        }
        HIP_OR_FAIL((launch_inject<real, DIM>(g_, p_, seg_, st_, ctr_, a, stream_)));
    }
    HIP_OR_FAIL(hipMemcpyAsync(h_ctr_ + CTR_STASH, ctr_ + CTR_STASH, sizeof(int32_t), hipMemcpyDeviceToHost, stream_));
    npart_ = npart_bound_;   // for the repack threshold
    return Status{};
}

template <typename real, int DIM>
Status Engine<real, DIM>::timing(int enable) {
    return timer_enable(timer_, stream_, enable);
}

template <typename real, int DIM>
Status Engine<real, DIM>::timing_read(double* ms, int64_t* launches, int cap) {
    return timer_read(timer_, stream_, ms, launches, cap);
}

// ---------------------------------------------------------------- batches

// Independent 2D runs of uneven size in shared stores: one segment list, one
// particle store and concatenated field arrays, each run at its own offsets.
// A step is one persistent push over all runs' tiles (largest first), one
// overflow push, one leaver insertion and one fused Yee pass over all runs
// at once.
class BatchBase {
public:
    virtual ~BatchBase() {}
    virtual Status step(int n) = 0;
    virtual Status polarization(int run, int species, double emin, double emax, double P[3], int64_t* N) = 0;
    virtual Status fields(int run, uint32_t mask, double* out, size_t cap) = 0;
    virtual Status particles(int run, int species, double* out, size_t cap, int64_t* n) = 0;
    virtual Status stats(int64_t* out, int cap) = 0;
    virtual Status run_time(bool enable, double* ns_out) = 0;
    virtual Status timing(int enable) = 0;
    virtual Status timing_read(double* ms, int64_t* launches, int cap) = 0;
    virtual void run_info(int r, int64_t* out) const = 0;   // tile x, tile y, particles, cells
    virtual int nruns() const = 0;
};

template <typename real>
class BatchEngine : public BatchBase {
public:
    BatchEngine(const pic_allocator* alloc, hipStream_t stream) : stream_(stream) {
        if (alloc && alloc->alloc && alloc->free) {
            alloc_ = *alloc;
            has_alloc_ = true;
        }
    }
    ~BatchEngine() { release(); }

    struct Run {
        Resolved R;
        Geom g;
        double d[3];
        long long cell_off = 0;
        int sid_base = 0, tile_base = 0, yee_blk_base = 0;
        long long count_sp[kMaxSpecies] = {0, 0, 0, 0};
        long long npart = 0;
    };

    Status init(const std::vector<Resolved>& Rs, const pic_state* st);
    Status step(int nsteps) override;
    Status polarization(int run, int species, double emin, double emax, double P[3], int64_t* N) override;
    Status fields(int run, uint32_t mask, double* out, size_t cap) override;
    Status particles(int run, int species, double* out, size_t cap, int64_t* n) override;
    Status stats(int64_t* out, int cap) override;
    Status run_time(bool enable, double* ns_out) override;   // per-run push time while enabled
    Status timing(int enable) override { return timer_enable(timer_, stream_, enable); }
    Status timing_read(double* ms, int64_t* launches, int cap) override {
        return timer_read(timer_, stream_, ms, launches, cap);
    }
    void run_info(int r, int64_t* out) const override {
        out[0] = runs_[r].g.T[0];
        out[1] = runs_[r].g.T[1];
        out[2] = runs_[r].npart;
        out[3] = runs_[r].g.ncells;
    }
    int nruns() const override { return (int)runs_.size(); }
    void release();

private:
    void* dalloc(size_t bytes) {
        if (bytes == 0) bytes = 256;
        void* p = nullptr;
        if (has_alloc_) p = alloc_.alloc(alloc_.user, bytes);
        else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
        if (p) live_.push_back(p);
        return p;
    }
    void dfree(void* p) {
        if (!p) return;
        auto it = std::find(live_.begin(), live_.end(), p);
        if (it != live_.end()) live_.erase(it);
        if (has_alloc_) alloc_.free(alloc_.user, p);
        else (void)hipFree(p);
    }
    Status alloc_store(PArrays<real>& a, long long cap, bool with_species);
    void free_store(PArrays<real>& a);
    Status repack();
    Status upload_descs();
    size_t push_lds() const {
        size_t lds = 0;
        for (const Run& r : runs_) {
            const size_t l = use_acc64_ ? tile_lds_bytes<real, double>(r.g, seg_.max_chunks)
                                        : tile_lds_bytes<real, real>(r.g, seg_.max_chunks);
            lds = std::max(lds, l);
        }
        return lds;
    }

    pic_allocator alloc_{};
    bool has_alloc_ = false;
    hipStream_t stream_;
    std::vector<void*> live_;
    std::vector<Run> runs_;
    int nsp_ = 0, nseg_ = 0, ntiles_ = 0;
    int use_acc64_ = 1, deposit_ = 1;
    long long cap_total_ = 0, npart_ = 0, ncells_ = 0;
    long long store_slots_ = 0;   // slots allocated in p_ (at least cap_total_ + kSpareSlots)
    int64_t nstep_ = 0, repacks_ = 0;
    int64_t check_at_ = kStashCheck;   // step of the next overflow check
    int push_blocks_ = 1;
    PArrays<real> p_{}, lv_{}, st_{};
    Segs seg_{};
    Fields<freal> f_{};
    freal* jbuf_[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    int jcur_ = 0;
    int32_t* ctr_ = nullptr;
    int32_t* h_ctr_ = nullptr;
    unsigned long long* moved_ = nullptr;
    unsigned long long* run_ns_ = nullptr;
    bool time_runs_ = false;
    double* acc_ = nullptr;
    RunDesc<real>* d_runs_ = nullptr;
    TileRef* d_order_ = nullptr;
    XcdQueues xq_{};
    int32_t* d_blk_run_ = nullptr;   // field-update block -> run
    int yee_nblk_ = 0;
    // the fused Yee step writes the new E and B here (pointers then swapped)
    freal* enext_[3] = {nullptr, nullptr, nullptr};
    freal* bnext_[3] = {nullptr, nullptr, nullptr};
    std::vector<TileRef> order_;
    Timer timer_;
};

template <typename real>
Status BatchEngine<real>::alloc_store(PArrays<real>& a, long long cap, bool with_species) {
    a = PArrays<real>{};
    const size_t n = (size_t)std::max(cap, 1LL);
    a.cell = (int32_t*)dalloc(n * sizeof(int32_t));
    for (int d = 0; d < 2; ++d) a.off[d] = (real*)dalloc(n * sizeof(real));
    for (int d = 0; d < 3; ++d) {
        a.u[d] = (real*)dalloc(n * sizeof(real));
        a.s[d] = (real*)dalloc(n * sizeof(real));
    }
    a.w = (real*)dalloc(n * sizeof(real));
    a.id = (int32_t*)dalloc(n * sizeof(int32_t));
    if (with_species) a.sp = (int32_t*)dalloc(n * sizeof(int32_t));
    bool ok = a.cell && a.w && a.id && a.off[0] && a.off[1] && (!with_species || a.sp);
    for (int d = 0; d < 3; ++d) ok = ok && a.u[d] && a.s[d];
    if (!ok) return fail(PIC_ENOMEM, "device allocation of a particle store (%lld slots) failed", cap);
    return Status{};
}

template <typename real>
void BatchEngine<real>::free_store(PArrays<real>& a) {
    dfree(a.cell);
    for (int d = 0; d < 3; ++d) {
        dfree(a.off[d]);
        dfree(a.u[d]);
        dfree(a.s[d]);
    }
    dfree(a.w);
    dfree(a.id);
    dfree(a.sp);
    a = PArrays<real>{};
}

template <typename real>
void BatchEngine<real>::release() {
    if (stream_ != nullptr || !live_.empty()) (void)hipStreamSynchronize(stream_);
    timer_free(timer_);
    std::vector<void*> all = live_;
    for (void* p : all) dfree(p);
    live_.clear();
    if (h_ctr_) (void)hipHostFree(h_ctr_);
    h_ctr_ = nullptr;
}

template <typename real>
Status BatchEngine<real>::upload_descs() {
    std::vector<RunDesc<real>> d(runs_.size());
    for (size_t r = 0; r < runs_.size(); ++r) {
        const Run& R = runs_[r];
        const pic_config& c = R.R.cfg;
        RunDesc<real>& D = d[r];
        D = RunDesc<real>{};
        D.g = R.g;
        D.k.dt = (real)c.dt;
        D.kf.dt = c.dt;
        for (int a = 0; a < 3; ++a) {
            D.k.dt_d[a] = (real)(c.dt / R.d[a]);
            D.k.dt_d_lo[a] = (real)(c.dt / R.d[a] - (double)D.k.dt_d[a]);
            D.k.d_dt[a] = (real)(R.d[a] / c.dt);
            D.kf.cb[a] = 0.5 * c.dt / R.d[a];
            D.kf.ce[a] = c.dt / R.d[a];
        }
        for (int s = 0; s < kMaxSpecies; ++s) {
            const bool on = s < c.nspecies;
            const double rr = on ? c.sp[s].Z / c.sp[s].mu : 0.0;
            D.k.r[s] = (real)rr;
            D.k.eps[s] = (real)(0.5 * rr * c.dt);
            D.k.a[s] = on ? (real)c.sp[s].a : real(0);
            D.k.Z[s] = on ? (real)c.sp[s].Z : real(0);
        }
        D.cell_off = R.cell_off;
        D.sid_base = R.sid_base;
        D.tile_base = R.tile_base;
        D.yee_blk_base = R.yee_blk_base;
    }
    HIP_OR_FAIL(hipMemcpyAsync(d_runs_, d.data(), d.size() * sizeof(RunDesc<real>), hipMemcpyHostToDevice, stream_));
    return Status{};
}

template <typename real>
Status BatchEngine<real>::init(const std::vector<Resolved>& Rs, const pic_state* st) {
    const int nrun = (int)Rs.size();
    runs_.resize(nrun);
    nsp_ = Rs[0].cfg.nspecies;
    use_acc64_ = Rs[0].use_acc64;
    deposit_ = (Rs[0].cfg.flags & PIC_FLAG_TEST_PARTICLE) ? 0 : 1;
    // ---- layout: tiles, segments and cells of every run, one after another
    long long cells = 0;
    int sids = 0, tiles = 0;
    npart_ = 0;
    for (int r = 0; r < nrun; ++r) {
        Run& R = runs_[r];
        R.R = Rs[r];
        const pic_config& c = R.R.cfg;
        R.g = Geom{};
        R.g.ndim = 2;
        R.g.nsp = nsp_;
        for (int a = 0; a < 3; ++a) {
            R.g.n[a] = R.R.n[a];
            R.g.T[a] = R.R.T[a];
            R.g.nt[a] = R.R.nt[a];
            R.d[a] = a < 2 ? c.d[a] : 1.0;
        }
        R.g.ntiles = R.g.nt[0] * R.g.nt[1];
        R.g.ncells = (long long)R.g.n[0] * R.g.n[1];
        R.cell_off = cells;
        R.sid_base = sids;
        R.tile_base = tiles;
        R.yee_blk_base = yee_nblk_;
        if ((long long)yee_nblk_ + yee_blocks(R.g.n[0], R.g.n[1]) > (1LL << 30))
            return fail(PIC_EINVAL, "batch too large for one field-update launch");
        yee_nblk_ += yee_blocks(R.g.n[0], R.g.n[1]);
        cells += R.g.ncells;
        sids += R.g.ntiles * nsp_;
        tiles += R.g.ntiles;
        R.npart = 0;
        for (int s = 0; s < nsp_; ++s) {
            R.count_sp[s] = st[r].count[s];
            R.npart += R.count_sp[s];
        }
        npart_ += R.npart;
    }
    ncells_ = cells;
    nseg_ = sids;
    ntiles_ = tiles;
    if (npart_ > (1LL << 31) - 1) return fail(PIC_EINVAL, "more than 2^31 particles in the batch");

    // ---- bin every particle: global segment and an in-segment order key
    std::vector<long long> count(nseg_, 0);
    std::vector<int32_t> segof((size_t)npart_);
    std::vector<uint32_t> key((size_t)npart_);
    std::vector<long long> run_first(nrun + 1, 0);
    auto place = [](const double* row, const Run& R, int cell[2], double off[2]) {
        for (int a = 0; a < 2; ++a) {
            const double xi = row[a] / R.d[a];
            const double fl = std::floor(xi);
            double o = xi - fl;
            long long ci = (long long)fl % R.g.n[a];
            if (ci < 0) ci += R.g.n[a];
            if ((real)o >= real(1)) {
                o = 0.0;
                ci = (ci + 1) % R.g.n[a];
            }
            cell[a] = (int)ci;
            off[a] = o;
        }
    };
    {
        long long q = 0;
        for (int r = 0; r < nrun; ++r) {
            Run& R = runs_[r];
            run_first[r] = q;
            const int tile_cells = R.g.T[0] * R.g.T[1];
            std::vector<int32_t> cellrank((size_t)nsp_ * R.g.ncells, 0);
            for (int s = 0; s < nsp_; ++s) {
                const double* P = st[r].particles[s];
                for (long long i = 0; i < R.count_sp[s]; ++i, ++q) {
                    const double* row = P + i * PIC_PARTICLE_IN_COLS;
                    for (int col = 0; col < PIC_PARTICLE_IN_COLS; ++col)
                        if (!std::isfinite(row[col]))
                            return fail(PIC_EINVAL, "run %d species %d particle %lld: non-finite input", r, s, i);
                    const double s2 = row[6] * row[6] + row[7] * row[7] + row[8] * row[8];
                    if (std::fabs(s2 - 1.0) > 1e-6)
                        return fail(PIC_EINVAL, "run %d species %d particle %lld: |s| must be 1", r, s, i);
                    int cell[2];
                    double off[2];
                    place(row, R, cell, off);
                    const int tile = cell[0] / R.g.T[0] + R.g.nt[0] * (cell[1] / R.g.T[1]);
                    const int sid = R.sid_base + tile * nsp_ + s;
                    segof[q] = sid;
                    count[sid]++;
                    const long long gcell = (long long)cell[1] * R.g.n[0] + cell[0];
                    const long long rank = cellrank[(size_t)s * R.g.ncells + gcell]++;
                    const int lc = (cell[0] % R.g.T[0]) + R.g.T[0] * (cell[1] % R.g.T[1]);
                    const unsigned long long k64 = (unsigned long long)rank * tile_cells + lc;
                    if (k64 > 0xFFFFFFFFull) return fail(PIC_EINVAL, "more than 2^32 particle ranks in a tile");
                    key[q] = (uint32_t)k64;
                }
            }
        }
        run_first[nrun] = q;
    }
    std::vector<int32_t> h_start(nseg_), h_cap(nseg_), h_count(nseg_);
    cap_total_ = 0;
    long long maxcap = 0;
    for (int s = 0; s < nseg_; ++s) {
        const double slack = runs_[0].R.slack;
        const long long cp = seg_capacity(count[s], slack);
        h_start[s] = (int32_t)cap_total_;
        h_cap[s] = (int32_t)cp;
        h_count[s] = (int32_t)count[s];
        cap_total_ += cp;
        maxcap = std::max(maxcap, cp);
        if (cap_total_ > kMaxSlots) return fail(PIC_ECAPACITY, "particle capacity exceeds 2^29 slots");
    }
    seg_.dummy = (int)cap_total_;
    seg_.max_chunks = (int)((maxcap + 63) / 64);
    if (push_lds() > 64 * 1024) return fail(PIC_ECAPACITY, "a tile needs more than 64 KiB of shared memory");

    // ---- device memory
    store_slots_ = cap_total_ + kSpareSlots;
    Status S = alloc_store(p_, store_slots_, false);
    if (S.code) return S;
    S = alloc_store(lv_, std::max(npart_, 1LL), true);
    if (S.code) return S;
    S = alloc_store(st_, std::max(npart_, 1LL), true);
    if (S.code) return S;
    seg_.start = (int32_t*)dalloc(nseg_ * sizeof(int32_t));
    seg_.cap = (int32_t*)dalloc(nseg_ * sizeof(int32_t));
    seg_.count = (int32_t*)dalloc(nseg_ * sizeof(int32_t));
    for (int a = 0; a < 3; ++a) {
        f_.E[a] = (freal*)dalloc(ncells_ * sizeof(freal));
        f_.B[a] = (freal*)dalloc(ncells_ * sizeof(freal));
        for (int b = 0; b < 2; ++b) jbuf_[b][a] = (freal*)dalloc(ncells_ * sizeof(freal));
        f_.J[a] = jbuf_[0][a];
        if (deposit_) {
            enext_[a] = (freal*)dalloc(ncells_ * sizeof(freal));
            bnext_[a] = (freal*)dalloc(ncells_ * sizeof(freal));
        }
    }
    ctr_ = (int32_t*)dalloc(CTR_NCTR * sizeof(int32_t));
    moved_ = (unsigned long long*)dalloc(sizeof(unsigned long long));
    run_ns_ = (unsigned long long*)dalloc(nrun * sizeof(unsigned long long));
    acc_ = (double*)dalloc(kRedSlots * kRedStride * sizeof(double));
    d_runs_ = (RunDesc<real>*)dalloc(nrun * sizeof(RunDesc<real>));
    d_order_ = (TileRef*)dalloc(ntiles_ * sizeof(TileRef));
    d_blk_run_ = (int32_t*)dalloc((size_t)yee_nblk_ * sizeof(int32_t));
    bool ok = seg_.start && seg_.cap && seg_.count && ctr_ && moved_ && run_ns_ && acc_ && d_runs_ && d_order_ &&
              d_blk_run_;
    for (int a = 0; a < 3; ++a)
        ok = ok && f_.E[a] && f_.B[a] && jbuf_[0][a] && jbuf_[1][a] && (!deposit_ || (enext_[a] && bnext_[a]));
    if (!ok) return fail(PIC_ENOMEM, "device allocation failed");
    HIP_OR_FAIL(hipHostMalloc((void**)&h_ctr_, CTR_NCTR * sizeof(int32_t), hipHostMallocDefault));
    std::memset(h_ctr_, 0, CTR_NCTR * sizeof(int32_t));

    // ---- particles in segment order
    {
        const size_t C = (size_t)cap_total_;
        std::vector<int32_t> hcell(C, 0), hid(C, 0);
        std::vector<real> hoff[2], hu[3], hs[3], hw(C, real(0));
        for (int a = 0; a < 2; ++a) hoff[a].assign(C, real(0));
        for (int a = 0; a < 3; ++a) {
            hu[a].assign(C, real(0));
            hs[a].assign(C, real(0));
        }
        std::vector<uint32_t> perm((size_t)npart_);
        std::vector<long long> first(nseg_ + 1, 0), fill(nseg_, 0);
        for (int sg = 0; sg < nseg_; ++sg) first[sg + 1] = first[sg] + count[sg];
        for (long long q = 0; q < npart_; ++q) perm[first[segof[q]] + fill[segof[q]]++] = (uint32_t)q;
        for (int sg = 0; sg < nseg_; ++sg)
            std::sort(perm.begin() + first[sg], perm.begin() + first[sg + 1],
                      [&](uint32_t a, uint32_t b) { return key[a] < key[b]; });
        for (int r = 0; r < nrun; ++r) {
            const Run& R = runs_[r];
            std::vector<long long> spbase(nsp_ + 1, run_first[r]);
            for (int s = 0; s < nsp_; ++s) spbase[s + 1] = spbase[s] + R.count_sp[s];
            for (int sg = R.sid_base; sg < R.sid_base + R.g.ntiles * nsp_; ++sg) {
                const int s = (sg - R.sid_base) % nsp_;
                const double* P = st[r].particles[s];
                long long slot = h_start[sg];
                for (long long m = first[sg]; m < first[sg + 1]; ++m, ++slot) {
                    const long long i = (long long)perm[m] - spbase[s];
                    const double* row = P + i * PIC_PARTICLE_IN_COLS;
                    int cell[2];
                    double off[2];
                    place(row, R, cell, off);
                    hcell[slot] = pack_cell<2>(cell[0], cell[1], 0);
                    for (int a = 0; a < 2; ++a) hoff[a][slot] = (real)off[a];
                    for (int a = 0; a < 3; ++a) {
                        hu[a][slot] = (real)row[3 + a];
                        hs[a][slot] = (real)row[6 + a];
                    }
                    hw[slot] = (real)row[9];
                    hid[slot] = (int32_t)i;
                }
            }
        }
        HIP_OR_FAIL(hipMemcpyAsync(p_.cell, hcell.data(), C * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
        HIP_OR_FAIL(hipMemcpyAsync(p_.id, hid.data(), C * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
        HIP_OR_FAIL(hipMemcpyAsync(p_.w, hw.data(), C * sizeof(real), hipMemcpyHostToDevice, stream_));
        for (int a = 0; a < 3; ++a) {
            if (a < 2)
                HIP_OR_FAIL(hipMemcpyAsync(p_.off[a], hoff[a].data(), C * sizeof(real), hipMemcpyHostToDevice, stream_));
            HIP_OR_FAIL(hipMemcpyAsync(p_.u[a], hu[a].data(), C * sizeof(real), hipMemcpyHostToDevice, stream_));
            HIP_OR_FAIL(hipMemcpyAsync(p_.s[a], hs[a].data(), C * sizeof(real), hipMemcpyHostToDevice, stream_));
        }
        HIP_OR_FAIL(hipStreamSynchronize(stream_));
    }
    HIP_OR_FAIL(hipMemcpyAsync(seg_.start, h_start.data(), nseg_ * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
    HIP_OR_FAIL(hipMemcpyAsync(seg_.cap, h_cap.data(), nseg_ * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
    HIP_OR_FAIL(hipMemcpyAsync(seg_.count, h_count.data(), nseg_ * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
    HIP_OR_FAIL(hipMemsetAsync(ctr_, 0, CTR_NCTR * sizeof(int32_t), stream_));
    HIP_OR_FAIL(hipMemsetAsync(moved_, 0, sizeof(unsigned long long), stream_));
    HIP_OR_FAIL(hipMemsetAsync(run_ns_, 0, nrun * sizeof(unsigned long long), stream_));

    // ---- fields, concatenated
    for (int comp = 0; comp < 6; ++comp) {
        freal* dst = comp < 3 ? f_.E[comp] : f_.B[comp - 3];
        for (int r = 0; r < nrun; ++r) {
            const Run& R = runs_[r];
            const size_t N = (size_t)R.g.ncells;
            if (st[r].fields) {
                const double* src = st[r].fields + comp * N;
                for (size_t i = 0; i < N; ++i)
                    if (!std::isfinite(src[i])) return fail(PIC_EINVAL, "run %d field %d: non-finite value", r, comp);
                HIP_OR_FAIL(hipMemcpyAsync(dst + R.cell_off, src, N * sizeof(freal), hipMemcpyHostToDevice, stream_));
                HIP_OR_FAIL(hipStreamSynchronize(stream_));
            } else {
                HIP_OR_FAIL(hipMemsetAsync(dst + R.cell_off, 0, N * sizeof(freal), stream_));
            }
        }
    }
    for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 3; ++a) HIP_OR_FAIL(hipMemsetAsync(jbuf_[b][a], 0, ncells_ * sizeof(freal), stream_));

    // ---- work list: each run's tiles in row-major order (neighbouring
    // tiles side by side, their guard cells shared in L2), the runs by
    // decreasing cost per tile, cut into 8 contiguous chunks of about equal
    // cost (particles + cells), one per XCD.  The persistent push takes the
    // chunks front to back, so the tiles left at the end, when workgroups
    // run out of work one by one, are the cheapest ones.
    order_.resize(ntiles_);
    {
        auto tile_cost = [&](const Run& R, int t) {
            long long c = 0;
            for (int s = 0; s < nsp_; ++s) c += count[R.sid_base + t * nsp_ + s];
            const int tx = t % R.g.nt[0], ty = t / R.g.nt[0];
            const long long cells = (long long)std::min(R.g.T[0], R.g.n[0] - tx * R.g.T[0]) *
                                    std::min(R.g.T[1], R.g.n[1] - ty * R.g.T[1]);
            return (double)(c + cells);
        };
        std::vector<double> run_cost(nrun, 0.0);
        std::vector<int> rorder(nrun);
        for (int r = 0; r < nrun; ++r) {
            rorder[r] = r;
            for (int t = 0; t < runs_[r].g.ntiles; ++t) run_cost[r] += tile_cost(runs_[r], t);
            run_cost[r] /= std::max(runs_[r].g.ntiles, 1);
        }
        std::stable_sort(rorder.begin(), rorder.end(), [&](int a, int b) { return run_cost[a] > run_cost[b]; });
        std::vector<double> cost(ntiles_);
        double total = 0.0;
        int i = 0;
        for (int r : rorder) {
            const Run& R = runs_[r];
            for (int t = 0; t < R.g.ntiles; ++t, ++i) {
                order_[i] = TileRef{r, t};
                cost[i] = tile_cost(R, t);
                total += cost[i];
            }
        }
        xq_.start[0] = 0;
        double acc = 0.0;
        int x = 1;
        for (int i = 0; i < ntiles_ && x < 8; ++i) {
            acc += cost[i];
            while (x < 8 && acc >= total * x / 8.0) xq_.start[x++] = i + 1;
        }
        while (x < 8) xq_.start[x++] = ntiles_;
        xq_.start[8] = ntiles_;
    }
    HIP_OR_FAIL(hipMemcpyAsync(d_order_, order_.data(), ntiles_ * sizeof(TileRef), hipMemcpyHostToDevice, stream_));
    {
        std::vector<int32_t> blk_run((size_t)yee_nblk_);
        for (int r = 0; r < nrun; ++r) {
            const Run& R = runs_[r];
            std::fill(blk_run.begin() + R.yee_blk_base,
                      blk_run.begin() + R.yee_blk_base + yee_blocks(R.g.n[0], R.g.n[1]), r);
        }
        HIP_OR_FAIL(hipMemcpyAsync(d_blk_run_, blk_run.data(), blk_run.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, stream_));
        HIP_OR_FAIL(hipStreamSynchronize(stream_));
    }
    S = upload_descs();
    if (S.code) return S;
    int dev = 0, cus = 256;
    HIP_OR_FAIL(hipGetDevice(&dev));
    HIP_OR_FAIL(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int per_cu = use_acc64_ ? push_batch_blocks_per_cu<real, double>(push_lds())
                                  : push_batch_blocks_per_cu<real, real>(push_lds());
    // a multiple of 8, so that every XCD runs the same number of workgroups
    push_blocks_ = std::max(8, std::min(ntiles_, cus * per_cu) / 8 * 8);
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    return Status{};
}

template <typename real>
Status BatchEngine<real>::step(int nsteps) {
    for (int it = 0; it < nsteps; ++it) {
        if (nstep_ > 0 && nstep_ == check_at_) {
            HIP_OR_FAIL(hipStreamSynchronize(stream_));
            if (h_ctr_[CTR_NONFINITE])
                return fail(PIC_ENONFINITE, "a push produced a non-finite momentum or spin before step %lld",
                            (long long)nstep_);
            long long left = h_ctr_[CTR_STASH];
            if (repack_due(nstep_, left, npart_)) {
                Status S = repack();
                if (S.code) return S;
                left = 0;
            }
            check_at_ = next_check(nstep_, left, npart_);
        }
        const int slot = (int)(nstep_ & 1);
        const int jnext = jcur_ ^ 1;
        for (int a = 0; a < 3; ++a) f_.J[a] = jbuf_[jnext][a];
        const size_t lds = push_lds();
        unsigned long long* rn = time_runs_ ? run_ns_ : nullptr;
        timer_start(timer_, stream_, 0);
        if (use_acc64_)
            HIP_OR_FAIL((launch_push_tiles_batch<real, double>(d_runs_, d_order_, xq_, push_blocks_, lds, p_, seg_,
                                                               lv_, ctr_, slot, f_, deposit_, rn, stream_)));
        else
            HIP_OR_FAIL((launch_push_tiles_batch<real, real>(d_runs_, d_order_, xq_, push_blocks_, lds, p_, seg_,
                                                             lv_, ctr_, slot, f_, deposit_, rn, stream_)));
        timer_stop(timer_, stream_, 0);
        timer_start(timer_, stream_, 1);
        HIP_OR_FAIL((launch_push_stash_batch<real>(d_runs_, st_, ctr_, f_, deposit_, kStashBlocks, stream_)));
        timer_stop(timer_, stream_, 1);
        timer_start(timer_, stream_, 2);
        HIP_OR_FAIL((launch_insert_batch<real>(d_runs_, p_, seg_, lv_, st_, ctr_, slot, moved_, 1024, stream_)));
        timer_stop(timer_, stream_, 2);
        if (deposit_) {
            timer_start(timer_, stream_, 3);
            Fields<freal> nf = f_;
            for (int a = 0; a < 3; ++a) {
                nf.E[a] = enext_[a];
                nf.B[a] = bnext_[a];
            }
            HIP_OR_FAIL((launch_yee_fused_batch<real>(d_runs_, d_blk_run_, yee_nblk_, f_, nf, jbuf_[jcur_], stream_)));
            for (int a = 0; a < 3; ++a) {
                std::swap(f_.E[a], enext_[a]);
                std::swap(f_.B[a], bnext_[a]);
            }
            timer_stop(timer_, stream_, 3);
        }
        // the overflow count for the next check only
        if (nstep_ + 1 == check_at_)
            HIP_OR_FAIL(hipMemcpyAsync(h_ctr_ + CTR_STASH, ctr_ + CTR_STASH, 2 * sizeof(int32_t),
                                       hipMemcpyDeviceToHost, stream_));
        if (deposit_) jcur_ = jnext;
        for (int a = 0; a < 3; ++a) f_.J[a] = jbuf_[jcur_][a];
        ++nstep_;
    }
    return Status{};
}

template <typename real>
Status BatchEngine<real>::repack() {
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    int32_t nst = 0;
    HIP_OR_FAIL(hipMemcpy(&nst, ctr_ + CTR_STASH, sizeof(int32_t), hipMemcpyDeviceToHost));
    h_ctr_[CTR_STASH] = nst;
    if (nst == 0) return Status{};
    const int saved_chunks = seg_.max_chunks;
    const long long capmax = max_segment_slots([&](int mc) {
        seg_.max_chunks = mc;
        return push_lds();
    });
    seg_.max_chunks = saved_chunks;
    std::vector<int32_t> cnt(nseg_), old_cap(nseg_);
    HIP_OR_FAIL(hipMemcpy(cnt.data(), seg_.count, nseg_ * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_OR_FAIL(hipMemcpy(old_cap.data(), seg_.cap, nseg_ * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int32_t> scell(nst), stag(nst);
    HIP_OR_FAIL(hipMemcpy(scell.data(), st_.cell, nst * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_OR_FAIL(hipMemcpy(stag.data(), st_.sp, nst * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<long long> want(cnt.begin(), cnt.end());
    for (int i = 0; i < nst; ++i) {
        const int run = stag[i] / kMaxSpecies, sp = stag[i] % kMaxSpecies;
        const Run& R = runs_[run];
        int c[3];
        unpack_cell<2>(scell[i], c[0], c[1], c[2]);
        const int tile = c[0] / R.g.T[0] + R.g.nt[0] * (c[1] / R.g.T[1]);
        want[R.sid_base + tile * nsp_ + sp]++;
    }
    std::vector<int32_t> nstart(nseg_), ncap(nseg_);
    long long total = 0, maxcap = 0;
    for (int s = 0; s < nseg_; ++s) {
        const long long cp = regrow_capacity(want[s], old_cap[s], runs_[0].R.slack, capmax);
        nstart[s] = (int32_t)total;
        ncap[s] = (int32_t)cp;
        total += cp;
        maxcap = std::max(maxcap, cp);
        if (total > kMaxSlots) return fail(PIC_ECAPACITY, "particle capacity exceeds 2^29 slots");
    }
    {
        const int saved = seg_.max_chunks;
        seg_.max_chunks = (int)((maxcap + 63) / 64);
        const size_t lds = push_lds();
        seg_.max_chunks = saved;
        if (lds > 64 * 1024) return fail(PIC_ECAPACITY, "a tile segment needs more than 64 KiB of shared memory");
    }
    PArrays<real> np{};
    const long long slots = store_alloc_slots(total + kSpareSlots, store_slots_);
    Status S = alloc_store(np, slots, false);
    if (S.code) return S;
    int32_t* d_nstart = (int32_t*)dalloc(nseg_ * sizeof(int32_t));
    if (!d_nstart) return fail(PIC_ENOMEM, "repack allocation failed");
    HIP_OR_FAIL(hipMemcpyAsync(d_nstart, nstart.data(), nseg_ * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
    HIP_OR_FAIL((launch_repack_segments<real>(p_, np, seg_.start, d_nstart, seg_.count, nseg_, 2, stream_)));
    HIP_OR_FAIL(hipMemcpyAsync(seg_.start, nstart.data(), nseg_ * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
    HIP_OR_FAIL(hipMemcpyAsync(seg_.cap, ncap.data(), nseg_ * sizeof(int32_t), hipMemcpyHostToDevice, stream_));
    HIP_OR_FAIL((launch_insert_batch<real>(d_runs_, np, seg_, st_, st_, ctr_, CTR_STASH, moved_, 256, stream_)));
    HIP_OR_FAIL(hipMemsetAsync(ctr_ + CTR_STASH, 0, sizeof(int32_t), stream_));
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    free_store(p_);
    dfree(d_nstart);
    p_ = np;
    store_slots_ = slots;
    cap_total_ = total;
    seg_.dummy = (int)total;
    seg_.max_chunks = (int)((maxcap + 63) / 64);
    h_ctr_[CTR_STASH] = 0;
    repacks_++;
    return Status{};
}

template <typename real>
Status BatchEngine<real>::polarization(int run, int species, double emin, double emax, double P[3], int64_t* N) {
    if (run < 0 || run >= nruns()) return fail(PIC_EINVAL, "run %d out of range", run);
    if (species < -1 || species >= nsp_) return fail(PIC_EINVAL, "species %d out of range", species);
    if (std::isnan(emin) || std::isnan(emax)) return fail(PIC_EINVAL, "energy window is NaN");
    const Run& R = runs_[run];
    ReduceArgs ra{};
    ra.run = run;
    ra.species = species;
    ra.emin = emin;
    ra.emax = emax;
    for (int s = 0; s < kMaxSpecies; ++s) {
        ra.mu[s] = s < nsp_ ? R.R.cfg.sp[s].mu : 1.0;
        ra.Z[s] = s < nsp_ ? R.R.cfg.sp[s].Z : 0.0;
    }
    Segs view = seg_;
    view.start = seg_.start + R.sid_base;
    view.cap = seg_.cap + R.sid_base;
    view.count = seg_.count + R.sid_base;
    double h[kRedSlots * kRedStride];
    HIP_OR_FAIL(hipMemsetAsync(acc_, 0, sizeof h, stream_));
    HIP_OR_FAIL((launch_reduce_particles<real, 2>(RED_POLARIZATION, R.g, p_, view, st_, ctr_, ra, acc_, nullptr, stream_)));
    HIP_OR_FAIL(hipMemcpyAsync(h, acc_, sizeof h, hipMemcpyDeviceToHost, stream_));
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    double acc[kRedStride] = {};
    for (int q = 0; q < kRedStride; ++q)
        for (int s = 0; s < kRedSlots; ++s) acc[q] += h[s * kRedStride + q];
    *N = (int64_t)std::llround(acc[3]);
    for (int a = 0; a < 3; ++a) P[a] = acc[3] > 0 ? acc[a] / acc[3] : 0.0;
    return Status{};
}

template <typename real>
Status BatchEngine<real>::fields(int run, uint32_t mask, double* out, size_t cap) {
    if (run < 0 || run >= nruns()) return fail(PIC_EINVAL, "run %d out of range", run);
    if (mask & ~0x1FFu) return fail(PIC_EINVAL, "field mask 0x%x: E, B and J only", mask);
    const Run& R = runs_[run];
    const size_t N = (size_t)R.g.ncells;
    int nc = 0;
    for (int b = 0; b < 9; ++b) nc += (mask >> b) & 1;
    if (!out && nc) return fail(PIC_EINVAL, "host_out is NULL");
    if (cap < (size_t)nc * N) return fail(PIC_EINVAL, "cap %zu < %zu", cap, (size_t)nc * N);
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    size_t o = 0;
    for (int b = 0; b < 9; ++b) {
        if (!((mask >> b) & 1)) continue;
        const freal* src = b < 3 ? f_.E[b] : (b < 6 ? f_.B[b - 3] : f_.J[b - 6]);
        HIP_OR_FAIL(hipMemcpy(out + o, src + R.cell_off, N * sizeof(freal), hipMemcpyDeviceToHost));
        o += N;
    }
    return Status{};
}

template <typename real>
Status BatchEngine<real>::particles(int run, int species, double* out, size_t cap, int64_t* n_out) {
    if (run < 0 || run >= nruns()) return fail(PIC_EINVAL, "run %d out of range", run);
    if (species < 0 || species >= nsp_) return fail(PIC_EINVAL, "species %d out of range", species);
    const Run& R = runs_[run];
    const long long n = R.count_sp[species];
    if (n_out) *n_out = n;
    if (cap < (size_t)n * PIC_PARTICLE_OUT_COLS) return fail(PIC_EINVAL, "cap too small for %lld particles", n);
    if (n > 0 && !out) return fail(PIC_EINVAL, "host_out is NULL");
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    const int ns = R.g.ntiles * nsp_;
    std::vector<int32_t> start(ns), count(ns);
    HIP_OR_FAIL(hipMemcpy(start.data(), seg_.start + R.sid_base, ns * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_OR_FAIL(hipMemcpy(count.data(), seg_.count + R.sid_base, ns * sizeof(int32_t), hipMemcpyDeviceToHost));
    int32_t nst = 0;
    HIP_OR_FAIL(hipMemcpy(&nst, ctr_ + CTR_STASH, sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<char> seen((size_t)n, 0);
    auto emit_range = [&](const PArrays<real>& A, long long lo, long long hi, bool stash) -> Status {
        const long long len = hi - lo;
        if (len <= 0) return Status{};
        std::vector<int32_t> cell(len), id(len), tag;
        std::vector<real> off[2], u[3], s[3], w(len);
        HIP_OR_FAIL(hipMemcpy(cell.data(), A.cell + lo, len * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIP_OR_FAIL(hipMemcpy(id.data(), A.id + lo, len * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIP_OR_FAIL(hipMemcpy(w.data(), A.w + lo, len * sizeof(real), hipMemcpyDeviceToHost));
        if (stash) {
            tag.resize(len);
            HIP_OR_FAIL(hipMemcpy(tag.data(), A.sp + lo, len * sizeof(int32_t), hipMemcpyDeviceToHost));
        }
        for (int a = 0; a < 3; ++a) {
            if (a < 2) {
                off[a].resize(len);
                HIP_OR_FAIL(hipMemcpy(off[a].data(), A.off[a] + lo, len * sizeof(real), hipMemcpyDeviceToHost));
            }
            u[a].resize(len);
            s[a].resize(len);
            HIP_OR_FAIL(hipMemcpy(u[a].data(), A.u[a] + lo, len * sizeof(real), hipMemcpyDeviceToHost));
            HIP_OR_FAIL(hipMemcpy(s[a].data(), A.s[a] + lo, len * sizeof(real), hipMemcpyDeviceToHost));
        }
        for (long long q = 0; q < len; ++q) {
            if (stash && tag[q] != run * kMaxSpecies + species) continue;
            const long long i = id[q];
            if (i < 0 || i >= n || seen[i]) return fail(PIC_ESTATE, "particle bookkeeping is corrupt (id %lld)", i);
            seen[i] = 1;
            double* row = out + i * PIC_PARTICLE_OUT_COLS;
            int c[3];
            unpack_cell<2>(cell[q], c[0], c[1], c[2]);
            row[0] = (double)i;
            for (int a = 0; a < 3; ++a) row[1 + a] = a < 2 ? ((double)c[a] + (double)off[a][q]) * R.d[a] : 0.0;
            for (int a = 0; a < 3; ++a) {
                row[4 + a] = (double)u[a][q];
                row[7 + a] = (double)s[a][q];
            }
            row[10] = (double)w[q];
        }
        return Status{};
    };
    for (int t = 0; t < R.g.ntiles; ++t) {
        const int k = t * nsp_ + species;
        Status S = emit_range(p_, start[k], (long long)start[k] + count[k], false);
        if (S.code) return S;
    }
    Status S = emit_range(st_, 0, nst, true);
    if (S.code) return S;
    for (long long i = 0; i < n; ++i)
        if (!seen[i]) return fail(PIC_ESTATE, "particle %lld of run %d species %d is missing", i, run, species);
    return Status{};
}

template <typename real>
Status BatchEngine<real>::stats(int64_t* out, int cap) {
    if (!out || cap < 5) return fail(PIC_EINVAL, "stats needs cap >= 5");
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    unsigned long long moved = 0;
    int32_t nst = 0;
    HIP_OR_FAIL(hipMemcpy(&moved, moved_, sizeof moved, hipMemcpyDeviceToHost));
    HIP_OR_FAIL(hipMemcpy(&nst, ctr_ + CTR_STASH, sizeof nst, hipMemcpyDeviceToHost));
    out[0] = nstep_;
    out[1] = (int64_t)moved;
    out[2] = nst;
    out[3] = repacks_;
    out[4] = npart_;
    if (cap > 5) out[5] = push_blocks_;
    if (cap > 6) out[6] = ntiles_;
    return Status{};
}

template <typename real>
Status BatchEngine<real>::run_time(bool enable, double* ns_out) {
    HIP_OR_FAIL(hipStreamSynchronize(stream_));
    if (ns_out) {
        std::vector<unsigned long long> h(runs_.size());
        HIP_OR_FAIL(hipMemcpy(h.data(), run_ns_, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
        for (size_t r = 0; r < h.size(); ++r) ns_out[r] = (double)h[r];
    }
    HIP_OR_FAIL(hipMemset(run_ns_, 0, runs_.size() * sizeof(unsigned long long)));
    time_runs_ = enable;
    return Status{};
}

}  // namespace

// ---------------------------------------------------------------- C ABI

struct pic_ctx {
    std::unique_ptr<EngineBase> eng;
    std::string err;
    bool failed = false;
};

static int finish(pic_ctx* ctx, const Status& s) {
    if (s.code != PIC_OK) {
        ctx->err = s.msg;
        if (s.code == PIC_EHIP || s.code == PIC_ESTATE) ctx->failed = true;
    }
    return s.code;
}

#define CTX_CHECK(ctx)                                        \
    do {                                                      \
        if (!(ctx)) return PIC_ESTATE;                        \
        if ((ctx)->failed || !(ctx)->eng) {                   \
            (ctx)->err = "context is unusable after an error"; \
            return PIC_ESTATE;                                \
        }                                                     \
    } while (0)

extern "C" {

int pic_init(const pic_config* cfg, const pic_state* init, const pic_allocator* alloc,
             void* hip_stream, pic_ctx** out) {
    g_init_error.clear();
    if (!out) {
        g_init_error = "out is NULL";
        return PIC_EINVAL;
    }
    *out = nullptr;
    Resolved R;
    Status s = resolve_config(cfg, init, R);
    if (s.code) {
        g_init_error = s.msg;
        return s.code;
    }
    if (alloc && (!alloc->alloc || !alloc->free)) {
        g_init_error = "allocator needs both alloc and free";
        return PIC_EINVAL;
    }
    std::unique_ptr<EngineBase> eng;
    hipStream_t stream = (hipStream_t)hip_stream;
    if (cfg->precision == PIC_FP64) {
        if (cfg->ndim == 2) eng.reset(new Engine<double, 2>(alloc, stream));
        else eng.reset(new Engine<double, 3>(alloc, stream));
    } else {
        if (cfg->ndim == 2) eng.reset(new Engine<float, 2>(alloc, stream));
        else eng.reset(new Engine<float, 3>(alloc, stream));
    }
    s = eng->init(R, init);
    if (s.code) {
        g_init_error = s.msg;
        eng->release();
        return s.code;
    }
    pic_ctx* ctx = new pic_ctx();
    ctx->eng = std::move(eng);
    *out = ctx;
    return PIC_OK;
}

int pic_step(pic_ctx* ctx, int32_t nsteps) {
    CTX_CHECK(ctx);
    if (nsteps < 0) {
        ctx->err = "nsteps must be >= 0";
        return PIC_EINVAL;
    }
    return finish(ctx, ctx->eng->step(nsteps));
}

int pic_polarization(pic_ctx* ctx, int32_t species, double emin, double emax, double P_out[3],
                     int64_t* N_out) {
    CTX_CHECK(ctx);
    if (!P_out || !N_out) {
        ctx->err = "P_out and N_out must not be NULL";
        return PIC_EINVAL;
    }
    return finish(ctx, ctx->eng->polarization(species, emin, emax, P_out, N_out));
}

int pic_polarization_record(pic_ctx* ctx, int32_t species, double ekin_min_mev, double ekin_max_mev,
                            int32_t capacity) {
    CTX_CHECK(ctx);
    return finish(ctx, ctx->eng->record(species, ekin_min_mev, ekin_max_mev, capacity));
}

int pic_polarization_history(pic_ctx* ctx, double* P_out, int64_t* N_out, int32_t cap, int32_t* nsteps_out) {
    CTX_CHECK(ctx);
    if (!nsteps_out) {
        ctx->err = "nsteps_out must not be NULL";
        return PIC_EINVAL;
    }
    int n = 0;
    const int code = finish(ctx, ctx->eng->record_read(P_out, N_out, cap, &n));
    *nsteps_out = n;
    return code;
}

int pic_fields(pic_ctx* ctx, uint32_t mask, double* host_out, size_t cap_doubles) {
    CTX_CHECK(ctx);
    return finish(ctx, ctx->eng->fields(mask, host_out, cap_doubles));
}

int pic_spectrum(pic_ctx* ctx, int32_t species, double emin, double emax, int32_t nbins,
                 double* count_out, double* weight_out, double* spin_out) {
    CTX_CHECK(ctx);
    return finish(ctx, ctx->eng->spectrum(species, emin, emax, nbins, count_out, weight_out, spin_out));
}

int pic_spectrum_noalloc(pic_ctx* ctx, int32_t species, double emin, double emax, int32_t nbins,
                         double* count_out, double* weight_out, double* spin_out) {
    CTX_CHECK(ctx);
    return finish(ctx, ctx->eng->spectrum_noalloc(species, emin, emax, nbins, count_out, weight_out, spin_out));
}

int pic_phase_space(pic_ctx* ctx, int32_t species, int32_t axis, double xmin, double xmax,
                    int32_t nx, int32_t comp, double pmin, double pmax, int32_t np, double* out) {
    CTX_CHECK(ctx);
    return finish(ctx, ctx->eng->phase_space(species, axis, xmin, xmax, nx, comp, pmin, pmax, np, out));
}

int pic_density(pic_ctx* ctx, int32_t species, double* out, size_t cap_doubles) {
    CTX_CHECK(ctx);
    return finish(ctx, ctx->eng->density(species, out, cap_doubles));
}

int pic_particles(pic_ctx* ctx, int32_t species, double* host_out, size_t cap_doubles, int64_t* n_out) {
    CTX_CHECK(ctx);
    return finish(ctx, ctx->eng->particles(species, host_out, cap_doubles, n_out));
}

int pic_particles_cells(pic_ctx* ctx, int32_t species, double* host_out, size_t cap_doubles, int64_t* n_out) {
    CTX_CHECK(ctx);
    return finish(ctx, ctx->eng->particles(species, host_out, cap_doubles, n_out, true));
}

int pic_test_poison(pic_ctx* ctx, int32_t species) {
    CTX_CHECK(ctx);
    return finish(ctx, ctx->eng->poison(species));
}

int pic_energy(pic_ctx* ctx, double* out, int32_t cap) {
    CTX_CHECK(ctx);
    return finish(ctx, ctx->eng->energy(out, cap));
}

int pic_stats(pic_ctx* ctx, int64_t* out, int32_t cap) {
    CTX_CHECK(ctx);
    return finish(ctx, ctx->eng->stats(out, cap));
}

int pic_window(pic_ctx* ctx, const pic_window_config* w) {
    CTX_CHECK(ctx);
    return finish(ctx, ctx->eng->window(w));
}

int pic_timing(pic_ctx* ctx, int32_t enable) {
    CTX_CHECK(ctx);
    return finish(ctx, ctx->eng->timing(enable));
}

int pic_timing_read(pic_ctx* ctx, double* ms_out, int64_t* launches_out, int32_t cap) {
    CTX_CHECK(ctx);
    return finish(ctx, ctx->eng->timing_read(ms_out, launches_out, cap));
}

const char* pic_last_error(const pic_ctx* ctx) {
    if (!ctx) return g_init_error.c_str();
    return ctx->err.c_str();
}

void pic_free(pic_ctx* ctx) {
    if (!ctx) return;
    if (ctx->eng) ctx->eng->release();
    delete ctx;
}

}  // extern "C"

// ---------------------------------------------------------------- batches: C ABI

struct pic_batch {
    std::unique_ptr<BatchBase> eng;
    std::string err;
    bool failed = false;
    std::vector<int32_t> cands;       // tile edges tried by the autotuner
    std::vector<double> tune;         // nrun x ncand: ns of push per particle-step (0: not tried)
    std::vector<double> kernel_ms;    // ncand + 1: push launch per uniform candidate, then per-run tiles
};

namespace {

constexpr int kTileCandidates[] = {8, 12, 16, 24, 32};

Status batch_resolve(int32_t nrun, const pic_config* cfgs, const pic_state* inits, std::vector<Resolved>& Rs) {
    Rs.resize(nrun);
    for (int r = 0; r < nrun; ++r) {
        Status S = resolve_config(&cfgs[r], &inits[r], Rs[r]);
        if (S.code) return fail(S.code, "run %d: %s", r, S.msg.c_str());
        const pic_config& c = cfgs[r];
        const pic_config& c0 = cfgs[0];
        if (c.ndim != 2) return fail(PIC_EINVAL, "run %d: batches hold 2D runs only", r);
        if (c.flags & (PIC_FLAG_DETERMINISTIC | PIC_FLAG_CELL_ROWS))
            return fail(PIC_EINVAL, "run %d: the deterministic mode and cell rows are not available in batches", r);
        bool same = c.precision == c0.precision && c.nspecies == c0.nspecies && c.flags == c0.flags &&
                    c.deposit_acc == c0.deposit_acc && Rs[r].slack == Rs[0].slack;
        for (int s = 0; s < c.nspecies && same; ++s)
            same = c.sp[s].Z == c0.sp[s].Z && c.sp[s].mu == c0.sp[s].mu && c.sp[s].a == c0.sp[s].a;
        if (!same)
            return fail(PIC_EINVAL, "run %d: precision, species, flags, deposit_acc and slack must match run 0", r);
    }
    return Status{};
}

Status batch_build(const std::vector<Resolved>& Rs, const pic_state* inits, const pic_allocator* alloc,
                   hipStream_t stream, std::unique_ptr<BatchBase>& out) {
    if (Rs[0].cfg.precision == PIC_FP64) {
        auto* e = new BatchEngine<double>(alloc, stream);
        out.reset(e);
        return e->init(Rs, inits);
    }
    auto* e = new BatchEngine<float>(alloc, stream);
    out.reset(e);
    return e->init(Rs, inits);
}

constexpr int kTuneSteps = 3;

// One autotuner trial: the batch built from cc, one step untimed, then
// kTuneSteps steps with the push launch and every run's tiles timed.
// kernel_ms: the mean push launch; share[r]: run r's tiles' summed time over
// the number of workgroups of the persistent push (which run side by side),
// per particle-step, in ns.
Status tune_trial(int nrun, const pic_config* cc, const pic_state* inits, const pic_allocator* alloc,
                  hipStream_t stream, double& kernel_ms, std::vector<double>& share) {
    std::vector<Resolved> Rc;
    Status S = batch_resolve(nrun, cc, inits, Rc);
    if (S.code) return S;
    std::unique_ptr<BatchBase> e;
    S = batch_build(Rc, inits, alloc, stream, e);
    if (S.code) return S;
    std::vector<double> ns(nrun, 0.0);
    double ms[kTimers];
    int64_t n[kTimers];
    int64_t st[7] = {0, 0, 0, 0, 0, 1, 0};
    if ((S = e->step(1)).code || (S = e->run_time(true, nullptr)).code || (S = e->timing(1)).code ||
        (S = e->step(kTuneSteps)).code || (S = e->run_time(false, ns.data())).code ||
        (S = e->timing_read(ms, n, kTimers)).code || (S = e->stats(st, 7)).code)
        return S;
    kernel_ms = ms[0] / (double)std::max<int64_t>(n[0], 1);
    const double width = (double)std::max<int64_t>(st[5], 1);
    share.assign(nrun, 0.0);
    for (int r = 0; r < nrun; ++r) {
        int64_t info[4];
        e->run_info(r, info);
        share[r] = ns[r] / width / (kTuneSteps * (double)std::max<int64_t>(info[2], 1));
    }
    return Status{};
}

// Tile autotuner for the runs whose cfg tile is 0 x 0 (tunable).
//  1. For each candidate edge c, every tunable run takes a c x c tile (a run
//     whose shared memory cannot hold it keeps the default) and the push
//     launch is timed: c* is the fastest candidate.
//  2. Each tunable run takes, among the candidates not larger than c*, the
//     one with the smallest share of the launch: larger tiles need more
//     shared memory per workgroup, and the largest tile of the batch sets
//     how many workgroups fit on a compute unit for all runs.
//  3. The per-run tiles are timed and kept only if faster than c* for all.
// cc receives the chosen configs.
void autotune_tiles(int nrun, const pic_config* cfgs, const pic_state* inits, const std::vector<int>& tunable,
                    const pic_allocator* alloc, hipStream_t stream, pic_batch* b, std::vector<pic_config>& cc) {
    const int ncand = (int)(sizeof kTileCandidates / sizeof kTileCandidates[0]);
    b->cands.assign(kTileCandidates, kTileCandidates + ncand);
    b->tune.assign((size_t)nrun * ncand, 0.0);
    b->kernel_ms.assign(ncand + 1, 0.0);
    std::vector<std::vector<pic_config>> trial(ncand);
    int cstar = -1;
    for (int ci = 0; ci < ncand; ++ci) {
        trial[ci].assign(cfgs, cfgs + nrun);
        std::vector<char> tried(nrun, 0);
        for (int r : tunable) {
            pic_config& c = trial[ci][r];
            c.tile[0] = c.tile[1] = kTileCandidates[ci];
            Resolved one;
            if (resolve_config(&c, &inits[r], one).code) c.tile[0] = c.tile[1] = 0;
            else tried[r] = 1;
        }
        if (std::find(tried.begin(), tried.end(), 1) == tried.end()) continue;   // no run takes it
        double kms = 0.0;
        std::vector<double> share;
        if (tune_trial(nrun, trial[ci].data(), inits, alloc, stream, kms, share).code) continue;
        b->kernel_ms[ci] = kms;
        for (int r : tunable)
            if (tried[r]) b->tune[(size_t)r * ncand + ci] = share[r];
        if (cstar < 0 || kms < b->kernel_ms[cstar]) cstar = ci;
    }
    cc.assign(cfgs, cfgs + nrun);
    if (cstar < 0) return;   // nothing could be timed: the default tiles
    cc = trial[cstar];
    std::vector<pic_config> mixed = trial[cstar];
    bool differs = false;
    for (int r : tunable) {
        int best = -1;
        for (int ci = 0; ci <= cstar; ++ci) {
            const double t = b->tune[(size_t)r * ncand + ci];
            if (t > 0.0 && (best < 0 || t < b->tune[(size_t)r * ncand + best])) best = ci;
        }
        if (best >= 0 && best != cstar) {
            mixed[r].tile[0] = mixed[r].tile[1] = kTileCandidates[best];
            differs = true;
        }
    }
    if (!differs) return;
    double kms = 0.0;
    std::vector<double> share;
    if (tune_trial(nrun, mixed.data(), inits, alloc, stream, kms, share).code) return;
    b->kernel_ms[ncand] = kms;
    if (kms < b->kernel_ms[cstar]) cc = mixed;
}

int batch_finish(pic_batch* b, const Status& s) {
    if (s.code != PIC_OK) {
        b->err = s.msg;
        if (s.code == PIC_EHIP || s.code == PIC_ESTATE) b->failed = true;
    }
    return s.code;
}

}  // namespace

#define BATCH_CHECK(b)                                        \
    do {                                                      \
        if (!(b)) return PIC_ESTATE;                          \
        if ((b)->failed || !(b)->eng) {                       \
            (b)->err = "batch is unusable after an error";    \
            return PIC_ESTATE;                                \
        }                                                     \
    } while (0)

extern "C" {

int pic_batch_init(int32_t nrun, const pic_config* cfgs, const pic_state* inits, int32_t autotune,
                   const pic_allocator* alloc, void* hip_stream, pic_batch** out) {
    g_init_error.clear();
    if (!out) {
        g_init_error = "out is NULL";
        return PIC_EINVAL;
    }
    *out = nullptr;
    if (nrun < 1 || nrun > 65535 || !cfgs || !inits) {
        g_init_error = "need 1 <= nrun <= 65535 (runs are a grid dimension of the field update) and non-NULL cfgs and inits";
        return PIC_EINVAL;
    }
    if (alloc && (!alloc->alloc || !alloc->free)) {
        g_init_error = "allocator needs both alloc and free";
        return PIC_EINVAL;
    }
    hipStream_t stream = (hipStream_t)hip_stream;
    std::vector<Resolved> Rs;
    Status S = batch_resolve(nrun, cfgs, inits, Rs);
    if (S.code) {
        g_init_error = S.msg;
        return S.code;
    }
    auto* b = new pic_batch();
    std::vector<int> tunable;
    for (int r = 0; r < nrun; ++r)
        if (autotune && cfgs[r].tile[0] == 0 && cfgs[r].tile[1] == 0) tunable.push_back(r);
    if (!tunable.empty()) {
        std::vector<pic_config> cc;
        autotune_tiles(nrun, cfgs, inits, tunable, alloc, stream, b, cc);
        S = batch_resolve(nrun, cc.data(), inits, Rs);
        if (S.code) {
            g_init_error = S.msg;
            delete b;
            return S.code;
        }
    }
    S = batch_build(Rs, inits, alloc, stream, b->eng);
    if (S.code) {
        g_init_error = S.msg;
        delete b;
        return S.code;
    }
    *out = b;
    return PIC_OK;
}

int pic_batch_step(pic_batch* b, int32_t nsteps) {
    BATCH_CHECK(b);
    if (nsteps < 0) {
        b->err = "nsteps must be >= 0";
        return PIC_EINVAL;
    }
    return batch_finish(b, b->eng->step(nsteps));
}

int pic_batch_polarization(pic_batch* b, int32_t run, int32_t species, double emin, double emax,
                           double P_out[3], int64_t* N_out) {
    BATCH_CHECK(b);
    if (!P_out || !N_out) {
        b->err = "P_out and N_out must not be NULL";
        return PIC_EINVAL;
    }
    return batch_finish(b, b->eng->polarization(run, species, emin, emax, P_out, N_out));
}

int pic_batch_fields(pic_batch* b, int32_t run, uint32_t mask, double* host_out, size_t cap_doubles) {
    BATCH_CHECK(b);
    return batch_finish(b, b->eng->fields(run, mask, host_out, cap_doubles));
}

int pic_batch_particles(pic_batch* b, int32_t run, int32_t species, double* host_out, size_t cap_doubles,
                        int64_t* n_out) {
    BATCH_CHECK(b);
    return batch_finish(b, b->eng->particles(run, species, host_out, cap_doubles, n_out));
}

int pic_batch_info(pic_batch* b, int32_t run, int64_t out[4]) {
    BATCH_CHECK(b);
    if (!out || run < 0 || run >= b->eng->nruns()) {
        b->err = "run out of range or out is NULL";
        return PIC_EINVAL;
    }
    b->eng->run_info(run, out);
    return PIC_OK;
}

int pic_batch_tuning(pic_batch* b, int32_t* cand_out, double* ns_out, double* kernel_ms_out, int32_t cap_cand,
                     int32_t* ncand_out) {
    BATCH_CHECK(b);
    const int nc = (int)b->cands.size();
    if (ncand_out) *ncand_out = nc;
    if (nc == 0) return PIC_OK;
    if (cap_cand < nc || !cand_out || !ns_out || !kernel_ms_out) {
        b->err = "cap_cand too small or NULL output";
        return PIC_EINVAL;
    }
    for (int i = 0; i < nc; ++i) cand_out[i] = b->cands[i];
    std::copy(b->tune.begin(), b->tune.end(), ns_out);
    std::copy(b->kernel_ms.begin(), b->kernel_ms.end(), kernel_ms_out);
    return PIC_OK;
}

int pic_batch_stats(pic_batch* b, int64_t* out, int32_t cap) {
    BATCH_CHECK(b);
    return batch_finish(b, b->eng->stats(out, cap));
}

int pic_batch_timing(pic_batch* b, int32_t enable) {
    BATCH_CHECK(b);
    return batch_finish(b, b->eng->timing(enable));
}

int pic_batch_timing_read(pic_batch* b, double* ms_out, int64_t* launches_out, int32_t cap) {
    BATCH_CHECK(b);
    return batch_finish(b, b->eng->timing_read(ms_out, launches_out, cap));
}

const char* pic_batch_last_error(const pic_batch* b) {
    if (!b) return g_init_error.c_str();
    return b->err.c_str();
}

void pic_batch_free(pic_batch* b) {
    delete b;
}

}  // extern "C"
