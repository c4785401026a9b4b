// picsar_hip.hip -- host engine and C ABI of the gfx950 PIC step.
//
// One context = one simulation on one GPU.  State lives in device memory
// for the life of the context: nine field planes in one padded layout, a
// second set of face-charge planes for the filter's ping-pong, two
// structure-of-arrays particle stores (the counting sort scatters from one
// into the other), metric tables built in FP64 on the host, and a few
// device counters (particle counts, step index, current buffer).
//
// A step is a fixed sequence of launches over a table of runs (Plan): a
// context steps a table of one, a batch steps the runs of many contexts
// with the same launches.  Without stage timing the sequence is captured
// once into a HIP graph and replayed; control returns to the host only at
// the end of pic_step / pic_batch_step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/picsar_hip.h"
#include "pic_device.h"
#include "pic_kernels.h"

using namespace pic;

// Device memory of the entry point that allocates nothing
// (pic_inject_particles_noalloc): the staging of at most
// kNoAllocMaxParticles particles -- six FP64 arrays and the uint64 ids -- on
// their way to the particle store.  Every GPU the library runs on holds one
// copy of it until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory: its address on each device is
// looked up once, with that device current (scratch_on, called by pic_init
// and pic_load), and only that address is used.
constexpr int64_t kNoAllocMaxParticles = 65536;
static __device__ __align__(256) double scratch[7 * kNoAllocMaxParticles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

struct HipError {
    hipError_t e;
    const char *what;
};

#define HIPCHK(expr)                                                                                                  \
    do {                                                                                                               \
        hipError_t e_ = (expr);                                                                                        \
        if (e_ != hipSuccess) throw HipError{e_, #expr};                                                               \
    } while (0)

struct StatusError {
    pic_status st;
    std::string msg;
};

template <typename U>
U *dev_alloc(size_t n)
{
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(U) * std::max<size_t>(n, 1)) != hipSuccess)
        throw StatusError{PIC_ENOMEM, "device allocation failed"};
    return (U *)p;
}

template <typename U>
void dev_fill(U *p, size_t n, U v, hipStream_t s)
{
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
    k_fill<U><<<std::max(blocks, 1), 256, 0, s>>>(p, n, v);
    HIPCHK(hipGetLastError());
}

// Device address of `scratch` on `device`, which must be current: looked up
// on the first call for the device and kept.
double *scratch_on(int device)
{
    if (device < 0 || device >= kMaxDevices) throw StatusError{PIC_EINVAL, "device index beyond the supported range"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch[device] = static_cast<double *>(p);
    }
    return g_scratch[device];
}

// The address scratch_on recorded for `device`, or null before it ran there.
double *scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[device];
}

// Per-stage device time from HIP events recorded between the launches of
// eagerly enqueued steps.
enum { kStSort = 0, kStFaraday, kStPush, kStFilter, kStAmpere, kStAbsorb, kStInject, kStZero, kStTotal, kStages };

class StageTimer {
public:
    ~StageTimer()
    {
        for (auto &e : pool_) (void)hipEventDestroy(e);
    }
    void begin(int n_steps)
    {
        const size_t need = (size_t)n_steps * kStages * 2;
        while (pool_.size() < need) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            pool_.push_back(e);
        }
        std::fill(used_, used_ + kStages, false);
        base_ = 0;
    }
    void next_step(int s) { base_ = (size_t)s * kStages * 2; }
    void mark(hipStream_t s, int q, bool start)
    {
        HIPCHK(hipEventRecord(pool_[base_ + 2 * q + (start ? 0 : 1)], s));
        used_[q] = true;
    }
    // mean per step over the n steps just enqueued (the stream must be idle)
    void finish(int n_steps, double *out)
    {
        for (int q = 0; q < kStages; ++q) {
            out[q] = 0.0;
            if (!used_[q] || n_steps <= 0) continue;
            for (int s = 0; s < n_steps; ++s) {
                float ms = 0.f;
                const size_t b = (size_t)s * kStages * 2 + 2 * q;
                HIPCHK(hipEventElapsedTime(&ms, pool_[b], pool_[b + 1]));
                out[q] += ms;
            }
            out[q] /= n_steps;
        }
    }

private:
    std::vector<hipEvent_t> pool_;
    size_t base_ = 0;
    bool used_[kStages] = {};
};

// ------------------------------------------------------------------
// Launch plan of one step over a table of runs
// ------------------------------------------------------------------
enum { kMapGrid = 0, kMapFilter, kMapAbsorb, kMapZero, kMapKeys, kMaps };

// The host's record of one run's sort schedule: its sort interval, the
// index of its next step and whether particles arrived since its last sort
// (the device counters kStep and kNeedSort, set alike by every host action
// that sets those, and advanced here step by step by the device's rule).
struct SortSched {
    int K;
    uint64_t *step;
    bool *need;
    bool due() const { return K > 0 && (*need || *step % (uint64_t)K == 0); }
    void advance(bool sorted) const
    {
        if (sorted && due()) *need = false;
        ++*step;
    }
};

template <typename T>
class Plan {
public:
    Plan() = default;
    Plan(const Plan &) = delete;
    Plan &operator=(const Plan &) = delete;
    ~Plan() { reset(); }

    void reset()
    {
        for (int g = 0; g < 2; ++g) {
            if (exec_[g]) (void)hipGraphExecDestroy(exec_[g]);
            if (graph_[g]) (void)hipGraphDestroy(graph_[g]);
            exec_[g] = nullptr;
            graph_[g] = nullptr;
        }
        if (cap_stream_) (void)hipStreamDestroy(cap_stream_);
        for (void *p : allocs_) (void)hipFree(p);
        cap_stream_ = nullptr;
        allocs_.clear();
    }

    // Work-group maps, grids and LDS size for these runs, and the table
    // (rebuilding drops the captured graph).
    void build(const std::vector<RunDev<T>> &rd, int ppt, hipStream_t s)
    {
        HIPCHK(hipStreamSynchronize(s));
        reset();
        n_ = (int)rd.size();
        ppt_ = ppt;
        runs_ = alloc<RunDev<T>>(n_);
        maps_ = alloc<int>((size_t)kMaps * (n_ + 1));
        chunk_off_ = alloc<unsigned long long>(n_ + 1);
        span_off_ = alloc<unsigned long long>(n_ + 1);
        work_ = alloc<unsigned int>(8);
        std::vector<int> h((size_t)kMaps * (n_ + 1), 0);
        long long cap_sum = 0, chunk_bound = 0;
        int max_cap = 0;
        const long long CH = 256LL * ppt_;
        for (int m = 0; m < kMaps; ++m) tot_[m] = 0;
        max_filt_ = 0;
        any_sort_ = false;
        for (int r = 0; r < n_; ++r) max_filt_ = std::max(max_filt_, rd[r].n_filt);
        // filter strips: 64 columns less a halo of H on each side, H the
        // filter kernel's build for the largest pass count
        const int fH = max_filt_ <= 2 ? 2 : (max_filt_ == 3 ? 3 : (max_filt_ <= 4 ? 4 : 8));
        const int fU = 64 - 2 * fH;
        for (int r = 0; r < n_; ++r) {
            const RunDev<T> &R = rd[r];
            const int nbx = (R.L.nth + 1 + 63) / 64;
            const int cnt[kMaps] = {
                nbx * ((R.L.nr + 1 + 4 * kFieldRows - 1) / (4 * kFieldRows)),
                R.n_filt > 0 ? ((R.L.nth + 1 + fU - 1) / fU * ((R.L.rows() + kFiltRB - 1) / kFiltRB) + 3) / 4 : 0,
                R.absorb_cells > 0 ? nbx * ((R.absorb_cells + 2 + 4 * kFieldRows - 1) / (4 * kFieldRows)) : 0,
                (int)((R.L.size() + 256 * kZeroPerThread - 1) / (256 * kZeroPerThread)),
                R.sort_interval > 0 ? (R.tm.n_keys + 1 + 255) / 256 : 0,
            };
            for (int m = 0; m < kMaps; ++m) {
                h[(size_t)m * (n_ + 1) + r] = tot_[m];
                tot_[m] += cnt[m];
            }
            any_sort_ = any_sort_ || R.sort_interval > 0;
            max_cap = std::max(max_cap, R.lds_cap);
            cap_sum += std::max<long long>(R.capacity, 1);
            chunk_bound += (std::max<long long>(R.capacity, 1) + CH - 1) / CH;
        }
        for (int m = 0; m < kMaps; ++m) h[(size_t)m * (n_ + 1) + n_] = tot_[m];
        HIPCHK(hipMemcpyAsync(maps_, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice, s));
        shm_ = max_cap > 0 ? lds_push_bytes<T>() : 0;
        if (shm_ > 0) {
            const int b = (int)shm_;
            HIPCHK(hipFuncSetAttribute((const void *)k_push<T, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, b));
            HIPCHK(hipFuncSetAttribute((const void *)k_push<T, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, b));
            HIPCHK(hipFuncSetAttribute((const void *)k_push<T, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, b));
        }
        // one wave per sort span (four per work-group); the kernels loop over
        // the spans of the step, so the grid only bounds the parallelism
        sort_blocks_ = (int)std::min<long long>(std::max<long long>((cap_sum + 4 * kSortSpan - 1) / (4 * kSortSpan), 1),
                                                4096);
        // the push work-groups fetch chunks until their XCD's range is done:
        // eight per CU at most, a multiple of eight
        push_grid_ = (int)std::max<long long>(8, std::min<long long>(8 * ((chunk_bound + 7) / 8), 8 * 256));
        upload(rd, s);
        HIPCHK(hipStreamSynchronize(s));
    }

    void upload(const std::vector<RunDev<T>> &rd, hipStream_t s) { upload(rd.data(), rd.size(), s); }
    // (no host allocation: the append that allocates nothing passes its one
    // run's entry directly)
    void upload(const RunDev<T> *rd, size_t n, hipStream_t s)
    {
        HIPCHK(hipMemcpyAsync(runs_, rd, sizeof(RunDev<T>) * n, hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }

    // n steps on stream s: eagerly with stage events when a timer is
    // given, else by replaying the captured graph of one step.  A step in
    // which no run sorts (by the host's record of each run's step index and
    // pending sort, which follows the device's rule) leaves the sort kernels
    // out and tells the step's bookkeeping that no run sorts; were the
    // record wrong, a sort would only come later, never half done.
    void run(int n, hipStream_t s, StageTimer *timer, const std::vector<SortSched> &sched)
    {
        if (n <= 0) return;
        if (timer) timer->begin(n);
        for (int q = 0; q < n; ++q) {
            bool sort = false;
            for (const SortSched &r : sched) sort = sort || r.due();
            sort = sort && any_sort_;
            if (timer) {
                timer->next_step(q);
                enqueue(s, timer, sort);
            } else {
                if (!exec_[sort]) capture(sort);
                HIPCHK(hipGraphLaunch(exec_[sort], s));
            }
            for (const SortSched &r : sched) r.advance(sort);
        }
    }

private:
    std::vector<void *> allocs_;
    int n_ = 0, ppt_ = 8, max_filt_ = 0;
    bool any_sort_ = false;
    RunDev<T> *runs_ = nullptr;
    int *maps_ = nullptr;
    int tot_[kMaps] = {};
    unsigned long long *chunk_off_ = nullptr, *span_off_ = nullptr;
    unsigned int *work_ = nullptr;
    size_t shm_ = 0;
    int sort_blocks_ = 1, push_grid_ = 8;
    hipStream_t cap_stream_ = nullptr;
    hipGraph_t graph_[2] = {};      // one step without, and with, the sort kernels
    hipGraphExec_t exec_[2] = {};

    template <typename U>
    U *alloc(size_t n)
    {
        U *p = dev_alloc<U>(n);
        allocs_.push_back(p);
        return p;
    }
    const int *map(int m) const { return maps_ + (size_t)m * (n_ + 1); }

    void capture(bool sort)
    {
        if (!cap_stream_) HIPCHK(hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(cap_stream_, hipStreamCaptureModeThreadLocal));
        try {
            enqueue(cap_stream_, nullptr, sort);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(cap_stream_, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        HIPCHK(hipStreamEndCapture(cap_stream_, &graph_[sort]));
        HIPCHK(hipGraphInstantiate(&exec_[sort], graph_[sort], nullptr, nullptr, 0));
    }

    void mark(StageTimer *t, hipStream_t s, int q, bool start)
    {
        if (t) t->mark(s, q, start);
    }

    // The launches of one step (order of Sec. 3 and App. A: half Faraday,
    // push and deposit, half Faraday, filter, Ampere, lossy layer, then
    // injection), preceded by the counting sort when `sort` is set (the
    // device then sorts the runs that are due).
    void enqueue(hipStream_t s, StageTimer *t, bool sort)
    {
        const dim3 blk2(64, 4);
        mark(t, s, kStTotal, true);
        // the sort stage is empty on a step without the sort kernels; the
        // opening kernel then also does the step's bookkeeping
        mark(t, s, kStSort, true);
        if (sort) {
            k_step_begin<T><<<1, 64, 0, s>>>(runs_, n_, kSortSpan, span_off_, 1);
            if (tot_[kMapKeys] > 0) k_sort_zero<T><<<tot_[kMapKeys], 256, 0, s>>>(runs_, n_, map(kMapKeys));
            k_sort_hist<T><<<sort_blocks_, 256, 0, s>>>(runs_, n_, span_off_);
            if (tot_[kMapKeys] > 0) k_sort_spans<T><<<tot_[kMapKeys], 256, 0, s>>>(runs_, n_, map(kMapKeys));
            k_sort_scan<T><<<n_, 1024, 0, s>>>(runs_);
            k_sort_scatter<T><<<sort_blocks_, 256, 0, s>>>(runs_, n_, span_off_);
            HIPCHK(hipGetLastError());
        }
        mark(t, s, kStSort, false);
        // the opening launch: bookkeeping and the cleared deposit planes beside
        // the first half Faraday update (timed as the Faraday stage; the
        // zeroing stage stays empty)
        mark(t, s, kStZero, true);
        mark(t, s, kStZero, false);
        mark(t, s, kStFaraday, true);
        {
            const int nz_pad = (tot_[kMapZero] + 7) / 8 * 8;
            k_open_faraday<T><<<nz_pad + tot_[kMapGrid], 256, 0, s>>>(runs_, n_, map(kMapZero), nz_pad, sort ? 0 : 1,
                                                                     kSortSpan, span_off_, 256 * ppt_, chunk_off_,
                                                                     work_, map(kMapGrid), tot_[kMapGrid], (T)0.5);
            HIPCHK(hipGetLastError());
        }
        mark(t, s, kStFaraday, false);
        mark(t, s, kStPush, true);
        if (ppt_ == 4) k_push<T, 4><<<push_grid_, 256, shm_, s>>>(runs_, n_, chunk_off_, work_);
        else if (ppt_ == 16) k_push<T, 16><<<push_grid_, 256, shm_, s>>>(runs_, n_, chunk_off_, work_);
        else k_push<T, 8><<<push_grid_, 256, shm_, s>>>(runs_, n_, chunk_off_, work_);
        HIPCHK(hipGetLastError());
        mark(t, s, kStPush, false);
        // the second half Faraday update beside the filter passes (timed as
        // the filter stage)
        mark(t, s, kStFilter, true);
        {
            const int nf = 3 * tot_[kMapFilter], nf_pad = (nf + 7) / 8 * 8, ng = tot_[kMapGrid];
            const int grid = nf_pad + ng;
            if (max_filt_ <= 2)
                k_faraday_filter<T, 2><<<grid, 256, 0, s>>>(runs_, n_, map(kMapFilter), nf, nf_pad, map(kMapGrid), ng,
                                                             (T)0.5);
            else if (max_filt_ == 3)
                k_faraday_filter<T, 3><<<grid, 256, 0, s>>>(runs_, n_, map(kMapFilter), nf, nf_pad, map(kMapGrid), ng,
                                                             (T)0.5);
            else if (max_filt_ <= 4)
                k_faraday_filter<T, 4><<<grid, 256, 0, s>>>(runs_, n_, map(kMapFilter), nf, nf_pad, map(kMapGrid), ng,
                                                             (T)0.5);
            else
                k_faraday_filter<T, 8><<<grid, 256, 0, s>>>(runs_, n_, map(kMapFilter), nf, nf_pad, map(kMapGrid), ng,
                                                             (T)0.5);
            HIPCHK(hipGetLastError());
        }
        mark(t, s, kStFilter, false);
        mark(t, s, kStAmpere, true);
        k_ampere<T><<<tot_[kMapGrid], blk2, 0, s>>>(runs_, n_, map(kMapGrid));
        HIPCHK(hipGetLastError());
        mark(t, s, kStAmpere, false);
        // injection and the lossy layer on B in one closing launch (its time
        // is reported as the injection stage; the absorb stage stays empty)
        mark(t, s, kStAbsorb, true);
        mark(t, s, kStAbsorb, false);
        mark(t, s, kStInject, true);
        k_close<T><<<n_ + (tot_[kMapAbsorb] + 3) / 4, 1024, 0, s>>>(runs_, n_, map(kMapAbsorb));
        HIPCHK(hipGetLastError());
        mark(t, s, kStInject, false);
        mark(t, s, kStTotal, false);
    }
};

// ------------------------------------------------------------------
// Geometry of the stretched coordinates (Sec. 3.2) and the area / line
// elements of App. A eq. (linearea), in FP64 on the host.
// ------------------------------------------------------------------
struct Geometry {
    int nr, nth, r_kind, th_kind;
    double r_in, r_out, dxi;

    double r(double x) const { return r_kind == PIC_R_LOG ? r_in * std::exp(x * dxi) : r_in + x * dxi; }
    double cth(double y) const
    {
        return th_kind == PIC_TH_EQAREA ? 1.0 - 2.0 * y / nth : std::cos(kPi * y / nth);
    }
    double sth(double y) const
    {
        if (th_kind == PIC_TH_EQAREA) return 2.0 / nth * std::sqrt(std::max(0.0, y * (nth - y)));
        return std::sin(kPi * y / nth);
    }
    double th(double y) const
    {
        if (th_kind == PIC_TH_EQAREA) return 2.0 * std::asin(std::sqrt(std::min(1.0, std::max(0.0, y / nth))));
        return kPi * y / nth;
    }
};

// Checkpoint file: this header, then the twelve field planes (E, B, the
// deposit planes, the filtered face charges; the padded device layout of
// field_elems entries each, in the context's precision), the injection carry
// (nth + 1 doubles), and the particle slots: cell indices (uint32), the six
// particle arrays (offsets, momenta, weight; the context's precision) and,
// with ids, the uint64 ids.
struct CkptHeader {
    char magic[8];
    uint32_t version;
    uint32_t real_bytes;
    pic_grid_desc grid;       // with the sort tile, interval and chunk size in use
    pic_phys_desc phys;
    uint64_t counters[kNumCounters];
    double qmax;              // largest |w| held: the fixed-point deposit scale
    uint64_t slots;           // particle slots written (live and deleted)
    uint64_t field_elems;     // entries per field plane
    uint32_t n_planes;
    uint32_t with_ids;
};
constexpr char kCkptMagic[8] = {'P', 'I', 'C', 'S', 'A', 'R', 'C', 'K'};
constexpr uint32_t kCkptVersion = 1;
constexpr uint32_t kCkptPlanes = 12;

inline void ck_write(FILE *f, const void *p, size_t bytes)
{
    if (bytes && std::fwrite(p, 1, bytes, f) != bytes) throw StatusError{PIC_EINVAL, "checkpoint write failed"};
}
inline void ck_read(FILE *f, void *p, size_t bytes)
{
    if (bytes && std::fread(p, 1, bytes, f) != bytes) throw StatusError{PIC_EINVAL, "checkpoint file truncated"};
}

class Engine {
public:
    virtual ~Engine() {}
    virtual void init() = 0;
    virtual void inject(int64_t n, const double *x, const double *y, const double *ur, const double *ut,
                        const double *up, const double *w, const uint64_t *id) = 0;
    virtual void inject_noalloc(int64_t n, const double *x, const double *y, const double *ur, const double *ut,
                                const double *up, const double *w, const uint64_t *id, double *scratch) = 0;
    virtual void step(int n) = 0;
    virtual void get_field(int comp, double *out) = 0;
    virtual void set_field(int comp, const double *in) = 0;
    virtual int64_t get_particles(double *x, double *y, double *ur, double *ut, double *up, double *w,
                                  uint64_t *id, int64_t cap) = 0;
    virtual int64_t get_cells(int32_t *ci, int32_t *cj, double *fx, double *fy, int64_t cap) = 0;
    virtual void counts(double *out) = 0;
    virtual void gauss(double *out) = 0;
    virtual void gauss_residual(double *out) = 0;
    virtual void rho_q(double *out) = 0;
    virtual void luminosity(double *out) = 0;
    // the state was changed from the host: the Gauss drift's reference lapses
    void gauss_unref() { gauss_ref_ = false; }
    bool gauss_ref_ = false;
    virtual void get_carry(double *out) = 0;
    virtual void set_carry(const double *in) = 0;
    virtual void set_step(int64_t step) = 0;
    virtual void stage_ms(double *out) = 0;
    virtual void set_sort(int tile_r, int tile_th, int sort_interval) = 0;
    virtual void get_sort(int32_t *out) const = 0;
    virtual double timed_steps(int n, double *psteps) = 0;
    // device status bits of the run (cleared on read)
    virtual int take_status() = 0;
    // checkpoint: the whole state to / from an open file (the header of a
    // restore has been read and checked by the caller)
    virtual void save(FILE *f) = 0;
    virtual void restore(FILE *f, const struct CkptHeader &h) = 0;

    pic_grid_desc gd{};
    pic_phys_desc ph{};
    hipStream_t stream = nullptr;
    bool timing = false;
    Layout L{};
    Geometry geo{};
    unsigned version = 0; // bumped whenever the run's table entry changes

    void field_shape(int comp, int32_t *rows, int32_t *cols, int32_t *row0) const
    {
        const int nr = gd.nr, nth = gd.nth, g = L.G;
        static const int half_r[9] = {1, 0, 0, 0, 1, 1, 1, 0, 0};
        static const int half_j[9] = {0, 1, 0, 1, 0, 1, 0, 1, 0};
        const int rr = half_r[comp] ? nr : nr + 1;
        if (rows) *rows = comp >= 6 ? rr + 2 * g : rr;
        if (cols) *cols = half_j[comp] ? nth : nth + 1;
        if (row0) *row0 = comp >= 6 ? -g : 0;
    }
};

void raise_status(int st, const std::string &where)
{
    if (st & 1) throw StatusError{PIC_ECFL, where + "a particle moved one cell or more in one step (CFL)"};
    if (st & 2) throw StatusError{PIC_ECAPACITY, where + "particle capacity exceeded by surface injection"};
    if (st & 4) throw StatusError{PIC_EDEVICE, where + "internal error: sort destination outside the particle store"};
}

template <typename T>
class EngineT final : public Engine {
public:
    ~EngineT() override
    {
        plan_.reset();
        for (void *p : allocs_) (void)hipFree(p);
        for (auto e : tev_)
            if (e) (void)hipEventDestroy(e);
    }

    void init() override
    {
        const int nr = gd.nr, nth = gd.nth;
        const int G = 2 * gd.n_filt + 3;
        L.nr = nr;
        L.nth = nth;
        L.G = G;
        L.pitch = ((nth + 1 + 15) / 16) * 16;
        geo.nr = nr;
        geo.nth = nth;
        geo.r_kind = gd.r_kind;
        geo.th_kind = gd.th_kind;
        geo.r_in = gd.r_in;
        geo.r_out = gd.r_out;
        geo.dxi = gd.r_kind == PIC_R_LOG ? std::log(gd.r_out / gd.r_in) / nr : (gd.r_out - gd.r_in) / nr;
        cap_ = gd.particle_capacity;
        if (ph.inject) qmax_ = std::fabs(ph.q_inj);
        with_ids_ = (gd.flags & PIC_FLAG_IDS) != 0;
        ppt_ = gd.chunk_ppt > 0 ? gd.chunk_ppt : 8;

        RunDev<T> &R = rd_;
        R = RunDev<T>{};
        R.L = L;
        const size_t fsz = L.size();
        for (int c = 0; c < 9; ++c) {
            fld_[c] = dalloc<T>(fsz);
            fill(fld_[c], fsz, (T)0);
            R.fld[c] = fld_[c];
        }
        for (int c = 0; c < 3; ++c) {
            ftmp_[c] = dalloc<T>(fsz);
            fill(ftmp_[c], fsz, (T)0);
            R.ftmp[c] = ftmp_[c];
            // the filter writes the second set of planes
            R.ffin[c] = gd.n_filt > 0 ? ftmp_[c] : fld_[6 + c];
        }
        build_tables();
        R.m = m_;
        R.r_push = r_push_;
        R.bg = Background{ph.bg_kind, ph.B0, gd.r_in};
        R.r_kind = gd.r_kind;
        R.th_kind = gd.th_kind;
        R.mover = gd.mover;
        R.n_filt = gd.n_filt;
        R.absorb_cells = std::min(gd.absorb_cells, nr);
        R.c = (T)gd.c;
        R.dxi = (T)geo.dxi;
        R.inv_dxi = (T)(1.0 / geo.dxi);
        R.nth_f = (T)nth;
        R.two_over_nth = (T)(2.0 / nth);
        R.pi_over_nth = (T)(kPi / nth);
        R.inv_pi_over_nth = (T)(nth / kPi);
        R.eps0 = (T)(ph.q_over_m / (2.0 * gd.c));
        R.omega = ph.omega;
        R.t_spin = ph.t_spin;
        R.cd = gd.c;
        for (int s = 0; s < 2; ++s) {
            // one push chunk of spare slots past the capacity takes the
            // loads and stores of lanes past the last particle
            cell_[s] = dalloc<uint32_t>(cap_ + kMaxChunk);
            R.cell[s] = cell_[s];
            for (int a = 0; a < 6; ++a) {
                arr_[s][a] = dalloc<T>(cap_ + kMaxChunk);
                R.arr[s][a] = arr_[s][a];
            }
            id_[s] = with_ids_ ? dalloc<uint64_t>(cap_ + kMaxChunk) : nullptr;
            R.id[s] = id_[s];
        }
        R.capacity = cap_;
        ctr_ = dalloc<unsigned long long>(kNumCounters);
        fill(ctr_, kNumCounters, 0ull);
        fill(ctr_ + kNeedSort, 1, 1ull); // the first step sorts
        sched_step_ = 0;
        sched_need_ = true;
        R.ctr = ctr_;
        status_ = dalloc<int>(1);
        fill(status_, 1, 0);
        R.status = status_;
        sort_state(gd.tile_r > 0 ? gd.tile_r : 8, gd.tile_th > 0 ? gd.tile_th : 8,
                   gd.sort_interval == 0 ? 4 : gd.sort_interval);
        set_dep_scale();
        R.inject = ph.inject && (ph.bg_kind == PIC_BG_MONOPOLE || ph.bg_kind == PIC_BG_DIPOLE);
        R.kn = dkn_;
        R.sn = dsn_;
        R.Aj = dAj_;
        R.rb0 = rb0_;
        R.f_inj = ph.f_inj;
        R.q_inj = ph.q_inj;
        carry_ = dalloc<double>(nth + 1);
        fill(carry_, (size_t)nth + 1, 0.0);
        R.carry = carry_;
        R.seed = ph.seed;
        // diagnostic planes, allocated once: node charge, its filter
        // ping-pong and the absolute charge (padded layout), the E flux and
        // the reference residual ((nr + 1) x (nth + 1)), the per-work-group
        // partial reductions, their total, and the luminosity per sphere
        const size_t nodes = (size_t)(nr + 1) * (nth + 1);
        gauss_grid_x_ = (nth + 1 + 63) / 64;
        gauss_grid_y_ = (nr + 1 + 3) / 4;
        grho_ = dalloc<double>(fsz);
        gtmp_ = dalloc<double>(fsz);
        gabs_ = dalloc<double>(fsz);
        fill(gtmp_, fsz, 0.0);
        gG_ = dalloc<double>(nodes);
        gR0_ = dalloc<double>(nodes);
        gparts_ = dalloc<double>((size_t)gauss_grid_x_ * gauss_grid_y_ * kGaussParts);
        gout_ = dalloc<double>(kGaussParts);
        gL_ = dalloc<double>((size_t)nr);
        gauss_ref_ = false;
        plan_.build({rd_}, ppt_, stream);
    }

    const RunDev<T> &run_desc() const { return rd_; }
    int ppt() const { return ppt_; }
    // this run's sort schedule as the host records it (see SortSched)
    SortSched sched() { return SortSched{rd_.sort_interval, &sched_step_, &sched_need_}; }

    // Checks of an append of n particles from the host (positions inside the
    // grid, finite momenta and weights, room in the store); returns the first
    // slot they take and the current buffer, and raises the largest |w| held
    // (the deposit's fixed-point scale, which a non-finite weight would void).
    unsigned long long inject_begin(int64_t n, const double *x, const double *y, const double *ur,
                                    const double *ut, const double *up, const double *w, int &cur)
    {
        const int nr = gd.nr, nth = gd.nth;
        const double lim = gd.n_filt + 1.0;
        for (int64_t q = 0; q < n; ++q) {
            if (!(x[q] >= -lim && x[q] <= nr + lim && y[q] >= 0.0 && y[q] <= nth))
                throw StatusError{PIC_EINVAL, "particle position outside the grid"};
            if (!(std::isfinite(ur[q]) && std::isfinite(ut[q]) && std::isfinite(up[q]) && std::isfinite(w[q])))
                throw StatusError{PIC_EINVAL, "non-finite particle momentum or weight"};
        }
        unsigned long long c[kNumCounters];
        read_counters(c);
        const unsigned long long ntot = c[kTotal];
        cur = (int)c[kCur];
        if ((int64_t)ntot + n > cap_) throw StatusError{PIC_ECAPACITY, "particle capacity exceeded"};
        for (int64_t q = 0; q < n; ++q) qmax_ = std::max(qmax_, std::fabs(w[q]));
        return ntot;
    }

    // Cell + offset conversion of m staged particles (stage: six arrays of m
    // doubles; sid: m ids or null) into slots at..at+m-1.
    void inject_load(const double *stage, const uint64_t *sid, int64_t m, unsigned long long at, int cur)
    {
        const int blocks = (int)std::min<int64_t>((m + 255) / 256, 4096);
        k_load<T><<<blocks, 256, 0, stream>>>(stage, sid, m, (long long)at, gd.nth, cell_[cur], arr_[cur][0],
                                              arr_[cur][1], arr_[cur][2], arr_[cur][3], arr_[cur][4], arr_[cur][5],
                                              id_[cur]);
        HIPCHK(hipGetLastError());
    }

    // The new particle count, a sort at the next step, the deposit scale.
    void inject_end(int64_t n, unsigned long long ntot)
    {
        const unsigned long long upd[2] = {ntot + n, 1ull};
        HIPCHK(hipMemcpyAsync(ctr_ + kTotal, &upd[0], sizeof(unsigned long long), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(ctr_ + kNeedSort, &upd[1], sizeof(unsigned long long), hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));
        sched_need_ = true;
        gauss_unref();
        if (set_dep_scale()) {
            plan_.upload(&rd_, 1, stream);
            ++version;
        }
    }

    void inject(int64_t n, const double *x, const double *y, const double *ur, const double *ut, const double *up,
                const double *w, const uint64_t *id) override
    {
        if (n == 0) return;
        int cur = 0;
        const unsigned long long ntot = inject_begin(n, x, y, ur, ut, up, w, cur);
        const int64_t chunk = 1 << 22;
        double *stage = dev_alloc<double>(6 * (size_t)std::min(n, chunk));
        uint64_t *sid = id ? dev_alloc<uint64_t>((size_t)std::min(n, chunk)) : nullptr;
        std::vector<double> hb;
        try {
            for (int64_t o = 0; o < n; o += chunk) {
                const int64_t m = std::min(chunk, n - o);
                hb.resize(6 * (size_t)m);
                const double *srcs[6] = {x, y, ur, ut, up, w};
                for (int a = 0; a < 6; ++a) std::memcpy(&hb[(size_t)a * m], srcs[a] + o, sizeof(double) * m);
                HIPCHK(hipMemcpyAsync(stage, hb.data(), sizeof(double) * 6 * m, hipMemcpyHostToDevice, stream));
                if (sid) HIPCHK(hipMemcpyAsync(sid, id + o, sizeof(uint64_t) * m, hipMemcpyHostToDevice, stream));
                inject_load(stage, sid, m, ntot + o, cur);
                HIPCHK(hipStreamSynchronize(stream));
            }
        } catch (...) {
            (void)hipStreamSynchronize(stream);
            (void)hipFree(stage);
            if (sid) (void)hipFree(sid);
            throw;
        }
        HIPCHK(hipStreamSynchronize(stream));
        HIPCHK(hipFree(stage));
        if (sid) HIPCHK(hipFree(sid));
        inject_end(n, ntot);
    }

    // The same append staged through caller-free device memory: the seven
    // arrays are copied straight from the caller's buffers into `scratch`
    // (room for kNoAllocMaxParticles particles), then converted in place.
    void inject_noalloc(int64_t n, const double *x, const double *y, const double *ur, const double *ut,
                        const double *up, const double *w, const uint64_t *id, double *scratch) override
    {
        if (n == 0) return;
        int cur = 0;
        const unsigned long long ntot = inject_begin(n, x, y, ur, ut, up, w, cur);
        const double *srcs[6] = {x, y, ur, ut, up, w};
        for (int a = 0; a < 6; ++a)
            HIPCHK(hipMemcpyAsync(scratch + (size_t)a * n, srcs[a], sizeof(double) * n, hipMemcpyHostToDevice,
                                  stream));
        uint64_t *sid = id ? reinterpret_cast<uint64_t *>(scratch + 6 * (size_t)n) : nullptr;
        if (sid) HIPCHK(hipMemcpyAsync(sid, id, sizeof(uint64_t) * n, hipMemcpyHostToDevice, stream));
        inject_load(scratch, sid, n, ntot, cur);
        HIPCHK(hipStreamSynchronize(stream));
        inject_end(n, ntot);
    }

    void step(int n) override
    {
        plan_.run(n, stream, timing ? &timer_ : nullptr, {sched()});
        HIPCHK(hipStreamSynchronize(stream));
        if (timing && n > 0) timer_.finish(n, stage_ms_);
        raise_status(take_status(), "");
    }

    int take_status() override
    {
        int st = 0;
        HIPCHK(hipMemcpyAsync(&st, status_, sizeof st, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        if (st) {
            fill(status_, 1, 0);
            HIPCHK(hipStreamSynchronize(stream));
        }
        return st;
    }

    void get_field(int comp, double *out) override
    {
        int32_t rows, cols, row0;
        field_shape(comp, &rows, &cols, &row0);
        const T *src = comp < 6 ? fld_[comp] : rd_.ffin[comp - 6];
        std::vector<T> h(L.size());
        HIPCHK(hipMemcpyAsync(h.data(), src, sizeof(T) * h.size(), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        for (int r = 0; r < rows; ++r)
            for (int cc = 0; cc < cols; ++cc) out[(size_t)r * cols + cc] = (double)h[L.at(row0 + r, cc)];
    }

    void set_field(int comp, const double *in) override
    {
        int32_t rows, cols, row0;
        field_shape(comp, &rows, &cols, &row0);
        std::vector<T> h(L.size(), (T)0);
        for (int r = 0; r < rows; ++r)
            for (int cc = 0; cc < cols; ++cc) h[L.at(row0 + r, cc)] = (T)in[(size_t)r * cols + cc];
        HIPCHK(hipMemcpyAsync(fld_[comp], h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));
        gauss_unref();
    }

    int64_t get_particles(double *x, double *y, double *ur, double *ut, double *up, double *w, uint64_t *id,
                          int64_t cap) override
    {
        unsigned long long c[kNumCounters];
        read_counters(c);
        const unsigned long long ntot = c[kTotal];
        const int cur = (int)c[kCur];
        std::vector<uint32_t> hc(ntot);
        HIPCHK(hipMemcpyAsync(hc.data(), cell_[cur], sizeof(uint32_t) * ntot, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        int64_t live = 0;
        for (auto cl : hc) live += cl != kDead;
        if (live > cap) return -live;
        std::vector<T> ha(ntot);
        double *outs[6] = {x, y, ur, ut, up, w};
        for (int a = 0; a < 6; ++a) {
            if (!outs[a]) continue;
            HIPCHK(hipMemcpyAsync(ha.data(), arr_[cur][a], sizeof(T) * ntot, hipMemcpyDeviceToHost, stream));
            HIPCHK(hipStreamSynchronize(stream));
            int64_t m = 0;
            for (size_t q = 0; q < ntot; ++q) {
                if (hc[q] == kDead) continue;
                double v = (double)ha[q];
                if (a == 0) v += cell_i(hc[q]);
                if (a == 1) v += cell_j(hc[q]);
                outs[a][m++] = v;
            }
        }
        if (id) {
            std::vector<uint64_t> hi(ntot);
            if (with_ids_) {
                HIPCHK(hipMemcpyAsync(hi.data(), id_[cur], sizeof(uint64_t) * ntot, hipMemcpyDeviceToHost, stream));
                HIPCHK(hipStreamSynchronize(stream));
            }
            int64_t m = 0;
            for (size_t q = 0; q < ntot; ++q)
                if (hc[q] != kDead) id[m++] = with_ids_ ? hi[q] : (uint64_t)q;
        }
        return live;
    }

    int64_t get_cells(int32_t *ci, int32_t *cj, double *fx, double *fy, int64_t cap) override
    {
        unsigned long long c[kNumCounters];
        read_counters(c);
        const unsigned long long ntot = c[kTotal];
        const int cur = (int)c[kCur];
        std::vector<uint32_t> hc(ntot);
        HIPCHK(hipMemcpyAsync(hc.data(), cell_[cur], sizeof(uint32_t) * ntot, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        int64_t live = 0;
        for (auto cl : hc) live += cl != kDead;
        if (live > cap) return -live;
        int64_t m = 0;
        for (size_t q = 0; q < ntot; ++q) {
            if (hc[q] == kDead) continue;
            if (ci) ci[m] = cell_i(hc[q]);
            if (cj) cj[m] = cell_j(hc[q]);
            ++m;
        }
        std::vector<T> ha(ntot);
        double *outs[2] = {fx, fy};
        for (int a = 0; a < 2; ++a) {
            if (!outs[a]) continue;
            HIPCHK(hipMemcpyAsync(ha.data(), arr_[cur][a], sizeof(T) * ntot, hipMemcpyDeviceToHost, stream));
            HIPCHK(hipStreamSynchronize(stream));
            m = 0;
            for (size_t q = 0; q < ntot; ++q)
                if (hc[q] != kDead) outs[a][m++] = (double)ha[q];
        }
        return live;
    }

    void counts(double *out) override
    {
        unsigned long long c[kNumCounters];
        read_counters(c);
        out[0] = (double)(c[kTotal] - c[kDeadSinceSort]);
        out[1] = (double)c[kInjected];
        out[2] = (double)c[kDeleted] + (double)c[kDeadSinceSort];
        out[3] = (double)c[kStep];
        out[4] = (double)c[kPartSteps];
        out[5] = (double)c[kGlobalChunks];
    }

    // The filtered bilinear node charge of the particles (and their
    // unfiltered absolute charge) in the persistent diagnostic planes;
    // returns the plane that holds the filtered charge.
    const double *charge_planes()
    {
        const size_t fsz = L.size();
        fill(grho_, fsz, 0.0);
        fill(gabs_, fsz, 0.0);
        const double qm = qmax_ > 0.0 ? qmax_ : 1.0;
        const int spans = (int)((cap_ + kNodeSpan - 1) / kNodeSpan);
        const NodeSrc<T> src{{cell_[0], cell_[1]}, {arr_[0][0], arr_[1][0]}, {arr_[0][1], arr_[1][1]},
                             {arr_[0][5], arr_[1][5]}, ctr_};
        k_node_charge<T><<<std::max(spans, 1), 256, 0, stream>>>(src, L, std::ldexp(1.0, 50) / qm,
                                                                qm * std::ldexp(1.0, -50), grho_, gabs_);
        HIPCHK(hipGetLastError());
        double *a = grho_, *b = gtmp_;
        const dim3 blk(64, 4), fg((gd.nth + 1 + 63) / 64, (L.rows() + 3) / 4);
        for (int pss = 0; pss < gd.n_filt; ++pss) {
            k_filter_nodes<double><<<fg, blk, 0, stream>>>(a, b, L);
            HIPCHK(hipGetLastError());
            std::swap(a, b);
        }
        return a;
    }

    // Gauss residual R = G - Qbar with its FP64 reductions on the device; the
    // first evaluation after the state was set from the host records R as
    // the reference R0 of the drift.  Returns the filtered charge plane.
    const double *gauss_eval()
    {
        const double *q = charge_planes();
        const dim3 blk(64, 4), grd(gauss_grid_x_, gauss_grid_y_);
        k_gauss_flux<T><<<grd, blk, 0, stream>>>(fld_[cER], fld_[cETH], L, gA_r_, gdkb_, gA_t_, gsb_, q, gabs_, gG_,
                                                 gR0_, gauss_ref_ ? 0 : 1, std::max(gd.nr - 1 - rd_.absorb_cells, 0),
                                                 gparts_);
        HIPCHK(hipGetLastError());
        k_gauss_final<<<1, 256, 0, stream>>>(gparts_, gauss_grid_x_ * gauss_grid_y_, gout_);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(gauss_last_, gout_, sizeof gauss_last_, hipMemcpyDeviceToHost, stream));
        if (!gauss_ref_) gauss_ref_step_ = (double)read_step();
        gauss_ref_ = true;
        return q;
    }

    void gauss(double *out) override
    {
        const double *q = gauss_eval();
        const size_t N = (size_t)(gd.nr + 1) * (gd.nth + 1);
        HIPCHK(hipMemcpyAsync(out, gG_, sizeof(double) * N, hipMemcpyDeviceToHost, stream));
        copy_node_plane(q, out + N);
        HIPCHK(hipStreamSynchronize(stream));
        if (gauss_last_[kGpNonFinite] > 0.0)
            throw StatusError{PIC_ENAN, "non-finite value in the Gauss diagnostic (E or particle charge)"};
    }

    void gauss_residual(double *out) override
    {
        gauss_eval();
        HIPCHK(hipStreamSynchronize(stream));
        for (int q = 0; q < kGaussParts; ++q) out[q] = gauss_last_[q];
        out[kGaussParts] = gauss_ref_step_;
        if (gauss_last_[kGpNonFinite] > 0.0)
            throw StatusError{PIC_ENAN, "non-finite value in the Gauss diagnostic (E or particle charge)"};
    }

    void rho_q(double *out) override
    {
        const double *q = charge_planes();
        copy_node_plane(q, out);
        HIPCHK(hipStreamSynchronize(stream));
    }

    void luminosity(double *out) override
    {
        const double t = (double)read_step();
        k_poynting<T><<<gd.nr, 256, 0, stream>>>(fld_[cETH], fld_[cEPH], fld_[cBTH], fld_[cBPH], L, rd_.bg,
                                                 inv_light_cylinder(ph.omega, ph.t_spin, gd.c, t), gd.c, grb_,
                                                 gA_r_, gkc_, gsb_, gdk_, gL_);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(out, gL_, sizeof(double) * gd.nr, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        for (int i = 0; i < gd.nr; ++i)
            if (!std::isfinite(out[i])) throw StatusError{PIC_ENAN, "non-finite value in the Poynting luminosity"};
    }

    void get_carry(double *out) override
    {
        HIPCHK(hipMemcpyAsync(out, carry_, sizeof(double) * (gd.nth + 1), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
    }

    void set_carry(const double *in) override
    {
        HIPCHK(hipMemcpyAsync(carry_, in, sizeof(double) * (gd.nth + 1), hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));
    }

    void set_step(int64_t step) override
    {
        const unsigned long long v = (unsigned long long)step;
        HIPCHK(hipMemcpyAsync(ctr_ + kStep, &v, sizeof v, hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));
        sched_step_ = v;
    }

    void stage_ms(double *out) override { std::memcpy(out, stage_ms_, sizeof stage_ms_); }

    // New sort tile and interval for a live run: new key arrays and LDS
    // plane size, a sort at the next step, a new launch plan.
    void set_sort(int tile_r, int tile_th, int sort_interval) override
    {
        HIPCHK(hipStreamSynchronize(stream));
        sort_state(tile_r, tile_th, sort_interval);
        fill(ctr_ + kNeedSort, 1, 1ull);
        sched_need_ = true;
        plan_.build({rd_}, ppt_, stream);
        ++version;
    }

    void get_sort(int32_t *out) const override
    {
        out[0] = rd_.tm.tile_r;
        out[1] = rd_.tm.tile_th;
        out[2] = rd_.sort_interval;
    }

    // device array -> file, through a host buffer of at most 16M entries
    template <typename U>
    void dump(FILE *f, const U *d, size_t n)
    {
        std::vector<U> h(std::min<size_t>(n, (size_t)1 << 24));
        for (size_t o = 0; o < n; o += h.size()) {
            const size_t m = std::min(h.size(), n - o);
            HIPCHK(hipMemcpyAsync(h.data(), d + o, sizeof(U) * m, hipMemcpyDeviceToHost, stream));
            HIPCHK(hipStreamSynchronize(stream));
            ck_write(f, h.data(), sizeof(U) * m);
        }
    }
    // file -> device array; `check(values, count, first index)` sees every
    // chunk on the host before it is uploaded
    template <typename U, typename F>
    void undump(FILE *f, U *d, size_t n, F check)
    {
        std::vector<U> h(std::min<size_t>(n, (size_t)1 << 24));
        for (size_t o = 0; o < n; o += h.size()) {
            const size_t m = std::min(h.size(), n - o);
            ck_read(f, h.data(), sizeof(U) * m);
            check(h.data(), m, o);
            HIPCHK(hipMemcpyAsync(d + o, h.data(), sizeof(U) * m, hipMemcpyHostToDevice, stream));
            HIPCHK(hipStreamSynchronize(stream));
        }
    }
    template <typename U>
    void undump(FILE *f, U *d, size_t n)
    {
        undump(f, d, n, [](const U *, size_t, size_t) {});
    }

    void save(FILE *f) override
    {
        HIPCHK(hipStreamSynchronize(stream));
        unsigned long long c[kNumCounters];
        read_counters(c);
        CkptHeader h{};
        std::memcpy(h.magic, kCkptMagic, sizeof h.magic);
        h.version = kCkptVersion;
        h.real_bytes = sizeof(T);
        h.grid = gd;
        h.grid.tile_r = rd_.tm.tile_r;
        h.grid.tile_th = rd_.tm.tile_th;
        h.grid.sort_interval = rd_.sort_interval;
        h.grid.chunk_ppt = ppt_;
        h.phys = ph;
        for (int k = 0; k < kNumCounters; ++k) h.counters[k] = c[k];
        h.qmax = qmax_;
        h.slots = c[kTotal];
        h.field_elems = L.size();
        h.n_planes = kCkptPlanes;
        h.with_ids = with_ids_ ? 1u : 0u;
        ck_write(f, &h, sizeof h);
        for (int q = 0; q < 9; ++q) dump(f, fld_[q], L.size());
        for (int q = 0; q < 3; ++q) dump(f, ftmp_[q], L.size());
        dump(f, carry_, (size_t)gd.nth + 1);
        const int cur = (int)c[kCur];
        dump(f, cell_[cur], h.slots);
        for (int a = 0; a < 6; ++a) dump(f, arr_[cur][a], h.slots);
        if (with_ids_) dump(f, id_[cur], h.slots);
    }

    // state of a fresh context (just initialised from the header's
    // descriptors) from the rest of the file
    void restore(FILE *f, const CkptHeader &h) override
    {
        if (h.field_elems != L.size() || h.n_planes != kCkptPlanes || h.real_bytes != sizeof(T) ||
            h.with_ids != (with_ids_ ? 1u : 0u))
            throw StatusError{PIC_EINVAL, "checkpoint does not match its own descriptors"};
        if ((int64_t)h.slots > cap_) throw StatusError{PIC_ECAPACITY, "checkpoint holds more particles than the capacity"};
        if (h.counters[kTotal] != h.slots || h.counters[kDeadSinceSort] > h.slots || h.counters[kLive] > h.slots ||
            h.counters[kCur] > 1 || !(h.qmax >= 0.0))
            throw StatusError{PIC_EINVAL, "checkpoint counters are inconsistent"};
        auto finite = [](const char *what) {
            return [what](const auto *v, size_t m, size_t) {
                for (size_t q = 0; q < m; ++q)
                    if (!std::isfinite((double)v[q]))
                        throw StatusError{PIC_EINVAL, std::string("checkpoint holds a non-finite ") + what};
            };
        };
        for (int q = 0; q < 9; ++q) undump(f, fld_[q], L.size(), finite("field value"));
        for (int q = 0; q < 3; ++q) undump(f, ftmp_[q], L.size(), finite("face charge"));
        undump(f, carry_, (size_t)gd.nth + 1, finite("injection carry"));
        // the kernels index fields and LDS by these: every cell must lie where
        // a particle may be, every offset inside its cell
        const int lim = gd.n_filt + 1, nr = gd.nr, nth = gd.nth;
        std::vector<uint8_t> last_row; // an offset of 1 in y belongs to the last row (or a deleted slot)
        last_row.reserve(h.slots);
        undump(f, cell_[0], h.slots, [&](const uint32_t *c, size_t m, size_t) {
            for (size_t q = 0; q < m; ++q) {
                const bool ok = c[q] == kDead || (cell_i(c[q]) >= -lim && cell_i(c[q]) <= nr + lim &&
                                                  cell_j(c[q]) >= 0 && cell_j(c[q]) <= nth - 1);
                if (!ok) throw StatusError{PIC_EINVAL, "checkpoint cell index out of range"};
                last_row.push_back(c[q] == kDead || cell_j(c[q]) == nth - 1);
            }
        });
        undump(f, arr_[0][0], h.slots, [&](const T *v, size_t m, size_t) {
            for (size_t q = 0; q < m; ++q)
                if (!(v[q] >= (T)0 && v[q] < (T)1)) throw StatusError{PIC_EINVAL, "checkpoint offset out of range"};
        });
        undump(f, arr_[0][1], h.slots, [&](const T *v, size_t m, size_t o) {
            for (size_t q = 0; q < m; ++q)
                if (!(v[q] >= (T)0 && (v[q] < (T)1 || (v[q] == (T)1 && last_row[o + q]))))
                    throw StatusError{PIC_EINVAL, "checkpoint offset out of range"};
        });
        for (int a = 2; a < 5; ++a) undump(f, arr_[0][a], h.slots, finite("momentum"));
        // the fixed-point deposit is scaled by the largest |w| the header
        // records (that of the FP64 weights as given, which an FP32 store
        // holds rounded to within 2^-24): every weight must lie within it
        undump(f, arr_[0][5], h.slots, [&](const T *v, size_t m, size_t) {
            for (size_t q = 0; q < m; ++q)
                if (!(std::fabs((double)v[q]) <= h.qmax * (1.0 + 0x1p-23)))
                    throw StatusError{PIC_EINVAL, "checkpoint weight non-finite or above its recorded maximum"};
        });
        if (with_ids_) undump(f, id_[0], h.slots);
        unsigned long long c[kNumCounters];
        for (int k = 0; k < kNumCounters; ++k) c[k] = h.counters[k];
        c[kCur] = 0;
        HIPCHK(hipMemcpyAsync(ctr_, c, sizeof c, hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));
        sched_step_ = c[kStep];
        sched_need_ = c[kNeedSort] != 0;
        qmax_ = h.qmax;
        if (set_dep_scale()) {
            plan_.upload(&rd_, 1, stream);
            ++version;
        }
    }

    // n steps replayed from the graph; device time in ms between HIP events
    // around them, and the particle-steps they advanced
    double timed_steps(int n, double *psteps) override
    {
        if (!tev_[0]) {
            HIPCHK(hipEventCreate(&tev_[0]));
            HIPCHK(hipEventCreate(&tev_[1]));
        }
        unsigned long long c0[kNumCounters], c1[kNumCounters];
        read_counters(c0);
        HIPCHK(hipEventRecord(tev_[0], stream));
        plan_.run(n, stream, nullptr, {sched()});
        HIPCHK(hipEventRecord(tev_[1], stream));
        HIPCHK(hipStreamSynchronize(stream));
        raise_status(take_status(), "");
        read_counters(c1);
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, tev_[0], tev_[1]));
        if (psteps) *psteps = (double)(c1[kPartSteps] - c0[kPartSteps]);
        return ms;
    }

private:
    hipEvent_t tev_[2] = {};

    void sort_state(int tile_r, int tile_th, int sort_interval)
    {
        RunDev<T> &R = rd_;
        for (void *p : {(void *)counts_, (void *)cursor_, (void *)offsets_, (void *)nspan_, (void *)slist_,
                        (void *)sbefore_}) dfree(p);
        // sort tiles over rows -G..nr+G
        const int ntr = (L.rows() + tile_r - 1) / tile_r;
        const int ntj = (L.nth + tile_th - 1) / tile_th;
        R.tm = TileMap{L.G, tile_r, tile_th, ntj, ntr * ntj, 1.0f / (float)tile_r, 1.0f / (float)tile_th};
        R.sort_interval = sort_interval;
        counts_ = dalloc<unsigned int>(R.tm.n_keys + 1);
        cursor_ = dalloc<unsigned int>(R.tm.n_keys + 1);
        offsets_ = dalloc<unsigned long long>(R.tm.n_keys + 1);
        nspan_ = dalloc<unsigned int>(R.tm.n_keys + 1);
        slist_ = dalloc<SpanEnt>((size_t)(R.tm.n_keys + 1) * kSpanList);
        sbefore_ = dalloc<unsigned int>((size_t)(R.tm.n_keys + 1) * kSpanList);
        R.counts = counts_;
        R.cursor = cursor_;
        R.offsets = offsets_;
        R.nspan = nspan_;
        R.slist = slist_;
        R.sbefore = sbefore_;
        // LDS plane size: a chunk spans at most two neighbouring tiles (serpentine
        // order), widened by the drift since the last sort (at most ~0.7 cell
        // per step in grid units) and the stencil halo (one cell below, two above)
        const int drift = sort_interval > 0 ? (7 * sort_interval + 9) / 10 : 0;
        const int Rr = 2 * tile_r + 2 * drift + 3, Cc = 2 * tile_th + 2 * drift + 3;
        R.lds_cap = sort_interval > 0 ? std::min(Rr * Cc, lds_plane<T>()) : 0;
    }


    std::vector<void *> allocs_;
    RunDev<T> rd_{};
    Plan<T> plan_;
    StageTimer timer_;
    int ppt_ = 8;
    T *fld_[9] = {};
    T *ftmp_[3] = {};
    uint32_t *cell_[2] = {};
    T *arr_[2][6] = {};
    uint64_t *id_[2] = {};
    unsigned long long *ctr_ = nullptr;
    int *status_ = nullptr;
    double *carry_ = nullptr;
    unsigned int *counts_ = nullptr, *cursor_ = nullptr, *nspan_ = nullptr;
    unsigned long long *offsets_ = nullptr;
    SpanEnt *slist_ = nullptr;
    unsigned int *sbefore_ = nullptr;
    int64_t cap_ = 0;
    uint64_t sched_step_ = 0; // the device's kStep and kNeedSort, as every host action and step sets them
    bool sched_need_ = true;
    double qmax_ = 0.0; // largest |w| held so far: sets the fixed-point deposit scale
    bool with_ids_ = false;
    Metric m_{};
    const T *r_push_ = nullptr;
    const double *dkn_ = nullptr, *dsn_ = nullptr, *dAj_ = nullptr;
    const double *gA_r_ = nullptr, *gdkb_ = nullptr, *gA_t_ = nullptr, *gsb_ = nullptr;
    const double *grb_ = nullptr, *gkc_ = nullptr, *gdk_ = nullptr;
    double rb0_ = 0.0;
    double stage_ms_[kStages] = {};
    double *grho_ = nullptr, *gtmp_ = nullptr, *gabs_ = nullptr, *gG_ = nullptr, *gR0_ = nullptr;
    double *gparts_ = nullptr, *gout_ = nullptr, *gL_ = nullptr;
    int gauss_grid_x_ = 1, gauss_grid_y_ = 1;
    double gauss_last_[kGaussParts] = {};
    double gauss_ref_step_ = 0.0; // step index at which the reference residual was recorded

    template <typename U>
    U *dalloc(size_t n)
    {
        U *p = dev_alloc<U>(n);
        allocs_.push_back(p);
        return p;
    }
    void dfree(void *p)
    {
        if (!p) return;
        auto it = std::find(allocs_.begin(), allocs_.end(), p);
        if (it != allocs_.end()) {
            allocs_.erase(it);
            HIPCHK(hipFree(p));
        }
    }
    template <typename U>
    void fill(U *p, size_t n, U v)
    {
        dev_fill(p, n, v, stream);
    }
    void read_counters(unsigned long long *c)
    {
        HIPCHK(hipMemcpyAsync(c, ctr_, sizeof(unsigned long long) * kNumCounters, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
    }
    uint64_t read_step()
    {
        unsigned long long c[kNumCounters];
        read_counters(c);
        return c[kStep];
    }
    // nodes (i, j), i = 0..nr, j = 0..nth, of a plane in the padded layout
    // into a row-major host array
    void copy_node_plane(const double *plane, double *host)
    {
        HIPCHK(hipMemcpy2DAsync(host, sizeof(double) * (gd.nth + 1), plane + L.at(0, 0), sizeof(double) * L.pitch,
                                sizeof(double) * (gd.nth + 1), gd.nr + 1, hipMemcpyDeviceToHost, stream));
    }
    // fixed-point scale of the LDS deposit from the largest |w| held,
    // bounded so that it stays finite in T for vanishing weights (test
    // particles): contributions of such weights then round to zero;
    // true when it changed
    bool set_dep_scale()
    {
        const double qm = qmax_ > 0.0 ? qmax_ : 1.0;
        const double top = std::ldexp(1.0, sizeof(T) == 4 ? 100 : 900);
        const double sc_d = std::min(std::ldexp(1.0, fixed_bits<T>()) / qm, top);
        const T sc = (T)sc_d;
        const T inv = (T)(sc_d < top ? qm * std::ldexp(1.0, -fixed_bits<T>()) : 1.0 / top);
        const bool changed = sc != rd_.dep_scale || inv != rd_.dep_inv;
        rd_.dep_scale = sc;
        rd_.dep_inv = inv;
        return changed;
    }

    template <typename U>
    const U *upload(const std::vector<double> &h)
    {
        std::vector<U> t(h.size());
        for (size_t q = 0; q < h.size(); ++q) t[q] = (U)h[q];
        U *d = dalloc<U>(t.size());
        HIPCHK(hipMemcpyAsync(d, t.data(), sizeof(U) * t.size(), hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));
        return d;
    }

    // Coefficients of the integral-form update (App. A), factored into
    // radial x meridional tables; each is formed in FP64 and rounded once.
    void build_tables()
    {
        const int nr = gd.nr, nth = gd.nth, G = L.G;
        const Geometry &g = geo;
        std::vector<double> r_node(nr + 2 * G + 1), rb(nr + 2 * G + 1);
        for (int i = -G; i <= nr + G; ++i) {
            r_node[i + G] = g.r(i);
            rb[i + G] = g.r(i + 0.5);
        }
        std::vector<double> invr(nr + 1), idr2(nr + 1, 0.0), dr(nr + 1, 0.0), invrb(nr + 1, 0.0), invA(nr + 1, 0.0),
            idrb2(nr + 1, 0.0), drb(nr + 1, 0.0), abi(nr + 1), abh(nr + 1, 1.0);
        for (int i = 0; i <= nr; ++i) {
            const double ri = g.r(i);
            invr[i] = 1.0 / ri;
            if (i < nr) {
                const double ra = ri, rbb = g.r(i + 1);
                idr2[i] = 2.0 / (rbb * rbb - ra * ra);
                dr[i] = rbb - ra;
                const double rh = g.r(i + 0.5);
                invrb[i] = 1.0 / rh;
                invA[i] = 1.0 / (2.0 * kPi * rh * rh);
            }
            if (i >= 1) {
                const double ra = g.r(i - 0.5), rbb = g.r(i + 0.5);
                idrb2[i] = 2.0 / (rbb * rbb - ra * ra);
                drb[i] = rbb - ra;
            }
        }
        // lossy layer: sigma* linear in the radial grid coordinate from the
        // inner edge of the layer (zero) to sigma_max at the outer conductor
        auto absorb = [&](double rho) {
            const int Lc = gd.absorb_cells;
            if (Lc <= 0) return 1.0;
            const double edge = (double)(nr - Lc);
            if (rho <= edge) return 1.0;
            return 1.0 - gd.sigma_max * (rho - edge) / Lc;
        };
        for (int i = 0; i <= nr; ++i) {
            abi[i] = absorb(i);
            if (i < nr) abh[i] = absorb(i + 0.5);
        }
        std::vector<double> s(nth + 1), k(nth + 1), sb(nth + 1, 0.0), icBr(nth + 1, 0.0), idth(nth + 1, 0.0),
            idkb(nth + 1), isb2pi(nth + 1, 0.0), idthb(nth + 1, 0.0), dkb(nth + 1);
        for (int j = 0; j <= nth; ++j) {
            s[j] = g.sth(j);
            k[j] = g.cth(j);
            if (j < nth) {
                sb[j] = g.sth(j + 0.5);
                icBr[j] = 1.0 / (g.cth(j) - g.cth(j + 1));
                idth[j] = 1.0 / (g.th(j + 1) - g.th(j));
                isb2pi[j] = 1.0 / (2.0 * kPi * sb[j]);
            }
            const double lo = j == 0 ? 1.0 : g.cth(j - 0.5);   // polar caps
            const double hi = j == nth ? -1.0 : g.cth(j + 0.5);
            dkb[j] = lo - hi;
            idkb[j] = 1.0 / dkb[j];
            if (j >= 1 && j < nth) idthb[j] = 1.0 / (g.th(j + 0.5) - g.th(j - 0.5));
        }
        m_.r_node = upload<double>(r_node);
        m_.rb = upload<double>(rb);
        m_.invr = upload<double>(invr);
        m_.idr2 = upload<double>(idr2);
        m_.dr = upload<double>(dr);
        m_.invrb = upload<double>(invrb);
        m_.invA = upload<double>(invA);
        m_.idrb2 = upload<double>(idrb2);
        m_.drb = upload<double>(drb);
        m_.s = upload<double>(s);
        m_.sb = upload<double>(sb);
        m_.icBr = upload<double>(icBr);
        m_.idth = upload<double>(idth);
        m_.idkb = upload<double>(idkb);
        m_.isb2pi = upload<double>(isb2pi);
        m_.idthb = upload<double>(idthb);
        m_.ab_int = upload<double>(abi);
        m_.ab_half = upload<double>(abh);
        r_push_ = upload<T>(r_node);
        // FP64 tables of the injection and the Gauss diagnostic
        std::vector<double> Aj(nth + 1);
        for (int j = 0; j <= nth; ++j) Aj[j] = 2.0 * kPi * gd.r_in * gd.r_in * dkb[j];
        dkn_ = upload<double>(k);
        dsn_ = upload<double>(s);
        dAj_ = upload<double>(Aj);
        rb0_ = g.r(0.5);
        std::vector<double> Ar(nr + 2 * G + 1), At(nr + 1, 0.0);
        for (int i = -G; i <= nr + G; ++i) Ar[i + G] = 2.0 * kPi * rb[i + G] * rb[i + G];
        for (int i = 1; i <= nr; ++i) At[i] = kPi * (rb[i + G] * rb[i + G] - rb[i - 1 + G] * rb[i - 1 + G]);
        gA_r_ = upload<double>(Ar);
        gdkb_ = upload<double>(dkb);
        gA_t_ = upload<double>(At);
        gsb_ = upload<double>(sb);
        // FP64 tables of the luminosity diagnostic
        std::vector<double> kc(nth), dk(nth);
        for (int j = 0; j < nth; ++j) {
            kc[j] = g.cth(j + 0.5);
            dk[j] = k[j] - k[j + 1];
        }
        grb_ = upload<double>(rb);
        gkc_ = upload<double>(kc);
        gdk_ = upload<double>(dk);
    }

};

// Many runs of one precision stepped by one launch sequence.
class Batch {
public:
    virtual ~Batch() {}
    virtual void step(int n) = 0;
    double last_ms = 0.0;
    bool timing = false;
    double stage_ms[kStages] = {};
};

template <typename T>
class BatchT final : public Batch {
public:
    BatchT(std::vector<EngineT<T> *> members, hipStream_t s) : members_(std::move(members)), stream_(s)
    {
        versions_.resize(members_.size());
        HIPCHK(hipEventCreate(&ev_[0]));
        HIPCHK(hipEventCreate(&ev_[1]));
        plan_.build(collect(), members_[0]->ppt(), stream_);
    }
    ~BatchT() override
    {
        (void)hipEventDestroy(ev_[0]);
        (void)hipEventDestroy(ev_[1]);
    }

    void step(int n) override
    {
        bool stale = false;
        for (size_t r = 0; r < members_.size(); ++r) stale = stale || versions_[r] != members_[r]->version;
        if (stale) plan_.build(collect(), members_[0]->ppt(), stream_);
        HIPCHK(hipEventRecord(ev_[0], stream_));
        std::vector<SortSched> sched;
        for (EngineT<T> *m : members_) sched.push_back(m->sched());
        plan_.run(n, stream_, timing ? &timer_ : nullptr, sched);
        HIPCHK(hipEventRecord(ev_[1], stream_));
        HIPCHK(hipStreamSynchronize(stream_));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ev_[0], ev_[1]));
        last_ms = ms;
        if (timing && n > 0) timer_.finish(n, stage_ms);
        int first = -1, st = 0;
        for (size_t r = 0; r < members_.size(); ++r) {
            const int s = members_[r]->take_status();
            if (s && first < 0) {
                first = (int)r;
                st = s;
            }
        }
        if (first >= 0) raise_status(st, "run " + std::to_string(first) + ": ");
    }

private:
    std::vector<EngineT<T> *> members_;
    std::vector<unsigned> versions_;
    hipStream_t stream_;
    hipEvent_t ev_[2] = {};
    Plan<T> plan_;
    StageTimer timer_;

    std::vector<RunDev<T>> collect()
    {
        std::vector<RunDev<T>> rd;
        for (size_t r = 0; r < members_.size(); ++r) {
            rd.push_back(members_[r]->run_desc());
            versions_[r] = members_[r]->version;
        }
        return rd;
    }
};

} // namespace

// ------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------

struct pic_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Engine *eng = nullptr;
    std::string err;
};

struct pic_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Batch *impl = nullptr;
    std::string err;
};

namespace {

template <typename C, typename F>
pic_status guarded(C *ctx, F &&f)
{
    if (!ctx) return PIC_EINVAL;
    try {
        HIPCHK(hipSetDevice(ctx->device));
        f();
        ctx->err.clear();
        return PIC_OK;
    } catch (const StatusError &e) {
        ctx->err = e.msg;
        return e.st;
    } catch (const HipError &e) {
        ctx->err = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
        return PIC_EDEVICE;
    } catch (const std::exception &e) {
        ctx->err = e.what();
        return PIC_EDEVICE;
    }
}

void need_engine(pic_ctx *ctx)
{
    if (!ctx->eng) throw StatusError{PIC_ESTATE, "pic_init has not been called"};
}

template <typename T>
Batch *make_batch(pic_ctx *const *runs, int n, hipStream_t s)
{
    std::vector<EngineT<T> *> m;
    for (int r = 0; r < n; ++r) m.push_back(static_cast<EngineT<T> *>(runs[r]->eng));
    return new BatchT<T>(std::move(m), s);
}

} // namespace

// Descriptors a context can be initialised with (pic_init and pic_load).
void validate(const pic_grid_desc &g, const pic_phys_desc &ph)
{
    if (g.nr < 2 || g.nth < 4 || g.nth > 8191 || g.nr > 16000 || !(g.r_in > 0) || !(g.r_out > g.r_in) ||
        !(g.c > 0) || g.n_filt < 0 || g.n_filt > 8 || g.absorb_cells < 0 || g.absorb_cells > g.nr ||
        g.particle_capacity < 0 || g.particle_capacity > INT32_MAX ||
        (g.precision != PIC_FP64 && g.precision != PIC_FP32) ||
        (g.mover != PIC_VAY && g.mover != PIC_BORIS) || (g.r_kind != PIC_R_LOG && g.r_kind != PIC_R_LIN) ||
        (g.th_kind != PIC_TH_EQAREA && g.th_kind != PIC_TH_LIN) || g.tile_r < 0 || g.tile_th < 0 ||
        !(g.chunk_ppt == 0 || g.chunk_ppt == 4 || g.chunk_ppt == 8 || g.chunk_ppt == 16))
        throw StatusError{PIC_EINVAL, "invalid grid descriptor"};
    if (ph.bg_kind < PIC_BG_NONE || ph.bg_kind > PIC_BG_DIPOLE_COROT || !(ph.q_inj > 0 || !ph.inject))
        throw StatusError{PIC_EINVAL, "invalid physics descriptor"};
}

extern "C" {

pic_status pic_create(pic_ctx **out, int device, void *hip_stream)
{
    if (!out) return PIC_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return PIC_EDEVICE;
    if (device < 0 || device >= ndev) return PIC_EINVAL;
    pic_ctx *c = new pic_ctx;
    c->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return PIC_EDEVICE;
    }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return PIC_EDEVICE;
        }
        c->own_stream = true;
    }
    *out = c;
    return PIC_OK;
}

pic_status pic_init(pic_ctx *ctx, const pic_grid_desc *grid, const pic_phys_desc *phys)
{
    return guarded(ctx, [&] {
        if (ctx->eng) throw StatusError{PIC_ESTATE, "pic_init called twice"};
        if (!grid || !phys) throw StatusError{PIC_EINVAL, "null descriptor"};
        validate(*grid, *phys);
        const pic_grid_desc &g = *grid;
        Engine *e = g.precision == PIC_FP32 ? (Engine *)new EngineT<float>() : (Engine *)new EngineT<double>();
        e->gd = g;
        e->ph = *phys;
        e->stream = ctx->stream;
        try {
            scratch_on(ctx->device);
            e->init();
        } catch (...) {
            delete e;
            throw;
        }
        ctx->eng = e;
    });
}

pic_status pic_init_grid(pic_ctx *ctx, const pic_grid_desc *grid, const pic_phys_desc *phys)
{
    return pic_init(ctx, grid, phys);
}

pic_status pic_inject_particles(pic_ctx *ctx, int64_t n, const double *x, const double *y, const double *ur,
                                const double *ut, const double *up, const double *w, const uint64_t *id)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        if (n < 0 || (n > 0 && (!x || !y || !ur || !ut || !up || !w)))
            throw StatusError{PIC_EINVAL, "invalid particle arrays"};
        ctx->eng->inject(n, x, y, ur, ut, up, w, id);
    });
}

pic_status pic_inject_particles_noalloc(pic_ctx *ctx, int64_t n, const double *x, const double *y,
                                        const double *ur, const double *ut, const double *up, const double *w,
                                        const uint64_t *id)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        if (n < 0 || (n > 0 && (!x || !y || !ur || !ut || !up || !w)))
            throw StatusError{PIC_EINVAL, "invalid particle arrays"};
        if (n > kNoAllocMaxParticles)
            throw StatusError{PIC_EINVAL, "pic_inject_particles_noalloc takes at most " +
                                              std::to_string(kNoAllocMaxParticles) + " particles per call"};
        double *sp = scratch_of(ctx->device);
        if (!sp) throw StatusError{PIC_ESTATE, "no staging memory on this device (pic_init has not run on it)"};
        ctx->eng->inject_noalloc(n, x, y, ur, ut, up, w, id, sp);
    });
}

pic_status pic_step(pic_ctx *ctx, int32_t n_steps)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        if (n_steps < 0) throw StatusError{PIC_EINVAL, "negative step count"};
        ctx->eng->step(n_steps);
    });
}

pic_status pic_field_shape(pic_ctx *ctx, int32_t comp, int32_t *rows, int32_t *cols, int32_t *row0)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        if (comp < 0 || comp > 8) throw StatusError{PIC_EINVAL, "invalid component"};
        ctx->eng->field_shape(comp, rows, cols, row0);
    });
}

pic_status pic_get_field(pic_ctx *ctx, int32_t comp, double *host, int64_t cap)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        if (comp < 0 || comp > 8 || !host) throw StatusError{PIC_EINVAL, "invalid component or buffer"};
        int32_t r, c, r0;
        ctx->eng->field_shape(comp, &r, &c, &r0);
        if (cap < (int64_t)r * c) throw StatusError{PIC_EINVAL, "output buffer too small"};
        ctx->eng->get_field(comp, host);
    });
}

pic_status pic_set_field(pic_ctx *ctx, int32_t comp, const double *host, int64_t n)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        if (comp < 0 || comp > 5 || !host) throw StatusError{PIC_EINVAL, "only E and B components can be set"};
        int32_t r, c, r0;
        ctx->eng->field_shape(comp, &r, &c, &r0);
        if (n != (int64_t)r * c) throw StatusError{PIC_EINVAL, "field size mismatch"};
        ctx->eng->set_field(comp, host);
    });
}

pic_status pic_get_particles(pic_ctx *ctx, double *x, double *y, double *ur, double *ut, double *up, double *w,
                             uint64_t *id, int64_t cap, int64_t *n_out)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        const int64_t n = ctx->eng->get_particles(x, y, ur, ut, up, w, id, cap);
        if (n_out) *n_out = n < 0 ? -n : n;
        if (n < 0) throw StatusError{PIC_EINVAL, "particle buffer too small"};
    });
}

pic_status pic_get_particle_cells(pic_ctx *ctx, int32_t *ci, int32_t *cj, double *fx, double *fy, int64_t cap,
                                  int64_t *n_out)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        const int64_t n = ctx->eng->get_cells(ci, cj, fx, fy, cap);
        if (n_out) *n_out = n < 0 ? -n : n;
        if (n < 0) throw StatusError{PIC_EINVAL, "particle buffer too small"};
    });
}

pic_status pic_get_moments(pic_ctx *ctx, int32_t kind, double *out, int64_t cap)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        if (!out) throw StatusError{PIC_EINVAL, "null output"};
        const int64_t N = (int64_t)(ctx->eng->gd.nr + 1) * (ctx->eng->gd.nth + 1);
        switch (kind) {
        case PIC_MOM_COUNTS: {
            if (cap < 5) throw StatusError{PIC_EINVAL, "output buffer too small"};
            double c[6];
            ctx->eng->counts(c);
            std::memcpy(out, c, sizeof(double) * (size_t)std::min<int64_t>(cap, 6));
            break;
        }
        case PIC_MOM_GAUSS:
            if (cap < 2 * N) throw StatusError{PIC_EINVAL, "output buffer too small"};
            ctx->eng->gauss(out);
            break;
        case PIC_MOM_CARRY:
            if (cap < ctx->eng->gd.nth + 1) throw StatusError{PIC_EINVAL, "output buffer too small"};
            ctx->eng->get_carry(out);
            break;
        case PIC_MOM_STAGE_MS:
            if (cap < 9) throw StatusError{PIC_EINVAL, "output buffer too small"};
            ctx->eng->stage_ms(out);
            break;
        case PIC_MOM_POYNTING:
            if (cap < ctx->eng->gd.nr) throw StatusError{PIC_EINVAL, "output buffer too small"};
            ctx->eng->luminosity(out);
            break;
        case PIC_MOM_GAUSS_RES:
            if (cap < kGaussParts + 1) throw StatusError{PIC_EINVAL, "output buffer too small"};
            ctx->eng->gauss_residual(out);
            break;
        case PIC_MOM_RHO_Q:
            if (cap < N) throw StatusError{PIC_EINVAL, "output buffer too small"};
            ctx->eng->rho_q(out);
            break;
        default:
            throw StatusError{PIC_EINVAL, "unknown moment"};
        }
    });
}

pic_status pic_set_step_index(pic_ctx *ctx, int64_t step)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        if (step < 0) throw StatusError{PIC_EINVAL, "negative step index"};
        ctx->eng->set_step(step);
    });
}

pic_status pic_set_carry(pic_ctx *ctx, const double *carry, int64_t n)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        if (!carry || n != ctx->eng->gd.nth + 1) throw StatusError{PIC_EINVAL, "carry size mismatch"};
        ctx->eng->set_carry(carry);
    });
}

pic_status pic_set_timing(pic_ctx *ctx, int32_t on)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        ctx->eng->timing = on != 0;
    });
}

pic_status pic_set_sort(pic_ctx *ctx, int32_t tile_r, int32_t tile_th, int32_t sort_interval)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        if (tile_r < 1 || tile_th < 1 || tile_r > 4096 || tile_th > 4096 || sort_interval == 0)
            throw StatusError{PIC_EINVAL, "invalid sort tile or interval"};
        ctx->eng->set_sort(tile_r, tile_th, sort_interval);
    });
}

pic_status pic_autotune(pic_ctx *ctx, const int32_t *cand, int32_t n_cand, int32_t steps, int32_t *best,
                        double *best_ns)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        if (!cand || n_cand < 1 || steps < 1 || !best) throw StatusError{PIC_EINVAL, "invalid autotune arguments"};
        for (int q = 0; q < n_cand; ++q) {
            const int32_t *c = cand + 3 * q;
            if (c[0] < 1 || c[1] < 1 || c[0] > 4096 || c[1] > 4096 || c[2] == 0)
                throw StatusError{PIC_EINVAL, "invalid autotune candidate"};
        }
        Engine *e = ctx->eng;
        int bq = 0;
        double bcost = 0.0;
        for (int q = 0; q < n_cand; ++q) {
            const int32_t *c = cand + 3 * q;
            e->set_sort(c[0], c[1], c[2]);
            e->timed_steps(1, nullptr); // sorts with the new tiles, captures the graph
            // whole sort periods, so that every candidate pays its sorts
            const int n = c[2] > 0 ? c[2] * ((steps + c[2] - 1) / c[2]) : steps;
            double ps = 0.0;
            const double ms = e->timed_steps(n, &ps);
            const double cost = 1e6 * ms / std::max(ps, 1.0);
            if (q == 0 || cost < bcost) {
                bq = q;
                bcost = cost;
            }
        }
        const int32_t *c = cand + 3 * bq;
        e->set_sort(c[0], c[1], c[2]);
        best[0] = c[0];
        best[1] = c[1];
        best[2] = c[2];
        if (best_ns) *best_ns = bcost;
    });
}

pic_status pic_save(pic_ctx *ctx, const char *path)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        if (!path) throw StatusError{PIC_EINVAL, "null path"};
        FILE *f = std::fopen(path, "wb");
        if (!f) throw StatusError{PIC_EINVAL, std::string("cannot create ") + path};
        try {
            ctx->eng->save(f);
        } catch (...) {
            std::fclose(f);
            throw;
        }
        if (std::fclose(f) != 0) throw StatusError{PIC_EINVAL, std::string("cannot write ") + path};
    });
}

pic_status pic_load(pic_ctx *ctx, const char *path)
{
    return guarded(ctx, [&] {
        if (ctx->eng) throw StatusError{PIC_ESTATE, "pic_load needs a context without pic_init"};
        if (!path) throw StatusError{PIC_EINVAL, "null path"};
        FILE *f = std::fopen(path, "rb");
        if (!f) throw StatusError{PIC_EINVAL, std::string("cannot open ") + path};
        Engine *e = nullptr;
        try {
            CkptHeader h{};
            ck_read(f, &h, sizeof h);
            if (std::memcmp(h.magic, kCkptMagic, sizeof h.magic) != 0 || h.version != kCkptVersion)
                throw StatusError{PIC_EINVAL, "not a checkpoint of this library version"};
            const bool fp32 = h.grid.precision == PIC_FP32;
            if ((fp32 ? 4u : 8u) != h.real_bytes || (!fp32 && h.grid.precision != PIC_FP64))
                throw StatusError{PIC_EINVAL, "checkpoint precision is inconsistent"};
            validate(h.grid, h.phys);
            e = fp32 ? (Engine *)new EngineT<float>() : (Engine *)new EngineT<double>();
            e->gd = h.grid;
            e->ph = h.phys;
            e->stream = ctx->stream;
            scratch_on(ctx->device);
            e->init();
            e->restore(f, h);
        } catch (...) {
            std::fclose(f);
            delete e;
            throw;
        }
        std::fclose(f);
        ctx->eng = e;
    });
}

const char *pic_last_error(const pic_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void pic_destroy(pic_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    delete ctx->eng;
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

pic_status pic_batch_create(pic_ctx *const *runs, int32_t n, void *hip_stream, pic_batch **out)
{
    if (!out) return PIC_EINVAL;
    *out = nullptr;
    if (!runs || n < 1) return PIC_EINVAL;
    for (int r = 0; r < n; ++r) {
        if (!runs[r]) return PIC_EINVAL;
        if (!runs[r]->eng) return PIC_ESTATE;
        if (runs[r]->device != runs[0]->device || runs[r]->eng->gd.precision != runs[0]->eng->gd.precision)
            return PIC_EINVAL;
        for (int q = 0; q < r; ++q)
            if (runs[q] == runs[r]) return PIC_EINVAL;
    }
    pic_batch *b = new pic_batch;
    b->device = runs[0]->device;
    const pic_status st = guarded(b, [&] {
        if (hip_stream) {
            b->stream = (hipStream_t)hip_stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
            b->own_stream = true;
        }
        b->impl = runs[0]->eng->gd.precision == PIC_FP32 ? make_batch<float>(runs, n, b->stream)
                                                         : make_batch<double>(runs, n, b->stream);
    });
    if (st != PIC_OK) {
        if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
        delete b;
        return st;
    }
    *out = b;
    return PIC_OK;
}

pic_status pic_batch_step(pic_batch *b, int32_t n_steps)
{
    return guarded(b, [&] {
        if (n_steps < 0) throw StatusError{PIC_EINVAL, "negative step count"};
        b->impl->step(n_steps);
    });
}

pic_status pic_batch_elapsed_ms(pic_batch *b, double *ms)
{
    return guarded(b, [&] {
        if (!ms) throw StatusError{PIC_EINVAL, "null output"};
        *ms = b->impl->last_ms;
    });
}

pic_status pic_batch_set_timing(pic_batch *b, int32_t on)
{
    return guarded(b, [&] { b->impl->timing = on != 0; });
}

pic_status pic_batch_stage_ms(pic_batch *b, double *out, int64_t cap)
{
    return guarded(b, [&] {
        if (!out || cap < kStages) throw StatusError{PIC_EINVAL, "output buffer too small"};
        std::memcpy(out, b->impl->stage_ms, sizeof(double) * kStages);
    });
}

const char *pic_batch_last_error(const pic_batch *b) { return b ? b->err.c_str() : "null batch"; }

void pic_batch_destroy(pic_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    delete b->impl;
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

} // extern "C"
