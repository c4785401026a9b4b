// picsar_hip.hip -- host engine and C ABI of the gfx950 PIC step.
//
// One context = one simulation on one GPU.  State lives in device memory
// for the life of the context: nine field planes in one padded layout, a
// second set of face-charge planes for the filter's ping-pong, two
// structure-of-arrays particle stores (the counting sort scatters from one
// into the other), FP64 metric tables built on the host, and a few device
// counters.  A step is a fixed sequence of kernel launches on the
// context's stream; control returns to the host only at the end of
// pic_step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/picsar_hip.h"
#include "pic_device.h"
#include "pic_kernels.h"

using namespace pic;

namespace {

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

class Engine {
public:
    virtual ~Engine() {}
    virtual void init() = 0;
    virtual void inject(int64_t n, const double *x, const double *y, const double *ur, const double *ut,
                        const double *up, const double *w, const uint64_t *id) = 0;
    virtual void step(int n) = 0;
    virtual void get_field(int comp, double *out) = 0;
    virtual void set_field(int comp, const double *in) = 0;
    virtual int64_t get_particles(double *x, double *y, double *ur, double *ut, double *up, double *w,
                                  uint64_t *id, int64_t cap) = 0;
    virtual void counts(double *out) = 0;
    virtual void gauss(double *out) = 0;
    virtual void get_carry(double *out) = 0;
    virtual void set_carry(const double *in) = 0;
    virtual void stage_ms(double *out) = 0;

    pic_grid_desc gd{};
    pic_phys_desc ph{};
    hipStream_t stream = nullptr;
    int64_t step_index = 0;
    bool timing = false;
    Layout L{};
    Geometry geo{};

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

template <typename T>
class EngineT final : public Engine {
public:
    ~EngineT() override
    {
        for (void *p : allocs_) (void)hipFree(p);
        for (auto &e : evpool_) (void)hipEventDestroy(e);
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
        tile_r_ = gd.tile_r > 0 ? gd.tile_r : 8;
        tile_th_ = gd.tile_th > 0 ? gd.tile_th : 8;
        sort_interval_ = gd.sort_interval == 0 ? 4 : gd.sort_interval;
        cap_ = gd.particle_capacity;
        if (ph.inject) qmax_ = std::fabs(ph.q_inj);
        with_ids_ = (gd.flags & PIC_FLAG_IDS) != 0;

        const size_t fsz = L.size();
        for (int c = 0; c < 9; ++c) {
            fld_[c] = dalloc<T>(fsz);
            fill(fld_[c], fsz, (T)0);
        }
        for (int c = 0; c < 3; ++c) {
            ftmp_[c] = dalloc<T>(fsz);
            fill(ftmp_[c], fsz, (T)0);
        }
        build_tables();
        for (int s = 0; s < 2; ++s) {
            cell_[s] = dalloc<uint32_t>(std::max<int64_t>(cap_, 1));
            for (int a = 0; a < 6; ++a) arr_[s][a] = dalloc<T>(std::max<int64_t>(cap_, 1));
            id_[s] = with_ids_ ? dalloc<uint64_t>(std::max<int64_t>(cap_, 1)) : nullptr;
        }
        ctr_ = dalloc<unsigned long long>(8);
        fill(ctr_, 8, 0ull);
        status_ = dalloc<int>(1);
        fill(status_, 1, 0);
        work_ = dalloc<unsigned int>(8);
        carry_ = dalloc<double>(nth + 1);
        fill(carry_, (size_t)nth + 1, 0.0);
        // sort tiles over rows -G..nr+G
        ntr_ = (L.rows() + tile_r_ - 1) / tile_r_;
        ntj_ = (nth + tile_th_ - 1) / tile_th_;
        n_keys_ = ntr_ * ntj_;
        counts_ = dalloc<unsigned int>(n_keys_ + 1);
        cursor_ = dalloc<unsigned int>(n_keys_ + 1);
        offsets_ = dalloc<unsigned long long>(n_keys_ + 1);
        // LDS plane size: a chunk spans at most two neighbouring tiles (serpentine
        // order), widened by the drift since the last sort (at most ~0.7 cell
        // per step in grid units) and the stencil halo (one cell below, two above)
        ppt_ = gd.chunk_ppt > 0 ? gd.chunk_ppt : 8;
        const int drift = sort_interval_ > 0 ? (7 * sort_interval_ + 9) / 10 : 0;
        const int R = 2 * tile_r_ + 2 * drift + 3, C = 2 * tile_th_ + 2 * drift + 3;
        lds_cap_ = sort_interval_ > 0 ? std::min(R * C, kMaxLdsBytes / (6 * (int)sizeof(T) + 24)) : 0;
        const int shm = (int)lds_push_bytes<T>(std::max(lds_cap_, 1));
        HIPCHK(hipFuncSetAttribute((const void *)k_push<T, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
        HIPCHK(hipFuncSetAttribute((const void *)k_push<T, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
        HIPCHK(hipFuncSetAttribute((const void *)k_push<T, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
        HIPCHK(hipStreamSynchronize(stream));
    }

    void inject(int64_t n, const double *x, const double *y, const double *ur, const double *ut, const double *up,
                const double *w, const uint64_t *id) override
    {
        if (n == 0) return;
        const int nr = gd.nr, nth = gd.nth;
        const double lim = gd.n_filt + 1.0;
        for (int64_t q = 0; q < n; ++q) {
            if (!(x[q] >= -lim && x[q] <= nr + lim && y[q] >= 0.0 && y[q] <= nth))
                throw StatusError{PIC_EINVAL, "particle position outside the grid"};
        }
        unsigned long long ntot = 0;
        HIPCHK(hipMemcpyAsync(&ntot, ctr_ + kTotal, sizeof ntot, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        if ((int64_t)ntot + n > cap_) throw StatusError{PIC_ECAPACITY, "particle capacity exceeded"};
        for (int64_t q = 0; q < n; ++q) qmax_ = std::max(qmax_, std::fabs(w[q]));
        const int64_t chunk = 1 << 22;
        double *stage = dalloc_tmp<double>(6 * (size_t)std::min(n, chunk));
        uint64_t *sid = id ? dalloc_tmp<uint64_t>((size_t)std::min(n, chunk)) : nullptr;
        std::vector<double> hb;
        for (int64_t o = 0; o < n; o += chunk) {
            const int64_t m = std::min(chunk, n - o);
            hb.resize(6 * (size_t)m);
            const double *srcs[6] = {x, y, ur, ut, up, w};
            for (int a = 0; a < 6; ++a) std::memcpy(&hb[(size_t)a * m], srcs[a] + o, sizeof(double) * m);
            HIPCHK(hipMemcpyAsync(stage, hb.data(), sizeof(double) * 6 * m, hipMemcpyHostToDevice, stream));
            if (sid) HIPCHK(hipMemcpyAsync(sid, id + o, sizeof(uint64_t) * m, hipMemcpyHostToDevice, stream));
            const int blocks = (int)std::min<int64_t>((m + 255) / 256, 4096);
            k_load<T><<<blocks, 256, 0, stream>>>(stage, sid, m, (long long)(ntot + o), nth, cell_[cur_],
                                                  arr_[cur_][0], arr_[cur_][1], arr_[cur_][2], arr_[cur_][3],
                                                  arr_[cur_][4], arr_[cur_][5], id_[cur_]);
            HIPCHK(hipGetLastError());
            HIPCHK(hipStreamSynchronize(stream));
        }
        free_tmp(stage);
        if (sid) free_tmp(sid);
        const unsigned long long nn = ntot + n;
        HIPCHK(hipMemcpyAsync(ctr_ + kTotal, &nn, sizeof nn, hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));
        n_bound_ = (int64_t)nn;
        need_sort_ = true;
    }

    void step(int n) override
    {
        if (timing) {
            const size_t need = (size_t)n * kStages * 2;
            while (evpool_.size() < need) {
                hipEvent_t e;
                HIPCHK(hipEventCreate(&e));
                evpool_.push_back(e);
            }
            std::fill(stage_used_, stage_used_ + (size_t)kStages, false);
        }
        for (int s = 0; s < n; ++s) {
            ev_base_ = (size_t)s * kStages * 2;
            one_step();
        }
        HIPCHK(hipStreamSynchronize(stream));
        int st = 0;
        HIPCHK(hipMemcpy(&st, status_, sizeof st, hipMemcpyDeviceToHost));
        unsigned long long c[8];
        HIPCHK(hipMemcpy(c, ctr_, sizeof c, hipMemcpyDeviceToHost));
        n_bound_ = (int64_t)c[kTotal];
        if (timing && n > 0) {
            // mean device time per step of each stage over the steps of this call
            for (int q = 0; q < kStages; ++q) {
                stage_ms_[q] = 0.0;
                if (!stage_used_[q]) continue;
                for (int s = 0; s < n; ++s) {
                    float ms = 0.f;
                    const size_t b = (size_t)s * kStages * 2 + 2 * q;
                    HIPCHK(hipEventElapsedTime(&ms, evpool_[b], evpool_[b + 1]));
                    stage_ms_[q] += ms;
                }
                stage_ms_[q] /= n;
            }
        }
        if (st & 1) {
            fill(status_, 1, 0);
            throw StatusError{PIC_ECFL, "a particle moved one cell or more in one step (CFL)"};
        }
        if (st & 2) {
            fill(status_, 1, 0);
            throw StatusError{PIC_ECAPACITY, "particle capacity exceeded by surface injection"};
        }
        if (st & 4) {
            fill(status_, 1, 0);
            throw StatusError{PIC_EDEVICE, "internal error: sort destination outside the particle store"};
        }
    }

    void get_field(int comp, double *out) override
    {
        int32_t rows, cols, row0;
        field_shape(comp, &rows, &cols, &row0);
        const T *src = comp < 6 ? fld_[comp] : fcur(comp - 6);
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
    }

    int64_t get_particles(double *x, double *y, double *ur, double *ut, double *up, double *w, uint64_t *id,
                          int64_t cap) override
    {
        unsigned long long ntot = 0;
        HIPCHK(hipMemcpyAsync(&ntot, ctr_ + kTotal, sizeof ntot, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        std::vector<uint32_t> hc(ntot);
        HIPCHK(hipMemcpyAsync(hc.data(), cell_[cur_], sizeof(uint32_t) * ntot, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        int64_t live = 0;
        for (auto c : hc) live += c != kDead;
        if (live > cap) return -live;
        std::vector<T> ha(ntot);
        double *outs[6] = {x, y, ur, ut, up, w};
        for (int a = 0; a < 6; ++a) {
            if (!outs[a]) continue;
            HIPCHK(hipMemcpyAsync(ha.data(), arr_[cur_][a], sizeof(T) * ntot, hipMemcpyDeviceToHost, stream));
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
                HIPCHK(hipMemcpyAsync(hi.data(), id_[cur_], sizeof(uint64_t) * ntot, hipMemcpyDeviceToHost, stream));
                HIPCHK(hipStreamSynchronize(stream));
            }
            int64_t m = 0;
            for (size_t q = 0; q < ntot; ++q)
                if (hc[q] != kDead) id[m++] = with_ids_ ? hi[q] : (uint64_t)q;
        }
        return live;
    }

    void counts(double *out) override
    {
        unsigned long long c[8];
        HIPCHK(hipMemcpyAsync(c, ctr_, sizeof c, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        out[0] = (double)(c[kTotal] - c[kDeadSinceSort]);
        out[1] = (double)c[kInjected];
        out[2] = (double)c[kDeleted] + (double)c[kDeadSinceSort];
        out[3] = (double)step_index;
        out[4] = (double)c[kPartSteps];
    }

    void gauss(double *out) override
    {
        const size_t fsz = L.size();
        double *rho = dalloc_tmp<double>(fsz), *tmp = dalloc_tmp<double>(fsz);
        double *G = dalloc_tmp<double>((size_t)(gd.nr + 1) * (gd.nth + 1));
        fill(rho, fsz, 0.0);
        fill(tmp, fsz, 0.0);
        k_node_charge<T><<<2048, 256, 0, stream>>>(cell_[cur_], arr_[cur_][0], arr_[cur_][1], arr_[cur_][5],
                                                   ctr_ + kTotal, L, rho);
        HIPCHK(hipGetLastError());
        double *a = rho, *b = tmp;
        for (int pss = 0; pss < gd.n_filt; ++pss) {
            FilterSet fs{};
            fs.src[0] = a;
            fs.dst[0] = b;
            fs.kind[0] = 0;
            fs.last_row[0] = gd.nr + L.G;
            dim3 blk(64, 4), grd((gd.nth + 1 + 63) / 64, (L.rows() + 3) / 4, 1);
            k_filter<double><<<grd, blk, 0, stream>>>(fs, L);
            HIPCHK(hipGetLastError());
            std::swap(a, b);
        }
        dim3 blk(64, 4), grd((gd.nth + 1 + 63) / 64, (gd.nr + 1 + 3) / 4);
        k_gauss_flux<T><<<grd, blk, 0, stream>>>(fld_[cER], fld_[cETH], L, gA_r_, gdkb_, gA_t_, gsb_, G);
        HIPCHK(hipGetLastError());
        const size_t N = (size_t)(gd.nr + 1) * (gd.nth + 1);
        std::vector<double> hr(fsz);
        HIPCHK(hipMemcpyAsync(out, G, sizeof(double) * N, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipMemcpyAsync(hr.data(), a, sizeof(double) * fsz, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        for (int i = 0; i <= gd.nr; ++i)
            for (int j = 0; j <= gd.nth; ++j) out[N + (size_t)i * (gd.nth + 1) + j] = hr[L.at(i, j)];
        free_tmp(rho);
        free_tmp(tmp);
        free_tmp(G);
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

    void stage_ms(double *out) override { std::memcpy(out, stage_ms_, sizeof stage_ms_); }

private:
    int ppt_ = 8;
    static constexpr int kMaxLdsBytes = 64 * 1024;
    enum { kTotal = 0, kDeadSinceSort = 1, kDeleted = 2, kInjected = 3, kLive = 4, kPartSteps = 5 };

    std::vector<void *> allocs_;
    T *fld_[9] = {};
    T *ftmp_[3] = {};
    bool f_in_tmp_ = false; // the filtered face charges of the last step live in ftmp_
    uint32_t *cell_[2] = {};
    T *arr_[2][6] = {};
    uint64_t *id_[2] = {};
    int cur_ = 0;
    unsigned long long *ctr_ = nullptr;
    int *status_ = nullptr;
    unsigned int *work_ = nullptr;
    double *carry_ = nullptr;
    unsigned int *counts_ = nullptr, *cursor_ = nullptr;
    unsigned long long *offsets_ = nullptr;
    int ntr_ = 0, ntj_ = 0, n_keys_ = 0;
    int tile_r_ = 8, tile_th_ = 8, sort_interval_ = 4;
    int lds_cap_ = 0;
    int64_t cap_ = 0, n_bound_ = 0;
    double qmax_ = 0.0; // largest |w| held so far: sets the fixed-point deposit scale
    bool with_ids_ = false, need_sort_ = true;
    Metric<T> m_{};
    const T *r_node_ = nullptr, *k_node_ = nullptr;
    const double *dkn_ = nullptr, *dsn_ = nullptr, *dAj_ = nullptr;
    const double *gA_r_ = nullptr, *gdkb_ = nullptr, *gA_t_ = nullptr, *gsb_ = nullptr;
    double rb0_ = 0.0;
    static constexpr int kStages = 9; // sort, faraday, push, filter, ampere, absorb, inject, zero, total
    std::vector<hipEvent_t> evpool_;
    size_t ev_base_ = 0;
    bool stage_used_[kStages] = {};
    double stage_ms_[kStages] = {};

    template <typename U>
    U *dalloc(size_t n)
    {
        void *p = nullptr;
        if (hipMalloc(&p, sizeof(U) * std::max<size_t>(n, 1)) != hipSuccess)
            throw StatusError{PIC_ENOMEM, "device allocation failed"};
        allocs_.push_back(p);
        return (U *)p;
    }
    template <typename U>
    U *dalloc_tmp(size_t n)
    {
        void *p = nullptr;
        if (hipMalloc(&p, sizeof(U) * std::max<size_t>(n, 1)) != hipSuccess)
            throw StatusError{PIC_ENOMEM, "device allocation failed"};
        return (U *)p;
    }
    void free_tmp(void *p)
    {
        HIPCHK(hipStreamSynchronize(stream));
        HIPCHK(hipFree(p));
    }
    template <typename U>
    void fill(U *p, size_t n, U v)
    {
        const int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
        k_fill<U><<<std::max(blocks, 1), 256, 0, stream>>>(p, n, v);
        HIPCHK(hipGetLastError());
    }
    T *fcur(int c) const { return f_in_tmp_ ? ftmp_[c] : fld_[6 + c]; }

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
        m_.r_node = upload<T>(r_node);
        m_.rb = upload<T>(rb);
        m_.invr = upload<T>(invr);
        m_.idr2 = upload<T>(idr2);
        m_.dr = upload<T>(dr);
        m_.invrb = upload<T>(invrb);
        m_.invA = upload<T>(invA);
        m_.idrb2 = upload<T>(idrb2);
        m_.drb = upload<T>(drb);
        m_.s = upload<T>(s);
        m_.k = upload<T>(k);
        m_.sb = upload<T>(sb);
        m_.icBr = upload<T>(icBr);
        m_.idth = upload<T>(idth);
        m_.idkb = upload<T>(idkb);
        m_.isb2pi = upload<T>(isb2pi);
        m_.idthb = upload<T>(idthb);
        m_.ab_int = upload<T>(abi);
        m_.ab_half = upload<T>(abh);
        r_node_ = m_.r_node;
        k_node_ = m_.k;
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
    }

    double inv_rl(double t) const
    {
        double om = ph.omega;
        if (ph.t_spin > 0.0 && t < ph.t_spin) om = ph.omega * t / ph.t_spin;
        return om / gd.c;
    }

    Fields<T> fields() const
    {
        Fields<T> f;
        for (int c = 0; c < 6; ++c) f.c[c] = fld_[c];
        for (int c = 0; c < 3; ++c) f.c[6 + c] = fld_[6 + c];
        return f;
    }

    void mark(int q, bool start)
    {
        if (!timing) return;
        HIPCHK(hipEventRecord(evpool_[ev_base_ + 2 * q + (start ? 0 : 1)], stream));
        stage_used_[q] = true;
    }

    void sort()
    {
        TileMap tm{L.G, tile_r_, tile_th_, ntj_, n_keys_};
        fill(counts_, (size_t)n_keys_ + 1, 0u);
        fill(cursor_, (size_t)n_keys_ + 1, 0u);
        // one wave per span of kSortSpan particles (4 waves per block)
        const int blocks = (int)std::min<int64_t>(std::max<int64_t>((n_bound_ + 4 * kSortSpan - 1) / (4 * kSortSpan), 1),
                                                  8192);
        k_sort_hist<<<blocks, 256, 0, stream>>>(cell_[cur_], ctr_ + kTotal, tm, counts_);
        HIPCHK(hipGetLastError());
        k_sort_scan<<<1, 1024, 0, stream>>>(counts_, n_keys_, offsets_, ctr_ + kTotal, ctr_ + kLive);
        HIPCHK(hipGetLastError());
        SortArgs<T> sa{};
        const int nxt = cur_ ^ 1;
        sa.cell = cell_[cur_];
        sa.cell_o = cell_[nxt];
        for (int a = 0; a < 6; ++a) {
            sa.a[a] = arr_[cur_][a];
            sa.a_o[a] = arr_[nxt][a];
        }
        sa.id = id_[cur_];
        sa.id_o = id_[nxt];
        sa.n_total = ctr_ + kTotal;
        sa.offsets = offsets_;
        sa.cursor = cursor_;
        sa.tm = tm;
        sa.capacity = (unsigned long long)cap_;
        sa.status = status_;
        k_sort_scatter<T><<<blocks, 256, 0, stream>>>(sa);
        HIPCHK(hipGetLastError());
        k_finish_sort<<<1, 1, 0, stream>>>(ctr_);
        HIPCHK(hipGetLastError());
        cur_ = nxt;
        need_sort_ = false;
    }

    void one_step()
    {
        mark(8, true);
        const int nr = gd.nr, nth = gd.nth;
        k_count_live<<<1, 1, 0, stream>>>(ctr_);
        HIPCHK(hipGetLastError());
        // sort
        mark(0, true);
        if (sort_interval_ > 0 && (need_sort_ || step_index % sort_interval_ == 0)) sort();
        mark(0, false);
        // zero the deposit planes
        mark(7, true);
        f_in_tmp_ = false;
        for (int c = 0; c < 3; ++c) fill(fld_[6 + c], L.size(), (T)0);
        mark(7, false);
        const dim3 blk(64, 4), grd((nth + 1 + 63) / 64, (nr + 1 + 3) / 4);
        const T hc = (T)(0.5 * gd.c);
        mark(1, true);
        k_faraday<T><<<grd, blk, 0, stream>>>(fields(), L, m_, hc);
        HIPCHK(hipGetLastError());
        mark(1, false);
        // particles
        mark(2, true);
        push(inv_rl((double)step_index));
        mark(2, false);
        k_faraday<T><<<grd, blk, 0, stream>>>(fields(), L, m_, hc);
        HIPCHK(hipGetLastError());
        // filter
        mark(3, true);
        T *src[3] = {fld_[6], fld_[7], fld_[8]}, *dst[3] = {ftmp_[0], ftmp_[1], ftmp_[2]};
        for (int pss = 0; pss < gd.n_filt; ++pss) {
            FilterSet fs{};
            for (int c = 0; c < 3; ++c) {
                fs.src[c] = src[c];
                fs.dst[c] = dst[c];
                fs.kind[c] = c == 1 ? 1 : 0;
                fs.last_row[c] = c == 0 ? nr + L.G - 1 : nr + L.G;
            }
            const dim3 fg((nth + 1 + 63) / 64, (L.rows() + 3) / 4, 3);
            k_filter<T><<<fg, blk, 0, stream>>>(fs, L);
            HIPCHK(hipGetLastError());
            std::swap(src[0], dst[0]);
            std::swap(src[1], dst[1]);
            std::swap(src[2], dst[2]);
        }
        f_in_tmp_ = src[0] == ftmp_[0];
        mark(3, false);
        mark(4, true);
        k_ampere<T><<<grd, blk, 0, stream>>>(fields(), src[0], src[1], src[2], L, m_, (T)gd.c);
        HIPCHK(hipGetLastError());
        mark(4, false);
        mark(5, true);
        if (gd.absorb_cells > 0) {
            const int i0 = std::max(0, nr - gd.absorb_cells - 1);
            const dim3 ag((nth + 1 + 63) / 64, (nr + 1 - i0 + 3) / 4);
            k_absorb_b<T><<<ag, blk, 0, stream>>>(fields(), L, m_, i0);
            HIPCHK(hipGetLastError());
        }
        mark(5, false);
        mark(6, true);
        if (ph.inject && (ph.bg_kind == PIC_BG_MONOPOLE || ph.bg_kind == PIC_BG_DIPOLE)) {
            InjectArgs<T> a{};
            a.L = L;
            a.Er = fld_[cER];
            a.bg = Background{ph.bg_kind, ph.B0, gd.r_in};
            a.inv_rl = inv_rl((double)(step_index + 1));
            a.rb0 = rb0_;
            a.kn = dkn_;
            a.sn = dsn_;
            a.Aj = dAj_;
            a.f_inj = ph.f_inj;
            a.q_inj = ph.q_inj;
            a.carry = carry_;
            a.seed = ph.seed;
            a.step = (uint64_t)step_index;
            a.cell = cell_[cur_];
            a.dx = arr_[cur_][0];
            a.dy = arr_[cur_][1];
            a.ur = arr_[cur_][2];
            a.ut = arr_[cur_][3];
            a.up = arr_[cur_][4];
            a.w = arr_[cur_][5];
            a.id = id_[cur_];
            a.n_total = ctr_ + kTotal;
            a.n_injected = ctr_ + kInjected;
            a.capacity = cap_;
            a.status = status_;
            k_inject<T><<<1, 1024, 0, stream>>>(a);
            HIPCHK(hipGetLastError());
            // upper bound of the count for the next launch grids: every node
            // can add at most f_inj |sigma| A / q + 1 pairs; the bound is only
            // used to size grids, which loop over the device-side count
            n_bound_ += 2 * (int64_t)(nth + 1) * 64;
        }
        mark(6, false);
        mark(8, false);
        ++step_index;
    }

    void push(double irl)
    {
        PushArgs<T> p{};
        p.L = L;
        p.f = fields();
        p.bg = Background{ph.bg_kind, ph.B0, gd.r_in};
        p.r_kind = gd.r_kind;
        p.th_kind = gd.th_kind;
        p.mover = gd.mover;
        p.n_filt = gd.n_filt;
        p.c = (T)gd.c;
        p.dxi = (T)geo.dxi;
        p.inv_dxi = (T)(1.0 / geo.dxi);
        p.nth_f = (T)gd.nth;
        p.two_over_nth = (T)(2.0 / gd.nth);
        p.pi_over_nth = (T)(kPi / gd.nth);
        p.inv_pi_over_nth = (T)(gd.nth / kPi);
        p.eps0 = (T)(ph.q_over_m / (2.0 * gd.c));
        p.inv_rl = (T)irl;
        p.r_node = r_node_;
        p.k_node = k_node_;
        p.cell = cell_[cur_];
        p.dx = arr_[cur_][0];
        p.dy = arr_[cur_][1];
        p.ur = arr_[cur_][2];
        p.ut = arr_[cur_][3];
        p.up = arr_[cur_][4];
        p.w = arr_[cur_][5];
        p.n_total = ctr_ + kTotal;
        p.n_dead = ctr_ + kDeadSinceSort;
        p.status = status_;
        p.work = work_;
        p.lds_cap = use_lds_ ? lds_cap_ : 0;
        const double qm = qmax_ > 0.0 ? qmax_ : 1.0;
        p.dep_scale = (T)(std::ldexp(1.0, fixed_bits<T>()) / qm);
        p.dep_inv = (T)(qm * std::ldexp(1.0, -fixed_bits<T>()));
        fill(work_, 8, 0u);
        const int CH = 256 * ppt_;
        const int64_t nch = (n_bound_ + CH - 1) / CH;
        const int grid = (int)std::max<int64_t>(8, std::min<int64_t>(8 * ((nch + 7) / 8), 8 * 256));
        const size_t shm = p.lds_cap > 0 ? lds_push_bytes<T>(lds_cap_) : 0;
        if (ppt_ == 4) k_push<T, 4><<<grid, 256, shm, stream>>>(p);
        else if (ppt_ == 16) k_push<T, 16><<<grid, 256, shm, stream>>>(p);
        else k_push<T, 8><<<grid, 256, shm, stream>>>(p);
        HIPCHK(hipGetLastError());
    }

public:
    bool use_lds_ = true;
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

namespace {

template <typename F>
pic_status guarded(pic_ctx *ctx, F &&f)
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

} // namespace

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
        const pic_grid_desc &g = *grid;
        if (g.nr < 2 || g.nth < 4 || g.nth > 8191 || g.nr > 16000 || !(g.r_in > 0) || !(g.r_out > g.r_in) ||
            !(g.c > 0) || g.n_filt < 0 || g.n_filt > 8 || g.absorb_cells < 0 || g.absorb_cells > g.nr ||
            g.particle_capacity < 0 || (g.precision != PIC_FP64 && g.precision != PIC_FP32) ||
            (g.mover != PIC_VAY && g.mover != PIC_BORIS) || (g.r_kind != PIC_R_LOG && g.r_kind != PIC_R_LIN) ||
            (g.th_kind != PIC_TH_EQAREA && g.th_kind != PIC_TH_LIN) || g.tile_r < 0 || g.tile_th < 0 ||
            !(g.chunk_ppt == 0 || g.chunk_ppt == 4 || g.chunk_ppt == 8 || g.chunk_ppt == 16))
            throw StatusError{PIC_EINVAL, "invalid grid descriptor"};
        if (phys->bg_kind < PIC_BG_NONE || phys->bg_kind > PIC_BG_DIPOLE_COROT || !(phys->q_inj > 0 || !phys->inject))
            throw StatusError{PIC_EINVAL, "invalid physics descriptor"};
        Engine *e = g.precision == PIC_FP32 ? (Engine *)new EngineT<float>() : (Engine *)new EngineT<double>();
        e->gd = g;
        e->ph = *phys;
        e->stream = ctx->stream;
        try {
            e->init();
        } catch (...) {
            delete e;
            throw;
        }
        ctx->eng = e;
    });
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

pic_status pic_get_moments(pic_ctx *ctx, int32_t kind, double *out, int64_t cap)
{
    return guarded(ctx, [&] {
        need_engine(ctx);
        if (!out) throw StatusError{PIC_EINVAL, "null output"};
        const int64_t N = (int64_t)(ctx->eng->gd.nr + 1) * (ctx->eng->gd.nth + 1);
        switch (kind) {
        case PIC_MOM_COUNTS:
            if (cap < 5) throw StatusError{PIC_EINVAL, "output buffer too small"};
            ctx->eng->counts(out);
            break;
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
        ctx->eng->step_index = step;
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

} // extern "C"
