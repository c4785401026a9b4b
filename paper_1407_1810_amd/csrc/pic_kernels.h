// pic_kernels.h -- HIP kernels of the gfx950 PIC step.
//
// Every kernel serves a table of independent runs; a single simulation is
// a table of one.  Field kernels find their run from a per-run prefix of
// their work-groups, particle kernels from a per-run prefix of their chunks
// or spans that the device computes each step, and the step index, the
// sort decision and the particle-buffer flip live in device counters.  A
// step is therefore a fixed sequence of launches, the same for one run or
// many uneven ones, which a HIP graph holds and replays.
//
//  k_step_begin ... particle-step count, sort decision, sort-span prefix
//  k_sort_* ....... counting sort of particles by tile (serpentine order)
//  k_open_faraday . close the sorts, lay out the push chunks, clear the
//                   deposit planes (and, on a step without the sort
//                   kernels, the bookkeeping of k_step_begin); beside it
//                   the first half Faraday update of B (App. A, eq.
//                   (discreteeq))
//  k_push ......... gather + Vay/Boris push + move + VB deposit, one
//                   work-group per chunk of cell-sorted particles, fields and
//                   face charges staged in LDS for the chunk's bounding box
//  k_faraday_filter the second half Faraday update, and beside it the
//                   n_filt 1-2-1 passes with the polar remap (App. B),
//                   by strips of 64 columns held in registers
//  k_ampere ....... Ampere update of E with the filtered face charges, polar
//                   caps (eq. (erpolarupdate)), walls, lossy layer on E
//  k_close ........ surface pair injection (Sec. 5.3, eq. (volinjeq)), then
//                   the step index advances; lossy layer on B (eq. (EBcond))
//  k_node_charge,
//  k_gauss_flux,
//  k_gauss_final .. FP64 Gauss diagnostic: node charge, residual, reductions
#pragma once
#include <climits>

#include "pic_device.h"

namespace pic {

// Per-run metric tables of the field update: the area and length elements
// of App. A eq. (linearea) factored into radial and meridional tables,
// formed in FP64 on the host and kept in FP64 on the device whatever the
// precision of the fields, so that the FP32 field kernels multiply by the
// stretch metric and the near-axis and polar-cap area factors in FP64 and
// round the updated field once.  Row tables are indexed by the radial node
// / half index, column tables by the meridional one; see
// Engine::build_tables for their definitions.
struct Metric {
    const double *r_node;  // r(i), i = -G..nr+G at [i + G]
    const double *rb;      // r(i + 1/2), i = -G..nr+G at [i + G]
    const double *invr;    // 1 / r_i
    const double *idr2;    // 2 / (r_{i+1}^2 - r_i^2)
    const double *dr;      // r_{i+1} - r_i
    const double *invrb;   // 1 / rbar_i
    const double *invA;    // 1 / (2 pi rbar_i^2)
    const double *idrb2;   // 2 / (rbar_i^2 - rbar_{i-1}^2)
    const double *drb;     // rbar_i - rbar_{i-1}
    const double *s;       // sin theta_j
    const double *sb;      // sin thetabar_j
    const double *icBr;    // 1 / (cos theta_j - cos theta_{j+1})
    const double *idth;    // 1 / (theta_{j+1} - theta_j)
    const double *idkb;    // 1 / (cos thetabar_{j-1} - cos thetabar_j), caps at the poles
    const double *isb2pi;  // 1 / (2 pi sin thetabar_j)
    const double *idthb;   // 1 / (thetabar_j - thetabar_{j-1})
    const double *ab_int;  // lossy-layer factor at rho = i
    const double *ab_half; // lossy-layer factor at rho = i + 1/2
};

// Device counters of a run (unsigned long long each).
enum : int {
    kTotal = 0,         // slots in use: live particles plus those deleted since the last sort
    kDeadSinceSort = 1,
    kDeleted = 2,       // deletions before the last sort
    kInjected = 3,
    kLive = 4,          // live count produced by the sort's scan
    kPartSteps = 5,     // particle-steps advanced
    kStep = 6,          // step index n (time t = n dt)
    kCur = 7,           // current particle buffer (0 or 1)
    kNeedSort = 8,      // particles were appended since the last sort
    kSortNow = 9,       // the current step sorts
    kGlobalChunks = 10, // push chunks whose cells did not fit the LDS planes
    kNumCounters = 16
};

// Counting-sort key of a packed cell: tiles of tile_r x tile_th cells over
// rows -G..nr+G, numbered in serpentine order so that consecutive tiles
// share an edge; deleted particles get the last key.  The tile index
// floor(x / d) of a row or column x (0 <= x < 2^21) is formed as
// trunc((x + 1/2) * r) with r = 1/d rounded to FP32 on the host: (x + 1/2) / d
// lies at least 1/(2d) from every integer, and the two roundings move it by
// at most 2^-23 of itself, below 2^-2 / d, so the truncation is exact (and
// much cheaper than an integer division by a value known only at run time).
struct TileMap {
    int G, tile_r, tile_th, ntj, n_keys;
    float inv_r, inv_th; // 1 / tile_r, 1 / tile_th rounded to FP32
    __device__ int key(uint32_t c) const
    {
        if (c == kDead) return n_keys;
        const int ti = (int)(((float)(cell_i(c) + G) + 0.5f) * inv_r);
        int tj = (int)(((float)cell_j(c) + 0.5f) * inv_th);
        if (ti & 1) tj = ntj - 1 - tj;
        return ti * ntj + tj;
    }
};

// One span of a sort that holds a key: its index among the run's spans and
// a particle count (see kSpanList).
struct SpanEnt {
    unsigned int s, c;
};

// Everything the kernels need to know about one run.  The host fills it
// once (and again when particles with a larger weight arrive); what changes
// from step to step lives in the counters `ctr`.
template <typename T>
struct RunDev {
    Layout L;
    T *fld[9];            // E_r, E_th, E_ph, B_r, B_th, B_ph, F_r, F_th, F_ph
    T *ftmp[3];           // second set of face-charge planes (filter ping-pong)
    const T *ffin[3];     // where the filtered face charges end up after n_filt passes
    Metric m;
    const T *r_push;      // r(i) at [i + G] in the context's precision: the push's start radii
    Background bg;
    int r_kind, th_kind, mover, n_filt, absorb_cells;
    T c, dxi, inv_dxi, nth_f, two_over_nth, pi_over_nth, inv_pi_over_nth, eps0;
    double omega, t_spin, cd; // final angular velocity, spin-up time, light speed
    uint32_t *cell[2];    // two particle stores; the sort scatters from one into the other
    T *arr[2][6];         // offsets dx, dy, momenta u_r, u_th, u_ph, weight w
    uint64_t *id[2];      // null when ids are not kept
    long long capacity;
    unsigned long long *ctr;
    int *status;          // bit 0 CFL, bit 1 capacity (injection), bit 2 sort destination
    int lds_cap;          // entries per LDS plane of the push, 0 = global-memory path
    T dep_scale, dep_inv; // fixed-point scale of the LDS deposit planes and its inverse
    TileMap tm;
    int sort_interval;    // <= 0: never
    unsigned int *counts, *cursor;
    unsigned long long *offsets;
    unsigned int *nspan;  // spans of the current sort that hold each key (kSpanOverflow: too many)
    SpanEnt *slist;       // per key, kSpanList entries (span index, particles there)
    unsigned int *sbefore; // per entry of slist: the key's particles in the spans before that one
    int inject;
    const double *kn, *sn, *Aj; // cos / sin theta_j, dual face area of node j on the inner conductor
    double rb0, f_inj, q_inj;
    double *carry;
    uint64_t seed;
};

// 1 / R_l = Omega(t) / c, Omega rising linearly over t_spin (Sec. 5.2).
__host__ __device__ inline double inv_light_cylinder(double omega, double t_spin, double c, double t)
{
    const double om = (t_spin > 0.0 && t < t_spin) ? omega * t / t_spin : omega;
    return om / c;
}

// Work-groups of a launch over many runs: run r owns [off[r], off[r+1]).
__device__ inline int run_of(const int *__restrict__ off, int n_runs, int b)
{
    int lo = 0, hi = n_runs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
__device__ inline int run_of(const unsigned long long *__restrict__ off, int n_runs, unsigned long long b)
{
    int lo = 0, hi = n_runs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The work-groups of a launch are dealt to the eight XCDs in turn (work-group
// b runs on XCD b % 8), and each XCD has its own L2.  Field kernels read the
// rows and columns next to their own tile, so a launch is renumbered to give
// each XCD a contiguous range of the tiles: neighbouring tiles then share an
// L2 and the shared rows are fetched from HBM once.  A bijection of
// [0, g): XCD x takes g / 8 (plus one for the first g % 8) consecutive tiles.
__device__ __forceinline__ int xcd_tile(int b, int g)
{
    const int x = b & 7, k = b >> 3, per = g >> 3, rem = g & 7;
    return x * per + min(x, rem) + k;
}

// Field kernels use 64 x 4 work-groups; each thread takes RS consecutive
// rows of one column, so a work-group covers 64 columns x 4 RS rows, the
// per-work-group run lookup is paid once per RS cells of a thread, and a
// thread's loads of neighbouring rows are shared and issued together.
// Faraday, Ampere and the lossy layer take 4 rows (more work-groups in
// flight).
constexpr int kFieldRows = 4;
constexpr int kZeroPerThread = 16;

// First (row, column) of thread (threadIdx.x, threadIdx.y) in the local
// work-group lb of a run whose rows are `ncol` wide.
struct Cell2 {
    int i, j;
};
template <int RS>
__device__ inline Cell2 block_cell(int lb, int ncol, int tx, int ty)
{
    const int nbx = (ncol + 63) / 64;
    const int by = lb / nbx, bx = lb - by * nbx;
    return Cell2{by * 4 * RS + RS * ty, bx * 64 + tx};
}
template <int RS>
__device__ inline Cell2 block_cell(int lb, int ncol)
{
    return block_cell<RS>(lb, ncol, (int)threadIdx.x, (int)threadIdx.y);
}

template <typename T>
__global__ void k_fill(T *__restrict__ p, size_t n, T v)
{
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
        p[q] = v;
}

// ------------------------------------------------------------------
// Step bookkeeping
// ------------------------------------------------------------------

// One thread: count the particle-steps this step advances, decide per run
// whether it sorts (never when may_sort is 0: a step launched without the
// sort kernels), and lay the sort spans of the sorting runs end to end.
template <typename T>
__device__ void step_begin_one(const RunDev<T> *__restrict__ runs, int n_runs, int span,
                               unsigned long long *__restrict__ span_off, int may_sort)
{
    unsigned long long acc = 0;
    for (int r = 0; r < n_runs; ++r) {
        const gptr<unsigned long long> c = glb(runs[r].ctr);
        c[kPartSteps] += c[kTotal] - c[kDeadSinceSort];
        const int K = runs[r].sort_interval;
        const bool now = may_sort && K > 0 && (c[kNeedSort] != 0 || c[kStep] % (unsigned long long)K == 0);
        c[kSortNow] = now ? 1ull : 0ull;
        span_off[r] = acc;
        if (now) acc += (c[kTotal] + span - 1) / span;
    }
    span_off[n_runs] = acc;
}

template <typename T>
__global__ void k_step_begin(const RunDev<T> *__restrict__ runs, int n_runs, int span,
                             unsigned long long *__restrict__ span_off, int may_sort)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) step_begin_one(runs, n_runs, span, span_off, may_sort);
}

// One thread: close the sort of every sorting run (the live count becomes
// the particle count, deletions since the last sort join the total, the
// buffers swap), then lay the push chunks of all runs end to end and reset
// the per-XCD chunk counters.
template <typename T>
__device__ void sort_finish_one(const RunDev<T> *__restrict__ runs, int n_runs, int chunk,
                                unsigned long long *__restrict__ chunk_off, unsigned int *__restrict__ work)
{
    unsigned long long acc = 0;
    for (int r = 0; r < n_runs; ++r) {
        const gptr<unsigned long long> c = glb(runs[r].ctr);
        if (c[kSortNow]) {
            c[kDeleted] += c[kDeadSinceSort];
            c[kDeadSinceSort] = 0;
            c[kTotal] = c[kLive];
            c[kCur] ^= 1ull;
            c[kNeedSort] = 0;
        }
        chunk_off[r] = acc;
        acc += (c[kTotal] + chunk - 1) / chunk;
    }
    chunk_off[n_runs] = acc;
    for (int x = 0; x < 8; ++x) work[x] = 0;
}

// ------------------------------------------------------------------
// Field kernels: 64 x 4 work-groups, run r owning work-groups
// [off[r], off[r+1]) of the launch
// ------------------------------------------------------------------

// The step's opening before the first Faraday half: work-group 0's first
// thread does the bookkeeping (with begin set, that of a step launched
// without the sort kernels: no run sorts; then the closing of the sorts and
// the layout of the push chunks), and every work-group clears its share of
// the three deposit planes (256 threads x kZeroPerThread entries each).
template <typename T>
__device__ inline void open_block(const RunDev<T> *__restrict__ runs, int n_runs, const int *__restrict__ off,
                                  int begin, int span, unsigned long long *__restrict__ span_off, int chunk,
                                  unsigned long long *__restrict__ chunk_off, unsigned int *__restrict__ work, int blk)
{
    if (blk == 0 && threadIdx.x == 0) {
        if (begin) step_begin_one(runs, n_runs, span, span_off, 0);
        sort_finish_one(runs, n_runs, chunk, chunk_off, work);
    }
    if (blk >= off[n_runs]) return; // padding
    const int r = run_of(off, n_runs, blk);
    const RunDev<T> &R = runs[r];
    const size_t n = R.L.size();
    const gptr<T> f0 = glb(R.fld[cFR]), f1 = glb(R.fld[cFTH]), f2 = glb(R.fld[cFPH]);
    const size_t b = (size_t)(blk - off[r]) * (256 * kZeroPerThread) + threadIdx.x;
#pragma unroll
    for (int q = 0; q < kZeroPerThread; ++q) {
        const size_t e = b + 256 * q;
        if (e < n) {
            f0[e] = (T)0;
            f1[e] = (T)0;
            f2[e] = (T)0;
        }
    }
}

// The updates of a thread's rows are formed first and stored together, so
// that no load waits behind a store it cannot be proven not to alias.  The
// loads are unconditional, at a row clamped to nr and columns clamped into
// the tables (rows -1 and nr + 1 are ghost rows; column nth + 1 lies in the
// row's padding or is the next row's first entry, column -1 in the previous
// row), so that all of them are issued before the first wait; only the
// stores are conditional, and where they happen the indices were not
// clamped.
template <typename T>
__device__ __forceinline__ void faraday_rows(gptr<const T> __restrict__ Er, gptr<const T> __restrict__ Eth,
                                             gptr<const T> __restrict__ Eph, gptr<T> __restrict__ Br,
                                             gptr<T> __restrict__ Bth, gptr<T> __restrict__ Bph, const Metric &m,
                                             const Layout &L, int i0, int j, double hc)
{
    const int nr = L.nr, nth = L.nth;
    const gptr<const double> s = glb(m.s), invr = glb(m.invr), icBr = glb(m.icBr), rn = glb(m.r_node),
                             idr2 = glb(m.idr2), dr = glb(m.dr), idth = glb(m.idth);
    double br[kFieldRows], bth[kFieldRows], bph[kFieldRows];
#pragma unroll
    for (int rs = 0; rs < kFieldRows; ++rs) {
        const int i = min(i0 + rs, nr);
        {
            const double circ = (double)Eph[L.at(i, j)] * s[j] - (double)Eph[L.at(i, j + 1)] * s[min(j + 1, nth)];
            br[rs] = (double)Br[L.at(i, j)] + hc * circ * invr[i] * icBr[j];
        }
        {
            const double circ = (double)Eph[L.at(i + 1, j)] * rn[i + 1 + L.G] - (double)Eph[L.at(i, j)] * rn[i + L.G];
            bth[rs] = (double)Bth[L.at(i, j)] + hc * circ * idr2[i];
        }
        {
            const double a = (double)Eth[L.at(i, j)] * rn[i + L.G] - (double)Eth[L.at(i + 1, j)] * rn[i + 1 + L.G];
            const double b = ((double)Er[L.at(i, j)] - (double)Er[L.at(i, j + 1)]) * dr[i] * idth[j];
            bph[rs] = (double)Bph[L.at(i, j)] + hc * (a - b) * idr2[i];
        }
    }
#pragma unroll
    for (int rs = 0; rs < kFieldRows; ++rs) {
        const int i = i0 + rs;
        if (i >= 1 && i < nr && j < nth) Br[L.at(i, j)] = (T)br[rs];
        if (i < nr && j >= 1 && j < nth) Bth[L.at(i, j)] = (T)bth[rs];
        if (i < nr && j < nth) Bph[L.at(i, j)] = (T)bph[rs];
    }
}

// B += hc * circulation(E) / area for B_r (i, j+1/2), B_th (i+1/2, j),
// B_ph (i+1/2, j+1/2).  B_r is held at zero on the conductors and B_th on
// the axis.
template <typename T>
__device__ inline void faraday_block(const RunDev<T> *__restrict__ runs, int n_runs, const int *__restrict__ off,
                                     T hc_frac, int b, int tx, int ty)
{
    const int r = run_of(off, n_runs, b);
    const RunDev<T> &R = runs[r];
    const Cell2 q = block_cell<kFieldRows>(b - off[r], R.L.nth + 1, tx, ty);
    if (q.j > R.L.nth) return;
    faraday_rows<T>(glb((const T *)R.fld[cER]), glb((const T *)R.fld[cETH]), glb((const T *)R.fld[cEPH]),
                    glb(R.fld[cBR]), glb(R.fld[cBTH]), glb(R.fld[cBPH]), R.m, R.L, q.i, q.j,
                    (double)hc_frac * R.cd);
}

// The step's opening launch: work-groups [0, nz_pad) close the sorts, lay
// out the push chunks and clear the face-charge planes (nz_pad: the zeroing
// map's work-groups padded to a multiple of eight, so that the XCD of a
// work-group is its index modulo eight in both parts); the rest take the
// first half Faraday update, which touches other arrays.
template <typename T>
__global__ __launch_bounds__(256) void k_open_faraday(const RunDev<T> *__restrict__ runs, int n_runs,
                                                      const int *__restrict__ off_zero, int nz_pad, int begin,
                                                      int span, unsigned long long *__restrict__ span_off,
                                                      int chunk, unsigned long long *__restrict__ chunk_off,
                                                      unsigned int *__restrict__ work,
                                                      const int *__restrict__ off_grid, int ng, T hc_frac)
{
    const int b = blockIdx.x;
    if (b < nz_pad) {
        open_block<T>(runs, n_runs, off_zero, begin, span, span_off, chunk, chunk_off, work, b);
        return;
    }
    faraday_block<T>(runs, n_runs, off_grid, hc_frac, xcd_tile(b - nz_pad, ng), (int)threadIdx.x & 63,
                     (int)threadIdx.x >> 6);
}

// E += (c circulation(B) - F) / area, then the lossy-layer factor on E;
// unconditional loads at clamped indices, conditional stores, as for B.
template <typename T>
__device__ __forceinline__ void ampere_rows(gptr<const T> __restrict__ Br, gptr<const T> __restrict__ Bth,
                                            gptr<const T> __restrict__ Bph, gptr<const T> __restrict__ Fr,
                                            gptr<const T> __restrict__ Fth, gptr<const T> __restrict__ Fph,
                                            gptr<T> __restrict__ Er, gptr<T> __restrict__ Eth,
                                            gptr<T> __restrict__ Eph, const Metric &m, const Layout &L, int i0,
                                            int j, double c)
{
    const int nr = L.nr, nth = L.nth;
    const gptr<const double> sb = glb(m.sb), invrb = glb(m.invrb), invA = glb(m.invA), idkb = glb(m.idkb),
                             ab_half = glb(m.ab_half), rb = glb(m.rb), isb2pi = glb(m.isb2pi),
                             idrb2 = glb(m.idrb2), ab_int = glb(m.ab_int), drb = glb(m.drb), idthb = glb(m.idthb);
    double er[kFieldRows], eth[kFieldRows], eph[kFieldRows];
    const double sbj = sb[j], sbw = sb[max(j - 1, 0)];
#pragma unroll
    for (int rs = 0; rs < kFieldRows; ++rs) {
        const int i = min(i0 + rs, nr);
        const size_t e = L.at(i, j);
        const double bph = Bph[e], bph_w = Bph[L.at(i, j - 1)]; // column -1 lies in the previous row
        {
            const double t1 = j < nth ? sbj * bph : 0.0;
            const double t0 = j > 0 ? sbw * bph_w : 0.0;
            er[rs] = ((double)Er[e] + (c * (t1 - t0) * invrb[i] - (double)Fr[e] * invA[i]) * idkb[j]) * ab_half[i];
        }
        {
            const double circ = rb[i - 1 + L.G] * (double)Bph[L.at(i - 1, j)] - rb[i + L.G] * bph;
            eth[rs] = ((double)Eth[e] + (c * circ - (double)Fth[e] * isb2pi[j]) * idrb2[i]) * ab_int[i];
        }
        {
            const double a = rb[i + L.G] * (double)Bth[e] - rb[i - 1 + L.G] * (double)Bth[L.at(i - 1, j)];
            const double b = ((double)Br[e] - (double)Br[L.at(i, j - 1)]) * drb[i] * idthb[j];
            eph[rs] = ((double)Eph[e] + (c * (a - b) - (double)Fph[e] * idthb[j]) * idrb2[i]) * ab_int[i];
        }
    }
#pragma unroll
    for (int rs = 0; rs < kFieldRows; ++rs) {
        const int i = i0 + rs;
        if (i < nr) Er[L.at(i, j)] = (T)er[rs];
        if (i >= 1 && i < nr && j < nth) Eth[L.at(i, j)] = (T)eth[rs];
        if (i >= 1 && i < nr && j >= 1 && j < nth) Eph[L.at(i, j)] = (T)eph[rs];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_ampere(const RunDev<T> *__restrict__ runs, int n_runs,
                                                const int *__restrict__ off)
{
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int r = run_of(off, n_runs, b);
    const RunDev<T> &R = runs[r];
    const Cell2 q = block_cell<kFieldRows>(b - off[r], R.L.nth + 1);
    if (q.j > R.L.nth) return;
    ampere_rows<T>(glb((const T *)R.fld[cBR]), glb((const T *)R.fld[cBTH]), glb((const T *)R.fld[cBPH]),
                   glb(R.ffin[0]), glb(R.ffin[1]), glb(R.ffin[2]), glb(R.fld[cER]), glb(R.fld[cETH]),
                   glb(R.fld[cEPH]), R.m, R.L, q.i, q.j, R.cd);
}

// Lossy layer on B (eq. (EBcond)) over rows nr - absorb_cells - 1 .. nr
// (the factor is 1 below), for one 64 x 4 block of threads: thread (tx, ty)
// of block lb of run R, kFieldRows rows each.
template <typename T>
__device__ inline void absorb_b_block(const RunDev<T> &R, int lb, int tx, int ty)
{
    const Layout L = R.L;
    const Cell2 q = block_cell<kFieldRows>(lb, L.nth + 1, tx, ty);
    const int j = q.j;
    if (j > L.nth) return;
    const gptr<const double> ab_int = glb(R.m.ab_int), ab_half = glb(R.m.ab_half);
    const gptr<T> Br = glb(R.fld[cBR]), Bth = glb(R.fld[cBTH]), Bph = glb(R.fld[cBPH]);
    const int i0 = L.nr - R.absorb_cells - 1 + q.i;
    // all loads of the thread's rows (unconditional, at a row clamped into
    // 0..nr) before its conditional stores
    T br[kFieldRows], bth[kFieldRows], bph[kFieldRows];
#pragma unroll
    for (int rs = 0; rs < kFieldRows; ++rs) {
        const int i = min(max(i0 + rs, 0), L.nr);
        br[rs] = (T)((double)Br[L.at(i, j)] * ab_int[i]);
        bth[rs] = (T)((double)Bth[L.at(i, j)] * ab_half[i]);
        bph[rs] = (T)((double)Bph[L.at(i, j)] * ab_half[i]);
    }
#pragma unroll
    for (int rs = 0; rs < kFieldRows; ++rs) {
        const int i = i0 + rs;
        if (i >= 0 && i <= L.nr && j < L.nth) Br[L.at(i, j)] = br[rs];
        if (i >= 0 && i < L.nr) Bth[L.at(i, j)] = bth[rs];
        if (i >= 0 && i < L.nr && j < L.nth) Bph[L.at(i, j)] = bph[rs];
    }
}

// One pass of the 1-2-1 filter.  kind 0: integer-j positions (F_r, F_ph,
// node charge), kind 1: half-integer j (F_th).  In theta the array is
// extended by zeros, filtered, and what spilled across a pole is folded
// back onto its mirror image, with a plus sign for integer-j components and
// a minus sign for the theta component; radially the array is extended by
// zeros beyond rows [-G, last row].
template <typename T, typename Ptr>
__device__ inline T theta_pass(Ptr a, const Layout &L, int i, int j, int kind)
{
    const int nth = L.nth;
    const int ncol = kind ? nth : nth + 1;
    const Ptr row = a + L.at(i, 0);
    T v = (T)0.5 * row[j];
    if (j > 0) v += (T)0.25 * row[j - 1];
    if (j + 1 < ncol) v += (T)0.25 * row[j + 1];
    if (kind == 0) {
        if (j == 1) v += (T)0.25 * row[0];
        if (j == nth - 1) v += (T)0.25 * row[nth];
    } else {
        if (j == 0) v -= (T)0.25 * row[0];
        if (j == nth - 1) v -= (T)0.25 * row[nth - 1];
    }
    return v;
}

// All n_filt passes of the 1-2-1 filter over one face-charge plane, by
// strips held in registers: a wave takes 64 consecutive columns, H of them
// halo on each side, over kFiltRB rows plus H halo rows above and below
// (H >= the run's passes).  Each pass forms the theta half (neighbouring
// columns from the next lanes; the edge and axis rules of the plane's
// parity: what spills across a pole folds back onto its mirror image, with
// a plus sign for integer-j components and a minus sign for the theta
// component) and then the radial half (the rows above and below in the
// lane's own registers); entries outside the array, and those whose
// neighbours lie outside the strip, are held at zero, so that the valid
// part shrinks by one column and row per pass and H passes leave the
// centre exact.  Each value is formed with the same operations, in the
// same order, as one pass over the whole plane.  No LDS, no barriers.
constexpr int kFiltRB = 32;
template <int H>
__host__ __device__ constexpr int filt_cols() { return 64 - 2 * H; } // useful columns of a strip

template <typename T, int H>
__device__ inline void filter_strip(const RunDev<T> &R, int comp, int q, int lane)
{
    constexpr int U = filt_cols<H>(), NW = kFiltRB + 2 * H;
    const Layout L = R.L;
    const int passes = R.n_filt;
    const int kind = comp == 1 ? 1 : 0;
    const int nth = L.nth, ncol = kind ? nth : nth + 1;
    const int first = -L.G, last = comp == 0 ? L.nr + L.G - 1 : L.nr + L.G;
    const int S = (nth + 1 + U - 1) / U;
    const int sb = q % S, rb = q / S;
    const int r0 = first + rb * kFiltRB; // first output row
    if (r0 > last) return;
    const int j = sb * U - H + lane;     // the lane's column
    const bool jin = j >= 0 && j < ncol;
    const int i0 = r0 - H;               // the strip's first row
    const gptr<const T> src = glb((const T *)R.fld[cFR + comp]);
    const gptr<T> dst = glb(R.ftmp[comp]);
    // theta-half flags of the lane: bit 0 the half is formed (the column is in
    // the array and both neighbours are in the strip), bit 1 j > 0, bit 2
    // j + 1 < ncol, bits 3 and 4 the axis node j = 0 or nth mirrored onto
    // j = 1 or nth - 1 (integer j), bits 5 and 6 the odd parity at j = 0 or
    // nth - 1 (half-integer j)
    const unsigned fl = (unsigned)(jin && lane >= 1 && lane <= 62) | (unsigned)(j > 0) << 1 |
                        (unsigned)(j + 1 < ncol) << 2 | (unsigned)(kind == 0 && j == 1) << 3 |
                        (unsigned)(kind == 0 && j == nth - 1) << 4 | (unsigned)(kind == 1 && j == 0) << 5 |
                        (unsigned)(kind == 1 && j == nth - 1) << 6;
    T v[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const int i = i0 + k;
        v[k] = (jin && i >= first && i <= last) ? src[L.at(i, j)] : (T)0;
    }
    for (int p = 0; p < passes; ++p) {
        // the theta half of row k, formed where the row is in the array
        auto theta = [&](int k) -> T {
            const T r0v = v[k];
            const T rm = __shfl_up(r0v, 1), rp = __shfl_down(r0v, 1);
            const int i = i0 + k;
            T t = (T)0;
            if ((fl & 1u) && i >= first && i <= last) {
                t = (T)0.5 * r0v;
                t += (fl & 2u) ? (T)0.25 * rm : (T)0;
                t += (fl & 4u) ? (T)0.25 * rp : (T)0;
                t += (fl & 8u) ? (T)0.25 * rm : (T)0;  // the axis node j = 0, mirrored
                t += (fl & 16u) ? (T)0.25 * rp : (T)0; // the axis node j = nth, mirrored
                t -= (fl & 32u) ? (T)0.25 * r0v : (T)0; // odd parity across the axis
                t -= (fl & 64u) ? (T)0.25 * r0v : (T)0;
            }
            return t;
        };
        // the radial half of row k from the theta halves of rows k - 1, k, k + 1
        T tm = (T)0, t0 = theta(0);
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const T t1 = k + 1 < NW ? theta(k + 1) : (T)0;
            const int i = i0 + k;
            T w = (T)0;
            if (jin && i >= first && i <= last && k >= 1 && k <= NW - 2) {
                w = (T)0.5 * t0;
                w += (T)0.25 * tm;
                w += (T)0.25 * t1;
            }
            v[k] = w;
            tm = t0;
            t0 = t1;
        }
    }
    if (lane >= H && lane < 64 - H && jin) {
#pragma unroll
        for (int k = H; k < H + kFiltRB; ++k) {
            const int i = i0 + k;
            if (i <= last) dst[L.at(i, j)] = v[k];
        }
    }
}

// The second half Faraday update and the filter of the face charges in one
// launch (they touch disjoint arrays): work-groups [0, nf_pad) filter, four
// waves each, one strip (filter_strip) per wave -- nf = 3 x the filter
// work-groups of all runs, padded to a multiple of eight so that the XCD of
// a work-group is its index modulo eight in both parts -- and the rest
// update B, 64 x 4 threads each.
template <typename T, int H>
__global__ __launch_bounds__(256) void k_faraday_filter(const RunDev<T> *__restrict__ runs, int n_runs,
                                                        const int *__restrict__ off_filt, int nf, int nf_pad,
                                                        const int *__restrict__ off_grid, int ng, T hc_frac)
{
    const int b = blockIdx.x;
    if (b < nf_pad) {
        const int v = xcd_tile(b, nf_pad);
        if (v >= nf) return; // the same for the whole work-group
        const int per = nf / 3, comp = v / per, lb = v - comp * per;
        const int r = run_of(off_filt, n_runs, lb);
        const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
        filter_strip<T, H>(runs[r], comp, 4 * (lb - off_filt[r]) + wv, lane);
        return;
    }
    faraday_block<T>(runs, n_runs, off_grid, hc_frac, xcd_tile(b - nf_pad, ng), (int)threadIdx.x & 63,
                     (int)threadIdx.x >> 6);
}

// The same pass on one integer-j array (the Gauss diagnostic's node charge).
template <typename T>
__global__ __launch_bounds__(256) void k_filter_nodes(const T *__restrict__ src, T *__restrict__ dst, Layout L)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = -L.G + (int)(blockIdx.y * blockDim.y + threadIdx.y);
    const int last = L.nr + L.G;
    if (i > last || j > L.nth) return;
    T v = (T)0.5 * theta_pass<T>(src, L, i, j, 0);
    if (i > -L.G) v += (T)0.25 * theta_pass<T>(src, L, i - 1, j, 0);
    if (i < last) v += (T)0.25 * theta_pass<T>(src, L, i + 1, j, 0);
    dst[L.at(i, j)] = v;
}

// ------------------------------------------------------------------
// Particle push
// ------------------------------------------------------------------

// A run as one particle sees it.
template <typename T>
struct PushArgs {
    Layout L;
    GFields<T> f;         // E, B (read) and F (deposit target)
    Background bg;
    int r_kind, th_kind, mover, n_filt;
    T c, dxi, inv_dxi, nth_f, two_over_nth, pi_over_nth, inv_pi_over_nth, eps0, inv_rl;
    gptr<const T> r_node; // r(i) at [i + G]
    gptr<uint32_t> cell;
    gptr<T> dx, dy, ur, ut, up;
    gptr<const T> w;
    gptr<unsigned long long> n_dead;
    gptr<int> status;
};

template <typename T>
__device__ inline PushArgs<T> push_args(const RunDev<T> &R, int cur, double step)
{
    PushArgs<T> p;
    p.L = R.L;
#pragma unroll
    for (int q = 0; q < 9; ++q) p.f.c[q] = glb(R.fld[q]);
    p.bg = R.bg;
    p.r_kind = R.r_kind;
    p.th_kind = R.th_kind;
    p.mover = R.mover;
    p.n_filt = R.n_filt;
    p.c = R.c;
    p.dxi = R.dxi;
    p.inv_dxi = R.inv_dxi;
    p.nth_f = R.nth_f;
    p.two_over_nth = R.two_over_nth;
    p.pi_over_nth = R.pi_over_nth;
    p.inv_pi_over_nth = R.inv_pi_over_nth;
    p.eps0 = R.eps0;
    p.inv_rl = (T)inv_light_cylinder(R.omega, R.t_spin, R.cd, step);
    p.r_node = glb(R.r_push);
    p.cell = glb(R.cell[cur]);
    p.dx = glb(R.arr[cur][0]);
    p.dy = glb(R.arr[cur][1]);
    p.ur = glb(R.arr[cur][2]);
    p.ut = glb(R.arr[cur][3]);
    p.up = glb(R.arr[cur][4]);
    p.w = glb((const T *)R.arr[cur][5]);
    p.n_dead = glb(R.ctr + kDeadSinceSort);
    p.status = glb(R.status);
    return p;
}

// Bilinear interpolation of one staggered lattice from its four values at
// (i, j), (i + 1, j), (i, j + 1), (i + 1, j + 1), at offsets (x, y).
template <typename T>
__device__ __forceinline__ T bilin(T v00, T v10, T v01, T v11, T x, T y)
{
    const T lo = v00 + x * (v10 - v00), hi = v01 + x * (v11 - v01);
    return lo + y * (hi - lo);
}

// Fields read straight from global memory (chunks not staged in LDS).
template <typename T>
struct GlobalView {
    const GFields<T> *f;
    Layout L;
    gptr<const T> rn; // r(i) at [i + G]
    __device__ T r_node(int i) const { return rn[i + L.G]; }
    __device__ T get(int c, int i, int j) const { return f->c[c][L.at(i, j)]; }
    // half-integer-j component continued across the axis with parity sgn
    __device__ T geth(int c, int i, int j, T sgn) const
    {
        if (j < 0) return sgn * f->c[c][L.at(i, 0)];
        if (j >= L.nth) return sgn * f->c[c][L.at(i, L.nth - 1)];
        return f->c[c][L.at(i, j)];
    }
    // Plasma field at offset (fx, fy) of cell (i, j): bilinear in grid
    // coordinates from each component's own staggered lattice; half-integer-j
    // components continue across the axis with their parity (r even, theta
    // and phi odd).
    __device__ void gather(int i, int j, T fx, T fy, T E[3], T B[3]) const
    {
        int ih = i, jh = j;
        T hx = fx - (T)0.5, hy = fy - (T)0.5;
        if (hx < (T)0) { ih = i - 1; hx += (T)1; }
        if (hy < (T)0) { jh = j - 1; hy += (T)1; }
        E[0] = bilin(get(cER, ih, j), get(cER, ih + 1, j), get(cER, ih, j + 1), get(cER, ih + 1, j + 1), hx, fy);
        E[1] = bilin(geth(cETH, i, jh, (T)-1), geth(cETH, i + 1, jh, (T)-1), geth(cETH, i, jh + 1, (T)-1),
                     geth(cETH, i + 1, jh + 1, (T)-1), fx, hy);
        E[2] = bilin(get(cEPH, i, j), get(cEPH, i + 1, j), get(cEPH, i, j + 1), get(cEPH, i + 1, j + 1), fx, fy);
        B[0] = bilin(geth(cBR, i, jh, (T)1), geth(cBR, i + 1, jh, (T)1), geth(cBR, i, jh + 1, (T)1),
                     geth(cBR, i + 1, jh + 1, (T)1), fx, hy);
        B[1] = bilin(get(cBTH, ih, j), get(cBTH, ih + 1, j), get(cBTH, ih, j + 1), get(cBTH, ih + 1, j + 1), hx, fy);
        B[2] = bilin(geth(cBPH, ih, jh, (T)-1), geth(cBPH, ih + 1, jh, (T)-1), geth(cBPH, ih, jh + 1, (T)-1),
                     geth(cBPH, ih + 1, jh + 1, (T)-1), hx, hy);
    }
};

// A deposit target gives the entry of node (i, j) (the same in its three
// face-charge planes), the entry step to node (i + a, j + b), the unit in
// which charges are added (each particle's charge is scaled to it once) and
// the add itself.  In global memory: FP atomics on the field arrays.
template <typename T>
struct GlobalDep {
    using Off = long long;
    gptr<T> F[3];
    Layout L;
    __device__ Off at(int i, int j) const { return (Off)L.at(i, j); }
    __device__ Off di() const { return L.pitch; }
    __device__ Off step(int a, int b) const { return (Off)a * L.pitch + b; }
    __device__ T unit() const { return (T)1; }
    __device__ void add(int c, Off e, T v) const { atomic_add(F[c] + e, v); }
};

// Entries per LDS plane of a push work-group: a compile-time stride, so
// that every plane of one (i, j) is reached with an immediate offset from
// one address.  FP32: nine planes (6 x 4 B fields, 3 x 8 B deposits), the
// radii of the region's rows and the work-group's few static bytes within
// 40 KB, so that four work-groups share a CU's 160 KB; FP64 (two
// work-groups per CU, as its registers allow; 6 x 8 B fields, 3 x 8 B +
// 3 x 4 B deposits): within 80 KB.
template <typename T>
constexpr int lds_plane();
template <>
constexpr int lds_plane<float>() { return 832; }
template <>
constexpr int lds_plane<double>() { return 956; }
constexpr int kLdsRows = 128; // most rows of a staged region

// Entry of node (i, j) in a staged plane of C columns whose first node is
// (i0, j0); offsets within a work-group's region stay far below 2^23, so
// the 24-bit multiply (full rate) serves.
__device__ __forceinline__ int lds_entry(int i, int j, int i0, int j0, int C)
{
    return __mul24(i - i0, C) + (j - j0);
}

template <typename T>
struct LdsView {
    static constexpr int P = lds_plane<T>();
    const T *s;
    const T *rn; // r(i) of the region's rows at [i - i0]
    int i0, j0, C;
    __device__ T r_node(int i) const { return rn[i - i0]; }
    // As GlobalView::gather; the axis mirror was applied when the planes
    // were staged, and the stencils of the four lattices are reached from
    // one entry by steps of one row (C) or one column.  All 24 values are
    // read before the first is used, so that the particle waits for LDS
    // once rather than once per component.
    __device__ void gather(int i, int j, T fx, T fy, T E[3], T B[3]) const
    {
        const int e = lds_entry(i, j, i0, j0, C);
        int ex = e, ey = e; // (i - 1, j) and (i, j - 1) when the half-node lies below
        T hx = fx - (T)0.5, hy = fy - (T)0.5;
        if (hx < (T)0) { ex = e - C; hx += (T)1; }
        if (hy < (T)0) { ey = e - 1; hy += (T)1; }
        const int exy = ex + (ey - e);
        const int at[6] = {ex, ey, e, ey, ex, exy};
        const int comp[6] = {cER, cETH, cEPH, cBR, cBTH, cBPH};
        T v[6][4];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const T *a = s + comp[q] * P + at[q];
            v[q][0] = a[0];
            v[q][1] = a[C];
            v[q][2] = a[1];
            v[q][3] = a[C + 1];
        }
        E[0] = bilin(v[0][0], v[0][1], v[0][2], v[0][3], hx, fy);
        E[1] = bilin(v[1][0], v[1][1], v[1][2], v[1][3], fx, hy);
        E[2] = bilin(v[2][0], v[2][1], v[2][2], v[2][3], fx, fy);
        B[0] = bilin(v[3][0], v[3][1], v[3][2], v[3][3], fx, hy);
        B[1] = bilin(v[4][0], v[4][1], v[4][2], v[4][3], hx, fy);
        B[2] = bilin(v[5][0], v[5][1], v[5][2], v[5][3], hx, hy);
    }
};

// Deposit planes in LDS hold fixed point, so that integer LDS atomics (much
// faster than floating-point ones) accumulate the contributions exactly and
// in any order.  Every contribution v is at most max|w| in magnitude.
//  FP32: one 64-bit plane per component, v stored as round(v * 2^40 /
//        max|w|), rounded to the integer through FP64 with the 1.5 * 2^52
//        shift; the quantum, 1e-12 max|w|, lies below the FP32 rounding of
//        contributions far smaller than max|w| (small azimuthal steps,
//        plasma particles beside heavier injected ones).
//  FP64: x = v * 2^48 / max|w| is split into its nearest integer (a 64-bit
//        plane, converted exactly with the 1.5 * 2^52 shift, valid below
//        2^51) and the exact remainder in [-1/2, 1/2] in units of 2^-16 (a
//        32-bit plane): the quantum is 2^-64 max|w|, far below FP64 rounding
//        even where the charges of co-located pairs cancel.
// A chunk of at most 4096 particles adds at most four contributions to an
// entry: below 2^54 (FP32) or 2^62 (FP64) in the 64-bit planes and 2^31 in
// the 32-bit ones.
template <typename T>
constexpr int fixed_bits();
template <>
constexpr int fixed_bits<float>() { return 40; }
template <>
constexpr int fixed_bits<double>() { return 48; }
constexpr double kLoScale = 65536.0; // units of the FP64 remainder plane per unit of the main plane

template <typename T>
struct LdsDep;

template <>
struct LdsDep<float> {
    using Off = int;
    static constexpr int P = lds_plane<float>();
    long long *s;
    int *lo; // unused in FP32
    int i0, j0, C;
    float scale;
    __device__ int at(int i, int j) const { return lds_entry(i, j, i0, j0, C); }
    __device__ int di() const { return C; }
    __device__ int step(int a, int b) const { return __mul24(a, C) + b; }
    __device__ float unit() const { return scale; }
    __device__ void add(int c, int e, float v) const
    {
        const double sh = (double)v + 6755399441055744.0; // 1.5 * 2^52
        const long long q = __double_as_longlong(sh) - 0x4338000000000000ll;
        atomicAdd((unsigned long long *)&s[c * P + e], (unsigned long long)q);
    }
};

template <>
struct LdsDep<double> {
    using Off = int;
    static constexpr int P = lds_plane<double>();
    long long *s;
    int *lo;
    int i0, j0, C;
    double scale;
    __device__ int at(int i, int j) const { return lds_entry(i, j, i0, j0, C); }
    __device__ int di() const { return C; }
    __device__ int step(int a, int b) const { return __mul24(a, C) + b; }
    __device__ double unit() const { return scale; }
    __device__ void add(int c, int e, double x) const
    {
        const double sh = x + 6755399441055744.0;                 // 1.5 * 2^52: the integer lands in the low bits
        const long long hi = __double_as_longlong(sh) - 0x4338000000000000ll;
        const double rem = x - (sh - 6755399441055744.0);         // exact, |rem| <= 1/2
        const int r = (int)__builtin_rint(rem * kLoScale);
        atomicAdd((unsigned long long *)&s[c * P + e], (unsigned long long)hi);
        atomicAdd(&lo[c * P + e], r);
    }
};

// Charge flux of a cell-sized cloud moving on a straight piece (xa, ya) ->
// (xb, yb) inside the cell whose first node is entry e, at grid offset
// (ox, oy) from the frame of the coordinates: the integral of the bilinear
// weights along the piece.
template <typename T, typename D>
__device__ __forceinline__ void vb_piece(const D &d, typename D::Off e, T xa, T ya, T xb, T yb, T ox, T oy, T Q)
{
    const T mx = (T)0.5 * (xa + xb) - ox, my = (T)0.5 * (ya + yb) - oy;
    const T qx = Q * (xb - xa), qy = Q * (yb - ya);
    const T ax = qx * my, ay = qy * mx;
    d.add(0, e, qx - ax);
    d.add(0, e + 1, ax);
    d.add(1, e, qy - ay);
    d.add(1, e + d.di(), ay);
}

// Villasenor-Buneman deposit of the move (x0, y0) -> (x1, y1), both in the
// frame of cell (i, j) (start in [0,1)^2, end within one cell of it): cut at
// the cell faces it crosses (at most one per axis), in the order met along
// the path; the first piece lies in cell (i, j), the last in the end cell
// (i + cx, j + cy), a middle one in the cell entered at the first crossing.
// Plus the ring charge Q dphi / 2 pi crossing a meridional half-plane,
// assigned bilinearly at the midpoint of the move.  The last row of cells
// holds y = nth.  Q is in the target's unit.
template <typename T, typename D>
__device__ inline void vb_deposit(const D &d, int i, int j, int nth, T x0, T y0, T x1, T y1, T Q, T dphi)
{
    const int cx = x1 >= (T)1 ? 1 : (x1 < (T)0 ? -1 : 0);
    const int cy = (y1 >= (T)1 && j < nth - 1) ? 1 : (y1 < (T)0 ? -1 : 0);
    const T X = cx > 0 ? (T)1 : (T)0, Y = cy > 0 ? (T)1 : (T)0;
    // path parameters of the crossings (2: none) and the other coordinate
    // there; formed on every lane and selected, so that lanes with different
    // crossings share one instruction stream
    const T dx = x1 - x0, dy = y1 - y0;
    const T tx = cx ? FM<T>::div(X - x0, dx) : (T)2, ty = cy ? FM<T>::div(Y - y0, dy) : (T)2;
    const T yx = y0 + tx * dy, xy = x0 + ty * dx;
    const bool both = cx != 0 && cy != 0, xf = tx < ty, yf = ty < tx;
    // split points s1, s2 (n of them) between the start and the end; the
    // middle piece lies in cell (i + a, j + b)
    const bool two = both && (xf || yf);
    const int n = two ? 2 : ((cx != 0 || cy != 0) ? 1 : 0);
    T s1x = x1, s1y = y1;
    if (xf) { s1x = X; s1y = yx; }
    else if (yf) { s1x = xy; s1y = Y; }
    else if (both) { s1x = X; s1y = Y; } // both faces at once: the corner
    const T s2x = two ? (xf ? xy : X) : x1, s2y = two ? (xf ? Y : yx) : y1;
    const int a = two && !xf ? 0 : cx, b = two && xf ? 0 : cy;
    const typename D::Off e = d.at(i, j);
    vb_piece(d, e, x0, y0, s1x, s1y, (T)0, (T)0, Q);
    if (n >= 1) vb_piece(d, e + d.step(a, b), s1x, s1y, s2x, s2y, (T)a, (T)b, Q);
    if (n >= 2) vb_piece(d, e + d.step(cx, cy), s2x, s2y, x1, y1, (T)cx, (T)cy, Q);
    const T mx = (T)0.5 * (x0 + x1), my = (T)0.5 * (y0 + y1);
    const T ci = floor(mx);
    T cj = floor(my);
    if (j + (int)cj > nth - 1) cj = (T)(nth - 1 - j);
    const T fx = mx - ci, fy = my - cj;
    const T q = Q * dphi * (T)(0.5 / kPi);
    const T q1 = q * fy, q0 = q - q1;                   // rows j and j + 1 of the cell
    const T a0 = q0 * fx, a1 = q1 * fx;
    const typename D::Off er = e + d.step((int)ci, (int)cj);
    d.add(2, er, q0 - a0);
    d.add(2, er + d.di(), a0);
    d.add(2, er + 1, q1 - a1);
    d.add(2, er + d.di() + 1, a1);
}

template <typename T>
__device__ inline T below_one();
template <>
__device__ inline float below_one<float>() { return 0x1.fffffep-1f; }
template <>
__device__ inline double below_one<double>() { return 0x1.fffffffffffffp-1; }

// Element k of a particle array addressed from the chunk's first slot: a
// scalar base plus a 32-bit byte offset, the form of a global access with
// a scalar base (chunks are far below 4 GiB).
template <typename U>
__device__ __forceinline__ auto &at_slot(gptr<U> a, uint32_t k)
{
    return *(gptr<U>)((gptr<char>)a + k * (uint32_t)sizeof(U));
}
template <typename U>
__device__ __forceinline__ U at_slot(gptr<const U> a, uint32_t k)
{
    return *(gptr<const U>)((gptr<const char>)a + k * (uint32_t)sizeof(U));
}

// The same accesses with the non-temporal hint, for the particle streams
// that a push reads once and writes once: they pass through L2 without
// displacing what a chunk reads twice (its cells, read for the bounding box
// and again by the loop, and the field planes shared by neighbouring chunks).
template <typename U>
__device__ __forceinline__ U ld_stream(gptr<U> a, uint32_t k)
{
    return __builtin_nontemporal_load((gptr<U>)((gptr<char>)a + k * (uint32_t)sizeof(U)));
}
template <typename U>
__device__ __forceinline__ U ld_stream(gptr<const U> a, uint32_t k)
{
    return __builtin_nontemporal_load((gptr<const U>)((gptr<const char>)a + k * (uint32_t)sizeof(U)));
}
template <typename U>
__device__ __forceinline__ void st_stream(gptr<U> a, uint32_t k, U v)
{
    __builtin_nontemporal_store(v, (gptr<U>)((gptr<char>)a + k * (uint32_t)sizeof(U)));
}

// The stored state of one particle, loaded ahead of its push, and the
// state it leaves.
template <typename T>
struct PIn {
    uint32_t c;
    T fx, fy, w, u0, u1, u2;
};
template <typename T>
struct POut {
    uint32_t c;
    T fx, fy, u0, u1, u2;
};

// Every slot of a chunk lies inside the arrays (a chunk starts below the
// run's particle count, and a chunk of spare slots follows the capacity),
// so the loads are unconditional; whether the slot holds a particle is
// decided where the state is used, so that nothing waits for the loads
// before then.
template <typename T>
__device__ __forceinline__ PIn<T> load_particle(const PushArgs<T> &p, uint32_t idx)
{
    PIn<T> a;
    a.c = at_slot(p.cell, idx);
    a.fx = ld_stream(p.dx, idx);
    a.fy = ld_stream(p.dy, idx);
    a.w = ld_stream(p.w, idx);
    a.u0 = ld_stream(p.ur, idx);
    a.u1 = ld_stream(p.ut, idx);
    a.u2 = ld_stream(p.up, idx);
    return a;
}

// Every iteration of the push stores one state per lane (a lane past the
// run's last particle writes back what it loaded from its own slot, which
// may lie in the chunk of spare slots every particle array holds past the
// capacity), so that the loop issues the same memory operations on every
// path and the wait for the next particle's loads, issued before these
// stores, never waits for the stores.
template <typename T>
__device__ __forceinline__ void store_particle(const PushArgs<T> &p, uint32_t idx, const POut<T> &o)
{
    st_stream(p.dx, idx, o.fx);
    st_stream(p.dy, idx, o.fy);
    st_stream(p.ur, idx, o.u0);
    st_stream(p.ut, idx, o.u1);
    st_stream(p.up, idx, o.u2);
    st_stream(p.cell, idx, o.c);
}

// One particle: gather, push, move with cancellation-free local increments,
// deposit, particle boundaries; returns the new state (the old one if the
// move breaks the CFL bound, which is flagged).
template <typename T, typename V, typename D>
__device__ inline POut<T> push_particle(const PushArgs<T> &p, const V &view, const D &dep, const PIn<T> &in)
{
    const int nr = p.L.nr, nth = p.L.nth;
    const uint32_t cl = in.c;
    const int i = cell_i(cl), j = cell_j(cl);
    const T fx = in.fx, fy = in.fy;
    const T w = in.w;
    T r = view.r_node(i);
    if (p.r_kind == 0) r *= FM<T>::exp(fx * p.dxi);
    else r += fx * p.dxi;
    const T ir = FM<T>::rcp(r);
    T k, s;
    if (p.th_kind == 0) {
        // sin theta = (2/nth) sqrt(y (nth - y)); both factors formed from the
        // cell index and the offset so that neither cancels near a pole
        const T ys = (T)j + fy, yn = (T)(nth - j) - fy;
        // cos theta = 1 - 2 y / nth, from the node value 1 - 2 j / nth (one rounding)
        k = fma(-fy, p.two_over_nth, fma(-(T)j, p.two_over_nth, (T)1));
        s = p.two_over_nth * FM<T>::sqrt(fmax(ys * yn, (T)0));
    } else if (2 * j < nth) {
        const T th = ((T)j + fy) * p.pi_over_nth;
        s = sin(th);
        k = cos(th);
    } else { // measure the angle from the south pole
        const T th = ((T)(nth - j) - fy) * p.pi_over_nth;
        s = sin(th);
        k = -cos(th);
    }
    // the momentum in the local basis (e_r, e_th, e_ph) at the start point;
    // the movers are vector operations, the same in any orthonormal basis,
    // so they work there on the local E and B as gathered
    T ul[3] = {in.u0, in.u1, in.u2};
    const bool outer = i > nr || (i == nr && fx > (T)0); // beyond the outer conductor: ballistic
    const bool inner = i < 0;                            // inside the star: corotation field only
    const T eps = w > (T)0 ? p.eps0 : (w < (T)0 ? -p.eps0 : (T)0);
    T ig; // 1 / gamma of the new momentum
    if (!outer && eps != (T)0) {
        T E[3], B[3];
        if (!inner) {
            view.gather(i, j, fx, fy, E, B);
        } else {
            E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = (T)0;
        }
        add_background(p.bg, p.inv_rl, inner, r, ir, k, s, E, B);
        if (p.mover == 0) {
            ig = vay_push(ul, E, B, eps);
        } else {
            boris_push(ul, E, B, eps);
            ig = FM<T>::rsqrt((T)1 + ul[0] * ul[0] + ul[1] * ul[1] + ul[2] * ul[2]);
        }
    } else {
        ig = FM<T>::rsqrt((T)1 + ul[0] * ul[0] + ul[1] * ul[1] + ul[2] * ul[2]);
    }
    // Cartesian frame at phi = 0: e_r = (s, 0, k), e_th = (k, 0, -s), e_ph = (0, 1, 0)
    const T uc[3] = {s * ul[0] + k * ul[1], ul[2], k * ul[0] - s * ul[1]};
    // displacement over the step, relative to r
    const T vg = p.c * ig;
    const T ex = uc[0] * vg * ir, ey = uc[1] * vg * ir, ez = uc[2] * vg * ir;
    const T xs = s + ex, zs = k + ez;                    // (R', Z') / r
    const T q = (T)2 * (s * ex + k * ez) + ex * ex + ey * ey + ez * ez;
    T sq, isq;                                           // r' / r and its inverse
    FM<T>::sqrt_rsqrt((T)1 + q, sq, isq);
    const T eta = FM<T>::div(q, (T)1 + sq);              // r' / r - 1
    const T dX = p.r_kind == 0 ? FM<T>::log1p(eta) * p.inv_dxi : r * eta * p.inv_dxi;
    const T Rn2 = xs * xs + ey * ey;
    T Rn = (T)0, iR = (T)0;                              // R' / r and its inverse
    if (Rn2 > (T)0) FM<T>::sqrt_rsqrt(Rn2, Rn, iR);
    T dY;
    if (p.th_kind == 0) dY = (T)-0.5 * p.nth_f * ((ez - k * eta) * isq);
    else dY = FM<T>::atan2(Rn * k - zs * s, Rn * s + zs * k) * p.inv_pi_over_nth;
    const T X1 = fx + dX;
    T Y1 = fy + dY;
    if (Y1 < (T)(-j)) Y1 = (T)(-j);                      // reflection at the poles: y' in [0, nth]
    if (Y1 > (T)(nth - j)) Y1 = (T)(nth - j);
    if (!(fabs(X1 - fx) < (T)1 && fabs(Y1 - fy) < (T)1)) { // CFL (or a non-finite value)
        atomic_or(p.status, 1);
        return POut<T>{in.c, in.fx, in.fy, in.u0, in.u1, in.u2};
    }
    T cph = (T)1, sph = (T)0;
    if (Rn > (T)0) {
        cph = xs * iR;
        sph = ey * iR;
    }
    vb_deposit(dep, i, j, nth, fx, fy, X1, Y1, w * dep.unit(), FM<T>::atan2(sph, cph));
    const T k1 = zs * isq, s1 = Rn * isq;
    const T ux = cph * uc[0] + sph * uc[1], uy = -sph * uc[0] + cph * uc[1], uz = uc[2];
    // new cell: X1, Y1 lie in (-1, 2); an offset below zero rounds up to at
    // most the largest value below one
    const T fxl = floor(X1), fyl = floor(Y1);
    int ni = i + (int)fxl, nj = j + (int)fyl;
    T nx = fmin(X1 - fxl, below_one<T>()), ny = fmin(Y1 - fyl, below_one<T>());
    if (nj > nth - 1) { nj = nth - 1; ny = (T)1; }      // y' = nth belongs to the last cell
    POut<T> o;
    o.fx = nx;
    o.fy = ny;
    o.u0 = s1 * ux + k1 * uz;
    o.u1 = k1 * ux - s1 * uz;
    o.u2 = uy;
    const int lim = p.n_filt + 1;                        // whole filtered shape inside a conductor
    if (ni < -lim || ni > nr + lim || (ni == nr + lim && nx > (T)0)) {
        o.c = kDead;
        atomic_add(p.n_dead, 1ull);
    } else {
        o.c = pack_cell(ni, nj);
    }
    return o;
}

// The particle loaded from chunk slot idx (a particle if idx < n and its
// cell is not the dead mark): pushed, and its new state stored.
template <typename T, typename V, typename D>
__device__ __forceinline__ void push_slot(const PushArgs<T> &p, const V &view, const D &dep, const PIn<T> &in,
                                          uint32_t idx, uint32_t n)
{
    POut<T> o{in.c, in.fx, in.fy, in.u0, in.u1, in.u2};
    if (idx < n && in.c != kDead) o = push_particle(p, view, dep, in);
    store_particle(p, idx, o);
}

__device__ inline int wave_min(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ inline int wave_max(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// LDS of a push work-group: six field planes of T, the radii of the
// region's rows, then three 64-bit fixed-point deposit planes (8-byte
// aligned), and for FP64 three 32-bit remainder planes, lds_plane<T>()
// entries each.
template <typename T>
__host__ __device__ constexpr size_t lds_rows_offset()
{
    return (size_t)6 * lds_plane<T>() * sizeof(T);
}
template <typename T>
__host__ __device__ constexpr size_t lds_field_bytes()
{
    return (lds_rows_offset<T>() + (size_t)kLdsRows * sizeof(T) + 7) / 8 * 8;
}
template <typename T>
__host__ __device__ constexpr size_t lds_dep_bytes()
{
    return (size_t)3 * lds_plane<T>() * sizeof(long long);
}
template <typename T>
__host__ __device__ constexpr size_t lds_push_bytes()
{
    return lds_field_bytes<T>() + lds_dep_bytes<T>() + (sizeof(T) == 8 ? (size_t)3 * lds_plane<T>() * sizeof(int) : 0);
}
static_assert(lds_push_bytes<float>() + 512 <= 40 * 1024, "FP32 push LDS: four work-groups per CU");
static_assert(lds_push_bytes<double>() + 512 <= 80 * 1024, "FP64 push LDS: two work-groups per CU");

// Slot of iteration q of thread t inside a chunk: each pass of the 256
// threads reads 256 consecutive particles (full cache lines in and out).
// The particle arrays are addressed from the chunk's first slot (a scalar
// base) with this small per-lane offset.
__device__ __forceinline__ uint32_t chunk_slot(int tid, int q)
{
    return 256u * (uint32_t)q + (uint32_t)tid;
}

// Most particles of one push chunk (256 threads x 16); every particle array
// holds this many spare slots past its capacity.
constexpr int kMaxChunk = 256 * 16;

template <typename T>
__device__ __forceinline__ void at_chunk(PushArgs<T> &p, uint32_t base)
{
    p.cell += base;
    p.dx += base;
    p.dy += base;
    p.ur += base;
    p.ut += base;
    p.up += base;
    p.w += base;
}


// One work-group per chunk of 256 * PPT consecutive (cell-sorted) particles
// of one run.  The chunk's cell bounding box, widened by one cell below and
// two above (gather stencils and one-cell moves), is staged in LDS when it
// fits: six field planes with the axis mirror applied, and three deposit
// planes that collect the chunk's face charges and are flushed with one
// global atomic per non-zero entry.  Chunks that do not fit (an unsorted
// tail) gather and deposit in global memory.  The chunks of all runs form
// one list (prefix chunk_off), cut into eight contiguous ranges, one per
// XCD, so that neighbouring chunks share an L2; work-group b takes chunks of
// range b % 8 from that range's atomic counter until the range is
// exhausted, so late-starting work-groups never leave a tail of unbalanced
// work.
// Waves per SIMD the push is compiled for: FP32 four (128 registers), FP64
// two (LDS and registers allow no more).
template <typename T>
constexpr int push_waves();
template <>
constexpr int push_waves<float>() { return 4; }
template <>
constexpr int push_waves<double>() { return 2; }

template <typename T, int PPT>
__global__ __launch_bounds__(256, push_waves<T>()) void k_push(const RunDev<T> *__restrict__ runs, int n_runs,
                                              const unsigned long long *__restrict__ chunk_off,
                                              unsigned int *__restrict__ work)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int red[4][4];
    __shared__ unsigned int s_next;
    constexpr int CH = 256 * PPT;
    const unsigned long long nch = chunk_off[n_runs];
    const int xcd = blockIdx.x & 7;
    const unsigned long long lo = nch * xcd / 8, hi = nch * (xcd + 1) / 8;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (;;) {
        if (tid == 0) s_next = atomic_add_fetch_old(glb(work + xcd), 1u);
        __syncthreads();
        const unsigned long long gch = lo + (unsigned long long)__builtin_amdgcn_readfirstlane(s_next);
        __syncthreads();
        if (gch >= hi) break;
        const int r = __builtin_amdgcn_readfirstlane(run_of(chunk_off, n_runs, gch));
        const RunDev<T> &R = runs[r];
        const gptr<const unsigned long long> ctr = glb((const unsigned long long *)R.ctr);
        const unsigned long long n = ctr[kTotal];
        const int cur = (int)ctr[kCur];
        PushArgs<T> p = push_args(R, cur, (double)ctr[kStep]);
        const int cap = R.lds_cap;
        const int nth = p.L.nth;
        constexpr int P = lds_plane<T>();
        T *sm = reinterpret_cast<T *>(smem_raw);                                  // 6 field planes
        T *srn = reinterpret_cast<T *>(smem_raw + lds_rows_offset<T>());          // radii of the rows
        long long *sd = reinterpret_cast<long long *>(smem_raw + lds_field_bytes<T>()); // 3 deposit planes
        int *sl = reinterpret_cast<int *>(smem_raw + lds_field_bytes<T>() + lds_dep_bytes<T>()); // FP64 remainders
        static_assert(CH <= kMaxChunk, "push chunk larger than the spare slots");
        const uint32_t base = (uint32_t)(gch - chunk_off[r]) * (uint32_t)CH;
        at_chunk(p, base);
        const uint32_t n32 = (uint32_t)min(n - base, (unsigned long long)CH); // particles of this chunk
        int imin = INT_MAX, imax = INT_MIN, jmin = INT_MAX, jmax = INT_MIN;
        if (cap > 0) {
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const uint32_t idx = chunk_slot(tid, q);
                const uint32_t c = idx < n32 ? at_slot(p.cell, idx) : kDead;
                if (c != kDead) {
                    const int ci = cell_i(c), cj = cell_j(c);
                    imin = min(imin, ci); imax = max(imax, ci);
                    jmin = min(jmin, cj); jmax = max(jmax, cj);
                }
            }
        }
        bool use = false;
        int i0 = 0, j0 = 0, C = 0;
        if (cap > 0) {
            imin = wave_min(imin); imax = wave_max(imax);
            jmin = wave_min(jmin); jmax = wave_max(jmax);
            if (lane == 0) { red[wv][0] = imin; red[wv][1] = imax; red[wv][2] = jmin; red[wv][3] = jmax; }
            __syncthreads();
            imin = min(min(red[0][0], red[1][0]), min(red[2][0], red[3][0]));
            imax = max(max(red[0][1], red[1][1]), max(red[2][1], red[3][1]));
            jmin = min(min(red[0][2], red[1][2]), min(red[2][2], red[3][2]));
            jmax = max(max(red[0][3], red[1][3]), max(red[2][3], red[3][3]));
            __syncthreads();
            if (imin <= imax) {
                const int Rr = imax - imin + 4;
                C = jmax - jmin + 4;
                use = (long long)Rr * C <= cap && Rr <= kLdsRows;
                i0 = imin - 1;
                j0 = jmin - 1;
            }
        }
        if (use) {
            const int RC = (imax - imin + 4) * C;
            // walk the region row-major with (row, column) carried along
            int rr = tid / C, cc = tid - (tid / C) * C;
            const int dr = 256 / C, dc = 256 - (256 / C) * C;
            for (int e = tid; e < RC; e += 256) {
                const int gi = i0 + rr, gj = j0 + cc;
                const bool vi = gj >= 0 && gj <= nth;
                int hj = gj;
                T so = (T)1;
                if (gj < 0) { hj = -1 - gj; so = (T)-1; }
                else if (gj >= nth) { hj = 2 * nth - 1 - gj; so = (T)-1; }
                const bool vh = hj >= 0 && hj < nth;
                sm[cER * P + e] = vi ? p.f.c[cER][p.L.at(gi, gj)] : (T)0;
                sm[cEPH * P + e] = vi ? p.f.c[cEPH][p.L.at(gi, gj)] : (T)0;
                sm[cBTH * P + e] = vi ? p.f.c[cBTH][p.L.at(gi, gj)] : (T)0;
                sm[cETH * P + e] = vh ? so * p.f.c[cETH][p.L.at(gi, hj)] : (T)0;
                sm[cBR * P + e] = vh ? p.f.c[cBR][p.L.at(gi, hj)] : (T)0;
                sm[cBPH * P + e] = vh ? so * p.f.c[cBPH][p.L.at(gi, hj)] : (T)0;
                sd[e] = 0;
                sd[P + e] = 0;
                sd[2 * P + e] = 0;
                if constexpr (sizeof(T) == 8) {
                    sl[e] = 0;
                    sl[P + e] = 0;
                    sl[2 * P + e] = 0;
                }
                rr += dr;
                cc += dc;
                if (cc >= C) { cc -= C; ++rr; }
            }
            for (int e = tid; e < imax - imin + 4; e += 256) srn[e] = p.r_node[i0 + e + p.L.G];
            __syncthreads();
            const LdsView<T> view{sm, srn, i0, j0, C};
            const LdsDep<T> dep{sd, sl, i0, j0, C, R.dep_scale};
            // the next particle's state is loaded while this one is pushed
            PIn<T> nxt = load_particle(p, chunk_slot(tid, 0));
#pragma unroll 1
            for (int q0 = 0; q0 < PPT; ++q0) {
                // the iteration index, opaque to the compiler, so that it does
                // not turn the seven array accesses into seven 64-bit pointers
                const int q = __builtin_amdgcn_readfirstlane(q0);
                const PIn<T> cur = nxt;
                if (q + 1 < PPT) nxt = load_particle(p, chunk_slot(tid, q + 1));
                push_slot(p, view, dep, cur, chunk_slot(tid, q), n32);
            }
            __syncthreads();
            {
                const T inv = R.dep_inv;
                int fr = tid / C, fc = tid - (tid / C) * C;
                for (int e = tid; e < RC; e += 256) {
                    const size_t g = p.L.at(i0 + fr, j0 + fc);
#pragma unroll
                    for (int comp = 0; comp < 3; ++comp) {
                        const long long v = sd[comp * P + e];
                        if constexpr (sizeof(T) == 8) {
                            const int l = sl[comp * P + e];
                            if (v != 0 || l != 0)
                                atomic_add(p.f.c[cFR + comp] + g, ((T)v + (T)l * (T)(1.0 / kLoScale)) * inv);
                        } else {
                            if (v != 0) atomic_add(p.f.c[cFR + comp] + g, (T)v * inv);
                        }
                    }
                    fr += dr;
                    fc += dc;
                    if (fc >= C) { fc -= C; ++fr; }
                }
            }
            __syncthreads();
        } else {
            if (tid == 0 && cap > 0) atomic_add(glb(R.ctr + kGlobalChunks), 1ull);
            const GlobalView<T> view{&p.f, p.L, p.r_node};
            const GlobalDep<T> dep{{p.f.c[cFR], p.f.c[cFTH], p.f.c[cFPH]}, p.L};
#pragma unroll 1
            for (int q0 = 0; q0 < PPT; ++q0) {
                const int q = __builtin_amdgcn_readfirstlane(q0);
                const uint32_t idx = chunk_slot(tid, q);
                push_slot(p, view, dep, load_particle(p, idx), idx, n32);
            }
        }
    }
}

// ------------------------------------------------------------------
// Surface injection: one work-group of 1024 threads per run; afterwards
// the step index of every run advances
// ------------------------------------------------------------------

constexpr int kInjMaxPer = 8; // nth + 1 <= 8192

template <typename T>
__device__ void inject_run(const RunDev<T> &R);

// The step's closing kernel (it runs after the Ampere update, which reads
// the B that the lossy layer then damps): work-group r < n_runs injects the
// pairs of run r and advances its step index; the other work-groups apply
// the lossy layer to B, four 64 x 4 blocks of the layer map `off` each.
template <typename T>
__global__ __launch_bounds__(1024) void k_close(const RunDev<T> *__restrict__ runs, int n_runs,
                                                const int *__restrict__ off)
{
    if ((int)blockIdx.x < n_runs) {
        inject_run(runs[blockIdx.x]);
        return;
    }
    const int sub = (int)threadIdx.x >> 8, t = (int)threadIdx.x & 255;
    const int b = ((int)blockIdx.x - n_runs) * 4 + sub;
    if (b >= off[n_runs]) return;
    const int r = run_of(off, n_runs, b);
    absorb_b_block(runs[r], b - off[r], t & 63, t >> 6);
}

template <typename T>
__device__ void inject_run(const RunDev<T> &R)
{
    __shared__ long long wsum[16];
    __shared__ int ok;
    const gptr<unsigned long long> ctr = glb(R.ctr);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint64_t step = ctr[kStep];
    const unsigned long long nbase = ctr[kTotal]; // fixed until this kernel's end
    if (!R.inject) {
        if (tid == 0) ctr[kStep] = step + 1;
        return;
    }
    const Layout L = R.L;
    const int cur = (int)ctr[kCur];
    const double irl = inv_light_cylinder(R.omega, R.t_spin, R.cd, (double)(step + 1));
    const int nth = L.nth, nodes = nth + 1;
    const int per = (nodes + 1023) / 1024;
    const int j0 = tid * per, j1 = min(j0 + per, nodes);
    // every input of this thread's nodes is loaded (at a node clamped into
    // the tables) before the first carry is stored
    double er[kInjMaxPer], kn[kInjMaxPer], sn[kInjMaxPer], cy[kInjMaxPer], aj[kInjMaxPer];
#pragma unroll
    for (int q = 0; q < kInjMaxPer; ++q) {
        if (q < per) {
            const int jj = min(j0 + q, nodes - 1);
            er[q] = (double)glb(R.fld[cER])[L.at(0, jj)];
            kn[q] = glb(R.kn)[jj];
            sn[q] = glb(R.sn)[jj];
            cy[q] = glb(R.carry)[jj];
            aj[q] = glb(R.Aj)[jj];
        }
    }
    long long m[kInjMaxPer];
    long long mine = 0;
#pragma unroll
    for (int q = 0; q < kInjMaxPer; ++q) {
        m[q] = 0;
        const int jj = j0 + q;
        if (q < per && jj < j1) {
            double E[3] = {0, 0, 0}, B[3] = {0, 0, 0};
            add_background(R.bg, irl, false, R.rb0, kn[q], sn[q], E, B);
            const double sigma = er[q] + E[0];
            const double cnew = cy[q] + R.f_inj * fabs(sigma) * aj[q] / R.q_inj;
            const double fl = floor(cnew);
            glb(R.carry)[jj] = cnew - fl;
            m[q] = (long long)fl;
            mine += (long long)fl;
        }
    }
    // exclusive prefix of the counts over the threads: within each wave by
    // shuffles, then over the sixteen wave totals
    long long incl = mine;
    for (int o = 1; o < 64; o <<= 1) {
        const long long v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    if (wv == 0) {
        long long w = lane < 16 ? wsum[lane] : 0;
        for (int o = 1; o < 16; o <<= 1) {
            const long long v = __shfl_up(w, o);
            if (lane >= o) w += v;
        }
        if (lane < 16) wsum[lane] = w;
    }
    __syncthreads();
    const long long total = wsum[15];
    long long off = (wv > 0 ? wsum[wv - 1] : 0) + incl - mine;
    if (tid == 0) ok = (long long)nbase + 2 * total <= R.capacity;
    __syncthreads();
    if (!ok) {
        if (tid == 0) {
            atomic_or(glb(R.status), 2);
            ctr[kStep] = step + 1;
        }
        return;
    }
    const gptr<uint32_t> cell = glb(R.cell[cur]);
    const gptr<T> a[6] = {glb(R.arr[cur][0]), glb(R.arr[cur][1]), glb(R.arr[cur][2]),
                          glb(R.arr[cur][3]), glb(R.arr[cur][4]), glb(R.arr[cur][5])};
    const gptr<uint64_t> id = R.id[cur] ? glb(R.id[cur]) : nullptr;
#pragma unroll
    for (int q = 0; q < kInjMaxPer; ++q) {
        const int jj = j0 + q;
        if (!(q < per && jj < j1)) continue;
        const double ylo = jj - 0.5 < 0.0 ? 0.0 : jj - 0.5;
        const double yhi = jj + 0.5 > nth ? (double)nth : jj + 0.5;
        for (long long kk = 0; kk < m[q]; ++kk) {
            uint64_t x[4] = {step, (uint64_t)jj, (uint64_t)kk, 0};
            philox4x64(x, R.seed, 0x50494353ull);
            const double U = (double)(x[0] >> 11) * 0x1.0p-53;
            const double y = ylo + U * (yhi - ylo);
            int jc = (int)floor(y);
            if (jc > nth - 1) jc = nth - 1;
            const T fy = (T)(y - jc);
            for (int sgn = 0; sgn < 2; ++sgn) {
                const size_t d = nbase + 2 * (size_t)(off + kk) + sgn;
                cell[d] = pack_cell(0, jc);
                a[0][d] = (T)0.5;
                a[1][d] = fy;
                a[2][d] = a[3][d] = a[4][d] = (T)0;
                a[5][d] = sgn == 0 ? (T)R.q_inj : (T)-R.q_inj;
                if (id)
                    id[d] = 0x8000000000000000ull | (step << 36) | ((uint64_t)jj << 20) | ((uint64_t)kk << 1) |
                            (uint64_t)sgn;
            }
        }
        off += m[q];
    }
    __syncthreads();
    if (tid == 0) {
        ctr[kTotal] = nbase + 2 * total;
        ctr[kInjected] += 2 * total;
        ctr[kStep] = step + 1;
    }
}

// ------------------------------------------------------------------
// Counting sort by tile, for the runs whose kSortNow is set
// ------------------------------------------------------------------

__device__ inline unsigned long long lanemask_le(int lane)
{
    return lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
}

// Particles per work-group of the sort kernels: each work-group takes a
// contiguous span of one run (16 particles per thread), so that the
// particles of one tile, kept together by the previous sort, are counted
// and placed by about one work-group, with one global atomic per tile.  The
// spans of all sorting runs are laid end to end (prefix span_off).
constexpr int kSortSpan = 256 * 16;
constexpr int kSortPer = kSortSpan / 256;

// Tile keys a work-group counts in LDS: a window centred on the key of the
// span's first live particle (of its first eight).  Particles move a few
// cells between sorts, so the keys of a span lie within a few tiles of each
// other (a few rows of tiles in the serpentine order, rows of up to a few
// hundred tiles); a key outside the window goes to the global counter
// directly.  The histogram and the scatter place the window alike.
constexpr int kSortWin = 2048;

// A key held by at most kSpanList spans of a sort is placed span by span in
// span order, so that the sort is stable: every particle keeps the order of
// its key's particles in storage.  The histogram records, per key, the spans
// that hold it and their counts, and the scan orders each key's spans and
// turns the counts into the key's particles in the spans before each.
// Between sorts particles move a few cells, so a key's particles lie in its
// own spans and in those of the tiles around it: with a key's particles in
// at most three spans, nine tiles hold at most 27.  A key held by more spans
// (an unsorted store: the first sort of particles loaded in any order), or
// met outside a span's LDS window, is placed in the order the spans claim
// it, and the sort is stable only within each span.
constexpr int kSpanList = 32;
constexpr unsigned int kSpanOverflow = 1u << 20;

__device__ __forceinline__ int sort_window_base(const TileMap &tm, gptr<const uint32_t> cs, uint32_t ns)
{
    int k0 = tm.key(cs[0]);
    for (uint32_t q = 1; q < min(ns, 8u) && k0 == tm.n_keys; ++q) k0 = tm.key(cs[q]);
    return k0 > kSortWin / 2 ? k0 - kSortWin / 2 : 0;
}
// Runs of equal keys among the 64 lanes of a wave (particles in lane
// order, mostly of one tile after the previous sort): whether the lane
// starts a run, the run's length (valid at its start) and the lane that
// starts the lane's run.  Counting one atomic per run instead of one per
// particle keeps the LDS atomics of a wave off one address.
struct KeyRun {
    bool head;
    int len, head_lane;
};
__device__ __forceinline__ KeyRun key_run(int key, int lane)
{
    const int prev = __shfl_up(key, 1);
    KeyRun k;
    k.head = lane == 0 || key != prev;
    const unsigned long long heads = __ballot(k.head);
    const unsigned long long after = heads & ~lanemask_le(lane);
    k.len = (after ? __ffsll((long long)after) - 1 : 64) - lane;
    k.head_lane = 63 - __clzll((long long)(heads & lanemask_le(lane)));
    return k;
}

// Clear the tile counters and cursors of the sorting runs (256 per
// work-group).
template <typename T>
__global__ __launch_bounds__(256) void k_sort_zero(const RunDev<T> *__restrict__ runs, int n_runs,
                                                   const int *__restrict__ off)
{
    const int r = run_of(off, n_runs, blockIdx.x);
    const RunDev<T> &R = runs[r];
    if (!glb(R.ctr)[kSortNow]) return;
    const int e = (blockIdx.x - off[r]) * 256 + threadIdx.x;
    if (e <= R.tm.n_keys) {
        glb(R.counts)[e] = 0;
        glb(R.cursor)[e] = 0;
        glb(R.nspan)[e] = 0;
    }
}

// Histogram of tile keys: LDS counts per span (one atomic per run of equal
// keys in a wave), then one global atomic per key present.  LDS atomics do not share the memory counter that the loads
// wait on, so a span costs one round trip to memory.
template <typename T>
__global__ __launch_bounds__(256) void k_sort_hist(const RunDev<T> *__restrict__ runs, int n_runs,
                                                   const unsigned long long *__restrict__ span_off)
{
    __shared__ unsigned int h[kSortWin];
    const int tid = threadIdx.x;
    for (int e = tid; e < kSortWin; e += 256) h[e] = 0;
    const unsigned long long nspan = span_off[n_runs];
    for (unsigned long long gs = blockIdx.x; gs < nspan; gs += gridDim.x) {
        const int r = __builtin_amdgcn_readfirstlane(run_of(span_off, n_runs, gs));
        const RunDev<T> &R = runs[r];
        const gptr<const unsigned long long> ctr = glb((const unsigned long long *)R.ctr);
        const unsigned long long n = ctr[kTotal];
        const gptr<const uint32_t> cell = glb((const uint32_t *)R.cell[ctr[kCur]]);
        const TileMap tm = R.tm;
        const gptr<unsigned int> counts = glb(R.counts);
        const unsigned long long s0 = (gs - span_off[r]) * kSortSpan;
        const uint32_t ns = (uint32_t)min(n - s0, (unsigned long long)kSortSpan);
        const gptr<const uint32_t> cs = cell + s0;
        uint32_t cw[kSortPer];
#pragma unroll
        for (int u = 0; u < kSortPer; ++u) {
            const uint32_t k = 256u * u + tid;
            cw[u] = k < ns ? cs[k] : kDead;
        }
        const int base = sort_window_base(tm, cs, ns);
        const gptr<unsigned int> nspan = glb(R.nspan);
        SpanEnt *const slist = R.slist; // struct copies need generic pointers
        const unsigned int sidx = (unsigned int)(gs - span_off[r]);
        __syncthreads(); // the window is clear
#pragma unroll
        for (int u = 0; u < kSortPer; ++u) {
            const int key = 256u * u + tid < ns ? tm.key(cw[u]) : INT_MAX;
            const KeyRun kr = key_run(key, tid & 63);
            if (kr.head && key != INT_MAX) {
                const unsigned int dw = (unsigned int)(key - base);
                if (dw < (unsigned int)kSortWin) {
                    atomicAdd(&h[dw], (unsigned int)kr.len);
                } else {
                    atomic_add(counts + key, (unsigned int)kr.len);
                    atomic_add(nspan + key, kSpanOverflow);
                }
            }
        }
        __syncthreads();
        for (int e = tid; e < kSortWin; e += 256) {
            const unsigned int v = h[e];
            if (v) {
                const int key = base + e;
                atomic_add(counts + key, v);
                const unsigned int slot = atomic_add_fetch_old(nspan + key, 1u);
                if (slot < (unsigned int)kSpanList) slist[(size_t)key * kSpanList + slot] = SpanEnt{sidx, v};
                h[e] = 0;
            }
        }
    }
}

// Exclusive scan of counts[0..n_keys] (the last key collects deleted
// particles) into offsets, one work-group per run; kLive becomes the number
// of live particles.
template <typename T>
__global__ __launch_bounds__(1024) void k_sort_scan(const RunDev<T> *__restrict__ runs)
{
    __shared__ unsigned long long s[1024];
    const RunDev<T> &R = runs[blockIdx.x];
    const gptr<unsigned long long> ctr = glb(R.ctr);
    if (!ctr[kSortNow]) return;
    const int n_keys = R.tm.n_keys;
    const gptr<const unsigned int> counts = glb((const unsigned int *)R.counts);
    const gptr<unsigned long long> offsets = glb(R.offsets);
    const int tid = threadIdx.x;
    const int per = (n_keys + 1 + 1023) / 1024;
    const int a = tid * per, b = min(a + per, n_keys + 1);
    unsigned long long mine = 0;
    for (int q = a; q < b; ++q) mine += counts[q];
    s[tid] = mine;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const unsigned long long v = tid >= o ? s[tid - o] : 0;
        __syncthreads();
        s[tid] += v;
        __syncthreads();
    }
    unsigned long long run = s[tid] - mine;
    for (int q = a; q < b; ++q) {
        offsets[q] = run;
        run += counts[q];
    }
    __syncthreads();
    if (tid == 0) ctr[kLive] = s[1023] - counts[n_keys];
}

// Per key held by at most kSpanList spans: for each of its spans, the
// key's particles in the spans before it (a lower span index), so that the
// scatter places the key span by span in span order.  One thread per key
// (the key map of the sort's zeroing), entries compared all against all:
// a key is held by a few spans, and no order of the list is needed.
template <typename T>
__global__ __launch_bounds__(256) void k_sort_spans(const RunDev<T> *__restrict__ runs, int n_runs,
                                                    const int *__restrict__ off)
{
    const int r = run_of(off, n_runs, blockIdx.x);
    const RunDev<T> &R = runs[r];
    if (!glb(R.ctr)[kSortNow]) return;
    const int q = (blockIdx.x - off[r]) * 256 + threadIdx.x;
    if (q > R.tm.n_keys) return;
    const unsigned int m = glb((const unsigned int *)R.nspan)[q];
    if (m > (unsigned int)kSpanList) return;
    const SpanEnt *const a = R.slist + (size_t)q * kSpanList; // struct copies need generic pointers
    const gptr<unsigned int> before = glb(R.sbefore) + (size_t)q * kSpanList;
    for (unsigned int k = 0; k < m; ++k) {
        const unsigned int sk = a[k].s;
        unsigned int b = 0;
        for (unsigned int l = 0; l < m; ++l) {
            const SpanEnt e = a[l];
            if (e.s < sk) b += e.c;
        }
        before[k] = b;
    }
}

// Scatter into the other buffer, stably.  Wave w of the work-group takes
// the quarter [1024 w, 1024 (w + 1)) of the span, 64 consecutive particles
// per slice, so that a particle's rank among the span's particles of its
// key in storage order is: the wave's particles of that key in its earlier
// slices (a running count per wave and key in LDS, which only that wave
// touches), the earlier lanes of its slice (a ballot per distinct key), and
// the particles of the key in the earlier waves' quarters (their counts,
// read after one barrier).  No rank depends on the order in which waves
// run.  The first wave that met a key then takes the span's block of slots
// for it: from the key's span list (the key's particles in the spans
// before this one) when the key is listed, else by a claim on the key's
// cursor; a key outside the window is claimed by runs of equal keys in a
// wave, on its cursor.  The particles are copied, four slices per thread at
// a time, to offsets[key] + block + rank.  Deleted particles (the last key)
// are dropped; lanes without a particle write a spare slot past the
// capacity, so that every lane stores.
__device__ inline unsigned long long lanemask_lt(int lane)
{
    return lane == 0 ? 0ull : ((1ull << lane) - 1ull);
}

template <typename T>
__global__ __launch_bounds__(256) void k_sort_scatter(const RunDev<T> *__restrict__ runs, int n_runs,
                                                      const unsigned long long *__restrict__ span_off)
{
    constexpr int Q = kSortSpan / 4;                // particles of a wave's quarter
    __shared__ unsigned int h[kSortWin];            // per key of the window: the span's first slot
    __shared__ unsigned short wc[4][kSortWin];      // per wave and key: the key's particles in its quarter
    __shared__ unsigned short tl[4][Q];             // per wave: the keys it met, as window offsets
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int e = tid; e < kSortWin; e += 256) h[e] = 0;
    for (int e = tid; e < 4 * kSortWin; e += 256) (&wc[0][0])[e] = 0;
    __syncthreads(); // the counts are clear; each span leaves them clear
    const unsigned long long nspan_all = span_off[n_runs];
    for (unsigned long long gs = blockIdx.x; gs < nspan_all; gs += gridDim.x) {
        const int r = __builtin_amdgcn_readfirstlane(run_of(span_off, n_runs, gs));
        const RunDev<T> &R = runs[r];
        const gptr<const unsigned long long> ctr = glb((const unsigned long long *)R.ctr);
        const unsigned long long n = ctr[kTotal];
        const int cur = (int)ctr[kCur], nxt = cur ^ 1;
        const TileMap tm = R.tm;
        const unsigned int sidx = (unsigned int)(gs - span_off[r]);
        const unsigned long long s0 = (unsigned long long)sidx * kSortSpan;
        const uint32_t ns = (uint32_t)min(n - s0, (unsigned long long)kSortSpan);
        const gptr<const uint32_t> cs = glb((const uint32_t *)R.cell[cur]) + s0;
        const gptr<const unsigned long long> offsets = glb((const unsigned long long *)R.offsets);
        const gptr<unsigned int> cursor = glb(R.cursor);
        const gptr<const unsigned int> nspan = glb((const unsigned int *)R.nspan);
        const SpanEnt *const slist = R.slist;
        const gptr<const unsigned int> sbefore = glb((const unsigned int *)R.sbefore);
        const uint32_t cap = (uint32_t)R.capacity;
        const uint32_t q0 = (uint32_t)wv * Q + (uint32_t)lane;
        uint32_t cw[kSortPer];
#pragma unroll
        for (int u = 0; u < kSortPer; ++u) {
            const uint32_t k = q0 + 64u * u;
            cw[u] = k < ns ? cs[k] : kDead;
        }
        const int base = sort_window_base(tm, cs, ns);
        // the wave's ranks: running counts of its keys, one ballot per
        // distinct key of a slice
        uint32_t rank[kSortPer];
        int nt = 0; // keys the wave met (the same on every lane)
#pragma unroll
        for (int u = 0; u < kSortPer; ++u) {
            const int key = q0 + 64u * u < ns ? tm.key(cw[u]) : INT_MAX;
            const bool live = key != INT_MAX && key != tm.n_keys;
            const unsigned int dw = (unsigned int)(key - base);
            const bool inw = live && dw < (unsigned int)kSortWin;
            // outside the window: one claim per run of equal keys in the wave
            const KeyRun kr = key_run(key, lane);
            uint32_t got = 0;
            if (kr.head && live && !inw)
                got = (uint32_t)(offsets[key] + atomic_add_fetch_old(cursor + key, (unsigned int)kr.len));
            const uint32_t out_rank = (uint32_t)__shfl((int)got, kr.head_lane) + (uint32_t)(lane - kr.head_lane);
            unsigned long long pending = __ballot(inw);
            uint32_t lrank = 0;
            while (pending) {
                const int leader = __ffsll((long long)pending) - 1;
                const unsigned int ld = (unsigned int)(__shfl(key, leader) - base);
                const unsigned long long m = __ballot(inw && dw == ld);
                const unsigned int c = wc[wv][ld];
                if (inw && dw == ld) lrank = c + (uint32_t)__popcll(m & lanemask_lt(lane));
                if (lane == 0) {
                    if (c == 0) tl[wv][nt] = (unsigned short)ld;
                    wc[wv][ld] = (unsigned short)(c + (unsigned int)__popcll(m));
                }
                nt += c == 0;
                pending &= ~m;
            }
            rank[u] = inw ? lrank : out_rank;
        }
        __syncthreads(); // every wave's counts are complete
        // the span's block of slots for each key, taken by the first wave
        // (in wave order) that met it
        for (int t = lane; t < nt; t += 64) {
            const unsigned int ld = tl[wv][t];
            bool first = true;
            unsigned int v = 0;
#pragma unroll
            for (int w2 = 0; w2 < 4; ++w2) {
                const unsigned int c = wc[w2][ld];
                first = first && !(w2 < wv && c != 0);
                v += c;
            }
            if (first) {
                const int key = base + (int)ld;
                const unsigned int m = nspan[key];
                unsigned long long blk = 0;
                bool listed = false;
                if (m <= (unsigned int)kSpanList) {
                    for (unsigned int q = 0; q < m; ++q) {
                        if (slist[(size_t)key * kSpanList + q].s == sidx) {
                            blk = sbefore[(size_t)key * kSpanList + q];
                            listed = true;
                        }
                    }
                }
                if (!listed) blk = atomic_add_fetch_old(cursor + key, v);
                h[ld] = (unsigned int)(offsets[key] + blk);
            }
        }
        __syncthreads(); // every block of slots is known
        uint32_t dest[kSortPer];
#pragma unroll
        for (int u = 0; u < kSortPer; ++u) {
            const int key = tm.key(cw[u]);
            const unsigned int dw = (unsigned int)(key - base);
            uint32_t d = cap + (uint32_t)lane; // spare slot
            if (q0 + 64u * u < ns && key != tm.n_keys) {
                uint32_t t = rank[u];
                if (dw < (unsigned int)kSortWin) {
                    t += h[dw];
                    for (int w2 = 0; w2 < wv; ++w2) t += wc[w2][dw];
                }
                if (t < cap) d = t;
                else atomic_or(glb(R.status), 4); // never write outside the store
            }
            dest[u] = d;
        }
        __syncthreads(); // every read of the counts and blocks is done
        for (int t = lane; t < nt; t += 64) {
            const unsigned int ld = tl[wv][t];
            wc[wv][ld] = 0;
            h[ld] = 0;
        }
        gptr<const T> src[6];
        gptr<T> dst[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            src[q] = glb((const T *)R.arr[cur][q]) + s0;
            dst[q] = glb(R.arr[nxt][q]);
        }
        const gptr<uint32_t> cell_o = glb(R.cell[nxt]);
        const gptr<const uint64_t> id = R.id[cur] ? glb((const uint64_t *)R.id[cur]) + s0 : nullptr;
        const gptr<uint64_t> id_o = glb(R.id[nxt]);
#pragma unroll
        for (int g = 0; g < kSortPer; g += 4) {
            T pay[4][6];
            uint64_t pid[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t k = q0 + 64u * (g + u);
                const bool in = k < ns;
#pragma unroll
                for (int q = 0; q < 6; ++q) pay[u][q] = in ? src[q][k] : (T)0;
                pid[u] = (in && id) ? id[k] : 0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t dd = dest[g + u];
                cell_o[dd] = cw[g + u];
#pragma unroll
                for (int q = 0; q < 6; ++q) dst[q][dd] = pay[u][q];
                if (id) id_o[dd] = pid[u];
            }
        }
    }
}

// ------------------------------------------------------------------
// Particle load (FP64 absolute coordinates -> cell + offsets)
// ------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_load(const double *__restrict__ src, const uint64_t *__restrict__ ids,
                                              long long n, long long at, int nth, uint32_t *cell, T *dx, T *dy,
                                              T *ur, T *ut, T *up, T *w, uint64_t *id)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const double x = src[q], y = src[n + q];
        const int i = (int)floor(x);
        int j = (int)floor(y);
        if (j > nth - 1) j = nth - 1;
        T fx = (T)(x - i), fy = (T)(y - j);
        if (fx >= (T)1) fx = below_one<T>();
        if (fy > (T)1) fy = (T)1;
        if (j < nth - 1 && fy >= (T)1) fy = below_one<T>();
        const long long d = at + q;
        cell[d] = pack_cell(i, j);
        dx[d] = fx;
        dy[d] = fy;
        ur[d] = (T)src[2 * n + q];
        ut[d] = (T)src[3 * n + q];
        up[d] = (T)src[4 * n + q];
        w[d] = (T)src[5 * n + q];
        if (id) id[d] = ids ? ids[q] : (uint64_t)d;
    }
}

// ------------------------------------------------------------------
// Gauss diagnostic in FP64
// ------------------------------------------------------------------

// Node charge of the particles, bilinear at the four nodes of each cell
// (the particle shape of Sec. 3.3, whose charge App. B's filter spreads),
// into two planes: the signed charge Q and the absolute charge |Q|, the
// scale against which the residual's drift is judged.  A work-group takes
// kNodeSpan consecutive particle slots.  When the nodes they reach fit in
// kNodeLds LDS entries (cell-sorted particles) the span's charges are summed
// there in 64-bit fixed point -- each contribution v rounded to an integer
// multiple of 2^-50 max|w| through the 1.5 * 2^52 shift (|v| <= max|w|, so
// the integer stays below 2^51; a span adds at most 2^12 max|w| to an entry,
// below 2^62) -- so that the sum of a span is exact and independent of the
// order of the atomics.  Positive and negative particles go to two planes
// (|Q| w each, four atomics per particle): rounding to the nearest integer
// is odd-symmetric, so their difference is exactly the signed sum and their
// sum the absolute one.  Each entry is flushed with one FP64 global atomic
// per plane; other spans add straight to global memory.  The grid covers
// the store's capacity; work-groups past the particle count return at once.
constexpr int kNodeSpan = 4096, kNodeLds = 2048;

__device__ __forceinline__ void lds_add_fixed(long long *a, double x)
{
    const double sh = x + 6755399441055744.0; // 1.5 * 2^52: the integer lands in the low bits
    atomicAdd((unsigned long long *)a, (unsigned long long)(__double_as_longlong(sh) - 0x4338000000000000ll));
}

// Both particle buffers of a context and its counters: the kernel reads
// which buffer is current from the counters, so that the host need not.
template <typename T>
struct NodeSrc {
    const uint32_t *cell[2];
    const T *dx[2], *dy[2], *w[2];
    const unsigned long long *ctr;
};

template <typename T>
__global__ __launch_bounds__(256) void k_node_charge(NodeSrc<T> src, Layout L, double scale, double inv,
                                                     double *__restrict__ rho, double *__restrict__ rabs)
{
    __shared__ long long acc[2][kNodeLds];
    __shared__ int red[4][4];
    const gptr<const unsigned long long> ctr = glb(src.ctr);
    const unsigned long long n = ctr[kTotal];
    const int cur = (int)ctr[kCur];
    const gptr<const uint32_t> cell = glb(src.cell[cur]);
    const gptr<const T> dx = glb(src.dx[cur]), dy = glb(src.dy[cur]), w = glb(src.w[cur]);
    const unsigned long long base = (unsigned long long)blockIdx.x * kNodeSpan;
    if (base >= n) return; // the same for the whole work-group
    const int cnt = (int)min((unsigned long long)kNodeSpan, n - base);
    const int tid = threadIdx.x, wv = tid >> 6;
    // cell bounding box of the span's live particles
    int imin = INT_MAX, imax = INT_MIN, jmin = INT_MAX, jmax = INT_MIN;
    for (int k = tid; k < cnt; k += 256) {
        const uint32_t c = cell[base + k];
        if (c == kDead) continue;
        const int i = cell_i(c), j = cell_j(c);
        imin = min(imin, i);
        imax = max(imax, i);
        jmin = min(jmin, j);
        jmax = max(jmax, j);
    }
    imin = wave_min(imin);
    imax = wave_max(imax);
    jmin = wave_min(jmin);
    jmax = wave_max(jmax);
    if ((tid & 63) == 0) {
        red[wv][0] = imin;
        red[wv][1] = imax;
        red[wv][2] = jmin;
        red[wv][3] = jmax;
    }
    __syncthreads();
    imin = min(min(red[0][0], red[1][0]), min(red[2][0], red[3][0]));
    imax = max(max(red[0][1], red[1][1]), max(red[2][1], red[3][1]));
    jmin = min(min(red[0][2], red[1][2]), min(red[2][2], red[3][2]));
    jmax = max(max(red[0][3], red[1][3]), max(red[2][3], red[3][3]));
    if (imin > imax) return; // no live particle in the span (the same for the whole work-group)
    const long long W = (long long)(jmax - jmin) + 2, NH = (long long)(imax - imin) + 2;
    if (W * NH <= kNodeLds) {
        const int nw = (int)W, ne = (int)(W * NH);
        for (int e = tid; e < ne; e += 256) {
            acc[0][e] = 0;
            acc[1][e] = 0;
        }
        __syncthreads();
        // four particles per thread at a time, all their loads issued first
        for (int k0 = tid; k0 < cnt; k0 += 4 * 256) {
            uint32_t c[4];
            double fx[4], fy[4], q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = k0 + 256 * u;
                const bool in = k < cnt;
                c[u] = in ? cell[base + k] : kDead;
                fx[u] = in ? (double)dx[base + k] : 0.0;
                fy[u] = in ? (double)dy[base + k] : 0.0;
                q[u] = in ? (double)w[base + k] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (c[u] == kDead) continue;
                const int e = (cell_i(c[u]) - imin) * nw + (cell_j(c[u]) - jmin); // (i + 1, j) is e + nw
                long long *const a = acc[q[u] < 0.0 ? 1 : 0];
                const double A = fabs(q[u]) * scale;
                const double gx = fx[u], gy = fy[u];
                lds_add_fixed(&a[e], A * ((1 - gx) * (1 - gy)));
                lds_add_fixed(&a[e + nw], A * (gx * (1 - gy)));
                lds_add_fixed(&a[e + 1], A * ((1 - gx) * gy));
                lds_add_fixed(&a[e + nw + 1], A * (gx * gy));
            }
        }
        __syncthreads();
        for (int e = tid; e < ne; e += 256) {
            const size_t g = L.at(imin + e / nw, jmin + e % nw);
            const long long p = acc[0][e], m = acc[1][e];
            if (p != m) unsafeAtomicAdd(&rho[g], (double)(p - m) * inv);
            if (p != 0 || m != 0)
                unsafeAtomicAdd(&rabs[g], (double)((unsigned long long)p + (unsigned long long)m) * inv);
        }
    } else {
        for (int k = tid; k < cnt; k += 256) {
            const uint32_t c = cell[base + k];
            if (c == kDead) continue;
            const int i = cell_i(c), j = cell_j(c);
            const double fx = dx[base + k], fy = dy[base + k], Q = w[base + k], A = fabs(Q);
            const double w00 = (1 - fx) * (1 - fy), w10 = fx * (1 - fy), w01 = (1 - fx) * fy, w11 = fx * fy;
            unsafeAtomicAdd(&rho[L.at(i, j)], Q * w00);
            unsafeAtomicAdd(&rho[L.at(i + 1, j)], Q * w10);
            unsafeAtomicAdd(&rho[L.at(i, j + 1)], Q * w01);
            unsafeAtomicAdd(&rho[L.at(i + 1, j + 1)], Q * w11);
            unsafeAtomicAdd(&rabs[L.at(i, j)], A * w00);
            unsafeAtomicAdd(&rabs[L.at(i + 1, j)], A * w10);
            unsafeAtomicAdd(&rabs[L.at(i, j + 1)], A * w01);
            unsafeAtomicAdd(&rabs[L.at(i + 1, j + 1)], A * w11);
        }
    }
}

// Spindown luminosity (Sec. 5.4): the Poynting flux of the total field
// (plasma plus the analytic initial field at the current step) through the
// sphere of each radial half-node, in FP64; one work-group per row
// i = 0..nr-1.  Per meridional cell: E_theta averaged over its two radial
// nodes, E_phi over its four corners, B_theta over its two meridional
// nodes, B_phi at its own point, times the cell's face 2 pi rbar^2 dk_j.
template <typename T>
__global__ __launch_bounds__(256) void k_poynting(const T *__restrict__ Eth, const T *__restrict__ Eph,
                                                  const T *__restrict__ Bth, const T *__restrict__ Bph, Layout L,
                                                  Background bg, double inv_rl, double c,
                                                  const double *__restrict__ rb, // rbar_i at [i + G]
                                                  const double *__restrict__ Ar, // 2 pi rbar_i^2 at [i + G]
                                                  const double *__restrict__ kc, // cos thetabar_j
                                                  const double *__restrict__ sc, // sin thetabar_j
                                                  const double *__restrict__ dk, // cos theta_j - cos theta_j+1
                                                  double *__restrict__ out)
{
    __shared__ double red[256];
    const int i = blockIdx.x, tid = threadIdx.x;
    const double r = rb[i + L.G], area = Ar[i + L.G];
    double acc = 0.0;
    for (int j = tid; j < L.nth; j += 256) {
        double E[3] = {0.0, 0.0, 0.0}, B[3] = {0.0, 0.0, 0.0};
        add_background<double>(bg, inv_rl, false, r, 1.0 / r, kc[j], sc[j], E, B);
        const double eth = 0.5 * ((double)Eth[L.at(i, j)] + (double)Eth[L.at(i + 1, j)]) + E[1];
        const double eph = 0.25 * ((double)Eph[L.at(i, j)] + (double)Eph[L.at(i + 1, j)] + (double)Eph[L.at(i, j + 1)] +
                                   (double)Eph[L.at(i + 1, j + 1)]) + E[2];
        const double bth = 0.5 * ((double)Bth[L.at(i, j)] + (double)Bth[L.at(i, j + 1)]) + B[1];
        const double bph = (double)Bph[L.at(i, j)] + B[2];
        acc += (eth * bph - eph * bth) * area * dk[j];
    }
    red[tid] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    if (tid == 0) out[i] = c * red[0];
}

// Closed-surface flux of E out of the dual cell of node (i, j) (Sec. 2
// eq. (maxti): the flux equals the charge the node holds, App. B eq.
// (multfiltcharge) with the filtered particle shape), and the residual
// R = G - Qbar, in FP64.  The kernel writes G on the interior rows
// 1 <= i <= nr-1 (zero on rows 0 and nr, whose nodes hold the conductors'
// surface charge) and reduces R over rows 1 <= i <= i_hi, all j: the rows
// below the lossy layer (i_hi = nr - 1 - absorb_cells), whose E the layer's
// damping leaves alone (Sec. 3.4.1), so that R is constant there in exact
// arithmetic.  Per work-group of 64 x 4 nodes it writes the partial
// reductions of the residual: max |R - R0| and sum (R - R0)^2 against the
// reference residual R0 (with ref_mode set, R0 := R instead and the drift is
// zero), max |R|, sum R^2, max of the absolute node charge, max |G|, the
// count of interior nodes and of non-finite values.  Every reduction is
// formed in a fixed order, so the result does not depend on scheduling.
constexpr int kGaussParts = 8;
enum : int { kGpDriftMax = 0, kGpDriftSq, kGpResMax, kGpResSq, kGpAbsMax, kGpFluxMax, kGpNodes, kGpNonFinite };

__device__ inline void gauss_combine(double *a, const double *b)
{
    a[kGpDriftMax] = fmax(a[kGpDriftMax], b[kGpDriftMax]);
    a[kGpDriftSq] += b[kGpDriftSq];
    a[kGpResMax] = fmax(a[kGpResMax], b[kGpResMax]);
    a[kGpResSq] += b[kGpResSq];
    a[kGpAbsMax] = fmax(a[kGpAbsMax], b[kGpAbsMax]);
    a[kGpFluxMax] = fmax(a[kGpFluxMax], b[kGpFluxMax]);
    a[kGpNodes] += b[kGpNodes];
    a[kGpNonFinite] += b[kGpNonFinite];
}

// Tree reduction of one value set per thread of a 256-thread work-group in
// LDS (fixed pairing); thread 0 ends with the total.
__device__ inline void gauss_block_reduce(double (*s)[kGaussParts], double *v)
{
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
#pragma unroll
    for (int q = 0; q < kGaussParts; ++q) s[tid][q] = v[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) gauss_combine(s[tid], s[tid + o]);
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kGaussParts; ++q) v[q] = s[0][q];
}

template <typename T>
__global__ __launch_bounds__(256) void k_gauss_flux(const T *__restrict__ Er, const T *__restrict__ Eth, Layout L,
                                                    const double *__restrict__ Ar,  // 2 pi rbar_i^2, [i + G]
                                                    const double *__restrict__ dkb, // cos thetabar_{j-1} - cos thetabar_j
                                                    const double *__restrict__ At,  // pi (rbar_i^2 - rbar_{i-1}^2)
                                                    const double *__restrict__ sb,  // sin thetabar_j
                                                    const double *__restrict__ Qbar, // filtered node charge (layout L)
                                                    const double *__restrict__ Qabs, // absolute node charge (layout L)
                                                    double *__restrict__ G, double *__restrict__ R0, int ref_mode,
                                                    int i_hi, double *__restrict__ parts)
{
    __shared__ double s[256][kGaussParts];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y * blockDim.y + threadIdx.y;
    double v[kGaussParts] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (i <= L.nr && j <= L.nth) {
        const size_t n = (size_t)i * (L.nth + 1) + j;
        double flux = 0.0;
        if (i >= 1 && i < L.nr) {
            flux = (double)Er[L.at(i, j)] * Ar[i + L.G] * dkb[j] -
                   (double)Er[L.at(i - 1, j)] * Ar[i - 1 + L.G] * dkb[j];
            if (j < L.nth) flux += (double)Eth[L.at(i, j)] * At[i] * sb[j];
            if (j > 0) flux -= (double)Eth[L.at(i, j - 1)] * At[i] * sb[j - 1];
            const double q = Qbar[L.at(i, j)], a = Qabs[L.at(i, j)];
            const double res = flux - q;
            double d = 0.0;
            if (ref_mode) R0[n] = res;
            else d = res - R0[n];
            const bool bad = !isfinite(flux) || !isfinite(q) || !isfinite(a) || !isfinite(d);
            v[kGpNonFinite] = bad ? 1.0 : 0.0;
            if (i <= i_hi) {
                if (!bad) {
                    v[kGpDriftMax] = fabs(d);
                    v[kGpDriftSq] = d * d;
                    v[kGpResMax] = fabs(res);
                    v[kGpResSq] = res * res;
                    v[kGpAbsMax] = a;
                    v[kGpFluxMax] = fabs(flux);
                }
                v[kGpNodes] = 1.0;
            }
        }
        G[n] = flux;
    }
    gauss_block_reduce(s, v);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        double *o = parts + (size_t)(blockIdx.y * gridDim.x + blockIdx.x) * kGaussParts;
#pragma unroll
        for (int q = 0; q < kGaussParts; ++q) o[q] = v[q];
    }
}

// The partial reductions of all work-groups of k_gauss_flux, combined by one
// work-group in a fixed order: out[0..7] = max |R - R0|, sqrt(sum (R - R0)^2),
// max |R|, sqrt(sum R^2), max absolute node charge, max |G|, interior nodes,
// non-finite values.
__global__ __launch_bounds__(256) void k_gauss_final(const double *__restrict__ parts, int n_parts,
                                                     double *__restrict__ out)
{
    __shared__ double s[256][kGaussParts];
    double v[kGaussParts] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < n_parts; b += 256) gauss_combine(v, parts + (size_t)b * kGaussParts);
    gauss_block_reduce(s, v);
    if (threadIdx.x == 0) {
        v[kGpDriftSq] = sqrt(v[kGpDriftSq]);
        v[kGpResSq] = sqrt(v[kGpResSq]);
#pragma unroll
        for (int q = 0; q < kGaussParts; ++q) out[q] = v[q];
    }
}

} // namespace pic
