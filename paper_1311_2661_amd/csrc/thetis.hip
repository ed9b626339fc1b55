// libthetis device path for MI355X (gfx950, CDNA4, 64-lane wavefronts).
//
// The solve step of "An Approximate, Efficient LP Solver for LP Rounding":
// stochastic coordinate descent (Algorithm 1, Section 3.3) on the penalty
// function of eq. (QP) (Section 3.2), in the asynchronous-parallel spirit of
// Section 3.4, followed by the pre-rounding scalings (Lemma
// infeasible:rounded:vc; Appendix C), the roundings (Section 2, Appendix B)
// and the feasibility check.
//
// Kernels (all 256-thread workgroups):
//   k_sweep_group  coordinate update of plain columns, G lanes per column
//                  (G = 4..64 by degree): gather A_j^T r with a coalesced
//                  index read, reduce with a lane butterfly, projected step,
//                  scatter delta*A_j into r (plain stores inside a colour
//                  class, hardware float atomics in the ASYNC schedule)
//   k_sweep_hub    the same for columns above 64 entries, one workgroup per
//                  column, residual entries staged in LDS between gather and
//                  scatter
//   k_sweep_block  block update with projection onto the k-simplex
//                  (multiway cut, Appendix E), one wavefront per block
//   k_sweep_slack  slack coordinates, one lane per inequality row
//   k_rows / k_cols / k_finalize   FP64 residual refresh r = Ay - b fused with
//                  the residual norms, row violation, penalty value F and the
//                  dual bound Phi, reduced in a fixed order (deterministic)
//   k_round_* / k_check_*          pre-rounding pass, roundings, check
#include <atomic>
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "thetis_internal.h"

using namespace thetis;

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(THETIS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

namespace {

// ---------------------------------------------------------------- precision
// X: storage of the structural x; R: storage of slacks and the residual and
// the type the updates are computed in
struct PF32 { using X = float;  using R = float; };
struct PF64 { using X = double; using R = double; };
struct PB16 { using X = __hip_bfloat16; using R = float; };

__device__ __forceinline__ float xval(float v) { return v; }
__device__ __forceinline__ double xval(double v) { return v; }
__device__ __forceinline__ float xval(__hip_bfloat16 v) { return __bfloat162float(v); }
// storage encoding (BF16: round to nearest even)
template <class X, class R> __device__ __forceinline__ X xenc(R v) { return (X)v; }
template <> __device__ __forceinline__ __hip_bfloat16 xenc<__hip_bfloat16, float>(float v) { return __float2bfloat16(v); }
template <> __device__ __forceinline__ __hip_bfloat16 xenc<__hip_bfloat16, double>(double v) { return __float2bfloat16((float)v); }

// stores y' into x[j] and returns the value actually stored (the step that
// reaches the residual is the realised one)
template <class P>
__device__ __forceinline__ typename P::R store_x(typename P::X *p, typename P::R v) {
    const typename P::X e = xenc<typename P::X, typename P::R>(v);
    *p = e;
    return (typename P::R)xval(e);
}
template <class P>
__device__ __forceinline__ typename P::R stored_value(typename P::R v) {
    return (typename P::R)xval(xenc<typename P::X, typename P::R>(v));
}

// ---------------------------------------------------------------- device arguments
template <class P>
struct Dev {
    using X = typename P::X;
    using R = typename P::R;
    // matrix
    const int32_t *col_ptr, *row_idx;
    const R *cval;            // CSC values, null when every entry is 1
    const int32_t *row_ptr, *csr_col;
    const R *csr_val;
    const double *b;
    const int8_t *sense;
    const double *c;          // objective (FP64, for the reductions)
    const R *ctil;            // c - A^T ubar over n + m (null: equals c, slacks 0)
    const R *ub;              // null: every structural bound is ub_value
    const R *norm2;           // ||A_j||^2, null when every entry is 1
    const R *ybar;            // prox centre over n + m (null: prox off or 0)
    const double *ubar;       // null: 0
    const int32_t *bfirst, *fixed, *col_block;
    const R *LB;              // block curvature bound, per block
    // state
    X *x;
    R *s, *r, *udual;
    // scalars
    R beta, rho, gamma, Lmax, ub_value;
    int32_t global_lmax, async_mode, prox_on;
    int32_t row_lanes;        // lanes per row in the row passes (1: a thread per row)
    int64_t n, m, nblocks;
    int32_t k;
};

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nwg) {
    // Workgroups are dispatched to the 8 XCDs round-robin; give each XCD a
    // contiguous run of logical workgroups so neighbouring columns (which
    // share residual cache lines) stay in one L2.
    const int64_t q = nwg >> 3, rem = nwg & 7, xcd = b & 7, idx = b >> 3;
    return xcd * q + (xcd < rem ? xcd : rem) + idx;
}

template <int G, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const T w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

template <class P>
__device__ __forceinline__ typename P::R col_bound(const Dev<P> &a, int64_t j) {
    return a.ub ? a.ub[j] : a.ub_value;
}

// projected coordinate step, same operation order as the update of Algorithm 1:
// y' = clip(y - gamma g / L, 0, U); an empty column without prox moves to
// its cheaper bound
template <class R>
__device__ __forceinline__ R coord_step(R y, R g, R L, R gamma, R U) {
    R yn;
    if (L > R(0)) yn = y - gamma * g / L;
    else yn = g > R(0) ? R(0) : (g < R(0) ? U : y);
    if (yn < R(0)) yn = R(0);
    if (yn > U) yn = U;
    return yn;
}

template <class R>
__device__ __forceinline__ void r_add(R *p, R cur, R d, bool async_mode) {
    if (async_mode) unsafeAtomicAdd(p, d);
    else *p = cur + d;
}

// A schedule as the kernels see it: unit ids in plan order and, for plain
// columns, their entries packed in the same order.
template <class R>
struct Sched {
    const int32_t *ids;
    const int32_t *ptr;
    const int32_t *row;
    const R *val;          // null when every entry is 1 or the signs are packed
    int32_t vmode;         // how entries are stored: see entry_at
    int64_t row_off = 0;   // VM 3 (one class's launch): row of entry e = e + row_off
    int32_t ids_ident = 0; // plain columns are numbered by plan position: id = q
};
// the unit at schedule position q (a plain column's id is q when the
// columns are laid out in plan order)
template <class R>
__device__ __forceinline__ int32_t sched_id(const Sched<R> &sc, int64_t q) {
    return sc.ids_ident ? (int32_t)q : sc.ids[q];
}

// One entry of a packed column.  VM 0: every value 1; 1: values stored
// beside the row indices; 2: every value +-1, the sign in the row index's
// top bit (rows stay below 2^31), so the sweep reads no value array.
template <int VM, class R>
__device__ __forceinline__ int32_t entry_at(const int32_t *row, const R *val, int64_t e, R &v) {
    const int32_t raw = row[e];
    if (VM == 2) {
        v = raw < 0 ? R(-1) : R(1);
        return raw & 0x7fffffff;
    }
    v = VM == 1 ? val[e] : R(1);
    return raw;
}

// VM 3: every value 1 and the rows of a class's entries are consecutive in
// entry order (a class whose columns own every row they touch, such as the
// first class in colouring order), so the row is computed, not loaded.
template <int VM> __host__ __device__ constexpr bool has_vals() { return VM == 1 || VM == 2; }
template <int VM, class R>
__device__ __forceinline__ int32_t sched_entry(const Sched<R> &sc, int64_t e, R &v) {
    if (VM == 3) {
        v = R(1);
        return (int32_t)(e + sc.row_off);
    }
    return entry_at<VM>(sc.row, sc.val, e, v);
}

// entry e of a fixed-stride column: -1 for an unused slot (kNoRow)
template <int VM, class R>
__device__ __forceinline__ int32_t padded_entry(const Sched<R> &sc, int64_t e, R &v) {
    if (VM == 3) {
        v = R(1);
        return (int32_t)(e + sc.row_off);
    }
    const int32_t raw = sc.row[e];
    if (raw == kNoRow) return -1;
    if (VM == 2) {
        v = raw < 0 ? R(-1) : R(1);
        return raw & 0x7fffffff;
    }
    v = VM == 1 ? sc.val[e] : R(1);
    return raw;
}

// Grid layout of one fused launch: the workgroup ranges of the segment
// kinds in this order (hubs first so their long gathers start early).
constexpr int kGridKinds = SEG_NKIND + 1;   // + the per-column terms of the dual pass
// grid position -> segment kind: HUB, G2..G64, BLOCK, SLACK, column terms
__host__ __device__ constexpr int grid_kind(int p) {
    return p == 0 ? SEG_HUB
                  : (p <= kGroupKinds ? p - 1
                                      : (p == kGroupKinds + 1 ? SEG_BLOCK : (p == kGroupKinds + 2 ? SEG_SLACK : SEG_NKIND)));
}
__host__ __device__ constexpr int grid_pos(int kind) {
    return kind == SEG_HUB ? 0
                           : (kind < kGroupKinds ? kind + 1
                                                 : (kind == SEG_BLOCK ? kGroupKinds + 1
                                                                      : (kind == SEG_SLACK ? kGroupKinds + 2 : kGroupKinds + 3)));
}
struct LaunchPlan {
    int64_t wg_start[kGridKinds + 1];   // by grid position
    int64_t first[kGridKinds];          // offset of the segment in its schedule
    int64_t count[kGridKinds];          // units of the segment
    int32_t lanes[kGridKinds];          // lanes per column of the lane-group ranges
    int32_t cols[kGridKinds];           // columns per lane group (sweep plans)
    int64_t hub_wg;                     // hub workgroups, a multiple of 8
    int64_t nwg;
    int32_t xsplit;                     // solo sweep: every range split over the XCDs (xcd_part)
    // fixed-stride lane-group ranges (sweep plans of the DET copy): the
    // entries of the range's i-th column start at ebase + i * stride
    int64_t ebase[kGridKinds];
    int32_t stride[kGridKinds];
};

// logical workgroup L of a plan -> grid position and workgroup inside it
__device__ __forceinline__ int locate_logical(const LaunchPlan &pl, int64_t L, int64_t *local) {
    int p = 0;
    while (p < kGridKinds - 1 && L >= pl.wg_start[p + 1]) ++p;
    *local = L - pl.wg_start[p];
    return p;
}
// hardware workgroup b -> logical workgroup (hubs first, the rest XCD-remapped)
__device__ __forceinline__ int64_t logical_wg(const LaunchPlan &pl, int64_t b) {
    return b < pl.hub_wg ? b : pl.hub_wg + xcd_remap(b - pl.hub_wg, pl.nwg - pl.hub_wg);
}

template <class P>
__device__ __forceinline__ typename P::R gradient(const Dev<P> &a, int64_t j, typename P::R y,
                                                  typename P::R dot) {
    using R = typename P::R;
    R g = (a.ctil ? a.ctil[j] : (R)a.c[j]) + a.beta * dot;
    if (a.prox_on) g += a.rho * (y - (a.ybar ? a.ybar[j] : R(0)));
    return g;
}

// ||A_j||^2 is the degree when every value is +-1
template <class P, int VM>
__device__ __forceinline__ typename P::R curvature(const Dev<P> &a, int64_t j, int32_t d) {
    using R = typename P::R;
    if (a.global_lmax) return a.Lmax;
    return a.beta * (VM == 1 ? a.norm2[j] : (R)d) + a.rho;
}

// Plain columns on groups of G lanes.  A column of a lane-group range has
// at most G entries (its degree bucket), so lane l holds entry l.  Each group
// takes C columns of the range (workgroup-interleaved) and issues the loads
// of all C together, so every lane keeps C residual loads in flight and a
// workgroup covers C times the columns; the sums, steps and stores of each
// column are exactly those of a lone column, so the results do not depend
// on C.

// With a fixed-stride range (stride > 0: entry l of the column at plan
// position q is sbase + q * stride + l) no entry pointer is loaded: a lane
// goes straight to its entry, and the column's degree, which the unit-value
// curvature needs, is the count of the group's filled slots (a ballot).
template <class P, int VM, int G, int C>
__device__ __forceinline__ void sweep_group(const Dev<P> &a, const Sched<typename P::R> &sc,
                                            int64_t first, int64_t count, int64_t lwg, int64_t sbase,
                                            int32_t stride) {
    using R = typename P::R;
    constexpr int NG = kWG / G;
    const int lane = threadIdx.x & (G - 1);
    const int64_t u0 = lwg * (NG * C) + threadIdx.x / G;
    int32_t j[C], row[C];
    R v[C], rv[C], y[C], cj[C], L[C], U[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int64_t u = u0 + c * NG;
        j[c] = -1;
        row[c] = -1;
        v[c] = R(1);
        if (u < count) {
            const int64_t q = first + u;
            j[c] = sched_id(sc, q);
            if (stride) {
                if (lane < stride) row[c] = padded_entry<VM>(sc, sbase + q * stride + lane, v[c]);
            } else {
                const int32_t e0 = sc.ptr[q], d = sc.ptr[q + 1] - e0;
                if (lane < d) row[c] = sched_entry<VM>(sc, e0 + lane, v[c]);
                L[c] = curvature<P, VM>(a, j[c], d);
            }
            y[c] = (R)xval(a.x[j[c]]);
            cj[c] = a.ctil ? a.ctil[j[c]] : (R)a.c[j[c]];
            U[c] = col_bound(a, j[c]);
        }
    }
    if (stride) {
        // degree = filled slots of the group (every lane of the wave takes part)
        const int gbase = (threadIdx.x & 63) & ~(G - 1);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const uint64_t bal = __ballot(row[c] >= 0);
            const uint64_t mine = G == 64 ? bal : (bal >> gbase) & ((uint64_t(1) << (G & 63)) - 1);
            if (j[c] >= 0) L[c] = curvature<P, VM>(a, j[c], (int32_t)__popcll(mine));
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) rv[c] = row[c] >= 0 ? a.r[row[c]] : R(0);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        R acc = R(0);
        if (row[c] >= 0) acc += has_vals<VM>() ? v[c] * rv[c] : rv[c];
        acc = group_sum<G>(acc);          // every lane of the wave takes part
        if (j[c] < 0) continue;
        R g = cj[c] + a.beta * acc;
        if (a.prox_on) g += a.rho * (y[c] - (a.ybar ? a.ybar[j[c]] : R(0)));
        const R yn = stored_value<P>(coord_step(y[c], g, L[c], a.gamma, U[c]));
        const R d = yn - y[c];
        if (lane == 0) store_x<P>(a.x + j[c], yn);
        if (d != R(0) && row[c] >= 0) r_add(a.r + row[c], rv[c], has_vals<VM>() ? d * v[c] : d, a.async_mode);
    }
}

// High-degree column: one workgroup.  The gather is unrolled four deep so
// each thread keeps four residual loads in flight; the first HubTile
// gathered entries and their rows are staged in LDS so their scatter does not
// re-read global memory, and the scatter of the rest keeps four entries per
// thread in flight.
template <class P>
struct HubTile {
    static constexpr int n = sizeof(typename P::R) == 4 ? 2048 : 1024;
};

template <class P, int VM>
__device__ __forceinline__ void sweep_hub(const Dev<P> &a, const Sched<typename P::R> &sc,
                                          int64_t q, typename P::R *st_r, int32_t *st_row,
                                          typename P::R *red) {
    using R = typename P::R;
    constexpr int TILE = HubTile<P>::n;
    const int tid = threadIdx.x;
    const int32_t j = sched_id(sc, q);
    const int32_t e0 = sc.ptr[q], e1 = sc.ptr[q + 1];
    R acc = R(0);
    for (int32_t base = e0; base < e1; base += 4 * kWG) {
        int32_t rw[4];
        R rv[4], vv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int32_t e = base + t * kWG + tid;
            rw[t] = e < e1 ? sched_entry<VM>(sc, e, vv[t]) : -1;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) rv[t] = rw[t] >= 0 ? a.r[rw[t]] : R(0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int32_t e = base + t * kWG + tid;
            if (rw[t] >= 0) {
                const int32_t o = e - e0;
                if (o < TILE) { st_r[o] = rv[t]; st_row[o] = rw[t]; }
                acc += has_vals<VM>() ? vv[t] * rv[t] : rv[t];
            }
        }
    }
    acc = group_sum<64>(acc);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    R tot = red[0];
#pragma unroll
    for (int w = 1; w < kWG / 64; ++w) tot += red[w];
    __syncthreads();   // red is reused by the next column of a batched loop
    const R y = (R)xval(a.x[j]);
    const R g = gradient(a, j, y, tot);
    const R yn = stored_value<P>(coord_step(y, g, curvature<P, VM>(a, j, e1 - e0), a.gamma, col_bound(a, j)));
    const R d = yn - y;
    if (tid == 0) store_x<P>(a.x + j, yn);
    if (d != R(0)) {
        // the staged entries: rows and old values from LDS, stores only
        const int32_t staged = min(e1 - e0, (int32_t)TILE);
        for (int32_t o = tid; o < staged; o += kWG) {
            R ve = R(1);
            if (has_vals<VM>()) (void)sched_entry<VM>(sc, e0 + o, ve);
            r_add(a.r + st_row[o], st_r[o], has_vals<VM>() ? d * ve : d, a.async_mode);
        }
        // the rest, four entries per thread in flight: their row loads, then
        // their residual loads, then the stores (the column's rows are
        // distinct, so no store feeds a later load)
        for (int32_t base = e0 + TILE; base < e1; base += 4 * kWG) {
            int32_t re[4];
            R ve[4], rv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int32_t e = base + t * kWG + tid;
                ve[t] = R(1);
                re[t] = e < e1 ? sched_entry<VM>(sc, e, ve[t]) : -1;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) rv[t] = re[t] >= 0 && !a.async_mode ? a.r[re[t]] : R(0);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (re[t] >= 0) r_add(a.r + re[t], rv[t], has_vals<VM>() ? d * ve[t] : d, a.async_mode);
        }
    }
}

// Simplex blocks (k columns of one pixel): BPW blocks per wavefront, each on
// 64/BPW lanes split into k groups of LPC lanes (LPC = largest power of two
// <= 64/(BPW k)); group i forms the gradient of column i.  The projection
// onto the simplex uses theta = max_j (P_j - 1)/c_j over the prefixes of the
// values sorted downwards (Held, Wolfe & Crowder; Duchi et al.), every lane
// evaluating one candidate j without sorting.  A lane's block has columns
// j0 .. j0+k-1; the entries of column i are [cptr[i], cptr[i+1]) of rows /
// vals (the CSC, or the packed block copy); `valid` is false for the lanes
// of a block position past the end (they still take part in the shuffles).
template <class P, int VM, int BPW>
__device__ __forceinline__ void sweep_block(const Dev<P> &a, bool valid, int32_t blk, int32_t j0, const int32_t *cptr,
                                            const int32_t *rows, const typename P::R *vals, int lpc) {
    using R = typename P::R;
    constexpr int LB = 64 / BPW;
    const int lane = threadIdx.x & 63;
    const int lb = lane % LB, base = lane - lb;
    const int32_t k = a.k;
    const int ci = lb / lpc, sub = lb % lpc;
    const bool own = valid && ci < k;
    const int32_t j = j0 + (own ? ci : 0);
    const int32_t e0 = own ? cptr[ci] : 0, e1 = own ? cptr[ci + 1] : 0;
    R acc = R(0);
    for (int32_t e = e0 + sub; e < e1; e += lpc) {
        R ve;
        const R rv = a.r[entry_at<VM>(rows, vals, e, ve)];
        acc += VM ? ve * rv : rv;
    }
    for (int o = lpc / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    const R L = a.global_lmax ? a.Lmax : (valid ? a.LB[blk] : R(0));
    R y = R(0), v = R(0);
    if (own) {
        y = (R)xval(a.x[j]);
        const R g = gradient(a, j, y, acc);
        v = L > R(0) ? y - a.gamma * g / L : y;
    }
    // lane q < k of a block takes the value of column q; every shuffle runs
    // with the whole wavefront active
    const R vq = __shfl(v, base + (lb < k ? lb : 0) * lpc, 64);
    R psum = R(0);
    int cnt = 0;
    for (int l = 0; l < k; ++l) {
        const R vl = __shfl(v, base + l * lpc, 64);
        if (vl > vq || (vl == vq && l <= lb)) { psum += vl; ++cnt; }
    }
    R theta = valid && lb < k ? (psum - R(1)) / (R)cnt : R(-INFINITY);
#pragma unroll
    for (int o = LB / 2; o > 0; o >>= 1) {
        const R t2 = __shfl_xor(theta, o, 64);
        theta = t2 > theta ? t2 : theta;
    }
    R w = v - theta;
    if (w < R(0)) w = R(0);
    w = stored_value<P>(w);
    const R d = own ? w - y : R(0);
    if (own && sub == 0) store_x<P>(a.x + j, w);
    if (own && d != R(0)) {
        for (int32_t e = e0 + sub; e < e1; e += lpc) {
            R ve;
            R *p = a.r + entry_at<VM>(rows, vals, e, ve);
            const R dv = VM ? d * ve : d;
            r_add(p, a.async_mode ? R(0) : *p, dv, a.async_mode);
        }
    }
}

// the packed DET blocks
template <class R>
struct BlockPack {
    const int32_t *id, *j0, *ptr, *row;
    const R *val;
    int32_t vmode;         // entries as in Sched
};
template <class P, int VM, int BPW>
__device__ __forceinline__ void sweep_block_packed(const Dev<P> &a, const BlockPack<typename P::R> &bp, bool valid,
                                                   int64_t t, int lpc) {
    const int32_t blk = valid ? bp.id[t] : 0, j0 = valid ? bp.j0[t] : 0;
    sweep_block<P, VM, BPW>(a, valid, blk, j0, bp.ptr + (valid ? t * a.k : 0), bp.row, bp.val, lpc);
}
// the column copy always stores its values (or none when all are 1)
template <class P, int VM, int BPW>
__device__ __forceinline__ void sweep_block_csc(const Dev<P> &a, bool valid, int32_t blk, int lpc) {
    const int32_t j0 = valid ? a.bfirst[blk] : 0;
    sweep_block<P, (VM == 0 ? 0 : 1), BPW>(a, valid, blk, j0, a.col_ptr + j0, a.row_idx, a.cval, lpc);
}
// blocks per wavefront for block size k (the layout of the sums depends on
// it, so the solo and batched sweeps take the same)
__host__ __device__ constexpr int block_bpw(int k) { return k <= 8 ? 4 : (k <= 16 ? 2 : 1); }

// slack s_i of an inequality row: column -e_i ('>=') or +e_i ('<='), s >= 0
template <class P>
__device__ __forceinline__ void sweep_slack(const Dev<P> &a, int64_t i) {
    using R = typename P::R;
    const R sg = a.sense[i] > 0 ? R(-1) : R(1);
    const R sv = a.s[i], rv = a.r[i];
    R g = (a.ctil ? a.ctil[a.n + i] : R(0)) + a.beta * (sg * rv);
    if (a.prox_on) g += a.rho * (sv - (a.ybar ? a.ybar[a.n + i] : R(0)));
    const R L = a.global_lmax ? a.Lmax : a.beta + a.rho;
    R sn = L > R(0) ? sv - a.gamma * g / L : (g > R(0) ? R(0) : sv);
    if (sn < R(0)) sn = R(0);
    const R d = sn - sv;
    a.s[i] = sn;
    if (d != R(0)) {
        if (a.async_mode) unsafeAtomicAdd(a.r + i, sg * d);
        else a.r[i] = rv + sg * d;
    }
}

template <class P, int VM, int G>
__device__ __forceinline__ void sweep_groups_c(const Dev<P> &a, const Sched<typename P::R> &sc, int cols,
                                               int64_t first, int64_t count, int64_t lwg, int64_t sbase,
                                               int32_t stride) {
    switch (cols) {
        case 1: sweep_group<P, VM, G, 1>(a, sc, first, count, lwg, sbase, stride); break;
        case 2: sweep_group<P, VM, G, 2>(a, sc, first, count, lwg, sbase, stride); break;
        case 4: sweep_group<P, VM, G, 4>(a, sc, first, count, lwg, sbase, stride); break;
        default: break;
    }
}
template <class P, int VM>
__device__ __forceinline__ void sweep_groups(const Dev<P> &a, const Sched<typename P::R> &sc, int lanes, int cols,
                                             int64_t first, int64_t count, int64_t lwg, int64_t sbase,
                                             int32_t stride) {
    switch (lanes) {
        case 2: sweep_groups_c<P, VM, 2>(a, sc, cols, first, count, lwg, sbase, stride); break;
        case 4: sweep_groups_c<P, VM, 4>(a, sc, cols, first, count, lwg, sbase, stride); break;
        case 8: sweep_groups_c<P, VM, 8>(a, sc, cols, first, count, lwg, sbase, stride); break;
        case 16: sweep_groups_c<P, VM, 16>(a, sc, cols, first, count, lwg, sbase, stride); break;
        case 32: sweep_groups_c<P, VM, 32>(a, sc, cols, first, count, lwg, sbase, stride); break;
        case 64: sweep_groups_c<P, VM, 64>(a, sc, cols, first, count, lwg, sbase, stride); break;
        default: break;
    }
}

// One class (DET) or one whole epoch part (ASYNC) in a single launch.
// logical workgroup L of a column plan.  A lane-group range may run wider
// groups than its degree bound (the tuner's choice): the extra lanes hold
// exact zeros, so the butterfly sums -- and every result -- are unchanged.
// With xsplit, L is the hardware workgroup: every range starts at a multiple
// of kXcds workgroups, and workgroup l of a range takes run l / kXcds of
// the range's part l % kXcds, so part x runs on XCD x.
template <class P, int VM>
__device__ __forceinline__ void sweep_item(const Dev<P> &a, const Sched<typename P::R> &sc, const LaunchPlan &pl,
                                           int64_t L, typename P::R *st_r, int32_t *st_row, typename P::R *red) {
    int64_t local;
    const int p = locate_logical(pl, L, &local);
    int64_t first = pl.first[p], count = pl.count[p];
    // entry base such that column q's slots start at sbase + q * stride
    const int64_t sbase = pl.ebase[p] - pl.first[p] * (int64_t)pl.stride[p];
    if (pl.xsplit) {
        const int64_t x = local % kXcds, lo = count * x / kXcds, hi = count * (x + 1) / kXcds;
        first += lo;
        count = hi - lo;
        local /= kXcds;
    }
    if (grid_kind(p) == SEG_HUB) {
        if (local < count) sweep_hub<P, VM>(a, sc, first + local, st_r, st_row, red);
        return;
    }
    sweep_groups<P, VM>(a, sc, pl.lanes[p], pl.cols[p], first, count, local, sbase, pl.stride[p]);
}

// The plain columns of one class (DET) or of a whole epoch (ASYNC) in one
// launch: hub workgroups first, then the lane-group ranges.
template <class P, int VM>
__global__ __launch_bounds__(kWG) void k_sweep(Dev<P> a, Sched<typename P::R> sc, LaunchPlan pl) {
    using R = typename P::R;
    __shared__ R st_r[HubTile<P>::n];
    __shared__ int32_t st_row[HubTile<P>::n];
    __shared__ R red[kWG / 64];
    sweep_item<P, VM>(a, sc, pl, pl.xsplit ? (int64_t)blockIdx.x : logical_wg(pl, blockIdx.x), st_r, st_row, red);
}

// the simplex blocks of one class: one wavefront per block, from the packed
// DET copy (list == null: blocks pb_first ..) or by id through the CSC
template <class P, int VM, int BPW>
__global__ __launch_bounds__(kWG) void k_sweep_block(Dev<P> a, const int32_t *__restrict__ list,
                                                     BlockPack<typename P::R> bp, int64_t pb_first,
                                                     int64_t count, int32_t lpc) {
    const int64_t w = xcd_remap(blockIdx.x, gridDim.x) * (kWG / 64) + (threadIdx.x >> 6);
    if (w * BPW >= count) return;        // the whole wavefront leaves together
    const int64_t u = w * BPW + (threadIdx.x & 63) / (64 / BPW);
    const bool valid = u < count;
    if (list) sweep_block_csc<P, VM, BPW>(a, valid, valid ? list[u] : 0, lpc);
    else sweep_block_packed<P, VM, BPW>(a, bp, valid, pb_first + u, lpc);
}

// the slack class: one lane per inequality row
template <class P>
__global__ __launch_bounds__(kWG) void k_sweep_slack(Dev<P> a, const int32_t *__restrict__ list,
                                                     int64_t count) {
    const int64_t u = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (u < count) sweep_slack<P>(a, list ? list[u] : u);
}

// ---------------------------------------------------------------- reductions
constexpr int kRowSlots = 6;   // sum w^2, max |w|, max violation, sum b u, sum (u-ubar)^2, sum -ubar w
constexpr int kColSlots = 3;   // sum of minima (Phi), c^T x, prox part of F

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// block reduction in fixed order into out[slot]; op 0 = sum, 1 = max
template <int NS>
__device__ void block_reduce(const double (&v)[NS], const int (&op)[NS], double *out) {
    __shared__ double sh[kWG / 64][NS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const double t = op[q] ? wmax(v[q]) : wsum(v[q]);
        if (lane == 0) sh[w][q] = t;
    }
    __syncthreads();
    if (threadIdx.x < NS) {
        const int q = threadIdx.x;
        double t = sh[0][q];
        for (int ww = 1; ww < kWG / 64; ++ww) t = op[q] ? fmax(t, sh[ww][q]) : t + sh[ww][q];
        out[q] = t;
    }
    __syncthreads();
}

// min over [0,U] of red*y + rho/2 (y - yb)^2
__device__ __forceinline__ double box_min(double red, double U, double rho, double yb) {
    if (rho > 0.0) {
        double y = yb - red / rho;
        if (y < 0.0) y = 0.0;
        if (y > U) y = U;
        return red * y + 0.5 * rho * (y - yb) * (y - yb);
    }
    if (red >= 0.0) return 0.0;
    return isinf(U) ? -INFINITY : red * U;
}

// Row pass: w = A x + slack - b in FP64, optionally stored as the new
// running residual; the dual estimate u = ubar - beta w (clipped so the
// unbounded slack columns keep a non-negative reduced cost when rho = 0),
// rounded once to storage precision and used for every term of Phi.
// rows a thread of the row pass takes (fewer partial records to fold)
constexpr int kRowsPerThread = 4;

template <class P>
__device__ __forceinline__ void rows_item(const Dev<P> &a, int64_t wg, int32_t write_r, int32_t with_dual,
                                          double *part) {
    using R = typename P::R;
    double v[kRowSlots] = {0, 0, 0, 0, 0, 0};
    const int op[kRowSlots] = {0, 1, 1, 0, 0, 0};
    // rows_lanes lanes per row (a power of two; long rows): the group's lanes
    // stride the row and reduce with a butterfly, its first lane finishes
    const int G = a.row_lanes, lane = threadIdx.x & (G - 1);
    for (int q = 0; q < kRowsPerThread; ++q) {
        const int64_t i = (wg * kRowsPerThread + q) * (kWG / G) + threadIdx.x / G;
        if (i >= a.m) break;                  // the whole group together
        double ax = 0.0;
        for (int32_t e = a.row_ptr[i] + lane; e < a.row_ptr[i + 1]; e += G)
            ax += (a.csr_val ? (double)a.csr_val[e] : 1.0) * (double)xval(a.x[a.csr_col[e]]);
        for (int o = G / 2; o > 0; o >>= 1) ax += __shfl_xor(ax, o, 64);
        if (lane) continue;
        const int8_t sn = a.sense[i];
        double acc = ax;
        if (sn > 0) acc -= (double)a.s[i];
        else if (sn < 0) acc += (double)a.s[i];
        const double w = acc - a.b[i];
        if (write_r) a.r[i] = (R)w;
        const double ub = a.ubar ? a.ubar[i] : 0.0;
        double ui = ub - (double)a.beta * w;
        if (!a.prox_on) {
            if (sn > 0 && ui < 0.0) ui = 0.0;
            if (sn < 0 && ui > 0.0) ui = 0.0;
        }
        const R ur = (R)ui;
        if (with_dual) a.udual[i] = ur;
        const double ud = (double)ur;
        double viol = sn > 0 ? a.b[i] - ax : (sn < 0 ? ax - a.b[i] : fabs(ax - a.b[i]));
        if (viol < 0.0) viol = 0.0;
        v[0] += w * w;
        v[1] = fmax(v[1], fabs(w));
        v[2] = fmax(v[2], viol);
        v[3] += a.b[i] * ud;
        v[4] += (ud - ub) * (ud - ub);
        v[5] += -ub * w;
    }
    block_reduce<kRowSlots>(v, op, part + wg * kRowSlots);
}

template <class P>
__global__ __launch_bounds__(kWG) void k_rows(Dev<P> a, int32_t write_r, int32_t with_dual, double *part) {
    rows_item<P>(a, blockIdx.x, write_r, with_dual, part);
}

// Workgroup sum of one double, returned to every thread (fixed order).
__device__ double block_sum_all(double v, double *sh) {
    v = wsum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = sh[0];
    for (int w = 1; w < kWG / 64; ++w) t += sh[w];
    __syncthreads();
    return t;
}

template <class P>
__device__ __forceinline__ double col_ubound(const Dev<P> &a, int64_t j) {
    return a.ub ? (double)a.ub[j] : (double)a.ub_value;
}

// Column pass of the refresh, on the ASYNC plan (every structural unit in
// degree buckets, then the slacks) plus one range over all columns for
// c^T x and the prox part of F.  Per variable: the minimum over its
// feasible set of its reduced-cost term (the inner minimisation of the dual
// function Phi), with the reduced cost gathered lane-group parallel like the
// sweep.  Every workgroup writes kColSlots partials.
template <class P, bool VALS>
__device__ __forceinline__ void dual_item(const Dev<P> &a, const Sched<typename P::R> &sc, const LaunchPlan &pl,
                                          int64_t L, int32_t slack_identity, double *part, double *sh) {
    int64_t local;
    const int p = locate_logical(pl, L, &local);
    const int64_t first = pl.first[p], count = pl.count[p];
    const int kind = grid_kind(p);
    const double rho = (double)a.rho;
    double v[kColSlots] = {0, 0, 0};
    const int op[kColSlots] = {0, 0, 0};
    if (kind == SEG_HUB) {
        const bool valid = local < count;
        double acc = 0.0;
        int32_t j = 0;
        if (valid) {
            const int64_t q = first + local;
            j = sc.ids[q];
            for (int32_t e = sc.ptr[q] + threadIdx.x; e < sc.ptr[q + 1]; e += kWG)
                acc += (VALS ? (double)sc.val[e] : 1.0) * (double)a.udual[sc.row[e]];
        }
        acc = block_sum_all(acc, sh);
        if (valid && threadIdx.x == 0)
            v[0] = box_min(a.c[j] - acc, col_ubound(a, j), rho, a.ybar ? (double)a.ybar[j] : 0.0);
    } else if (kind < kGroupKinds) {
        // kRowsPerThread columns per lane group
        const int G = pl.lanes[p];
        const int lane = threadIdx.x & (G - 1);
        for (int rq = 0; rq < kRowsPerThread; ++rq) {
            const int64_t u = (local * kRowsPerThread + rq) * (kWG / G) + threadIdx.x / G;
            const bool valid = u < count;
            double acc = 0.0;
            int32_t j = 0;
            if (valid) {
                const int64_t q = first + u;
                j = sc.ids[q];
                for (int32_t e = sc.ptr[q] + lane; e < sc.ptr[q + 1]; e += G)
                    acc += (VALS ? (double)sc.val[e] : 1.0) * (double)a.udual[sc.row[e]];
            }
            for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
            if (valid && lane == 0)
                v[0] += box_min(a.c[j] - acc, col_ubound(a, j), rho, a.ybar ? (double)a.ybar[j] : 0.0);
        }
    } else if (kind == SEG_BLOCK) {
        // one wavefront per block, lpc lanes per column as in the sweep; the
        // minimum over the simplex without prox is the smallest reduced
        // cost, with prox the value at the projection of yb - red/rho;
        // kRowsPerThread blocks per wavefront
        const int lane = threadIdx.x & 63;
        for (int rq = 0; rq < kRowsPerThread; ++rq) {
            const int64_t u = (local * kRowsPerThread + rq) * (kWG / 64) + (threadIdx.x >> 6);
            if (u >= count) break;                // the whole wavefront together
            const int32_t bl = sc.ids[first + u];
            const int32_t k = a.k;
            int lpc = 64;
            while (lpc * k > 64) lpc >>= 1;
            const int ci = lane / lpc, sub = lane % lpc;
            const bool own = ci < k;
            const int32_t j = a.bfirst[bl] + (own ? ci : 0);
            double acc = 0.0;
            if (own)
                for (int32_t e = a.col_ptr[j] + sub; e < a.col_ptr[j + 1]; e += lpc)
                    acc += (VALS ? (double)a.cval[e] : 1.0) * (double)a.udual[a.row_idx[e]];
            for (int o = lpc / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
            const double red = own ? a.c[j] - acc : INFINITY;
            double term;
            if (a.prox_on) {
                const double yb = own && a.ybar ? (double)a.ybar[j] : 0.0;
                const double w = own ? yb - red / rho : 0.0;
                const double wq = __shfl(w, (lane < k ? lane : 0) * lpc, 64);
                double ps = 0.0;
                int cnt = 0;
                for (int l = 0; l < k; ++l) {
                    const double wl = __shfl(w, l * lpc, 64);
                    if (wl > wq || (wl == wq && l <= lane)) { ps += wl; ++cnt; }
                }
                const double theta = wmax(lane < k ? (ps - 1.0) / cnt : -INFINITY);
                const double yi = fmax(w - theta, 0.0);
                term = wsum(own && sub == 0 ? red * yi + 0.5 * rho * (yi - yb) * (yi - yb) : 0.0);
            } else {
                term = -wmax(-red);
            }
            if (lane == 0) v[0] += term;
        }
    } else if (kind == SEG_SLACK) {
        for (int rq = 0; rq < kRowsPerThread; ++rq) {
            const int64_t u = (local * kRowsPerThread + rq) * kWG + threadIdx.x;
            if (u >= count) break;
            const int64_t i = slack_identity ? u : sc.ids[first + u];
            const int8_t sn = a.sense[i];
            const double sv = (double)a.s[i];
            const double yb = a.ybar ? (double)a.ybar[a.n + i] : 0.0;
            if (a.prox_on) v[2] += 0.5 * rho * (sv - yb) * (sv - yb);
            v[0] += box_min((sn > 0 ? 1.0 : -1.0) * (double)a.udual[i], INFINITY, rho, yb);
        }
    } else {
        // every structural column (kRowsPerThread per thread): c^T x, the
        // prox part of F, and the fixed simplex blocks' contribution to Phi
        // (their first column's thread)
        for (int q = 0; q < kRowsPerThread; ++q) {
            const int64_t j = (local * kRowsPerThread + q) * kWG + threadIdx.x;
            if (j >= a.n) break;
            const double xj = (double)xval(a.x[j]);
            v[1] += a.c[j] * xj;
            const double yb = a.ybar ? (double)a.ybar[j] : 0.0;
            if (a.prox_on) v[2] += 0.5 * rho * (xj - yb) * (xj - yb);
            const int32_t bl = a.col_block ? a.col_block[j] : -1;
            if (bl >= 0 && a.fixed[bl] >= 0 && j == a.bfirst[bl]) {
                const int f = a.fixed[bl], k = a.k;
                const int32_t jf = a.bfirst[bl] + f;
                double val = a.c[jf];
                for (int32_t e = a.col_ptr[jf]; e < a.col_ptr[jf + 1]; ++e)
                    val -= (VALS ? (double)a.cval[e] : 1.0) * (double)a.udual[a.row_idx[e]];
                if (a.prox_on)
                    for (int i = 0; i < k; ++i) {
                        const double ybi = a.ybar ? (double)a.ybar[a.bfirst[bl] + i] : 0.0;
                        const double d = (i == f ? 1.0 : 0.0) - ybi;
                        val += 0.5 * rho * d * d;
                    }
                v[0] += val;
            }
        }
    }
    block_reduce<kColSlots>(v, op, part + L * kColSlots);
}

template <class P, bool VALS>
__global__ __launch_bounds__(kWG) void k_dual(Dev<P> a, Sched<typename P::R> sc, LaunchPlan pl,
                                              int32_t slack_identity, double *part) {
    __shared__ double sh[kWG / 64];
    dual_item<P, VALS>(a, sc, pl, logical_wg(pl, blockIdx.x), slack_identity, part, sh);
}

// metrics slots
enum { MT_F = 0, MT_CX, MT_LINF, MT_L2, MT_VIOL, MT_PHI, MT_GAP, MT_BAD, MT_NSLOT = 16 };

// One workgroup folds nb records of NS partial slots in a fixed order:
// thread t takes records t, t+256, ..., then a pairwise tree.  op: 0 sum,
// 1 max, 2 min.  The result is valid in thread 0.
template <int NS>
__device__ void fold_records(const double *part, int64_t nb, const int (&op)[NS], double (&out)[NS]) {
    __shared__ double sh[kWG][NS];
    const int t = threadIdx.x;
    double acc[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) acc[q] = op[q] == 0 ? 0.0 : (op[q] == 1 ? -INFINITY : INFINITY);
    // eight records' loads are issued together, then combined in record
    // order: the same sequence of operations as one record at a time
    constexpr int U = 8;
    int64_t b = t;
    for (; b + (U - 1) * kWG < nb; b += U * kWG) {
        double x[U][NS];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < NS; ++q) x[u][q] = part[(b + u * kWG) * NS + q];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < NS; ++q)
                acc[q] = op[q] == 0 ? acc[q] + x[u][q] : (op[q] == 1 ? fmax(acc[q], x[u][q]) : fmin(acc[q], x[u][q]));
    }
    for (; b < nb; b += kWG)
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const double x = part[b * NS + q];
            acc[q] = op[q] == 0 ? acc[q] + x : (op[q] == 1 ? fmax(acc[q], x) : fmin(acc[q], x));
        }
#pragma unroll
    for (int q = 0; q < NS; ++q) sh[t][q] = acc[q];
    __syncthreads();
    for (int w = kWG / 2; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const double x = sh[t + w][q];
                sh[t][q] = op[q] == 0 ? sh[t][q] + x : (op[q] == 1 ? fmax(sh[t][q], x) : fmin(sh[t][q], x));
            }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) out[q] = sh[0][q];
    __syncthreads();
}

__device__ __forceinline__ void finalize_item(const double *rp, int64_t nr, const double *cp, int64_t nc,
                                              double beta, int32_t with_dual, double *mt) {
    const int rop[kRowSlots] = {0, 1, 1, 0, 0, 0};
    const int cop[kColSlots] = {0, 0, 0};
    double rs[kRowSlots], cs[kColSlots];
    fold_records<kRowSlots>(rp, nr, rop, rs);
    fold_records<kColSlots>(cp, nc, cop, cs);
    if (threadIdx.x == 0) {
        const double F = cs[1] + rs[5] + 0.5 * beta * rs[0] + cs[2];
        const double phi = rs[3] - rs[4] / (2.0 * beta) + cs[0];
        mt[MT_F] = F;
        mt[MT_CX] = cs[1];
        mt[MT_LINF] = rs[1];
        mt[MT_L2] = sqrt(rs[0]);
        mt[MT_VIOL] = rs[2];
        const double den = fabs(F) > 1.0 ? fabs(F) : 1.0;
        mt[MT_PHI] = with_dual ? phi : NAN;
        mt[MT_GAP] = with_dual ? (F - phi) / den : NAN;
        mt[MT_BAD] = (isfinite(F) && isfinite(rs[0])) ? 0.0 : 1.0;
    }
}

__global__ __launch_bounds__(kWG) void k_finalize(const double *rp, int64_t nr, const double *cp,
                                                  int64_t nc, double beta, int32_t with_dual, double *mt) {
    finalize_item(rp, nr, cp, nc, beta, with_dual, mt);
}

// ---------------------------------------------------------------- multiplier step
// Augmented-Lagrangian update between two penalty solves (Section 3.2):
// ubar <- ubar - beta (A y - b), optionally ybar <- y, and ctil = c - A^T ubar
// recomputed in FP64, together with the LP dual function D at the new
// multiplier clipped to the sign each inequality row's slack allows
// (covering >= 0, packing <= 0): D(u) = b^T u + sum over variables of the
// minimum of its reduced-cost term over its feasible set, a lower bound on
// the LP optimum.  After the clip every slack's reduced cost is
// non-negative, so the slacks add nothing to D.
constexpr int kMulRowSlots = 2;   // sum b u, max |w|
constexpr int kMulColSlots = 2;   // sum of minima, c^T x

__device__ __forceinline__ double clip_dual(double u, int8_t sn) {
    return sn > 0 ? fmax(u, 0.0) : (sn < 0 ? fmin(u, 0.0) : u);
}

// Row pass: w from x and s in FP64 (kRowsPerThread rows per thread), the new
// multiplier, the slack entries of ctil (covering +ubar, packing -ubar) and,
// when ybar_w is set, the slack part of the new prox centre.
template <class P>
__global__ __launch_bounds__(kWG) void k_mul_rows(Dev<P> a, double *ubar_w, double2 *upair, typename P::R *ctil_w,
                                                  typename P::R *ybar_w, double beta, double *part) {
    using R = typename P::R;
    double v[kMulRowSlots] = {0, 0};
    const int op[kMulRowSlots] = {0, 1};
    const int G = a.row_lanes, lane = threadIdx.x & (G - 1);
    for (int q = 0; q < kRowsPerThread; ++q) {
        const int64_t i = ((int64_t)blockIdx.x * kRowsPerThread + q) * (kWG / G) + threadIdx.x / G;
        if (i >= a.m) break;                  // the whole group together
        double acc = 0.0;
        for (int32_t e = a.row_ptr[i] + lane; e < a.row_ptr[i + 1]; e += G)
            acc += (a.csr_val ? (double)a.csr_val[e] : 1.0) * (double)xval(a.x[a.csr_col[e]]);
        for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane) continue;
        const int8_t sn = a.sense[i];
        if (sn > 0) acc -= (double)a.s[i];
        else if (sn < 0) acc += (double)a.s[i];
        const double w = acc - a.b[i];
        const double un = ubar_w[i] - beta * w;
        const double uc = clip_dual(un, sn);
        ubar_w[i] = un;
        // the column pass reads both values of a row with one 16-byte load
        upair[i] = make_double2(un, uc);
        ctil_w[a.n + i] = (R)(sn > 0 ? un : (sn < 0 ? -un : 0.0));
        if (ybar_w) ybar_w[a.n + i] = a.s[i];
        v[0] += a.b[i] * uc;
        v[1] = fmax(v[1], fabs(w));
    }
    block_reduce<kMulRowSlots>(v, op, part + (int64_t)blockIdx.x * kMulRowSlots);
}

// Column pass on the refresh's column plan (every free unit in degree
// buckets, then one range over all columns): per column the two gathers
// A_j^T ubar (new ctil_j) and A_j^T clip(ubar) (reduced cost of D); plain
// columns add their box minimum, free blocks the smallest reduced cost of
// the block, fixed blocks the reduced cost of their fixed label; the range
// over all columns adds c^T x, writes ctil of fixed-block columns and moves
// the structural part of ybar.
template <class P, bool VALS>
__device__ __forceinline__ void mul_item(const Dev<P> &a, const Sched<typename P::R> &sc, const LaunchPlan &pl,
                                         int64_t L, const double2 *upair, typename P::R *ctil_w,
                                         typename P::R *ybar_w, double *part, double *sh) {
    using R = typename P::R;
    int64_t local;
    const int p = locate_logical(pl, L, &local);
    const int64_t first = pl.first[p], count = pl.count[p];
    const int kind = grid_kind(p);
    double v[kMulColSlots] = {0, 0};
    const int op[kMulColSlots] = {0, 0};
    auto gather = [&](int32_t e0, int32_t e1, int32_t step, const R *val, const int32_t *row,
                      double &t_u, double &t_c) {
        for (int32_t e = e0; e < e1; e += step) {
            const double av = VALS ? (double)val[e] : 1.0;
            const double2 up = upair[row[e]];
            t_u += av * up.x;
            t_c += av * up.y;
        }
    };
    if (kind == SEG_HUB) {
        const bool valid = local < count;
        double tu = 0.0, tc = 0.0;
        int32_t j = 0;
        if (valid) {
            const int64_t q = first + local;
            j = sc.ids[q];
            gather(sc.ptr[q] + threadIdx.x, sc.ptr[q + 1], kWG, sc.val, sc.row, tu, tc);
        }
        tu = block_sum_all(tu, sh);
        tc = block_sum_all(tc, sh);
        if (valid && threadIdx.x == 0) {
            ctil_w[j] = (R)(a.c[j] - tu);
            v[0] = box_min(a.c[j] - tc, col_ubound(a, j), 0.0, 0.0);
        }
    } else if (kind < kGroupKinds) {
        const int G = pl.lanes[p];
        const int lane = threadIdx.x & (G - 1);
        for (int rq = 0; rq < kRowsPerThread; ++rq) {
            const int64_t u = (local * kRowsPerThread + rq) * (kWG / G) + threadIdx.x / G;
            const bool valid = u < count;
            double tu = 0.0, tc = 0.0;
            int32_t j = 0;
            if (valid) {
                const int64_t q = first + u;
                j = sc.ids[q];
                gather(sc.ptr[q] + lane, sc.ptr[q + 1], G, sc.val, sc.row, tu, tc);
            }
            for (int o = G / 2; o > 0; o >>= 1) {
                tu += __shfl_xor(tu, o, 64);
                tc += __shfl_xor(tc, o, 64);
            }
            if (valid && lane == 0) {
                ctil_w[j] = (R)(a.c[j] - tu);
                v[0] += box_min(a.c[j] - tc, col_ubound(a, j), 0.0, 0.0);
            }
        }
    } else if (kind == SEG_BLOCK) {
        const int lane = threadIdx.x & 63;
        for (int rq = 0; rq < kRowsPerThread; ++rq) {
            const int64_t u = (local * kRowsPerThread + rq) * (kWG / 64) + (threadIdx.x >> 6);
            if (u >= count) break;                // the whole wavefront together
            const int32_t bl = sc.ids[first + u];
            const int32_t k = a.k;
            int lpc = 64;
            while (lpc * k > 64) lpc >>= 1;
            const int ci = lane / lpc, sub = lane % lpc;
            const bool own = ci < k;
            const int32_t j = a.bfirst[bl] + (own ? ci : 0);
            double tu = 0.0, tc = 0.0;
            if (own) gather(a.col_ptr[j] + sub, a.col_ptr[j + 1], lpc, a.cval, a.row_idx, tu, tc);
            for (int o = lpc / 2; o > 0; o >>= 1) {
                tu += __shfl_xor(tu, o, 64);
                tc += __shfl_xor(tc, o, 64);
            }
            if (own && sub == 0) ctil_w[j] = (R)(a.c[j] - tu);
            const double red = own ? a.c[j] - tc : INFINITY;
            const double term = -wmax(-red);
            if (lane == 0) v[0] += term;
        }
    } else if (kind == SEG_NKIND) {
        for (int q = 0; q < kRowsPerThread; ++q) {
            const int64_t j = (local * kRowsPerThread + q) * kWG + threadIdx.x;
            if (j >= a.n) break;
            const auto xs = a.x[j];
            v[1] += a.c[j] * (double)xval(xs);
            if (ybar_w) ybar_w[j] = (R)xval(xs);
            const int32_t bl = a.col_block ? a.col_block[j] : -1;
            if (bl >= 0 && a.fixed[bl] >= 0) {
                double tu = 0.0, tc = 0.0;
                gather(a.col_ptr[j], a.col_ptr[j + 1], 1, a.cval, a.row_idx, tu, tc);
                ctil_w[j] = (R)(a.c[j] - tu);
                if (j == a.bfirst[bl] + a.fixed[bl]) v[0] += a.c[j] - tc;
            }
        }
    }
    // slack units add nothing (clipped multiplier: reduced cost >= 0)
    block_reduce<kMulColSlots>(v, op, part + L * kMulColSlots);
}

template <class P, bool VALS>
__global__ __launch_bounds__(kWG) void k_mul_cols(Dev<P> a, Sched<typename P::R> sc, LaunchPlan pl,
                                                  const double2 *upair, typename P::R *ctil_w,
                                                  typename P::R *ybar_w, double *part) {
    __shared__ double sh[kWG / 64];
    mul_item<P, VALS>(a, sc, pl, logical_wg(pl, blockIdx.x), upair, ctil_w, ybar_w, part, sh);
}

// out: c^T x, max |w|, D, (c^T x - D) / max(1, |c^T x|)
__global__ __launch_bounds__(kWG) void k_mul_final(const double *rp, int64_t nr, const double *cp, int64_t nc,
                                                   double *out) {
    const int rop[kMulRowSlots] = {0, 1};
    const int cop[kMulColSlots] = {0, 0};
    double rs[kMulRowSlots], cs[kMulColSlots];
    fold_records<kMulRowSlots>(rp, nr, rop, rs);
    fold_records<kMulColSlots>(cp, nc, cop, cs);
    if (threadIdx.x == 0) {
        const double d = rs[0] + cs[0];
        out[0] = cs[1];
        out[1] = rs[1];
        out[2] = d;
        out[3] = (cs[1] - d) / (fabs(cs[1]) > 1.0 ? fabs(cs[1]) : 1.0);
    }
}

// ---------------------------------------------------------------- rounding
// edge pass for the two-entry rows: op 0 min (x_u+x_v)/2, 1 max (x_u+x_v)/2,
// 2 max (x_u+x_v-1)
template <class P>
__global__ __launch_bounds__(kWG) void k_edge_extreme(Dev<P> a, int32_t op, double *part) {
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    double v = op == 0 ? INFINITY : -INFINITY;
    if (i < a.m) {
        const int32_t e = a.row_ptr[i];
        const double xu = (double)xval(a.x[a.csr_col[e]]), xv = (double)xval(a.x[a.csr_col[e + 1]]);
        v = op == 2 ? (xu + xv) - 1.0 : (xu + xv) * 0.5;
    }
    if (op == 0) v = -v;
    v = wmax(v);
    __shared__ double sh[kWG / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int w = 1; w < kWG / 64; ++w) t = fmax(t, sh[w]);
        part[blockIdx.x] = op == 0 ? -t : t;
    }
}

// fold of the edge partials into the threshold (VC: min(1/2, m), MIS:
// max(1/2, m), alpha: max(0, m)); one workgroup
__global__ __launch_bounds__(kWG) void k_edge_fold(const double *part, int64_t nb, int32_t op, double *out) {
    const int o[1] = {op == 0 ? 2 : 1};
    double r[1];
    fold_records<1>(part, nb, o, r);
    if (threadIdx.x == 0) *out = op == 0 ? fmin(0.5, r[0]) : (op == 1 ? fmax(0.5, r[0]) : fmax(0.0, r[0]));
}

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }
__device__ __forceinline__ double unit53_dev(uint64_t w) { return (double)(w >> 11) * (1.0 / 9007199254740992.0); }

__device__ uint64_t philox_word_dev(uint64_t seed, uint64_t stream, uint64_t c0, uint64_t c1, uint64_t c2) {
    uint64_t x0 = c0, x1 = c1, x2 = c2, x3 = 0, k0 = seed, k1 = stream;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round) { k0 += Philox4x64::W0; k1 += Philox4x64::W1; }
        const uint64_t hi0 = mulhi64(Philox4x64::M0, x0), lo0 = Philox4x64::M0 * x0;
        const uint64_t hi1 = mulhi64(Philox4x64::M1, x2), lo1 = Philox4x64::M1 * x2;
        const uint64_t n0 = hi1 ^ x1 ^ k0, n2 = hi0 ^ x3 ^ k1;
        x0 = n0; x1 = lo1; x2 = n2; x3 = lo0;
    }
    return x0;
}

// the covering rounding's scaled point: x/(1-alpha) capped at 1, all ones
// once alpha reaches 1
__device__ __forceinline__ double cover_scaled(double x, double alpha) {
    const double v = alpha < 1.0 ? x / (1.0 - alpha) : 1.0;
    return v > 1.0 ? 1.0 : v;
}

// rule VC / COVER threshold: x >= T; MIS threshold: x > T; COVER_RAND: any
// of `rounds` draws below the scaled x; MIS_RAND / PACK_RAND: U_v <
// x/(1+alpha); writes 0/1 and the cost partial
template <class P>
__global__ __launch_bounds__(kWG) void k_pick(Dev<P> a, int32_t rule, const double *thr,
                                              uint64_t seed, int32_t rep, int32_t rounds, int32_t *sol,
                                              double *part, const int32_t *col_orig) {
    const int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x;
    double v = 0.0;
    if (j < a.n) {
        const double xj = (double)xval(a.x[j]);
        int32_t keep;
        if (rule == THETIS_ROUND_VC_THRESH || rule == THETIS_ROUND_COVER_THRESH) keep = xj >= *thr;
        else if (rule == THETIS_ROUND_MIS_THRESH) keep = xj > *thr;
        else if (rule == THETIS_ROUND_COVER_RAND) {
            // the union needs one draw below xt: stop at the first, and draw
            // nothing when xt <= 0 (no draw in [0, 1) is below it)
            const double xt = cover_scaled(xj, *thr);
            keep = 0;
            for (int32_t r = 0; r < rounds && xt > 0.0 && !keep; ++r)
                keep = unit53_dev(philox_word_dev(seed, RNG_ROUND, (uint64_t)rep, (uint64_t)col_orig[j], 16 + (uint64_t)r)) < xt;
        } else {
            const double xt = xj / (1.0 + *thr);
            keep = unit53_dev(philox_word_dev(seed, RNG_ROUND, (uint64_t)rep, (uint64_t)col_orig[j], 0)) < xt;
        }
        sol[j] = keep;
        v = keep ? a.c[j] : 0.0;
    }
    v = wsum(v);
    __shared__ double sh[kWG / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int w = 1; w < kWG / 64; ++w) t += sh[w];
        part[blockIdx.x] = t;
    }
}

// alteration: mark both ends of every row whose two vertices were picked
template <class P>
__global__ __launch_bounds__(kWG) void k_conflicts(Dev<P> a, const int32_t *pick, int32_t *drop) {
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i >= a.m) return;
    const int32_t e = a.row_ptr[i];
    const int32_t u = a.csr_col[e], v = a.csr_col[e + 1];
    if (pick[u] && pick[v]) { drop[u] = 1; drop[v] = 1; }
}

template <class P>
__global__ __launch_bounds__(kWG) void k_apply_drop(Dev<P> a, int32_t *sol, const int32_t *drop,
                                                    double *part) {
    const int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x;
    double v = 0.0;
    if (j < a.n) {
        const int32_t keep = sol[j] && !drop[j];
        sol[j] = keep;
        v = keep ? a.c[j] : 0.0;
    }
    v = wsum(v);
    __shared__ double sh[kWG / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int w = 1; w < kWG / 64; ++w) t += sh[w];
        part[blockIdx.x] = t;
    }
}

// Row pass of the general roundings (one thread per row, sums in entry
// order without contraction, as the scalings define them): COVER_THRESH
// min(S/f, max x) (f passed in `fx`), COVER_RAND b - S, PACK_RAND (S - b)/b,
// with S = A_j x; one partial per workgroup (min for the threshold, max
// otherwise)
template <class P>
__global__ __launch_bounds__(kWG) void k_row_scale(Dev<P> a, int32_t rule, double fx, double *part) {
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    const bool is_min = rule == THETIS_ROUND_COVER_THRESH;
    double v = is_min ? INFINITY : -INFINITY;
    if (i < a.m) {
        double sm = 0.0, mx = -INFINITY;
        for (int32_t e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e) {
            const double xv = (double)xval(a.x[a.csr_col[e]]);
            sm = __dadd_rn(sm, __dmul_rn(a.csr_val ? (double)a.csr_val[e] : 1.0, xv));
            mx = fmax(mx, xv);
        }
        if (rule == THETIS_ROUND_COVER_THRESH) v = fmin(sm / fx, mx);
        else if (rule == THETIS_ROUND_COVER_RAND) v = a.b[i] - sm;
        else v = (sm - a.b[i]) / a.b[i];
    }
    if (is_min) v = -v;
    v = wmax(v);
    __shared__ double sh[kWG / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int w = 1; w < kWG / 64; ++w) t = fmax(t, sh[w]);
        part[blockIdx.x] = is_min ? -t : t;
    }
}

// fold into the rule's scalar: COVER_THRESH T = min(1/f, min); COVER_RAND
// alpha = max(0, max)/q (0 without rows); PACK_RAND alpha = max(0, max)
__global__ __launch_bounds__(kWG) void k_row_scale_fold(const double *part, int64_t nb, int32_t rule, double fx,
                                                        double q, double *out) {
    const bool is_min = rule == THETIS_ROUND_COVER_THRESH;
    const int o[1] = {is_min ? 2 : 1};
    double r[1];
    fold_records<1>(part, nb, o, r);
    if (threadIdx.x == 0) {
        if (is_min) *out = fmin(1.0 / fx, r[0]);
        else if (rule == THETIS_ROUND_COVER_RAND) *out = isinf(q) ? 0.0 : fmax(0.0, r[0]) / q;
        else *out = fmax(0.0, r[0]);
    }
}

// Covering completion: a row whose picked sets fall short of b takes, from
// the picked set alone, its unpicked sets of positive weight in decreasing
// scaled x (ties: entry order) until it is covered; marks them in `add`.
// Every row decides from the same picked set, so the result does not depend
// on the order rows run in.
template <class P>
__global__ __launch_bounds__(kWG) void k_cover_repair(Dev<P> a, const int32_t *pick, const double *alpha,
                                                      int32_t *add) {
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i >= a.m) return;
    const int32_t e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];
    double cov = 0.0;
    for (int32_t e = e0; e < e1; ++e)
        cov = __dadd_rn(cov, __dmul_rn(a.csr_val ? (double)a.csr_val[e] : 1.0, (double)pick[a.csr_col[e]]));
    const double al = *alpha;
    double prev_x = INFINITY;
    int32_t prev_e = -1;
    while (cov < a.b[i]) {
        // next in the order (scaled x descending, entry position ascending)
        double bx = -1.0;
        int32_t be = -1;
        for (int32_t e = e0; e < e1; ++e) {
            const double av = a.csr_val ? (double)a.csr_val[e] : 1.0;
            const int32_t j = a.csr_col[e];
            if (pick[j] || av <= 0.0) continue;
            const double xt = cover_scaled((double)xval(a.x[j]), al);
            const bool after = xt < prev_x || (xt == prev_x && e > prev_e);
            if (after && xt > bx) { bx = xt; be = e; }
        }
        if (be < 0) break;
        add[a.csr_col[be]] = 1;
        cov = __dadd_rn(cov, a.csr_val ? (double)a.csr_val[be] : 1.0);
        prev_x = bx;
        prev_e = be;
    }
}

// sol |= add; cost partial
template <class P>
__global__ __launch_bounds__(kWG) void k_apply_add(Dev<P> a, int32_t *sol, const int32_t *add, double *part) {
    const int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x;
    double v = 0.0;
    if (j < a.n) {
        const int32_t keep = sol[j] || add[j];
        sol[j] = keep;
        v = keep ? a.c[j] : 0.0;
    }
    v = wsum(v);
    __shared__ double sh[kWG / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int w = 1; w < kWG / 64; ++w) t += sh[w];
        part[blockIdx.x] = t;
    }
}

// Packing alteration (Bansal et al., Appendix B) with weights w = A_js/b_j:
// a picked set is marked for deletion when, in a row where it has weight,
// the picked sets of weight >= its own (itself included) weigh more than 1
template <class P>
__global__ __launch_bounds__(kWG) void k_pack_conflicts(Dev<P> a, const int32_t *pick, int32_t *drop) {
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i >= a.m) return;
    const int32_t e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];
    const double bi = a.b[i];
    // rows of up to 16 entries: the picked entries' weights gathered once
    constexpr int kShort = 16;
    if (e1 - e0 <= kShort) {
        double w[kShort];
        int32_t col[kShort];
        bool has[kShort];
        int np = 0;
        for (int32_t e = e0; e < e1; ++e) {
            const int32_t j = a.csr_col[e];
            if (!pick[j]) continue;
            const double av = a.csr_val ? (double)a.csr_val[e] : 1.0;
            w[np] = av / bi;
            has[np] = av > 0.0;
            col[np] = j;
            ++np;
        }
        // the same sums in the same (entry) order as the general loop below
        for (int q = 0; q < np; ++q) {
            if (!has[q]) continue;
            double tot = 0.0;
            for (int q2 = 0; q2 < np; ++q2)
                if (w[q2] >= w[q]) tot = __dadd_rn(tot, w[q2]);
            if (tot > 1.0) drop[col[q]] = 1;
        }
        return;
    }
    for (int32_t e = e0; e < e1; ++e) {
        const int32_t j = a.csr_col[e];
        const double av = a.csr_val ? (double)a.csr_val[e] : 1.0;
        if (!pick[j] || av <= 0.0) continue;
        const double w = av / bi;
        double tot = 0.0;
        for (int32_t e2 = e0; e2 < e1; ++e2) {
            if (!pick[a.csr_col[e2]]) continue;
            const double w2 = (a.csr_val ? (double)a.csr_val[e2] : 1.0) / bi;
            if (w2 >= w) tot = __dadd_rn(tot, w2);
        }
        if (tot > 1.0) drop[j] = 1;
    }
}

// MAP LP, node-based roundings: a fixed block keeps its label; ARGMAX takes
// the largest marginal (first maximum), SAMPLE the first label whose running
// sum of marginals (label order, FP64) exceeds a Philox uniform, else the
// last label with positive mass
template <class P>
__global__ __launch_bounds__(kWG) void k_map_label(Dev<P> a, int32_t rule, uint64_t seed, int32_t rep,
                                                   int32_t *lab) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (t >= a.nblocks) return;
    const int32_t j0 = a.bfirst[t], k = a.k;
    int32_t l = 0;
    if (a.fixed[t] >= 0) {
        l = a.fixed[t];
    } else if (rule == THETIS_ROUND_MAP_ARGMAX) {
        double best = (double)xval(a.x[j0]);
        for (int32_t i = 1; i < k; ++i) {
            const double v = (double)xval(a.x[j0 + i]);
            if (v > best) { best = v; l = i; }
        }
    } else {
        const double u = unit53_dev(philox_word_dev(seed, RNG_ROUND, (uint64_t)rep, (uint64_t)t, 3));
        double cum = 0.0;
        int32_t got = -1, lastpos = 0;
        for (int32_t i = 0; i < k; ++i) {
            const double v = (double)xval(a.x[j0 + i]);
            if (v > 0.0) lastpos = i;
            cum = __dadd_rn(cum, v);
            if (got < 0 && u < cum) got = i;
        }
        l = got < 0 ? lastpos : got;
    }
    lab[t] = l;
}

// energy partials: block t's objective at its label, factor t's at its
// label pair (one index serves both)
template <class P>
__global__ __launch_bounds__(kWG) void k_map_energy(Dev<P> a, const int32_t *lab, const int32_t *pw_ends,
                                                    const int32_t *pw_first, int64_t npw, double *part) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    double v = 0.0;
    if (t < a.nblocks) v += a.c[a.bfirst[t] + lab[t]];
    if (t < npw)
        v += a.c[(int64_t)pw_first[t] + (int64_t)lab[pw_ends[2 * t]] * a.k + lab[pw_ends[2 * t + 1]]];
    v = wsum(v);
    __shared__ double sh[kWG / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tt = sh[0];
        for (int w = 1; w < kWG / 64; ++w) tt += sh[w];
        part[blockIdx.x] = tt;
    }
}

// region growing: block t takes the first label of the order whose entry
// reaches 1 - rad, else the last label of the order
template <class P>
__global__ __launch_bounds__(kWG) void k_ckr_label(Dev<P> a, double rad, const int32_t *order,
                                                   int32_t *lab) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (t >= a.nblocks) return;
    const int32_t j0 = a.bfirst[t], k = a.k;
    int32_t l = order[k - 1];
    for (int q = 0; q < k - 1; ++q) {
        const int32_t i = order[q];
        if ((double)xval(a.x[j0 + i]) >= 1.0 - rad) { l = i; break; }
    }
    lab[t] = l;
}

// cut cost read off the rows: a row holding two block columns of label li
// and one free column charges that column's cost when exactly one of the
// two blocks carries label li; every (edge, label) pair owns two rows
template <class P>
__global__ __launch_bounds__(kWG) void k_ckr_cost(Dev<P> a, const int32_t *lab, double *part) {
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    double v = 0.0;
    if (i < a.m) {
        int32_t zc = -1, b1 = -1, b2 = -1, li = -1;
        for (int32_t e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e) {
            const int32_t j = a.csr_col[e];
            const int32_t bl = a.col_block[j];
            if (bl < 0) zc = j;
            else if (b1 < 0) { b1 = bl; li = j - a.bfirst[bl]; }
            else b2 = bl;
        }
        if (zc >= 0 && b1 >= 0 && b2 >= 0 && ((lab[b1] == li) != (lab[b2] == li))) v = a.c[zc];
    }
    v = wsum(v);
    __shared__ double sh[kWG / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int w = 1; w < kWG / 64; ++w) t += sh[w];
        part[blockIdx.x] = t;
    }
}

// cost fold + keep-best decision: out[0] cost of this repetition, out[1]
// best cost so far, out[2] 1 when this repetition became the best, out[3]
// the best repetition (ties keep the earlier one); one workgroup
__global__ __launch_bounds__(kWG) void k_cost_fold(const double *part, int64_t nb, double scale, int32_t rep,
                                                   double *out) {
    const int o[1] = {0};
    double r[1];
    fold_records<1>(part, nb, o, r);
    if (threadIdx.x == 0) {
        const double t = r[0] * scale;
        out[0] = t;
        const int better = rep == 0 || t < out[1];
        if (better) { out[1] = t; out[3] = (double)rep; }
        out[2] = better ? 1.0 : 0.0;
    }
}

__global__ __launch_bounds__(kWG) void k_copy_if(const double *flag, const int32_t *src, int32_t *dst,
                                                 int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (j < n && flag[2] != 0.0) dst[j] = src[j];
}

// per-column integers between the internal and the caller's column order:
// out == 1 scatters to the caller's order, else gathers from it
__global__ __launch_bounds__(kWG) void k_col_map(const int32_t *src, int32_t *dst, const int32_t *col_orig,
                                                 int64_t n, int32_t out) {
    const int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (j >= n) return;
    if (out) dst[col_orig[j]] = src[j];
    else dst[j] = src[col_orig[j]];
}

// feasibility of a 0/1 solution: A sol against b, row by row
template <class P>
__global__ __launch_bounds__(kWG) void k_check_rows(Dev<P> a, const int32_t *sol, double *part) {
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    double v = 0.0;
    if (i < a.m) {
        double ax = 0.0;
        for (int32_t e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e)
            ax += (a.csr_val ? (double)a.csr_val[e] : 1.0) * (double)sol[a.csr_col[e]];
        const int8_t sn = a.sense[i];
        const bool ok = sn > 0 ? ax >= a.b[i] : (sn < 0 ? ax <= a.b[i] : ax == a.b[i]);
        v = ok ? 0.0 : 1.0;
    }
    if (i < a.n) {
        const int32_t sv = sol[i];
        if (sv != 0 && sv != 1) v += 1.0;
    }
    v = wsum(v);
    __shared__ double sh[kWG / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int w = 1; w < kWG / 64; ++w) t += sh[w];
        part[blockIdx.x] = t;
    }
}

template <class P>
__global__ __launch_bounds__(kWG) void k_check_labels(Dev<P> a, const int32_t *lab, double *part) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    double v = 0.0;
    if (t < a.nblocks) {
        const int32_t l = lab[t];
        if (l < 0 || l >= a.k) v = 1.0;
        else if (a.fixed[t] >= 0 && l != a.fixed[t]) v = 1.0;
    }
    v = wsum(v);
    __shared__ double sh[kWG / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t2 = sh[0];
        for (int w = 1; w < kWG / 64; ++w) t2 += sh[w];
        part[blockIdx.x] = t2;
    }
}

template <class P>
__global__ __launch_bounds__(kWG) void k_set_start(Dev<P> a) {
    // y = 0, fixed blocks at their unit vector; each entry is written by
    // exactly one thread
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (t < a.n) {
        const int32_t bl = a.col_block ? a.col_block[t] : -1;
        const bool one = bl >= 0 && a.fixed[bl] >= 0 && t == (int64_t)a.bfirst[bl] + a.fixed[bl];
        a.x[t] = xenc<typename P::X, float>(one ? 1.0f : 0.0f);
    }
    if (t < a.m) a.s[t] = 0;
}

// y arrives and leaves in the caller's order; row_orig[r] (col_orig[j]) is
// the caller's index of internal row r (column j)
template <class P>
__global__ __launch_bounds__(kWG) void k_load_y(Dev<P> a, const double *y, const int32_t *row_orig,
                                                const int32_t *col_orig) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    using R = typename P::R;
    if (t < a.n) {
        double v = y[col_orig[t]];
        const double U = a.ub ? (double)a.ub[t] : (double)a.ub_value;
        if (v < 0.0) v = 0.0;
        if (v > U) v = U;
        // a fixed block (a terminal, an observed variable) keeps its unit vector
        const int32_t blk = a.col_block ? a.col_block[t] : -1;
        if (blk >= 0 && a.fixed[blk] >= 0) v = (t - a.bfirst[blk] == a.fixed[blk]) ? 1.0 : 0.0;
        a.x[t] = xenc<typename P::X, double>(v);
    }
    if (t < a.m) {
        double v = y[a.n + row_orig[t]];
        if (v < 0.0 || a.sense[t] == 0) v = 0.0;
        a.s[t] = (R)v;
    }
}

template <class P>
__global__ __launch_bounds__(kWG) void k_store_y(Dev<P> a, double *x, double *s, const int32_t *row_orig,
                                                 const int32_t *col_orig) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (t < a.n) x[col_orig[t]] = (double)xval(a.x[t]);
    if (s && t < a.m) s[row_orig[t]] = (double)a.s[t];
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
constexpr int32_t kMaxReps = 64;

}  // namespace

// ==================================================================== solver

// launches of one class (DET) or one epoch part (ASYNC)
struct ClassLaunch {
    bool has_cols = false;
    int32_t group_cols = 1;                 // columns per lane group (the tuner's choice)
    LaunchPlan cols{};                      // hub + lane-group ranges (k_sweep)
    std::vector<Segment> col_segs;          // the segments that plan covers
    int64_t block_first = 0, block_count = 0, block_pb = -1;   // block_pb: first packed block (DET)
    int64_t slack_first = 0, slack_count = 0;
    double bytes_cols = 0, bytes_block = 0, bytes_slack = 0;   // algorithmic, per launch
    bool ident_rows = false;                // DET, unit values: row of entry e is e + row_off
    int64_t row_off = 0;
};

struct ClassEvent {
    int32_t cls;
    hipEvent_t e0, e1;
};

struct thetis_solver {
    // tuner: events around every class launch while set
    std::vector<ClassEvent> *class_events = nullptr;
    // host copy of what the launches need
    int64_t m = 0, n = 0, nnz = 0, nblocks = 0;
    int32_t k = 0, nclasses = 0;
    bool unit_vals = true, uniform_ub = true, all_rows_slack = true;
    double ub_value = 1.0;
    std::vector<ClassLaunch> det;              // per colour class
    ClassLaunch async_launch;                  // ASYNC: everything of one epoch
    LaunchPlan dual{};                         // column pass of the refresh, with the dual bound
    LaunchPlan colterms{};                     // column pass without it (c^T x, prox part of F)
    bool metrics_dual = false;                 // the fresh metrics include the dual bound
    bool edge_shape_cover = false, edge_shape_pack = false;
    bool sign_vals = false;                    // every matrix value +-1, not all 1 (signs packed)
    bool cover_int = false, set_cover = false, packing = false;   // shapes of the general roundings
    int64_t npw = -1;                                              // pairwise factors (MAP LP)
    double cover_q = 0.0;
    int64_t max_row_len = 0;
    int64_t nunits = 0, updates_per_epoch = 0, max_degree = 0;
    int32_t row_lanes = 1;                     // lanes per row of the row passes
    int32_t lpc = 1;                           // lanes per column of a simplex block
    bool det_ids_ident = false;                // DET plain columns: id = schedule position
    int static_dev = -1;                       // device whose static workspace this solver holds
    // parameters
    thetis_params p{};
    double rho = 0.0, Lmax = 0.0;
    // curvature factors without beta: every unit's curvature is beta * a + rho
    // (a = ||A_j||^2, the block's largest ||A_i||^2, or 1 for a slack)
    double amax = 0.0;
    std::vector<double> lb_factor;             // a per simplex block (-1 for fixed ones)
    bool has_ybar = false, has_ubar = false;
    double beta0 = 0.0;                        // beta at creation
    uint64_t inst_digest = 0;                  // the instance's digest (checkpoints)
    uint64_t layout_digest = 0;                // its internal row and column orders (checkpoints)
    bool mul_dirty = false;                    // ubar / ctil / ybar / beta moved since creation
    // device
    hipStream_t stream = nullptr;
    bool own_ws = false;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    // device pointers (typed at launch)
    void *col_ptr, *row_idx, *cval, *row_ptr, *csr_col, *csr_val, *b, *sense, *c, *ctil, *ub,
        *norm2, *ybar, *ubar, *bfirst, *fixed, *col_block, *LB, *x, *s, *r, *udual, *sched,
        *async_sched, *pk_det_ptr, *pk_det_row, *pk_det_val, *pk_async_ptr, *pk_async_row,
        *pk_async_val, *pb_id, *pb_j0, *pb_ptr, *pb_row, *pb_val, *rpart, *cpart, *metrics, *sol, *best, *drop,
        *ckr_order, *thr, *costbuf,
        *chkbuf, *mulstats, *ystage, *row_orig, *col_orig, *ctil0, *ybar0, *ubar0, *upair, *pw_ends, *pw_first;
    int64_t nwg_rows = 0, nwg_cols = 0;
    int64_t epoch = 0;
    std::atomic<int32_t> batch_slots{0};       // batch slots holding this solver (destroy refuses while > 0)
    bool metrics_fresh = false;
    double mt[MT_NSLOT] = {0};
    bool have_round = false;
    int32_t last_rule = 0;
    // timing: HIP events around every launch of every `timing`-th epoch
    int32_t timing = 0;
    bool timing_now = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    // per kernel group: (start, stop) event indices and the algorithmic
    // bytes of each timed launch
    std::vector<std::pair<int, int>> ev[THETIS_K_NKINDS];
    std::vector<double> ev_bytes[THETIS_K_NKINDS];
    double ms[THETIS_K_NKINDS] = {0}, bytes[THETIS_K_NKINDS] = {0};
    int64_t launches[THETIS_K_NKINDS] = {0};
    double refresh_bytes = 0, refresh_bytes_nodual = 0;
};

namespace {

struct Carver {
    size_t off = 0;
    char *base = nullptr;
    void *take(size_t bytes) {
        off = (off + 255) & ~size_t(255);
        void *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

size_t prec_bytes(int32_t prec) { return prec == THETIS_PREC_FP64 ? 8 : 4; }
size_t x_bytes(int32_t prec) { return prec == THETIS_PREC_FP64 ? 8 : (prec == THETIS_PREC_BF16X ? 2 : 4); }

int64_t units_per_wg(int kind) {
    if (kind == SEG_HUB) return 1;
    if (kind < kGroupKinds) return kWG / kGroupLanes[kind];
    if (kind == SEG_BLOCK) return kWG / 64;
    return kWG;
}

// workgroups of a row pass: kRowsPerThread rows per group of row_lanes lanes
int64_t row_wgs(int64_t m, int32_t lanes) {
    return cdiv(std::max<int64_t>(m, 1), (int64_t)(kWG / lanes) * kRowsPerThread);
}
int64_t row_wgs(const thetis_solver &S) { return row_wgs(S.m, S.row_lanes); }

// lanes per row for the row passes: 1 for short rows (edges), else the
// largest power of two up to half the mean row length, at most 16
int32_t choose_row_lanes(int64_t nnz, int64_t m) {
    const double len = m ? (double)nnz / (double)m : 0.0;
    if (len < 4.0) return 1;
    int32_t g = 2;
    while (g < 16 && 2.0 * g <= len / 2.0) g *= 2;
    return g;
}

// Workgroup ranges of one fused launch over the given segments (at most one
// segment per kind) plus, for the dual pass, ncolterms per-column threads.
// widen multiplies the lanes per column, cols sets the columns per lane
// group of the lane-group ranges (sweep plans only; at most 2 on 64 lanes).
// xsplit (solo sweep plans): every range is split into kXcds parts, each on
// the same number of workgroups.
LaunchPlan make_plan(const std::vector<Segment> &segs, bool dual, int64_t ncolterms, int widen = 1,
                     int cols = 1, bool xsplit = false) {
    LaunchPlan pl{};
    pl.xsplit = xsplit && !dual;
    for (int p = 0; p < kGridKinds; ++p) {
        const int kind = grid_kind(p);
        pl.lanes[p] = kind < kGroupKinds ? std::min(64, kGroupLanes[kind] * widen) : 0;
        pl.cols[p] = kind < kGroupKinds && !dual ? (pl.lanes[p] == 64 ? std::min(cols, 2) : cols) : 1;
    }
    for (const Segment &sg : segs) {
        const int p = grid_pos(sg.kind);
        pl.first[p] = sg.first;
        pl.count[p] = sg.count;
        if (!dual && sg.stride) {
            pl.ebase[p] = sg.ebase;
            pl.stride[p] = sg.stride;
        }
    }
    pl.count[kGridKinds - 1] = ncolterms;
    int64_t wg = 0;
    for (int p = 0; p < kGridKinds; ++p) {
        pl.wg_start[p] = wg;
        const int kind = grid_kind(p);
        // dual plans: kRowsPerThread units per group / wavefront / thread
        const int64_t upw = kind < kGroupKinds ? kWG / pl.lanes[p] * pl.cols[p] * (dual ? kRowsPerThread : 1)
                          : (kind == SEG_NKIND ? kWG * kRowsPerThread
                                               : units_per_wg(kind) * (dual && kind != SEG_HUB ? kRowsPerThread : 1));
        int64_t w = pl.count[p] ? cdiv(pl.count[p], upw) : 0;
        if (pl.xsplit && pl.count[p]) w = kXcds * cdiv(cdiv(pl.count[p], kXcds), upw);
        if (kind == SEG_HUB) { w = cdiv(w, 8) * 8; pl.hub_wg = w; }
        wg += w;
    }
    pl.wg_start[kGridKinds] = wg;
    pl.nwg = wg;
    return pl;
}

// carve the workspace in a fixed order; with base == nullptr it only sizes
void carve(thetis_solver &S, const Inst &in, char *base, size_t *total) {
    Carver cv;
    cv.base = base;
    const size_t R = prec_bytes(S.p.precision), X = x_bytes(S.p.precision);
    const int64_t n = in.n, m = in.m, nnz = in.nnz, nb = in.nblocks;
    S.col_ptr = cv.take(4 * (n + 1));
    S.row_idx = cv.take(4 * std::max<int64_t>(nnz, 1));
    S.cval = in.unit_vals ? nullptr : cv.take(R * nnz);
    S.norm2 = in.unit_vals ? nullptr : cv.take(R * n);
    S.row_ptr = cv.take(4 * (m + 1));
    S.csr_col = cv.take(4 * std::max<int64_t>(nnz, 1));
    S.csr_val = in.unit_vals ? nullptr : cv.take(R * nnz);
    S.b = cv.take(8 * std::max<int64_t>(m, 1));
    S.sense = cv.take(std::max<int64_t>(m, 1));
    S.c = cv.take(8 * std::max<int64_t>(n, 1));
    S.ctil = S.has_ubar ? cv.take(R * (n + m)) : nullptr;
    S.ub = in.uniform_ub ? nullptr : cv.take(R * n);
    S.ybar = S.has_ybar ? cv.take(R * (n + m)) : nullptr;
    S.ubar = S.has_ubar ? cv.take(8 * m) : nullptr;
    // the values given at creation, restored by a reset after multiplier steps
    S.ctil0 = S.has_ubar ? cv.take(R * (n + m)) : nullptr;
    S.ybar0 = S.has_ybar ? cv.take(R * (n + m)) : nullptr;
    S.ubar0 = S.has_ubar ? cv.take(8 * m) : nullptr;
    S.upair = S.has_ubar ? cv.take(16 * std::max<int64_t>(m, 1)) : nullptr;   // multiplier step's row records
    S.bfirst = nb ? cv.take(4 * nb) : nullptr;
    S.fixed = nb ? cv.take(4 * nb) : nullptr;
    S.col_block = nb ? cv.take(4 * n) : nullptr;
    S.LB = nb ? cv.take(R * nb) : nullptr;
    S.x = cv.take(X * std::max<int64_t>(n, 1));
    S.s = cv.take(R * std::max<int64_t>(m, 1));
    S.r = cv.take(R * std::max<int64_t>(m, 1));
    S.udual = cv.take(R * std::max<int64_t>(m, 1));
    S.sched = cv.take(4 * std::max<size_t>(in.sched.size(), 1));
    S.async_sched = cv.take(4 * std::max<size_t>(in.async_sched.size(), 1));
    S.pk_det_ptr = cv.take(4 * in.pk_det.ptr.size());
    S.pk_det_row = cv.take(4 * std::max<size_t>(in.pk_det.row.size(), 1));
    S.pk_det_val = in.unit_vals || in.sign_vals ? nullptr : cv.take(R * std::max<size_t>(in.pk_det.val.size(), 1));
    S.pk_async_ptr = cv.take(4 * in.pk_async.ptr.size());
    S.pk_async_row = cv.take(4 * std::max<size_t>(in.pk_async.row.size(), 1));
    S.pk_async_val = in.unit_vals ? nullptr : cv.take(R * std::max<size_t>(in.pk_async.val.size(), 1));
    S.pb_id = nb ? cv.take(4 * in.pb_det.id.size()) : nullptr;
    S.pb_j0 = nb ? cv.take(4 * in.pb_det.j0.size()) : nullptr;
    S.pb_ptr = nb ? cv.take(4 * in.pb_det.ptr.size()) : nullptr;
    S.pb_row = nb ? cv.take(4 * std::max<size_t>(in.pb_det.row.size(), 1)) : nullptr;
    S.pb_val = nb && !in.unit_vals && !in.sign_vals ? cv.take(R * std::max<size_t>(in.pb_det.val.size(), 1)) : nullptr;
    S.row_lanes = choose_row_lanes(nnz, m);
    // row-pass records (row_wgs) and the rounding's per-thread partials
    S.nwg_rows = std::max<int64_t>(std::max<int64_t>(cdiv(std::max(m, n), kWG), row_wgs(m, S.row_lanes)), 1);
    std::vector<Segment> dsegs = in.async_struct.segs;
    dsegs.insert(dsegs.end(), in.async_slack.segs.begin(), in.async_slack.segs.end());
    S.dual = make_plan(dsegs, true, n);
    S.colterms = make_plan({}, true, n);
    S.nwg_cols = std::max<int64_t>(S.dual.nwg, 1);
    S.rpart = cv.take(8 * kRowSlots * S.nwg_rows);
    S.cpart = cv.take(8 * kColSlots * S.nwg_cols);
    S.metrics = cv.take(8 * MT_NSLOT);
    const int64_t ns = std::max<int64_t>(std::max(n, nb), 1);
    S.sol = cv.take(4 * ns);
    S.best = cv.take(4 * ns);
    S.drop = cv.take(4 * ns);
    S.ckr_order = cv.take(4 * 64 * kMaxReps);
    S.thr = cv.take(8 * 4);
    S.costbuf = cv.take(8 * 4);
    S.chkbuf = cv.take(8 * 4);
    S.mulstats = cv.take(8 * 4);
    S.pw_ends = in.npw > 0 ? cv.take(8 * in.npw) : nullptr;
    S.pw_first = in.npw > 0 ? cv.take(4 * in.npw) : nullptr;
    S.ystage = cv.take(8 * std::max<int64_t>(n + m, 1));
    S.row_orig = cv.take(4 * std::max<int64_t>(m, 1));
    S.col_orig = cv.take(4 * std::max<int64_t>(n, 1));
    *total = cv.off + 256;
}

template <class P>
Dev<P> make_dev(const thetis_solver &S) {
    using R = typename P::R;
    Dev<P> a;
    a.col_ptr = (const int32_t *)S.col_ptr;
    a.row_idx = (const int32_t *)S.row_idx;
    a.cval = (const R *)S.cval;
    a.row_ptr = (const int32_t *)S.row_ptr;
    a.csr_col = (const int32_t *)S.csr_col;
    a.csr_val = (const R *)S.csr_val;
    a.b = (const double *)S.b;
    a.sense = (const int8_t *)S.sense;
    a.c = (const double *)S.c;
    a.ctil = (const R *)S.ctil;
    a.ub = (const R *)S.ub;
    a.norm2 = (const R *)S.norm2;
    a.ybar = (const R *)S.ybar;
    a.ubar = (const double *)S.ubar;
    a.bfirst = (const int32_t *)S.bfirst;
    a.fixed = (const int32_t *)S.fixed;
    a.col_block = (const int32_t *)S.col_block;
    a.LB = (const R *)S.LB;
    a.x = (typename P::X *)S.x;
    a.s = (R *)S.s;
    a.r = (R *)S.r;
    a.udual = (R *)S.udual;
    a.beta = (R)S.p.beta;
    a.rho = (R)S.rho;
    a.gamma = (R)S.p.step_scale;
    a.Lmax = (R)S.Lmax;
    a.ub_value = (R)S.ub_value;
    a.global_lmax = S.p.step_rule == THETIS_STEP_GLOBAL_LMAX;
    a.async_mode = S.p.schedule == THETIS_SCHED_ASYNC;
    a.prox_on = S.p.prox != 0;
    a.row_lanes = S.row_lanes;
    a.n = S.n;
    a.m = S.m;
    a.nblocks = S.nblocks;
    a.k = S.k;
    return a;
}

// how the DET copies store their entries (the ASYNC copy and the column copy
// keep their values): see entry_at
int32_t det_vmode(const thetis_solver &S) { return S.unit_vals ? 0 : (S.sign_vals ? 2 : 1); }

template <class P>
Sched<typename P::R> det_sched(const thetis_solver &S) {
    Sched<typename P::R> sc{(const int32_t *)S.sched, (const int32_t *)S.pk_det_ptr, (const int32_t *)S.pk_det_row,
                            (const typename P::R *)S.pk_det_val, det_vmode(S)};
    sc.ids_ident = S.det_ids_ident ? 1 : 0;
    return sc;
}
template <class P>
BlockPack<typename P::R> block_pack(const thetis_solver &S) {
    return {(const int32_t *)S.pb_id, (const int32_t *)S.pb_j0, (const int32_t *)S.pb_ptr, (const int32_t *)S.pb_row,
            (const typename P::R *)S.pb_val, det_vmode(S)};
}
template <class P>
Sched<typename P::R> async_sched(const thetis_solver &S) {
    return {(const int32_t *)S.async_sched, (const int32_t *)S.pk_async_ptr, (const int32_t *)S.pk_async_row,
            (const typename P::R *)S.pk_async_val, S.unit_vals ? 0 : 1};
}

hipEvent_t next_event(thetis_solver &S, int *idx) {
    if (S.ev_used == S.ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        S.ev_pool.push_back(e);
    }
    *idx = (int)S.ev_used;
    return S.ev_pool[S.ev_used++];
}

struct TimedScope {
    thetis_solver &S;
    int kind;
    double bytes;
    int i0 = -1;
    TimedScope(thetis_solver &s, int k, double b) : S(s), kind(k), bytes(b) {
        if (S.timing && S.timing_now) {
            hipEvent_t e = next_event(S, &i0);
            if (e) (void)hipEventRecord(e, S.stream);
        }
    }
    ~TimedScope() {
        if (i0 >= 0) {
            int i1;
            hipEvent_t e = next_event(S, &i1);
            if (e) {
                (void)hipEventRecord(e, S.stream);
                S.ev[kind].push_back({i0, i1});
                S.ev_bytes[kind].push_back(bytes);
            }
        }
    }
};

template <class P, int VM>
void launch_cols(thetis_solver &S, const Dev<P> &a, const Sched<typename P::R> &sc, const LaunchPlan &pl) {
    hipLaunchKernelGGL((k_sweep<P, VM>), dim3(pl.nwg), dim3(kWG), 0, S.stream, a, sc, pl);
}

template <class P, int VM>
void launch_blocks(thetis_solver &S, const Dev<P> &a, const int32_t *list, const BlockPack<typename P::R> &bp,
                   int64_t pb_first, int64_t count) {
    const int bpw = block_bpw(S.k);
    const int64_t grid = cdiv(count, (int64_t)bpw * (kWG / 64));
    if (bpw == 4) hipLaunchKernelGGL((k_sweep_block<P, VM, 4>), dim3(grid), dim3(kWG), 0, S.stream, a, list, bp, pb_first, count, S.lpc);
    else if (bpw == 2) hipLaunchKernelGGL((k_sweep_block<P, VM, 2>), dim3(grid), dim3(kWG), 0, S.stream, a, list, bp, pb_first, count, S.lpc);
    else hipLaunchKernelGGL((k_sweep_block<P, VM, 1>), dim3(grid), dim3(kWG), 0, S.stream, a, list, bp, pb_first, count, S.lpc);
}

// the launches of one class: plain columns (hubs + lane groups) in one
// fused launch, simplex blocks, slacks; all conflict-free among themselves
template <class P>
void launch_class(thetis_solver &S, const Dev<P> &a, const ClassLaunch &cl, const Sched<typename P::R> &sc) {
    if (cl.has_cols) {
        TimedScope ts(S, THETIS_K_SWEEP_COLUMNS, cl.bytes_cols);
        if (sc.vmode == 2) launch_cols<P, 2>(S, a, sc, cl.cols);
        else if (sc.vmode == 1) launch_cols<P, 1>(S, a, sc, cl.cols);
        else if (cl.ident_rows) {
            Sched<typename P::R> si = sc;
            si.row_off = cl.row_off;
            launch_cols<P, 3>(S, a, si, cl.cols);
        } else launch_cols<P, 0>(S, a, sc, cl.cols);
    }
    if (cl.block_count) {
        TimedScope ts(S, THETIS_K_SWEEP_BLOCK, cl.bytes_block);
        // the packed DET copy, else by id through the column copy
        const int32_t *list = cl.block_pb >= 0 ? nullptr : sc.ids + cl.block_first;
        const BlockPack<typename P::R> bp = block_pack<P>(S);
        const int vm = list ? (S.unit_vals ? 0 : 1) : bp.vmode;
        if (vm == 2) launch_blocks<P, 2>(S, a, list, bp, cl.block_pb, cl.block_count);
        else if (vm == 1) launch_blocks<P, 1>(S, a, list, bp, cl.block_pb, cl.block_count);
        else launch_blocks<P, 0>(S, a, list, bp, cl.block_pb, cl.block_count);
    }
    if (cl.slack_count) {
        TimedScope ts(S, THETIS_K_SWEEP_SLACK, cl.bytes_slack);
        const int32_t *list = S.all_rows_slack ? nullptr : sc.ids + cl.slack_first;
        hipLaunchKernelGGL((k_sweep_slack<P>), dim3(cdiv(cl.slack_count, kWG)), dim3(kWG), 0, S.stream, a, list, cl.slack_count);
    }
}

// FP64 refresh: row pass (+ new r when write_r), column pass, fold.  The
// dual bound needs a gather of the dual estimate over every column; it is
// computed only when asked for (stop test, metric queries).  Without it the
// column pass covers just c^T x and the prox part of F.
template <class P>
thetis_status refresh(thetis_solver &S, bool write_r, bool with_dual) {
    Dev<P> a = make_dev<P>(S);
    const int64_t gr = row_wgs(S);
    const LaunchPlan &pl = with_dual ? S.dual : S.colterms;
    {
        TimedScope ts(S, THETIS_K_REFRESH, with_dual ? S.refresh_bytes : S.refresh_bytes_nodual);
        hipLaunchKernelGGL((k_rows<P>), dim3(gr), dim3(kWG), 0, S.stream, a, (int32_t)write_r, (int32_t)with_dual,
                           (double *)S.rpart);
        const int32_t ident = S.all_rows_slack ? 1 : 0;
        if (pl.nwg > 0) {
            if (S.unit_vals) hipLaunchKernelGGL((k_dual<P, false>), dim3(pl.nwg), dim3(kWG), 0, S.stream, a, async_sched<P>(S), pl, ident, (double *)S.cpart);
            else hipLaunchKernelGGL((k_dual<P, true>), dim3(pl.nwg), dim3(kWG), 0, S.stream, a, async_sched<P>(S), pl, ident, (double *)S.cpart);
        }
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kWG), 0, S.stream, (const double *)S.rpart, gr,
                           (const double *)S.cpart, pl.nwg, S.p.beta, (int32_t)with_dual, (double *)S.metrics);
    }
    HIP_TRY(hipGetLastError());
    S.metrics_fresh = true;
    S.metrics_dual = with_dual;
    return THETIS_OK;
}

template <class P>
thetis_status read_metrics(thetis_solver &S) {
    if (!S.metrics_fresh || !S.metrics_dual) {
        thetis_status st = refresh<P>(S, false, true);
        if (st) return st;
    }
    HIP_TRY(hipMemcpyAsync(S.mt, S.metrics, sizeof(S.mt), hipMemcpyDeviceToHost, S.stream));
    HIP_TRY(hipStreamSynchronize(S.stream));
    S.metrics_fresh = true;
    if (S.mt[MT_BAD] != 0.0) return fail(THETIS_EDIVERGED, "NaN or Inf in the penalty reductions");
    return THETIS_OK;
}

template <class P>
thetis_status run_epochs_impl(thetis_solver &S, int32_t max_epochs, double gap_tol, int32_t *done) {
    Dev<P> a = make_dev<P>(S);
    const Sched<typename P::R> dsc = det_sched<P>(S), asc = async_sched<P>(S);
    std::vector<int32_t> order(std::max(S.nclasses, 1));
    S.ev_used = 0;
    for (int q = 0; q < THETIS_K_NKINDS; ++q) { S.ev[q].clear(); S.ev_bytes[q].clear(); }
    int32_t e = 0;
    thetis_status st = THETIS_OK;
    for (; e < max_epochs; ++e) {
        S.timing_now = S.timing > 0 && (S.epoch % S.timing) == 0;
        if (S.p.schedule == THETIS_SCHED_DET) {
            class_order(S.nclasses, S.p.seed, S.epoch, order.data());
            for (int32_t q = 0; q < S.nclasses; ++q) {
                if (S.class_events) {
                    hipEvent_t e0 = nullptr, e1 = nullptr;
                    HIP_TRY(hipEventCreate(&e0));
                    HIP_TRY(hipEventCreate(&e1));
                    HIP_TRY(hipEventRecord(e0, S.stream));
                    launch_class<P>(S, a, S.det[order[q]], dsc);
                    HIP_TRY(hipEventRecord(e1, S.stream));
                    S.class_events->push_back({order[q], e0, e1});
                } else {
                    launch_class<P>(S, a, S.det[order[q]], dsc);
                }
            }
        } else {
            launch_class<P>(S, a, S.async_launch, asc);
        }
        S.epoch++;
        S.metrics_fresh = false;
        if (S.p.refresh_every > 0 && S.epoch % S.p.refresh_every == 0) {
            S.timing_now = S.timing > 0 && (S.epoch / S.p.refresh_every) % S.timing == 0;
            st = refresh<P>(S, true, gap_tol > 0.0);
            if (st) { ++e; break; }      // the epoch itself was applied
            if (gap_tol > 0.0) {
                HIP_TRY(hipMemcpyAsync(S.mt, S.metrics, sizeof(S.mt), hipMemcpyDeviceToHost, S.stream));
                HIP_TRY(hipStreamSynchronize(S.stream));
                if (S.mt[MT_BAD] != 0.0) { ++e; st = fail(THETIS_EDIVERGED, "NaN or Inf in the refresh"); break; }
                if (S.mt[MT_GAP] <= gap_tol) { ++e; break; }
            }
        }
    }
    if (done) *done = e;
    HIP_TRY(hipGetLastError());
    if (S.timing) {
        HIP_TRY(hipStreamSynchronize(S.stream));
        for (int q = 0; q < THETIS_K_NKINDS; ++q) {
            S.ms[q] = 0;
            S.bytes[q] = 0;
            for (size_t t = 0; t < S.ev[q].size(); ++t) {
                float ms = 0;
                HIP_TRY(hipEventElapsedTime(&ms, S.ev_pool[S.ev[q][t].first], S.ev_pool[S.ev[q][t].second]));
                S.ms[q] += ms;
                S.bytes[q] += S.ev_bytes[q][t];
            }
            S.launches[q] = (int64_t)S.ev[q].size();
        }
    }
    return st;
}

thetis_status apply_beta(thetis_solver &S, double beta);

template <class P>
thetis_status reset_impl(thetis_solver &S) {
    if (S.mul_dirty) {
        const size_t R = prec_bytes(S.p.precision);
        if (S.has_ubar) {
            HIP_TRY(hipMemcpyAsync(S.ubar, S.ubar0, 8 * S.m, hipMemcpyDeviceToDevice, S.stream));
            HIP_TRY(hipMemcpyAsync(S.ctil, S.ctil0, R * (S.n + S.m), hipMemcpyDeviceToDevice, S.stream));
        }
        if (S.has_ybar) HIP_TRY(hipMemcpyAsync(S.ybar, S.ybar0, R * (S.n + S.m), hipMemcpyDeviceToDevice, S.stream));
        if (S.p.beta != S.beta0) {
            thetis_status st = apply_beta(S, S.beta0);
            if (st) return st;
        }
        S.mul_dirty = false;
    }
    Dev<P> a = make_dev<P>(S);
    const int64_t N = std::max<int64_t>(std::max(S.n, S.m), 1);
    hipLaunchKernelGGL((k_set_start<P>), dim3(cdiv(N, kWG)), dim3(kWG), 0, S.stream, a);
    S.epoch = 0;
    S.have_round = false;
    HIP_TRY(hipGetLastError());
    return refresh<P>(S, true, false);
}

// Multiplier step: row pass, column pass on the refresh's column plan, fold;
// out[0..3] as k_mul_final writes them, out[4] the device time (ms) of the
// three launches.
template <class P>
thetis_status multiplier_impl(thetis_solver &S, bool move_centre, double *out) {
    using R = typename P::R;
    Dev<P> a = make_dev<P>(S);
    R *ybar_w = move_centre ? (R *)S.ybar : nullptr;
    const int64_t gr = row_wgs(S);
    const LaunchPlan &pl = S.dual;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(THETIS_EDEVICE, "hipEventCreate failed");
    }
    (void)hipEventRecord(e0, S.stream);
    hipLaunchKernelGGL((k_mul_rows<P>), dim3(gr), dim3(kWG), 0, S.stream, a, (double *)S.ubar, (double2 *)S.upair,
                       (R *)S.ctil, ybar_w, S.p.beta, (double *)S.rpart);
    if (pl.nwg > 0) {
        if (S.unit_vals) hipLaunchKernelGGL((k_mul_cols<P, false>), dim3(pl.nwg), dim3(kWG), 0, S.stream, a, async_sched<P>(S), pl, (const double2 *)S.upair, (R *)S.ctil, ybar_w, (double *)S.cpart);
        else hipLaunchKernelGGL((k_mul_cols<P, true>), dim3(pl.nwg), dim3(kWG), 0, S.stream, a, async_sched<P>(S), pl, (const double2 *)S.upair, (R *)S.ctil, ybar_w, (double *)S.cpart);
    }
    hipLaunchKernelGGL(k_mul_final, dim3(1), dim3(kWG), 0, S.stream, (const double *)S.rpart, gr,
                       (const double *)S.cpart, pl.nwg, (double *)S.mulstats);
    (void)hipEventRecord(e1, S.stream);
    hipError_t err = hipGetLastError();
    if (err == hipSuccess) err = hipMemcpyAsync(out, S.mulstats, 4 * sizeof(double), hipMemcpyDeviceToHost, S.stream);
    if (err == hipSuccess) err = hipStreamSynchronize(S.stream);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_TRY(err);
    out[4] = ms;
    S.metrics_fresh = false;
    S.mul_dirty = true;
    return THETIS_OK;
}

// Algorithmic bytes of one multiplier step (R real, X stored x, V a matrix
// value when stored): row pass per row: pointer 4, b 8, sense 1, s R, ubar
// read and written 16, the row record {ubar, clipped ubar} 16, slack ctil R
// (+ ybar R), per entry column index 4 + V + x X; column pass per structural
// column: list entry 4, pointer 4, c 8, bound R when stored, ctil R, per
// entry row index 4 + V + the row record 16; the range over all columns:
// c 8, x X (+ block id 4, + ybar R).
double multiplier_traffic(const thetis_solver &S, bool move_centre) {
    const double R = (double)prec_bytes(S.p.precision), X = (double)x_bytes(S.p.precision);
    const double V = S.unit_vals ? 0.0 : R;
    const double m = (double)S.m, n = (double)S.n, nnz = (double)S.nnz;
    const double rows = m * (4 + 8 + 1 + R + 16 + 16 + R + (move_centre ? R : 0)) + nnz * (4 + V + X);
    const double cols = n * (4 + 4 + 8 + (S.uniform_ub ? 0 : R) + R) + nnz * (4 + V + 16);
    const double all = n * (8 + X + (S.nblocks ? 4 : 0) + (move_centre ? R : 0));
    return rows + cols + all;
}

template <class P>
thetis_status set_y_impl(thetis_solver &S, const double *y) {
    HIP_TRY(hipMemcpyAsync(S.ystage, y, 8 * (S.n + S.m), hipMemcpyHostToDevice, S.stream));
    Dev<P> a = make_dev<P>(S);
    const int64_t N = std::max<int64_t>(std::max(S.n, S.m), 1);
    hipLaunchKernelGGL((k_load_y<P>), dim3(cdiv(N, kWG)), dim3(kWG), 0, S.stream, a, (const double *)S.ystage,
                       (const int32_t *)S.row_orig, (const int32_t *)S.col_orig);
    HIP_TRY(hipGetLastError());
    thetis_status st = refresh<P>(S, true, false);
    S.have_round = false;
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(S.stream));
    return THETIS_OK;
}

template <class P>
thetis_status get_x_impl(thetis_solver &S, double *x, double *s) {
    Dev<P> a = make_dev<P>(S);
    double *dx = (double *)S.ystage, *ds = dx + S.n;
    const int64_t N = std::max<int64_t>(std::max(S.n, S.m), 1);
    hipLaunchKernelGGL((k_store_y<P>), dim3(cdiv(N, kWG)), dim3(kWG), 0, S.stream, a, dx, s ? ds : nullptr,
                       (const int32_t *)S.row_orig, (const int32_t *)S.col_orig);
    HIP_TRY(hipGetLastError());
    if (x) HIP_TRY(hipMemcpyAsync(x, dx, 8 * S.n, hipMemcpyDeviceToHost, S.stream));
    if (s) HIP_TRY(hipMemcpyAsync(s, ds, 8 * S.m, hipMemcpyDeviceToHost, S.stream));
    HIP_TRY(hipStreamSynchronize(S.stream));
    return THETIS_OK;
}

template <class P>
thetis_status round_impl(thetis_solver &S, int32_t rule, uint64_t seed, int32_t reps, int32_t *sol_host,
                         double *cost, double *aux) {
    Dev<P> a = make_dev<P>(S);
    const int64_t gm = std::max<int64_t>(cdiv(S.m, kWG), 1), gn = std::max<int64_t>(cdiv(S.n, kWG), 1);
    double *part = (double *)S.rpart;
    double *thr = (double *)S.thr, *cb = (double *)S.costbuf;
    int32_t *sol = (int32_t *)S.sol, *best = (int32_t *)S.best, *drop = (int32_t *)S.drop;
    double auxv[2] = {0, 0};
    int64_t nsol = S.n;          // a label per simplex block for the label rules (set below)
    bool per_column = true;
    if (rule == THETIS_ROUND_VC_THRESH || rule == THETIS_ROUND_MIS_THRESH) {
        if (rule == THETIS_ROUND_VC_THRESH && !S.edge_shape_cover)
            return fail(THETIS_EINVAL, "VC rounding needs rows x_u + x_v >= 1");
        if (rule == THETIS_ROUND_MIS_THRESH && !S.edge_shape_pack)
            return fail(THETIS_EINVAL, "MIS rounding needs rows x_u + x_v <= 1");
        const int32_t op = rule == THETIS_ROUND_VC_THRESH ? 0 : 1;
        hipLaunchKernelGGL((k_edge_extreme<P>), dim3(gm), dim3(kWG), 0, S.stream, a, op, part);
        hipLaunchKernelGGL(k_edge_fold, dim3(1), dim3(kWG), 0, S.stream, (const double *)part, gm, op, thr);
        hipLaunchKernelGGL((k_pick<P>), dim3(gn), dim3(kWG), 0, S.stream, a, rule, (const double *)thr, seed, 0, 0, best, part,
                           (const int32_t *)S.col_orig);
        hipLaunchKernelGGL(k_cost_fold, dim3(1), dim3(kWG), 0, S.stream, (const double *)part, gn, 1.0, 0, cb);
        HIP_TRY(hipMemcpyAsync(auxv, thr, 8, hipMemcpyDeviceToHost, S.stream));
    } else if (rule == THETIS_ROUND_MIS_RAND) {
        if (!S.edge_shape_pack) return fail(THETIS_EINVAL, "MIS rounding needs rows x_u + x_v <= 1");
        if (reps < 1) return fail(THETIS_EINVAL, "reps must be >= 1");
        hipLaunchKernelGGL((k_edge_extreme<P>), dim3(gm), dim3(kWG), 0, S.stream, a, 2, part);
        hipLaunchKernelGGL(k_edge_fold, dim3(1), dim3(kWG), 0, S.stream, (const double *)part, gm, 2, thr);
        for (int32_t rep = 0; rep < reps; ++rep) {
            HIP_TRY(hipMemsetAsync(drop, 0, 4 * S.n, S.stream));
            hipLaunchKernelGGL((k_pick<P>), dim3(gn), dim3(kWG), 0, S.stream, a, rule, (const double *)thr, seed, rep, 0, sol, part,
                               (const int32_t *)S.col_orig);
            hipLaunchKernelGGL((k_conflicts<P>), dim3(gm), dim3(kWG), 0, S.stream, a, (const int32_t *)sol, drop);
            hipLaunchKernelGGL((k_apply_drop<P>), dim3(gn), dim3(kWG), 0, S.stream, a, sol, (const int32_t *)drop, part);
            hipLaunchKernelGGL(k_cost_fold, dim3(1), dim3(kWG), 0, S.stream, (const double *)part, gn, 1.0, rep, cb);
            hipLaunchKernelGGL(k_copy_if, dim3(gn), dim3(kWG), 0, S.stream, (const double *)cb, (const int32_t *)sol, best, S.n);
        }
        HIP_TRY(hipMemcpyAsync(auxv, thr, 8, hipMemcpyDeviceToHost, S.stream));
    } else if (rule == THETIS_ROUND_COVER_THRESH) {
        if (!S.set_cover) return fail(THETIS_EINVAL, "COVER_THRESH needs set-cover rows (0/1 entries, >= 1) and binary columns");
        const double f = (double)std::max<int64_t>(S.max_row_len, 1);
        hipLaunchKernelGGL((k_row_scale<P>), dim3(gm), dim3(kWG), 0, S.stream, a, rule, f, part);
        hipLaunchKernelGGL(k_row_scale_fold, dim3(1), dim3(kWG), 0, S.stream, (const double *)part, gm, rule, f, 1.0, thr);
        hipLaunchKernelGGL((k_pick<P>), dim3(gn), dim3(kWG), 0, S.stream, a, rule, (const double *)thr, seed, 0, 0, best, part,
                           (const int32_t *)S.col_orig);
        hipLaunchKernelGGL(k_cost_fold, dim3(1), dim3(kWG), 0, S.stream, (const double *)part, gn, 1.0, 0, cb);
        HIP_TRY(hipMemcpyAsync(auxv, thr, 8, hipMemcpyDeviceToHost, S.stream));
    } else if (rule == THETIS_ROUND_COVER_RAND || rule == THETIS_ROUND_PACK_RAND) {
        const bool cover = rule == THETIS_ROUND_COVER_RAND;
        if (cover && !S.cover_int)
            return fail(THETIS_EINVAL, "COVER_RAND needs rows >= with non-negative integer entries and b, and binary columns");
        if (!cover && !S.packing)
            return fail(THETIS_EINVAL, "PACK_RAND needs rows <= with non-negative entries and b > 0, and binary columns");
        if (reps < 1) return fail(THETIS_EINVAL, "reps must be >= 1");
        // independent rounds whose union is kept: ceil(ln(2m)), so that a
        // row stays uncovered with probability at most 1/(2m)
        int32_t rounds = 0;
        if (cover) rounds = std::max<int32_t>(1, S.m > 0 ? (int32_t)std::ceil(std::log(2.0 * (double)S.m)) : 1);
        hipLaunchKernelGGL((k_row_scale<P>), dim3(gm), dim3(kWG), 0, S.stream, a, rule, 1.0, part);
        hipLaunchKernelGGL(k_row_scale_fold, dim3(1), dim3(kWG), 0, S.stream, (const double *)part, gm, rule, 1.0,
                           S.cover_q, thr);
        for (int32_t rep = 0; rep < reps; ++rep) {
            HIP_TRY(hipMemsetAsync(drop, 0, 4 * S.n, S.stream));
            hipLaunchKernelGGL((k_pick<P>), dim3(gn), dim3(kWG), 0, S.stream, a, rule, (const double *)thr, seed, rep,
                               rounds, sol, part, (const int32_t *)S.col_orig);
            if (cover) {
                hipLaunchKernelGGL((k_cover_repair<P>), dim3(gm), dim3(kWG), 0, S.stream, a, (const int32_t *)sol,
                                   (const double *)thr, drop);
                hipLaunchKernelGGL((k_apply_add<P>), dim3(gn), dim3(kWG), 0, S.stream, a, sol, (const int32_t *)drop, part);
            } else {
                hipLaunchKernelGGL((k_pack_conflicts<P>), dim3(gm), dim3(kWG), 0, S.stream, a, (const int32_t *)sol, drop);
                hipLaunchKernelGGL((k_apply_drop<P>), dim3(gn), dim3(kWG), 0, S.stream, a, sol, (const int32_t *)drop, part);
            }
            hipLaunchKernelGGL(k_cost_fold, dim3(1), dim3(kWG), 0, S.stream, (const double *)part, gn, 1.0, rep, cb);
            hipLaunchKernelGGL(k_copy_if, dim3(gn), dim3(kWG), 0, S.stream, (const double *)cb, (const int32_t *)sol, best, S.n);
        }
        HIP_TRY(hipMemcpyAsync(auxv, thr, 8, hipMemcpyDeviceToHost, S.stream));
    } else if (rule == THETIS_ROUND_MAP_ARGMAX || rule == THETIS_ROUND_MAP_SAMPLE) {
        if (S.nblocks <= 0 || S.npw < 0) return fail(THETIS_EINVAL, "MAP rounding needs simplex blocks and pairwise factors");
        const int32_t nrep = rule == THETIS_ROUND_MAP_ARGMAX ? 1 : reps;
        if (nrep < 1) return fail(THETIS_EINVAL, "reps must be >= 1");
        nsol = S.nblocks;
        per_column = false;
        const int64_t gb = std::max<int64_t>(cdiv(S.nblocks, kWG), 1);
        const int64_t ge = std::max<int64_t>(cdiv(std::max(S.nblocks, S.npw), kWG), 1);
        for (int32_t rep = 0; rep < nrep; ++rep) {
            hipLaunchKernelGGL((k_map_label<P>), dim3(gb), dim3(kWG), 0, S.stream, a, rule, seed, rep, sol);
            hipLaunchKernelGGL((k_map_energy<P>), dim3(ge), dim3(kWG), 0, S.stream, a, (const int32_t *)sol,
                               (const int32_t *)S.pw_ends, (const int32_t *)S.pw_first, S.npw, part);
            hipLaunchKernelGGL(k_cost_fold, dim3(1), dim3(kWG), 0, S.stream, (const double *)part, ge, 1.0, rep, cb);
            hipLaunchKernelGGL(k_copy_if, dim3(gb), dim3(kWG), 0, S.stream, (const double *)cb, (const int32_t *)sol, best, S.nblocks);
        }
    } else if (rule == THETIS_ROUND_MC_CKR) {
        if (S.nblocks <= 0) return fail(THETIS_EINVAL, "MC rounding needs simplex blocks");
        if (reps < 1 || reps > kMaxReps) return fail(THETIS_EINVAL, "reps must be in [1, 64]");
        nsol = S.nblocks;
        per_column = false;
        const int64_t gb = std::max<int64_t>(cdiv(S.nblocks, kWG), 1);
        std::vector<int32_t> orders(64 * (size_t)reps);  // one label order per repetition
        std::vector<double> rads(reps);
        for (int32_t rep = 0; rep < reps; ++rep) {
            rads[rep] = unit53(philox_word_host(seed, RNG_ROUND, (uint64_t)rep, 0, 1));
            std::vector<std::pair<uint64_t, int32_t>> ks(S.k);
            for (int32_t i = 0; i < S.k; ++i) ks[i] = {philox_word_host(seed, RNG_ROUND, (uint64_t)rep, (uint64_t)i, 2), i};
            std::sort(ks.begin(), ks.end());
            for (int32_t i = 0; i < S.k; ++i) orders[64 * (size_t)rep + i] = ks[i].second;
        }
        HIP_TRY(hipMemcpyAsync(S.ckr_order, orders.data(), 4 * orders.size(), hipMemcpyHostToDevice, S.stream));
        for (int32_t rep = 0; rep < reps; ++rep) {
            hipLaunchKernelGGL((k_ckr_label<P>), dim3(gb), dim3(kWG), 0, S.stream, a, rads[rep],
                               (const int32_t *)S.ckr_order + 64 * (size_t)rep, sol);
            hipLaunchKernelGGL((k_ckr_cost<P>), dim3(gm), dim3(kWG), 0, S.stream, a, (const int32_t *)sol, part);
            hipLaunchKernelGGL(k_cost_fold, dim3(1), dim3(kWG), 0, S.stream, (const double *)part, gm, 0.5, rep, cb);
            hipLaunchKernelGGL(k_copy_if, dim3(gb), dim3(kWG), 0, S.stream, (const double *)cb, (const int32_t *)sol, best, S.nblocks);
        }
        auxv[0] = -1.0;   // radius of the winning repetition, filled below
    } else {
        return fail(THETIS_EINVAL, "unknown rounding rule");
    }
    HIP_TRY(hipGetLastError());
    double cbh[4];
    HIP_TRY(hipMemcpyAsync(cbh, cb, 32, hipMemcpyDeviceToHost, S.stream));
    if (sol_host) {
        const int32_t *src = best;
        if (per_column && S.n) {
            // one entry per column: back to the caller's column order
            int32_t *stage = (int32_t *)S.ystage;
            hipLaunchKernelGGL(k_col_map, dim3(gn), dim3(kWG), 0, S.stream, (const int32_t *)best, stage,
                               (const int32_t *)S.col_orig, S.n, 1);
            HIP_TRY(hipGetLastError());
            src = stage;
        }
        HIP_TRY(hipMemcpyAsync(sol_host, src, 4 * nsol, hipMemcpyDeviceToHost, S.stream));
    }
    HIP_TRY(hipStreamSynchronize(S.stream));
    if (cost) *cost = cbh[1];
    auxv[1] = cbh[3];
    if (rule == THETIS_ROUND_MC_CKR)
        auxv[0] = unit53(philox_word_host(seed, RNG_ROUND, (uint64_t)cbh[3], 0, 1));
    if (aux) { aux[0] = auxv[0]; aux[1] = auxv[1]; }
    S.have_round = true;
    S.last_rule = rule;
    return THETIS_OK;
}

template <class P>
thetis_status check_impl(thetis_solver &S, int32_t rule, const int32_t *sol_host, int32_t *feasible,
                         int64_t *nviol) {
    Dev<P> a = make_dev<P>(S);
    const int32_t *sol = (const int32_t *)S.best;
    const bool labels = rule == THETIS_ROUND_MC_CKR || rule == THETIS_ROUND_MAP_ARGMAX || rule == THETIS_ROUND_MAP_SAMPLE;
    if (labels && S.nblocks <= 0) return fail(THETIS_EINVAL, "label check needs simplex blocks");
    if (!labels && (rule < THETIS_ROUND_VC_THRESH || rule > THETIS_ROUND_PACK_RAND))
        return fail(THETIS_EINVAL, "unknown rule");
    const int64_t nsol = labels ? S.nblocks : S.n;
    if (sol_host) {
        if (labels) {
            HIP_TRY(hipMemcpyAsync(S.drop, sol_host, 4 * nsol, hipMemcpyHostToDevice, S.stream));
        } else if (nsol) {
            // one entry per column, in the caller's order: into the internal one
            int32_t *stage = (int32_t *)S.ystage;
            HIP_TRY(hipMemcpyAsync(stage, sol_host, 4 * nsol, hipMemcpyHostToDevice, S.stream));
            hipLaunchKernelGGL(k_col_map, dim3(cdiv(nsol, kWG)), dim3(kWG), 0, S.stream, (const int32_t *)stage,
                               (int32_t *)S.drop, (const int32_t *)S.col_orig, nsol, 0);
            HIP_TRY(hipGetLastError());
        }
        sol = (const int32_t *)S.drop;
    } else if (!S.have_round) {
        return fail(THETIS_EINVAL, "no rounded solution on the device");
    }
    double *part = (double *)S.rpart;
    int64_t g;
    if (labels) {
        g = std::max<int64_t>(cdiv(S.nblocks, kWG), 1);
        hipLaunchKernelGGL((k_check_labels<P>), dim3(g), dim3(kWG), 0, S.stream, a, sol, part);
    } else {
        g = std::max<int64_t>(cdiv(std::max(S.m, S.n), kWG), 1);
        hipLaunchKernelGGL((k_check_rows<P>), dim3(g), dim3(kWG), 0, S.stream, a, sol, part);
    }
    double *cb = (double *)S.chkbuf;
    hipLaunchKernelGGL(k_cost_fold, dim3(1), dim3(kWG), 0, S.stream, (const double *)part, g, 1.0, 0, cb);
    HIP_TRY(hipGetLastError());
    double h[4];
    HIP_TRY(hipMemcpyAsync(h, cb, 32, hipMemcpyDeviceToHost, S.stream));
    HIP_TRY(hipStreamSynchronize(S.stream));
    const int64_t bad = (int64_t)h[0];
    if (nviol) *nviol = bad;
    if (feasible) *feasible = bad == 0;
    return THETIS_OK;
}

#define DISPATCH(S, CALL)                                                       \
    ((S).p.precision == THETIS_PREC_FP64 ? CALL<PF64> : ((S).p.precision == THETIS_PREC_BF16X ? CALL<PB16> : CALL<PF32>))

bool edge_shape(const Inst &in, int8_t want) {
    if (in.m == 0) return false;
    for (int64_t i = 0; i < in.m; ++i) {
        if (in.row_ptr[i + 1] - in.row_ptr[i] != 2) return false;
        if (in.sense[i] != want || in.b[i] != 1.0) return false;
        if (!in.unit_vals) {
            if (in.val[in.row_ptr[i]] != 1.0 || in.val[in.row_ptr[i] + 1] != 1.0) return false;
        }
    }
    return true;
}

// curvature of every unit and the largest one (eq. Lmax with the prox
// weight rho in place of 1/beta)
void compute_curvatures(thetis_solver &S, const Inst &in, std::vector<double> &norm2, std::vector<double> &LB) {
    norm2.assign(in.n, 0.0);
    for (int64_t j = 0; j < in.n; ++j) {
        double a2 = 0.0;
        for (int32_t e = in.col_ptr[j]; e < in.col_ptr[j + 1]; ++e) {
            const double v = in.unit_vals ? 1.0 : in.cval[e];
            a2 += v * v;
        }
        norm2[j] = a2;
    }
    LB.assign(in.nblocks, 0.0);
    S.lb_factor.assign(in.nblocks, -1.0);
    double amax = 0.0;
    // the columns of a block share no row (checked when the blocks are
    // declared), so the block of A^T A is diag(||A_i||^2): its largest entry
    // is the Lipschitz constant of the block gradient (Appendix E), and the
    // block step is the exact block minimiser when the entries are equal
    // (the multiway-cut and MAP blocks)
    for (int64_t t = 0; t < in.nblocks; ++t) {
        if (in.fixed[t] >= 0) continue;
        double best = 0.0;
        for (int32_t i = 0; i < in.k; ++i) best = std::max(best, norm2[in.bfirst[t] + i]);
        S.lb_factor[t] = best;
        LB[t] = S.p.beta * best + S.rho;
        amax = std::max(amax, best);
    }
    for (int64_t j = 0; j < in.n; ++j) {
        if (in.nblocks && in.col_block[j] >= 0) continue;
        amax = std::max(amax, norm2[j]);
    }
    for (int64_t i = 0; i < in.m; ++i)
        if (in.sense[i] != 0) amax = std::max(amax, 1.0);
    S.amax = amax;
    // beta * a + rho is monotone in a (also after rounding): the largest
    // curvature is the one of the largest factor
    S.Lmax = in.nunits ? S.p.beta * amax + S.rho : 0.0;
}

template <class T>
thetis_status upload(thetis_solver &S, void *dst, const std::vector<T> &src) {
    if (src.empty() || !dst) return THETIS_OK;
    HIP_TRY(hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, S.stream));
    return THETIS_OK;
}

template <class R>
thetis_status upload_conv(thetis_solver &S, void *dst, const std::vector<double> &src) {
    if (src.empty() || !dst) return THETIS_OK;
    std::vector<R> tmp(src.begin(), src.end());
    HIP_TRY(hipMemcpyAsync(dst, tmp.data(), sizeof(R) * tmp.size(), hipMemcpyHostToDevice, S.stream));
    HIP_TRY(hipStreamSynchronize(S.stream));
    return THETIS_OK;
}

thetis_status hip_status(hipError_t e) {
    if (e == hipSuccess) return THETIS_OK;
    return fail(THETIS_EDEVICE, std::string("HIP: ") + hipGetErrorString(e));
}

thetis_status upload_real(thetis_solver &S, void *dst, const std::vector<double> &src) {
    return S.p.precision == THETIS_PREC_FP64 ? upload_conv<double>(S, dst, src) : upload_conv<float>(S, dst, src);
}

// Algorithmic bytes of one launch of a segment (R = bytes of a stored real,
// X = bytes of a stored x).  Plain column j with d entries: list entry 4,
// packed pointers 8, per entry row index 4 + residual read R + write R
// (+ value R), x read and write 2X, cost 8 (FP64 c; R when shifted by ubar)
// (+ bound R, + ||A_j||^2 R when not implied, + prox centre R).  Simplex
// block: the same per column plus the block's first column and curvature.
// Slack: s and r read and written (+ row list 4 when not every row has one).
double segment_bytes(const thetis_solver &S, const Inst &in, const std::vector<int32_t> &sched,
                     const Segment &sg) {
    const double R = (double)prec_bytes(S.p.precision);
    const double X = (double)x_bytes(S.p.precision);
    // the DET copies of a +-1 matrix carry the signs in the row indices
    // (no value, no stored ||A_j||^2)
    const bool noval = in.unit_vals || (in.sign_vals && &sched == &in.sched);
    const double V = noval ? 0.0 : R;
    const double per_col = 8 + 2 * X + (S.has_ubar ? R : 8.0) + (in.uniform_ub ? 0 : R) +
                           (noval ? 0 : R) + (S.has_ybar ? R : 0);
    double b = 0.0;
    if (sg.kind == SEG_SLACK) return (double)sg.count * (4 * R + (in.all_rows_slack ? 0.0 : 4.0));
    for (int64_t q = 0; q < sg.count; ++q) {
        const int32_t id = sched[sg.first + q];
        b += 4;
        if (sg.kind == SEG_BLOCK) {
            b += 4 + R;
            for (int32_t i = 0; i < in.k; ++i) {
                const int32_t j = in.bfirst[id] + i;
                const double d = in.col_ptr[j + 1] - in.col_ptr[j];
                b += per_col + d * (4 + 2 * R + V);
            }
        } else {
            const double d = in.col_ptr[id + 1] - in.col_ptr[id];
            b += per_col + d * (4 + 2 * R + V);
        }
    }
    return b;
}

// pk: the packed DET copy when the class is one of the DET schedule's (its
// entries are then checked for consecutive rows), else null
ClassLaunch make_class_launch(const thetis_solver &S, const Inst &in, const std::vector<int32_t> &sched,
                              const std::vector<Segment> &segs, const Packed *pk) {
    ClassLaunch cl;
    std::vector<Segment> cols;
    for (const Segment &sg : segs) {
        const double b = segment_bytes(S, in, sched, sg);
        if (sg.kind == SEG_BLOCK) {
            cl.block_first = sg.first; cl.block_count = sg.count; cl.block_pb = sg.pb_first; cl.bytes_block = b;
        }
        else if (sg.kind == SEG_SLACK) { cl.slack_first = sg.first; cl.slack_count = sg.count; cl.bytes_slack = b; }
        else { cols.push_back(sg); cl.bytes_cols += b; }
    }
    if (!cols.empty()) {
        cl.has_cols = true;
        cl.cols = make_plan(cols, false, 0, 1, 1, true);
        cl.col_segs = cols;
    }
    if (pk && cl.has_cols && det_vmode(S) == 0) {
        bool ident = true, any = false;
        int64_t off = 0;
        for (const Segment &sg : cols)
            for (int64_t q = sg.first; q < sg.first + sg.count && ident; ++q)
                for (int64_t e = pk->ptr[q]; e < pk->ptr[q + 1] && ident; ++e) {
                    if (!any) { off = (int64_t)pk->row[e] - e; any = true; }
                    ident = (int64_t)pk->row[e] == e + off;
                }
        cl.ident_rows = ident && any;
        cl.row_off = cl.ident_rows ? off : 0;
    }
    return cl;
}

// one refresh: row pass (row pointers, indices, x gathered, s, b, sense, r
// written, and the dual estimate written when the bound is wanted) and
// column pass (c and x; with the bound also the packed pointers, indices,
// dual estimate gathered, and s and sense of the slacks)
double refresh_traffic(const thetis_solver &S, bool with_dual) {
    const double R = (double)prec_bytes(S.p.precision);
    const double V = S.unit_vals ? 0.0 : R;
    const double rows = 4.0 * (S.m + 1) + S.nnz * (4 + R + V) + S.m * (R + 8 + 1 + R + (with_dual ? R : 0));
    double cols = S.n * (8 + R);
    if (with_dual) cols += 4.0 * (S.n + 1) + S.nnz * (4 + R + V) + S.m * (1 + 2 * R);
    return rows + cols;
}

thetis_status check_params(const thetis_params *p) {
    if (!p) return fail(THETIS_EINVAL, "params is NULL");
    if (!(p->beta > 0.0) || !std::isfinite(p->beta)) return fail(THETIS_EINVAL, "beta must be positive and finite");
    if (p->step_rule != THETIS_STEP_PER_COORD && p->step_rule != THETIS_STEP_GLOBAL_LMAX)
        return fail(THETIS_EINVAL, "unknown step rule");
    if (!(p->step_scale > 0.0 && p->step_scale <= 1.0)) return fail(THETIS_EINVAL, "step_scale must be in (0, 1]");
    if (p->schedule != THETIS_SCHED_DET && p->schedule != THETIS_SCHED_ASYNC)
        return fail(THETIS_EINVAL, "unknown schedule");
    if (p->precision != THETIS_PREC_FP32 && p->precision != THETIS_PREC_FP64 && p->precision != THETIS_PREC_BF16X)
        return fail(THETIS_EINVAL, "unknown precision");
    if (p->refresh_every < 1) return fail(THETIS_EINVAL, "refresh_every must be >= 1");
    return THETIS_OK;
}

}  // namespace

// ==================================================================== C ABI

extern "C" thetis_status thetis_solver_workspace_bytes(const thetis_inst *h, const thetis_params *p,
                                                       size_t *bytes) {
    try {
        clear_error();
        if (!h || !bytes) return fail(THETIS_EINVAL, "NULL argument");
        thetis_status st = check_params(p);
        if (st) return st;
        st = ensure_layout(h);
        if (st) return st;
        thetis_solver S;
        S.p = *p;
        S.has_ybar = p->prox && p->ybar;
        S.has_ubar = p->ubar != nullptr;
        carve(S, h->in, nullptr, bytes);
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

// The workspace of thetis_solver_create_static: a file-scope device array
// (a copy on every device the library runs on, for the life of the
// process).  Host code never passes `scratch` itself to a kernel or a copy:
// it takes the device's address of it once per device with
// hipGetSymbolAddress and uses that.
static __device__ __align__(256) char scratch[THETIS_STATIC_WORKSPACE_BYTES];

namespace {
struct StaticWorkspace {
    void *ptr = nullptr;               // this device's address of `scratch`
    const thetis_solver *holder = nullptr;
};
std::mutex g_static_mu;
std::vector<StaticWorkspace> g_static;   // by device ordinal

// the device's address of `scratch` (the device must be current), resolved
// on the first use on that device
thetis_status static_workspace(int dev, void **ptr) {
    if ((size_t)dev >= g_static.size()) g_static.resize((size_t)dev + 1);
    StaticWorkspace &w = g_static[(size_t)dev];
    if (!w.ptr) {
        void *q = nullptr;
        const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !q) {
            (void)hipGetLastError();
            return fail(THETIS_EDEVICE, std::string("hipGetSymbolAddress of the static workspace failed: ") +
                                            hipGetErrorString(e));
        }
        w.ptr = q;
    }
    *ptr = w.ptr;
    return THETIS_OK;
}

// a solver made on the static workspace gives it back when destroyed
void release_static(const thetis_solver *s) {
    if (s->static_dev < 0) return;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if ((size_t)s->static_dev < g_static.size() && g_static[(size_t)s->static_dev].holder == s)
        g_static[(size_t)s->static_dev].holder = nullptr;
}
}  // namespace

extern "C" thetis_status thetis_solver_create(const thetis_inst *h, const thetis_params *p,
                                              void *dev_workspace, size_t ws_bytes, void *stream,
                                              thetis_solver **out) {
    thetis_solver *Sp = nullptr;   // released by the handler below if the host side throws
    try {
        clear_error();
        if (!h || !out) return fail(THETIS_EINVAL, "NULL argument");
        *out = nullptr;
        thetis_status st = check_params(p);
        if (st) return st;
        st = ensure_layout(h);
        if (st) return st;
        const Inst &in = h->in;
        Sp = new (std::nothrow) thetis_solver;
        if (!Sp) return fail(THETIS_ENOMEM, "host allocation failed");
        thetis_solver &S = *Sp;
        S.p = *p;
        S.p.ybar = nullptr;
        S.p.ubar = nullptr;
        S.beta0 = p->beta;
        S.rho = p->prox ? 1.0 / p->beta : 0.0;
        S.has_ybar = p->prox && p->ybar;
        S.has_ubar = p->ubar != nullptr;
        S.m = in.m; S.n = in.n; S.nnz = in.nnz; S.nblocks = in.nblocks; S.k = in.k;
        S.nclasses = in.nclasses; S.nunits = in.nunits;
        S.unit_vals = in.unit_vals; S.uniform_ub = in.uniform_ub; S.ub_value = in.ub_value;
        S.all_rows_slack = in.all_rows_slack;
        while (S.lpc * 2 * std::max(S.k, 1) * block_bpw(S.k) <= 64) S.lpc *= 2;
        S.max_degree = in.max_col_degree;
        S.edge_shape_cover = edge_shape(in, 1);
        S.edge_shape_pack = edge_shape(in, -1);
        S.sign_vals = in.sign_vals;
        S.cover_int = in.cover_int;
        S.set_cover = in.set_cover;
        S.packing = in.packing;
        S.cover_q = in.cover_q;
        S.inst_digest = in.digest;
        S.layout_digest = layout_digest(in);
        S.max_row_len = in.max_row_len;
        S.npw = in.npw;
        for (const ClassPlan &cp : in.classes) S.det.push_back(make_class_launch(S, in, in.sched, cp.segs, &in.pk_det));
        // columns laid out in plan order: a plain column's id is its position
        S.det_ids_ident = true;
        for (const ClassPlan &cp : in.classes)
            for (const Segment &sg : cp.segs)
                if (sg.kind < kGroupKinds || sg.kind == SEG_HUB)
                    for (int64_t q = sg.first; q < sg.first + sg.count && S.det_ids_ident; ++q)
                        S.det_ids_ident = in.sched[q] == q;
        {
            std::vector<Segment> all = in.async_struct.segs;
            all.insert(all.end(), in.async_slack.segs.begin(), in.async_slack.segs.end());
            S.async_launch = make_class_launch(S, in, in.async_sched, all, nullptr);
        }
        S.updates_per_epoch = 0;
        for (const ClassPlan &cp : in.classes)
            for (const Segment &sg : cp.segs) S.updates_per_epoch += sg.kind == SEG_BLOCK ? sg.count * in.k : sg.count;
        S.refresh_bytes = refresh_traffic(S, true);
        S.refresh_bytes_nodual = refresh_traffic(S, false);
        S.stream = (hipStream_t)stream;
        size_t need = 0;
        carve(S, in, nullptr, &need);
        if (dev_workspace) {
            if (ws_bytes < need) { delete Sp; return fail(THETIS_ENOMEM, "workspace smaller than thetis_solver_workspace_bytes"); }
            S.ws = (char *)dev_workspace;
            S.ws_bytes = ws_bytes;
        } else {
            if (hipMalloc(&S.ws, need) != hipSuccess) { delete Sp; (void)hipGetLastError(); return fail(THETIS_ENOMEM, "hipMalloc of the workspace failed"); }
            S.own_ws = true;
            S.ws_bytes = need;
        }
        char *base = (char *)(((uintptr_t)S.ws + 255) & ~uintptr_t(255));
        size_t dummy;
        carve(S, in, base, &dummy);
        std::vector<double> norm2, LB;
        compute_curvatures(S, in, norm2, LB);
#define UP(expr) do { thetis_status s_ = (expr); if (s_) { thetis_solver_destroy(Sp); return s_; } } while (0)
        UP(upload(S, S.col_ptr, in.col_ptr));
        UP(upload(S, S.row_idx, in.row_idx));
        UP(upload(S, S.row_ptr, in.row_ptr));
        UP(upload(S, S.csr_col, in.col_idx));
        UP(upload(S, S.b, in.b));
        UP(upload(S, S.sense, in.sense));
        UP(upload(S, S.c, in.c));
        UP(upload(S, S.row_orig, in.row_orig));
        UP(upload(S, S.col_orig, in.col_orig));
        if (in.npw > 0) {
            UP(upload(S, S.pw_ends, in.pw_ends));
            UP(upload(S, S.pw_first, in.pw_first));
        }
        UP(upload(S, S.sched, in.sched));
        UP(upload(S, S.async_sched, in.async_sched));
        UP(upload(S, S.pk_det_ptr, in.pk_det.ptr));
        UP(upload(S, S.pk_det_row, in.pk_det.row));
        UP(upload(S, S.pk_async_ptr, in.pk_async.ptr));
        UP(upload(S, S.pk_async_row, in.pk_async.row));
        if (!in.unit_vals) {
            UP(upload_real(S, S.cval, in.cval));
            UP(upload_real(S, S.csr_val, in.val));
            UP(upload_real(S, S.norm2, norm2));
            UP(upload_real(S, S.pk_det_val, in.pk_det.val));
            UP(upload_real(S, S.pk_async_val, in.pk_async.val));
        }
        if (!in.uniform_ub) UP(upload_real(S, S.ub, in.u));
        if (in.nblocks) {
            UP(upload(S, S.bfirst, in.bfirst));
            UP(upload(S, S.pb_id, in.pb_det.id));
            UP(upload(S, S.pb_j0, in.pb_det.j0));
            UP(upload(S, S.pb_ptr, in.pb_det.ptr));
            UP(upload(S, S.pb_row, in.pb_det.row));
            if (!in.unit_vals) UP(upload_real(S, S.pb_val, in.pb_det.val));
            UP(upload(S, S.fixed, in.fixed));
            UP(upload(S, S.col_block, in.col_block));
            UP(upload_real(S, S.LB, LB));
        }
        if (S.has_ybar) {
            // the slack part of ybar follows the internal row order
            std::vector<double> yb(in.n + in.m);
            for (int64_t j = 0; j < in.n; ++j) yb[j] = p->ybar[in.col_orig[j]];
            for (int64_t r = 0; r < in.m; ++r) yb[in.n + r] = p->ybar[in.n + in.row_orig[r]];
            UP(upload_real(S, S.ybar, yb));
            UP(hip_status(hipMemcpyAsync(S.ybar0, S.ybar, prec_bytes(S.p.precision) * (in.n + in.m),
                                         hipMemcpyDeviceToDevice, S.stream)));
        }
        if (S.has_ubar) {
            std::vector<double> ub(in.m);
            for (int64_t r = 0; r < in.m; ++r) ub[r] = p->ubar[in.row_orig[r]];
            UP(upload(S, S.ubar, ub));
            // ctil = c - A^T ubar over the structural columns, -sign * ubar_i for slacks
            std::vector<double> ct(in.n + in.m, 0.0);
            for (int64_t j = 0; j < in.n; ++j) {
                double acc = 0.0;
                for (int32_t e = in.col_ptr[j]; e < in.col_ptr[j + 1]; ++e)
                    acc += (in.unit_vals ? 1.0 : in.cval[e]) * ub[in.row_idx[e]];
                ct[j] = in.c[j] - acc;
            }
            for (int64_t i = 0; i < in.m; ++i) {
                const double sg = in.sense[i] > 0 ? -1.0 : (in.sense[i] < 0 ? 1.0 : 0.0);
                ct[in.n + i] = -sg * ub[i];
            }
            UP(upload_real(S, S.ctil, ct));
            UP(hip_status(hipMemcpyAsync(S.ctil0, S.ctil, prec_bytes(S.p.precision) * (in.n + in.m),
                                         hipMemcpyDeviceToDevice, S.stream)));
            UP(hip_status(hipMemcpyAsync(S.ubar0, S.ubar, 8 * in.m, hipMemcpyDeviceToDevice, S.stream)));
        }
        const_cast<thetis_inst *>(h)->in.has_solver = true;
        st = DISPATCH(S, reset_impl)(S);
        if (st) { thetis_solver_destroy(Sp); return st; }
        if (hipStreamSynchronize(S.stream) != hipSuccess) {
            thetis_solver_destroy(Sp);
            return fail(THETIS_EDEVICE, "device error while creating the solver");
        }
#undef UP
        *out = Sp;
        return THETIS_OK;
    } catch (...) {
        const thetis_status st = exception_status();
        if (Sp) thetis_solver_destroy(Sp);
        return st;
    }
}

extern "C" thetis_status thetis_solver_create_static(const thetis_inst *h, const thetis_params *p, void *stream,
                                                     thetis_solver **out) {
    try {
        clear_error();
        if (!h || !out) return fail(THETIS_EINVAL, "NULL argument");
        *out = nullptr;
        size_t need = 0;
        thetis_status st = thetis_solver_workspace_bytes(h, p, &need);
        if (st) return st;
        if (need > THETIS_STATIC_WORKSPACE_BYTES)
            return fail(THETIS_EBUDGET, "the instance needs " + std::to_string(need) +
                                            " workspace bytes; the static workspace holds " +
                                            std::to_string(THETIS_STATIC_WORKSPACE_BYTES));
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) {
            (void)hipGetLastError();
            return fail(THETIS_EDEVICE, "no current HIP device");
        }
        std::lock_guard<std::mutex> lock(g_static_mu);
        void *ws = nullptr;
        st = static_workspace(dev, &ws);
        if (st) return st;
        if (g_static[(size_t)dev].holder)
            return fail(THETIS_EBUSY, "a solver made by thetis_solver_create_static still lives on this device");
        thetis_solver *s = nullptr;
        st = thetis_solver_create(h, p, ws, THETIS_STATIC_WORKSPACE_BYTES, stream, &s);
        if (st) return st;
        s->static_dev = dev;
        g_static[(size_t)dev].holder = s;
        *out = s;
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_solver_reset(thetis_solver *s) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        return DISPATCH(*s, reset_impl)(*s);
    } catch (...) {
        return exception_status();
    }
}

namespace {

// new beta: rho follows with prox; the plain columns' curvatures are formed
// from beta in the kernels, the blocks' bounds are stored and re-uploaded
thetis_status apply_beta(thetis_solver &S, double beta) {
    S.p.beta = beta;
    S.rho = S.p.prox ? 1.0 / beta : 0.0;
    S.Lmax = S.nunits ? beta * S.amax + S.rho : 0.0;
    S.metrics_fresh = false;
    if (S.nblocks) {
        std::vector<double> LB(S.nblocks, 0.0);
        for (int64_t t = 0; t < S.nblocks; ++t)
            if (S.lb_factor[t] >= 0.0) LB[t] = beta * S.lb_factor[t] + S.rho;
        thetis_status st = upload_real(S, S.LB, LB);
        if (st) return st;
    }
    return THETIS_OK;
}

}  // namespace

extern "C" thetis_status thetis_set_beta(thetis_solver *s, double beta) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        if (!(beta > 0.0) || !std::isfinite(beta)) return fail(THETIS_EINVAL, "beta must be positive");
        s->beta0 = beta;          // the beta a reset returns to
        return apply_beta(*s, beta);
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_multiplier_step(thetis_solver *s, int32_t move_centre, double new_beta,
                                                thetis_mul_stats *stats_host) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        thetis_solver &S = *s;
        if (!S.has_ubar) return fail(THETIS_EUNSUPPORTED, "the solver was created without ubar");
        if (move_centre && !S.has_ybar) return fail(THETIS_EUNSUPPORTED, "moving the prox centre needs prox on and a ybar");
        if (!(new_beta == 0.0 || (new_beta > 0.0 && std::isfinite(new_beta))))
            return fail(THETIS_EINVAL, "new_beta must be 0 (keep) or positive");
        double out[5] = {0, 0, 0, 0, 0};
        thetis_status st = DISPATCH(S, multiplier_impl)(S, move_centre != 0, out);
        if (st) return st;
        if (new_beta > 0.0) {
            st = apply_beta(S, new_beta);
            if (st) return st;
        }
        if (stats_host) {
            stats_host->lp_value = out[0];
            stats_host->linf = out[1];
            stats_host->lp_dual = out[2];
            stats_host->lp_gap = out[3];
            stats_host->device_ms = out[4];
            stats_host->alg_bytes = multiplier_traffic(S, move_centre != 0);
        }
        if (!std::isfinite(out[0]) || std::isnan(out[2])) return fail(THETIS_EDIVERGED, "NaN or Inf in the multiplier step");
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_get_multipliers(thetis_solver *s, double *ubar_host, double *ybar_host) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        thetis_solver &S = *s;
        if (ubar_host && !S.has_ubar) return fail(THETIS_EUNSUPPORTED, "the solver was created without ubar");
        if (ybar_host && !S.has_ybar) return fail(THETIS_EUNSUPPORTED, "the solver has no prox centre");
        const int64_t n = S.n, m = S.m;
        std::vector<int32_t> ro(m);
        std::vector<double> u(ubar_host ? m : 0);
        const size_t R = prec_bytes(S.p.precision);
        std::vector<char> yb(ybar_host ? R * (n + m) : 0);
        if (m) HIP_TRY(hipMemcpyAsync(ro.data(), S.row_orig, 4 * m, hipMemcpyDeviceToHost, S.stream));
        std::vector<int32_t> co(ybar_host ? n : 0);
        if (ybar_host && n) HIP_TRY(hipMemcpyAsync(co.data(), S.col_orig, 4 * n, hipMemcpyDeviceToHost, S.stream));
        if (ubar_host && m) HIP_TRY(hipMemcpyAsync(u.data(), S.ubar, 8 * m, hipMemcpyDeviceToHost, S.stream));
        if (ybar_host && n + m) HIP_TRY(hipMemcpyAsync(yb.data(), S.ybar, yb.size(), hipMemcpyDeviceToHost, S.stream));
        HIP_TRY(hipStreamSynchronize(S.stream));
        // rows and columns are stored in the layout's order; hand them back in the caller's
        if (ubar_host)
            for (int64_t r = 0; r < m; ++r) ubar_host[ro[r]] = u[r];
        if (ybar_host) {
            auto get = [&](int64_t j) {
                if (R == 8) { double v; std::memcpy(&v, yb.data() + 8 * j, 8); return v; }
                float v; std::memcpy(&v, yb.data() + 4 * j, 4); return (double)v;
            };
            for (int64_t j = 0; j < n; ++j) ybar_host[co[j]] = get(j);
            for (int64_t r = 0; r < m; ++r) ybar_host[n + ro[r]] = get(n + r);
        }
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_run_multipliers(thetis_solver *s, int32_t max_outer, int32_t inner_epochs,
                                                double inner_gap_tol, double beta_growth, double beta_max,
                                                double feas_tol, double lp_gap_tol, int32_t move_centre,
                                                int32_t *outer_done, int64_t *epochs_done,
                                                thetis_mul_stats *last_host) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        if (max_outer < 0 || inner_epochs < 0) return fail(THETIS_EINVAL, "max_outer and inner_epochs must be >= 0");
        if (beta_growth > 1.0 && !(beta_max > 0.0 && std::isfinite(beta_max)))
            return fail(THETIS_EINVAL, "beta_max must be positive and finite when beta grows");
        if (!(beta_growth >= 0.0) || !std::isfinite(beta_growth)) return fail(THETIS_EINVAL, "beta_growth must be finite and >= 0");
        int32_t outer = 0;
        int64_t epochs = 0;
        thetis_mul_stats st_last{};
        thetis_status st = THETIS_OK;
        for (; outer < max_outer; ) {
            int32_t done = 0;
            st = thetis_run_epochs(s, inner_epochs, inner_gap_tol, &done);
            epochs += done;
            if (st) break;
            const double nb = beta_growth > 1.0 ? std::min(s->p.beta * beta_growth, std::max(beta_max, s->p.beta)) : 0.0;
            st = thetis_multiplier_step(s, move_centre, nb, &st_last);
            ++outer;
            if (st) break;
            if (st_last.linf <= feas_tol && st_last.lp_gap <= lp_gap_tol) break;
        }
        if (outer_done) *outer_done = outer;
        if (epochs_done) *epochs_done = epochs;
        if (last_host) *last_host = st_last;
        return st;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_set_step_rule(thetis_solver *s, int32_t rule, double scale) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        if (rule != THETIS_STEP_PER_COORD && rule != THETIS_STEP_GLOBAL_LMAX) return fail(THETIS_EINVAL, "unknown step rule");
        if (!(scale > 0.0 && scale <= 1.0)) return fail(THETIS_EINVAL, "step_scale must be in (0, 1]");
        s->p.step_rule = rule;
        s->p.step_scale = scale;
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_run_epochs(thetis_solver *s, int32_t max_epochs, double gap_tol,
                                           int32_t *epochs_done) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        if (max_epochs < 0) return fail(THETIS_EINVAL, "max_epochs < 0");
        s->have_round = false;
        return DISPATCH(*s, run_epochs_impl)(*s, max_epochs, gap_tol, epochs_done);
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_solver_autotune(thetis_solver *s, int32_t epochs_per_candidate, int32_t *choice_host) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        if (epochs_per_candidate < 1) return fail(THETIS_EINVAL, "epochs_per_candidate < 1");
        thetis_solver &S = *s;
        const int32_t nc = (int32_t)S.det.size();
        if (S.p.schedule != THETIS_SCHED_DET) {
            if (choice_host) for (int32_t c = 0; c < nc; ++c) choice_host[c] = S.det[c].group_cols;
            return THETIS_OK;
        }
        const int cands[3] = {1, 2, 4};
        std::vector<double> ms(3 * (size_t)std::max(nc, 1), 0.0);
        std::vector<ClassEvent> evs;
        // one untimed epoch first, so that no candidate runs on cold caches
        thetis_status st = DISPATCH(S, run_epochs_impl)(S, 1, 0.0, nullptr);
        for (int ci = 0; ci < 3 && st == THETIS_OK; ++ci) {
            for (ClassLaunch &cl : S.det)
                if (cl.has_cols) { cl.group_cols = cands[ci]; cl.cols = make_plan(cl.col_segs, false, 0, 1, cands[ci], true); }
            evs.clear();
            S.class_events = &evs;
            st = DISPATCH(S, run_epochs_impl)(S, epochs_per_candidate, 0.0, nullptr);
            S.class_events = nullptr;
            if (st == THETIS_OK && hipStreamSynchronize(S.stream) != hipSuccess) st = fail(THETIS_EDEVICE, "tuner sync failed");
            for (const ClassEvent &ev : evs) {
                float t = 0.f;
                if (st == THETIS_OK && hipEventElapsedTime(&t, ev.e0, ev.e1) == hipSuccess) ms[3 * ev.cls + ci] += t;
                (void)hipEventDestroy(ev.e0);
                (void)hipEventDestroy(ev.e1);
            }
        }
        for (int32_t c = 0; c < nc; ++c) {
            ClassLaunch &cl = S.det[c];
            // one column per group unless another shape is clearly faster
            int best = 0;
            for (int ci = 1; ci < 3; ++ci) if (ms[3 * c + ci] < 0.97 * ms[3 * c + best]) best = ci;
            if (cl.has_cols) { cl.group_cols = cands[best]; cl.cols = make_plan(cl.col_segs, false, 0, 1, cands[best], true); }
            if (choice_host) choice_host[c] = cl.group_cols;
        }
        s->have_round = false;
        return st;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_residual(thetis_solver *s, double *linf, double *l2, double *viol) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        thetis_status st = DISPATCH(*s, read_metrics)(*s);
        if (st) return st;
        if (linf) *linf = s->mt[MT_LINF];
        if (l2) *l2 = s->mt[MT_L2];
        if (viol) *viol = s->mt[MT_VIOL];
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_objective(thetis_solver *s, double *lp_value, double *penalty,
                                          double *dual_bound, double *gap) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        thetis_status st = DISPATCH(*s, read_metrics)(*s);
        if (st) return st;
        if (lp_value) *lp_value = s->mt[MT_CX];
        if (penalty) *penalty = s->mt[MT_F];
        if (dual_bound) *dual_bound = s->mt[MT_PHI];
        if (gap) *gap = s->mt[MT_GAP];
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_get_x(thetis_solver *s, double *x, double *sl) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        return DISPATCH(*s, get_x_impl)(*s, x, sl);
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_set_y(thetis_solver *s, const double *y) {
    try {
        clear_error();
        if (!s || !y) return fail(THETIS_EINVAL, "NULL argument");
        for (int64_t j = 0; j < s->n + s->m; ++j)
            if (!std::isfinite(y[j])) return fail(THETIS_EINVAL, "non-finite y");
        return DISPATCH(*s, set_y_impl)(*s, y);
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_epoch(const thetis_solver *s, int64_t *epoch) {
    try {
        clear_error();
        if (!s || !epoch) return fail(THETIS_EINVAL, "NULL argument");
        *epoch = s->epoch;
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_round(thetis_solver *s, int32_t rule, uint64_t seed, int32_t reps,
                                      int32_t *sol_host, double *cost, double *aux) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        return DISPATCH(*s, round_impl)(*s, rule, seed, reps, sol_host, cost, aux);
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_check_feasible(thetis_solver *s, int32_t rule, const int32_t *sol_host,
                                               int32_t *feasible, int64_t *n_violated) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        return DISPATCH(*s, check_impl)(*s, rule, sol_host, feasible, n_violated);
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_set_timing(thetis_solver *s, int32_t enable) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        if (enable < 0) return fail(THETIS_EINVAL, "timing period must be >= 0");
        s->timing = enable;
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_get_timing(const thetis_solver *s, int32_t kind, double *ms,
                                           int64_t *launches, double *alg_bytes) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        if (kind < 0 || kind >= THETIS_K_NKINDS) return fail(THETIS_EINVAL, "unknown kernel group");
        if (ms) *ms = s->ms[kind];
        if (launches) *launches = s->launches[kind];
        if (alg_bytes) *alg_bytes = s->bytes[kind];
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_epoch_traffic(const thetis_solver *s, double *sweep_bytes,
                                              double *refresh_bytes, int64_t *updates) {
    try {
        clear_error();
        if (!s) return fail(THETIS_EINVAL, "solver is NULL");
        double sw = 0.0;
        if (s->p.schedule == THETIS_SCHED_ASYNC) {
            sw = s->async_launch.bytes_cols + s->async_launch.bytes_block + s->async_launch.bytes_slack;
        } else {
            for (const ClassLaunch &cl : s->det) sw += cl.bytes_cols + cl.bytes_block + cl.bytes_slack;
        }
        if (sweep_bytes) *sweep_bytes = sw;
        if (refresh_bytes) *refresh_bytes = s->refresh_bytes;
        if (updates) *updates = s->updates_per_epoch;
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

namespace {

// Checkpoint layout: a header, then x, s, r, and, when the solver holds
// them, ubar (FP64), the shifted costs and the prox centre, each as stored.
struct CheckpointHeader {
    char magic[8];
    int32_t version, precision, has_ubar, has_ybar;
    int64_t n, m, epoch;
    double beta;
    uint64_t inst_digest;
    uint64_t layout_digest;    // the internal orders y and r are stored in
};
constexpr int32_t kCheckpointVersion = 2;
constexpr char kCheckpointMagic[8] = {'T', 'H', 'E', 'T', 'I', 'S', 'C', 'K'};

struct CheckpointPart {
    void *dev;
    size_t bytes;
};

std::vector<CheckpointPart> checkpoint_parts(const thetis_solver &S) {
    const size_t R = prec_bytes(S.p.precision), X = x_bytes(S.p.precision);
    std::vector<CheckpointPart> parts = {{S.x, X * (size_t)S.n}, {S.s, R * (size_t)S.m}, {S.r, R * (size_t)S.m}};
    if (S.has_ubar) {
        parts.push_back({S.ubar, 8 * (size_t)S.m});
        parts.push_back({S.ctil, R * (size_t)(S.n + S.m)});
    }
    if (S.has_ybar) parts.push_back({S.ybar, R * (size_t)(S.n + S.m)});
    return parts;
}

}  // namespace

extern "C" thetis_status thetis_solver_save(thetis_solver *s, void *host_buf, size_t *bytes) {
    try {
        clear_error();
        if (!s || !bytes) return fail(THETIS_EINVAL, "NULL argument");
        thetis_solver &S = *s;
        const std::vector<CheckpointPart> parts = checkpoint_parts(S);
        size_t need = sizeof(CheckpointHeader);
        for (const CheckpointPart &q : parts) need += q.bytes;
        if (!host_buf) { *bytes = need; return THETIS_OK; }
        if (*bytes < need) { *bytes = need; return fail(THETIS_EINVAL, "checkpoint buffer too small"); }
        CheckpointHeader h{};
        std::memcpy(h.magic, kCheckpointMagic, 8);
        h.version = kCheckpointVersion;
        h.precision = S.p.precision;
        h.has_ubar = S.has_ubar;
        h.has_ybar = S.has_ybar;
        h.n = S.n;
        h.m = S.m;
        h.epoch = S.epoch;
        h.beta = S.p.beta;
        h.inst_digest = S.inst_digest;
        h.layout_digest = S.layout_digest;
        char *out = (char *)host_buf;
        std::memcpy(out, &h, sizeof(h));
        size_t off = sizeof(h);
        for (const CheckpointPart &q : parts) {
            if (q.bytes) HIP_TRY(hipMemcpyAsync(out + off, q.dev, q.bytes, hipMemcpyDeviceToHost, S.stream));
            off += q.bytes;
        }
        HIP_TRY(hipStreamSynchronize(S.stream));
        *bytes = need;
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_solver_load(thetis_solver *s, const void *host_buf, size_t bytes) {
    try {
        clear_error();
        if (!s || !host_buf) return fail(THETIS_EINVAL, "NULL argument");
        thetis_solver &S = *s;
        if (bytes < sizeof(CheckpointHeader)) return fail(THETIS_EINVAL, "checkpoint too short");
        CheckpointHeader h;
        std::memcpy(&h, host_buf, sizeof(h));
        if (std::memcmp(h.magic, kCheckpointMagic, 8) != 0 || h.version != kCheckpointVersion)
            return fail(THETIS_EINVAL, "not a checkpoint of this library version");
        if (h.layout_digest != S.layout_digest)
            return fail(THETIS_EINVAL, "checkpoint of another internal layout (rows or columns ordered differently)");
        if (h.precision != S.p.precision || h.n != S.n || h.m != S.m || h.inst_digest != S.inst_digest ||
            h.has_ubar != (int32_t)S.has_ubar || h.has_ybar != (int32_t)S.has_ybar)
            return fail(THETIS_EINVAL, "checkpoint of a different instance, precision or parameter set");
        if (!(h.beta > 0.0) || !std::isfinite(h.beta) || h.epoch < 0) return fail(THETIS_EINVAL, "corrupt checkpoint header");
        const std::vector<CheckpointPart> parts = checkpoint_parts(S);
        size_t need = sizeof(h);
        for (const CheckpointPart &q : parts) need += q.bytes;
        if (bytes != need) return fail(THETIS_EINVAL, "checkpoint size does not match the solver");
        const char *in = (const char *)host_buf;
        size_t off = sizeof(h);
        for (const CheckpointPart &q : parts) {
            if (q.bytes) HIP_TRY(hipMemcpyAsync(q.dev, in + off, q.bytes, hipMemcpyHostToDevice, S.stream));
            off += q.bytes;
        }
        HIP_TRY(hipStreamSynchronize(S.stream));
        if (h.beta != S.p.beta) {
            thetis_status st = apply_beta(S, h.beta);
            if (st) return st;
        }
        S.epoch = h.epoch;
        S.metrics_fresh = false;
        S.have_round = false;
        if (S.has_ubar || S.has_ybar || h.beta != S.beta0) S.mul_dirty = true;   // a reset returns to creation
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_solver_destroy(thetis_solver *s) {
    try {
        clear_error();
        if (!s) return THETIS_OK;
        if (s->batch_slots.load() > 0)
            return fail(THETIS_EBUSY, "the solver occupies a batch slot: empty the slot or destroy the batch first");
        (void)hipStreamSynchronize(s->stream);
        for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
        if (s->own_ws && s->ws) (void)hipFree(s->ws);
        release_static(s);
        delete s;
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

// ==================================================================== batches
//
// A batch advances many solvers with one sequence of launches per epoch.
// k_border draws every active instance's class order for the epoch (its own
// Philox order).  k_bplan then, for every step q at once, looks up each
// instance's class of that step and its workgroup count and turns the counts
// into offsets, and k_bsweep of step q walks the resulting (instance,
// workgroup) items: each XCD takes a
// contiguous share of the items (so an instance's columns stay in one L2)
// and each of its workgroups a contiguous run of that share.  Kernel boundaries are the class barriers.  After the
// last step, k_bepoch advances the epoch counters and marks the instances
// whose refresh is due; k_brows / k_bdual / k_bfinal refresh them and retire
// those whose certified gap reached the tolerance.  Every per-column and
// per-row computation is the solo kernels' own device code with the same
// logical workgroup numbering, so a batched solve equals the solve alone.

namespace {

template <class P>
struct BInst {
    Dev<P> a;
    Sched<typename P::R> sc, asc;       // DET schedule, all-columns schedule
    BlockPack<typename P::R> pb;        // packed DET blocks
    LaunchPlan dual;                    // column pass of the refresh
    double *rpart, *cpart, *metrics;
    int64_t epoch, rows_wg;
    uint64_t seed;
    double gap_tol, beta;
    int32_t nclasses, class_base, refresh_every, active, due, with_dual, slack_identity, lpc;
    int32_t epochs_done, max_epochs, diverged, reason;   // reason: 0 running, 1 gap, 2 epochs, 3 NaN
    int32_t pending;                    // waits for a place in the window
};

struct BClass {
    LaunchPlan cols;
    int64_t block_first, block_count, block_pb, slack_first, slack_count;
    int64_t wg_cols, wg_block, wg_slack;
};

constexpr int kMaxBatchClasses = 64;
// most epochs one captured batch graph runs
constexpr int64_t kGraphEpochs = 8;
// a batch work item covers one logical workgroup of plain columns, or this
// many simplex blocks per wavefront, or this many slacks per thread (larger
// items amortise the walk to the item's instance and plan)
constexpr int kBatchBlocks = 4;
constexpr int kBatchSlacks = 4;

// The running instances: alist[0 .. ctl[CTL_NACT]) holds their slots in
// slot order, and the per-epoch kernels visit only those.  ctl[CTL_CURSOR]
// is the first slot not yet considered for a start, ctl[CTL_PENDING] the
// number of waiting slots, ctl[CTL_LEFT] running + waiting (read by the host).
enum { CTL_NACT = 0, CTL_CURSOR, CTL_PENDING, CTL_LEFT, CTL_N };

// class order of every active instance for its current epoch: classes
// sorted by (Philox word, class id).  One wavefront per instance, lane c
// draws the word of class c and counts the classes ahead of it.
template <class P>
__global__ __launch_bounds__(kWG) void k_border(const BInst<P> *bi, const int32_t *alist, const int32_t *ctl,
                                                int8_t *order) {
    const int32_t w = blockIdx.x * (kWG / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= ctl[CTL_NACT]) return;       // the whole wavefront leaves together
    const int32_t i = alist[w];
    const BInst<P> &I = bi[i];
    if (!I.active) return;
    const int32_t C = I.nclasses;
    const uint64_t key = lane < C ? philox_word_dev(I.seed, RNG_CLASS_ORDER, (uint64_t)I.epoch, (uint64_t)lane, 0) : 0;
    const uint32_t klo = (uint32_t)key, khi = (uint32_t)(key >> 32);
    int32_t rank = 0;
    for (int32_t c = 0; c < C; ++c) {
        const uint64_t kc = ((uint64_t)(uint32_t)__shfl((int)khi, c, 64) << 32) | (uint32_t)__shfl((int)klo, c, 64);
        rank += (kc < key || (kc == key && c < lane)) ? 1 : 0;
    }
    if (lane < C) order[(int64_t)i * kMaxBatchClasses + rank] = (int8_t)lane;
}

// A directory of the work items of one launch: the instances with work, in
// slot order, with their class, the offset of their first item and, for
// every kDirChunk-th item, the directory entry that owns it.  A walk finds
// an item's instance with one table load and a short forward step, however
// many slots are empty.
constexpr int kDirChunk = 16;
struct Dir {
    int64_t *total, *start;                   // start: nact + 1 entries
    int32_t *inst, *cls, *wtmp, *ctmp, *itmp, *chunk;
    int64_t chunk_cap;
};
__host__ __device__ inline int64_t dir_bytes(int32_t count, int64_t chunk_cap) {
    const int64_t b = 8 + 8 * ((int64_t)count + 1) + 20 * (int64_t)count + 4 * chunk_cap;
    return (b + 255) / 256 * 256;
}
__host__ __device__ inline Dir dir_at(char *base, int32_t count, int64_t chunk_cap, int d) {
    char *p = base + (int64_t)d * dir_bytes(count, chunk_cap);
    Dir r;
    r.total = (int64_t *)p;
    r.start = r.total + 1;
    r.inst = (int32_t *)(r.start + count + 1);
    r.cls = r.inst + count;
    r.wtmp = r.cls + count;
    r.ctmp = r.wtmp + count;
    r.itmp = r.ctmp + count;
    r.chunk = r.itmp + count;
    r.chunk_cap = chunk_cap;
    return r;
}

// one workgroup: builds the directory from n entries (the weight functor
// gives entry k's item count, class and slot)
template <class Wf>
__device__ void build_dir(const Dir &d, int32_t count, Wf weight) {
    __shared__ int64_t psum[kWG + 1];
    __shared__ int32_t pnz[kWG + 1];
    const int t = threadIdx.x;
    const int32_t per = (count + kWG - 1) / kWG;
    const int32_t lo = min(count, t * per), hi = min(count, lo + per);
    int64_t sum = 0;
    int32_t nz = 0;
    for (int32_t i = lo; i < hi; ++i) {
        int32_t c = 0, id = i;
        const int32_t w = weight(i, &c, &id);
        d.wtmp[i] = w;
        d.ctmp[i] = c;
        d.itmp[i] = id;
        sum += w;
        nz += w > 0;
    }
    psum[t + 1] = sum;
    pnz[t + 1] = nz;
    __syncthreads();
    if (t == 0) {
        psum[0] = 0;
        pnz[0] = 0;
        for (int u = 1; u <= kWG; ++u) { psum[u] += psum[u - 1]; pnz[u] += pnz[u - 1]; }
    }
    __syncthreads();
    int64_t s = psum[t];
    int32_t q = pnz[t];
    for (int32_t i = lo; i < hi; ++i) {
        const int32_t w = d.wtmp[i];
        if (w == 0) continue;
        d.inst[q] = d.itmp[i];
        d.cls[q] = d.ctmp[i];
        d.start[q] = s;
        for (int64_t c = (s + kDirChunk - 1) / kDirChunk; c * kDirChunk < s + w && c < d.chunk_cap; ++c)
            d.chunk[c] = q;
        s += w;
        ++q;
    }
    if (t == 0) {
        d.start[pnz[kWG]] = psum[kWG];
        *d.total = psum[kWG];
    }
}

// every step q of the epoch (workgroup q): the directory of the step's items,
// each active instance contributing its class of step q
template <class P>
__global__ __launch_bounds__(kWG) void k_bplan(const BInst<P> *bi, const BClass *bc, int32_t count,
                                               const int32_t *alist, const int32_t *ctl, const int8_t *order,
                                               char *dirs, int64_t chunk_cap) {
    const int32_t q = blockIdx.x;
    const Dir d = dir_at(dirs, count, chunk_cap, q);
    build_dir(d, ctl[CTL_NACT], [&](int32_t k, int32_t *c, int32_t *id) -> int32_t {
        const int32_t i = alist[k];
        *id = i;
        const BInst<P> &I = bi[i];
        if (!I.active || q >= I.nclasses) return 0;
        *c = order[(int64_t)i * kMaxBatchClasses + q];
        const BClass &C = bc[I.class_base + *c];
        return (int32_t)(C.wg_cols + C.wg_block + C.wg_slack);
    });
}

// the directory of the running instances' workgroup counts (refresh
// passes; counts[k] belongs to alist[k])
__global__ __launch_bounds__(kWG) void k_bdir(const int32_t *counts, const int32_t *alist, const int32_t *ctl,
                                              int32_t count, char *dirs, int64_t chunk_cap, int32_t which) {
    const Dir d = dir_at(dirs, count, chunk_cap, which);
    build_dir(d, ctl[CTL_NACT], [&](int32_t k, int32_t *c, int32_t *id) -> int32_t {
        *c = 0;
        *id = alist[k];
        return counts[k];
    });
}

// the directory entry of item `it`, from a hint at or before it
__device__ __forceinline__ int32_t dir_find(const Dir &d, int64_t it, int32_t p, bool jump) {
    if (jump) p = d.chunk[it / kDirChunk];
    while (d.start[p + 1] <= it) ++p;
    return p;
}

// this workgroup's share of `total` items.  XCD x (= block & 7) takes the
// x-th contiguous eighth.  Inside it, either each workgroup of the XCD takes
// a contiguous run (stride 1), or the XCD's workgroups take neighbouring
// items and stride by their count, so that at any moment one XCD works on
// one or two instances whose state fits its L2.  Both walks visit items in
// increasing order, so the owner is found by stepping forward.
struct Share {
    int64_t lo, hi, step;
};
__device__ __forceinline__ Share xcd_share(int64_t total, int32_t strided) {
    const int64_t xcd = blockIdx.x & 7, per = gridDim.x >> 3, lw = blockIdx.x >> 3;
    const int64_t chunk = (total + 7) >> 3;
    const int64_t xlo = xcd * chunk, xhi = min(total, xlo + chunk);
    Share s;
    if (strided) {
        s.lo = xlo + lw;
        s.hi = xhi;
        s.step = per;
    } else {
        const int64_t sub = (xhi - xlo + per - 1) / per;
        s.lo = xlo + lw * sub;
        s.hi = min(xhi, s.lo + sub);
        s.step = 1;
    }
    return s;
}

// waves per SIMD the batch sweep is compiled for: the FP32 forms fit 64
// registers (full occupancy); the FP64 validation form keeps its registers
template <class P>
struct BsweepWaves {
    static constexpr int value = sizeof(typename P::R) == 4 ? 8 : 4;
};

// bi and bc are only read while the sweep runs (restrict: the sweep's stores
// cannot change them, so their fields are loaded once, as scalars)
template <class P, int VM>
__global__ __launch_bounds__(kWG, BsweepWaves<P>::value) void k_bsweep(const BInst<P> *__restrict__ bi,
                                                                        const BClass *__restrict__ bc,
                                                                        char *dirs, int32_t count, int64_t chunk_cap,
                                                                        int32_t q, int32_t strided) {
    using R = typename P::R;
    __shared__ R st_r[HubTile<P>::n];
    __shared__ int32_t st_row[HubTile<P>::n];
    __shared__ R red[kWG / 64];
    const Dir d = dir_at(dirs, count, chunk_cap, q);
    const Share sh = xcd_share(*d.total, strided);
    int32_t p = 0;
    for (int64_t it = sh.lo; it < sh.hi; it += sh.step) {
        p = dir_find(d, it, p, it == sh.lo || sh.step > 1);
        const BInst<P> &I = bi[d.inst[p]];
        const BClass &C = bc[I.class_base + d.cls[p]];
        const int64_t local = it - d.start[p];
        const Dev<P> &a = I.a;
        const Sched<R> &sc = I.sc;
        const int64_t wg_cols = C.wg_cols, wg_block = C.wg_block;
        if (local < wg_cols) {
            sweep_item<P, VM>(a, sc, C.cols, local, st_r, st_row, red);
        } else if (local < wg_cols + wg_block) {
            // kBatchBlocks blocks per wavefront
            // kBatchBlocks wavefront positions, each with BPW blocks
            const int64_t first = C.block_pb, count = C.block_count;
            const int32_t lpc = I.lpc;
            const int64_t base = (local - wg_cols) * (kWG / 64) * kBatchBlocks + (threadIdx.x >> 6);
            if (block_bpw(a.k) == 4) {
                for (int b = 0; b < kBatchBlocks; ++b) {
                    const int64_t w = base + b * (kWG / 64);
                    if (w * 4 >= count) break;
                    const int64_t u = w * 4 + (threadIdx.x & 63) / 16;
                    sweep_block_packed<P, VM, 4>(a, I.pb, u < count, first + u, lpc);
                }
            } else if (block_bpw(a.k) == 2) {
                for (int b = 0; b < kBatchBlocks; ++b) {
                    const int64_t w = base + b * (kWG / 64);
                    if (w * 2 >= count) break;
                    const int64_t u = w * 2 + (threadIdx.x & 63) / 32;
                    sweep_block_packed<P, VM, 2>(a, I.pb, u < count, first + u, lpc);
                }
            } else {
                for (int b = 0; b < kBatchBlocks; ++b) {
                    const int64_t w = base + b * (kWG / 64);
                    if (w >= count) break;
                    sweep_block_packed<P, VM, 1>(a, I.pb, true, first + w, lpc);
                }
            }
        } else {
            // kBatchSlacks slacks per thread
            const int64_t first = C.slack_first, count = C.slack_count;
            const bool ident = I.slack_identity;
            const int64_t base = (local - wg_cols - wg_block) * kWG * kBatchSlacks + threadIdx.x;
            for (int b = 0; b < kBatchSlacks; ++b) {
                const int64_t u = base + b * kWG;
                if (u < count) sweep_slack<P>(a, ident ? u : sc.ids[first + u]);
            }
        }
    }
}

template <class P>
__global__ __launch_bounds__(kWG) void k_bepoch(BInst<P> *bi, const int32_t *alist, const int32_t *ctl,
                                                int32_t *rows_wg, int32_t *dual_wg) {
    const int32_t k = blockIdx.x * kWG + threadIdx.x;
    if (k >= ctl[CTL_NACT]) return;
    BInst<P> &I = bi[alist[k]];
    int32_t rw = 0, dw = 0;
    if (I.active) {
        I.epoch += 1;
        I.epochs_done += 1;
        I.due = (I.epoch % I.refresh_every) == 0;
        if (I.due) { rw = (int32_t)I.rows_wg; dw = (int32_t)I.dual.nwg; }
        else if (I.epochs_done >= I.max_epochs) { I.active = 0; I.reason = 2; }
    } else {
        I.due = 0;
    }
    rows_wg[k] = rw;
    dual_wg[k] = dw;
}

template <class P>
__global__ __launch_bounds__(kWG) void k_brows(const BInst<P> *__restrict__ bi, char *dirs, int32_t count, int64_t chunk_cap,
                                               int32_t which, int32_t strided) {
    const Dir d = dir_at(dirs, count, chunk_cap, which);
    const Share sh = xcd_share(*d.total, strided);
    int32_t p = 0;
    for (int64_t it = sh.lo; it < sh.hi; it += sh.step) {
        p = dir_find(d, it, p, it == sh.lo || sh.step > 1);
        const BInst<P> &I = bi[d.inst[p]];
        rows_item<P>(I.a, it - d.start[p], 1, I.with_dual, I.rpart);
    }
}

template <class P, bool VALS>
__global__ __launch_bounds__(kWG) void k_bdual(const BInst<P> *__restrict__ bi, char *dirs, int32_t count, int64_t chunk_cap,
                                               int32_t which, int32_t strided) {
    __shared__ double sh2[kWG / 64];
    const Dir d = dir_at(dirs, count, chunk_cap, which);
    const Share sh = xcd_share(*d.total, strided);
    int32_t p = 0;
    for (int64_t it = sh.lo; it < sh.hi; it += sh.step) {
        p = dir_find(d, it, p, it == sh.lo || sh.step > 1);
        const BInst<P> &I = bi[d.inst[p]];
        dual_item<P, VALS>(I.a, I.asc, I.dual, it - d.start[p], I.slack_identity, I.cpart, sh2);
    }
}

// one workgroup per due instance: fold its partials into its metrics, then
// retire it on a reached gap, the epoch cap or a NaN
template <class P>
__global__ __launch_bounds__(kWG) void k_bfinal(BInst<P> *bi, const int32_t *alist, const int32_t *ctl) {
    const int32_t n = ctl[CTL_NACT];
    for (int32_t k = blockIdx.x; k < n; k += gridDim.x) {
        BInst<P> &I = bi[alist[k]];
        if (!I.due) continue;
        finalize_item(I.rpart, I.rows_wg, I.cpart, I.dual.nwg, I.beta, I.with_dual, I.metrics);
        if (threadIdx.x == 0) {
            const double *mt = I.metrics;
            if (I.epochs_done >= I.max_epochs) { I.active = 0; I.reason = 2; }
            if (I.gap_tol > 0.0 && mt[MT_GAP] <= I.gap_tol) { I.active = 0; I.reason = 1; }
            if (mt[MT_BAD] != 0.0) { I.diverged = 1; I.active = 0; I.reason = 3; }
            I.due = 0;
        }
        __syncthreads();
    }
}

// end of an epoch, one workgroup: the running list drops the instances that
// retired, then waiting slots (in slot order, from the cursor) start until
// `window` run at once
template <class P>
__global__ __launch_bounds__(kWG) void k_bwindow(BInst<P> *bi, int32_t count, int32_t window, int32_t *alist,
                                                 int32_t *ctl) {
    __shared__ int32_t part[kWG + 1];
    __shared__ int32_t keep[kWG];
    __shared__ int32_t n_run, cursor, pending;
    const int t = threadIdx.x;
    const int32_t n = ctl[CTL_NACT];
    if (t == 0) { n_run = 0; cursor = ctl[CTL_CURSOR]; pending = ctl[CTL_PENDING]; }
    __syncthreads();
    // compaction in kWG-wide rounds: entries only move to lower positions,
    // and a round reads all of its entries before any is written
    for (int32_t base = 0; base < n; base += kWG) {
        const int32_t k = base + t;
        const int32_t slot = k < n ? alist[k] : -1;
        const int32_t alive = slot >= 0 && bi[slot].active ? 1 : 0;
        keep[t] = alive;
        __syncthreads();
        if (t == 0) {
            part[0] = 0;
            for (int u = 0; u < kWG; ++u) part[u + 1] = part[u] + keep[u];
        }
        __syncthreads();
        if (alive) alist[n_run + part[t]] = slot;
        __syncthreads();
        if (t == 0) n_run += part[kWG];
        __syncthreads();
    }
    // starts: scan the slots after the cursor, kWG at a time
    while (n_run < window && pending > 0 && cursor < count) {
        const int32_t s = cursor + t;
        const int32_t waiting = s < count && bi[s].pending ? 1 : 0;
        keep[t] = waiting;
        __syncthreads();
        if (t == 0) {
            part[0] = 0;
            for (int u = 0; u < kWG; ++u) part[u + 1] = part[u] + keep[u];
        }
        __syncthreads();
        const int32_t room = window - n_run;
        const int32_t rank = part[t];
        if (waiting && rank < room) {
            bi[s].pending = 0;
            bi[s].active = 1;
            alist[n_run + rank] = s;
        }
        __syncthreads();
        if (t == 0) {
            const int32_t started = min(room, part[kWG]);
            // the cursor stops after the last slot started when the room ran out
            int32_t adv = kWG;
            if (part[kWG] > room) {
                // the last slot started is the first u with room waiting
                // slots in [0, u]; the slots after it are looked at again
                int u = 0;
                while (part[u + 1] < room) ++u;
                adv = u + 1;
            }
            cursor += adv;
            n_run += started;
            pending -= started;
        }
        __syncthreads();
    }
    if (t == 0) {
        ctl[CTL_NACT] = n_run;
        ctl[CTL_CURSOR] = cursor;
        ctl[CTL_PENDING] = pending;
        ctl[CTL_LEFT] = n_run + pending;
    }
}

}  // namespace

struct thetis_batch {
    int32_t count = 0, precision = 0, max_classes = 0;
    bool vals = false;
    int32_t vmode = -1;                  // how the solvers' DET copies store values (entry_at); -1: none yet
    int64_t bc_capacity = 0;             // BClass records the device table holds
    std::vector<thetis_solver *> solvers;
    bool slots_counted = false;          // the solvers' batch_slots count this batch's slots
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int widen = 1, grid_mult = 2, strided = 1, cols = 4;
    int64_t most_items = 1;             // the largest item count of any launch
    int32_t window = 0;                 // most instances running at once (0: all)
    int64_t resident_wg = 2048;
    // device
    void *bi = nullptr, *bc = nullptr;
    int32_t *rows_wg = nullptr, *dual_wg = nullptr;
    int32_t *alist = nullptr, *ctl = nullptr;      // running slots, window control (CTL_*)
    int8_t *order = nullptr;
    // item directories: one per step of an epoch, then rows and dual refresh
    char *dirs = nullptr;
    int64_t chunk_cap = 0;
    size_t bi_bytes = 0;
    std::vector<char> bi_host;          // host image of the BInst array
    int64_t nclass_total = 0;
    // captured epochs: graph_epochs copies of one epoch's launches
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int captured_widen = 0, captured_grid = -1, captured_strided = -1, captured_cols = 0, captured_window = -1;
    int32_t graph_epochs = 1, captured_epochs = 0;
    // instances left after a graph launch, copied to pinned host memory
    // (two slots: the host reads one while the next launch runs)
    int32_t *poll = nullptr;
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
    int64_t captured_most = 0;
    uint64_t signature = 0;
};

namespace {

struct Choice {
    int widen, grid_mult, strided, cols;
};
// the tuner's choices by batch shape, for the life of the process; batches
// made or tuned on different threads share it under this lock
std::mutex g_tuned_mu;
std::map<uint64_t, Choice> &tuned_choices() {
    static std::map<uint64_t, Choice> m;
    return m;
}

void batch_drop_graph(thetis_batch &B) {
    if (B.exec) (void)hipGraphExecDestroy(B.exec);
    if (B.graph) (void)hipGraphDestroy(B.graph);
    B.exec = nullptr;
    B.graph = nullptr;
}

// host image of the per-instance records and the per-class plans for the
// current launch configuration
template <class P>
thetis_status batch_upload(thetis_batch &B, int32_t max_epochs, double gap_tol) {
    std::vector<BInst<P>> bi(B.count);
    std::vector<BClass> bc;
    int32_t occupied = 0;
    for (int32_t i = 0; i < B.count; ++i) {
        BInst<P> &I = bi[i];
        std::memset((void *)&I, 0, sizeof(I));
        if (!B.solvers[i]) continue;        // empty slot: inactive, no classes
        thetis_solver &S = *B.solvers[i];
        I.a = make_dev<P>(S);
        I.sc = det_sched<P>(S);
        I.pb = block_pack<P>(S);
        I.asc = async_sched<P>(S);
        I.with_dual = gap_tol > 0.0;
        I.dual = I.with_dual ? S.dual : S.colterms;
        I.rpart = (double *)S.rpart;
        I.cpart = (double *)S.cpart;
        I.metrics = (double *)S.metrics;
        I.epoch = S.epoch;
        I.rows_wg = row_wgs(S);
        I.seed = S.p.seed;
        I.gap_tol = gap_tol;
        I.beta = S.p.beta;
        I.nclasses = S.nclasses;
        I.class_base = (int32_t)bc.size();
        I.refresh_every = S.p.refresh_every;
        // with a window, the first `window` occupied slots start and the
        // rest wait
        I.pending = (max_epochs > 0 && B.window > 0 && occupied >= B.window) ? 1 : 0;
        I.active = (max_epochs > 0 && !I.pending) ? 1 : 0;
        ++occupied;
        I.due = 0;
        I.slack_identity = S.all_rows_slack ? 1 : 0;
        I.lpc = S.lpc;
        I.epochs_done = 0;
        I.max_epochs = max_epochs;
        I.diverged = 0;
        I.reason = 0;
        for (const ClassLaunch &cl : S.det) {
            BClass C{};
            C.cols = cl.has_cols ? make_plan(cl.col_segs, false, 0, B.widen, B.cols) : LaunchPlan{};
            C.wg_cols = cl.has_cols ? C.cols.nwg : 0;
            C.block_first = cl.block_first;
            C.block_count = cl.block_count;
            C.block_pb = cl.block_pb;
            C.wg_block = cdiv(cl.block_count, (kWG / 64) * kBatchBlocks * block_bpw(S.k));
            C.slack_first = cl.slack_first;
            C.slack_count = cl.slack_count;
            C.wg_slack = cdiv(cl.slack_count, kWG * kBatchSlacks);
            bc.push_back(C);
        }
    }
    if ((int64_t)bc.size() > B.bc_capacity) {
        HIP_TRY(hipStreamSynchronize(B.stream));
        (void)hipFree(B.bc);
        B.bc = nullptr;
        const int64_t cap = std::max<int64_t>((int64_t)bc.size() * 2, 64);
        HIP_TRY(hipMalloc(&B.bc, sizeof(BClass) * cap));
        B.bc_capacity = cap;
        batch_drop_graph(B);                 // the captured launches point at the old table
    }
    int32_t mc = 0;
    for (thetis_solver *S : B.solvers) if (S) mc = std::max(mc, S->nclasses);
    if (mc != B.max_classes) { B.max_classes = mc; batch_drop_graph(B); }
    // directory chunk tables: enough for the most items any launch can have
    int64_t most = 1;
    {
        int64_t steps = 0, rows = 0, dual = 0;
        for (int32_t i = 0; i < B.count; ++i) {
            if (!B.solvers[i]) continue;
            int64_t w = 0;
            for (int32_t c = 0; c < bi[i].nclasses; ++c) {
                const BClass &C = bc[bi[i].class_base + c];
                w = std::max<int64_t>(w, C.wg_cols + C.wg_block + C.wg_slack);
            }
            steps += w;
            rows += bi[i].rows_wg;
            dual += bi[i].dual.nwg;
        }
        most = std::max<int64_t>({most, steps, rows, dual});
    }
    B.most_items = most;
    const int64_t cap_needed = most / kDirChunk + 2;
    if (!B.dirs || cap_needed > B.chunk_cap) {
        HIP_TRY(hipStreamSynchronize(B.stream));
        if (B.dirs) (void)hipFree(B.dirs);
        B.dirs = nullptr;
        const int64_t cap = cap_needed * 2;
        HIP_TRY(hipMalloc((void **)&B.dirs, dir_bytes(B.count, cap) * (kMaxBatchClasses + 2)));
        B.chunk_cap = cap;
        batch_drop_graph(B);                 // the captured launches point at the old tables
    }
    // the running list and window control: the first `window` occupied
    // slots run, the rest wait from the first waiting slot on
    std::vector<int32_t> alist;
    int32_t ctl[CTL_N] = {0, B.count, 0, 0};
    for (int32_t i = 0; i < B.count; ++i) {
        if (!B.solvers[i]) continue;
        if (bi[i].active) alist.push_back(i);
        else if (bi[i].pending) { ctl[CTL_PENDING]++; ctl[CTL_CURSOR] = std::min(ctl[CTL_CURSOR], i); }
    }
    ctl[CTL_NACT] = (int32_t)alist.size();
    ctl[CTL_LEFT] = ctl[CTL_NACT] + ctl[CTL_PENDING];
    if (!alist.empty())
        HIP_TRY(hipMemcpyAsync(B.alist, alist.data(), 4 * alist.size(), hipMemcpyHostToDevice, B.stream));
    HIP_TRY(hipMemcpyAsync(B.ctl, ctl, sizeof(ctl), hipMemcpyHostToDevice, B.stream));
    HIP_TRY(hipMemcpyAsync(B.bi, bi.data(), sizeof(BInst<P>) * B.count, hipMemcpyHostToDevice, B.stream));
    if (!bc.empty())
        HIP_TRY(hipMemcpyAsync(B.bc, bc.data(), sizeof(BClass) * bc.size(), hipMemcpyHostToDevice, B.stream));
    HIP_TRY(hipStreamSynchronize(B.stream));
    return THETIS_OK;
}

// the launches of one epoch (captured once per configuration)
template <class P>
void batch_epoch_launches(thetis_batch &B) {
    const int32_t n = B.count;
    // grid_mult 0: one workgroup per work item of the largest launch (the
    // hardware dispatcher balances the items); else a multiple of the
    // resident workgroups walking the items
    const int64_t grid = B.grid_mult > 0 ? std::max<int64_t>(8, (B.resident_wg * B.grid_mult) / 8 * 8)
                                         : std::max<int64_t>(8, (B.most_items + 7) / 8 * 8);
    BInst<P> *bi = (BInst<P> *)B.bi;
    const BClass *bc = (const BClass *)B.bc;
    const int32_t win = B.window > 0 ? std::min(B.window, n) : n;
    hipLaunchKernelGGL((k_border<P>), dim3(cdiv(win, kWG / 64)), dim3(kWG), 0, B.stream, (const BInst<P> *)bi,
                       (const int32_t *)B.alist, (const int32_t *)B.ctl, B.order);
    hipLaunchKernelGGL((k_bplan<P>), dim3(std::max(B.max_classes, 1)), dim3(kWG), 0, B.stream, (const BInst<P> *)bi, bc, n,
                       (const int32_t *)B.alist, (const int32_t *)B.ctl, (const int8_t *)B.order, B.dirs, B.chunk_cap);
    for (int32_t q = 0; q < B.max_classes; ++q) {
        if (B.vmode == 2) hipLaunchKernelGGL((k_bsweep<P, 2>), dim3(grid), dim3(kWG), 0, B.stream, bi, bc, B.dirs, n, B.chunk_cap, q, B.strided);
        else if (B.vmode == 1) hipLaunchKernelGGL((k_bsweep<P, 1>), dim3(grid), dim3(kWG), 0, B.stream, bi, bc, B.dirs, n, B.chunk_cap, q, B.strided);
        else hipLaunchKernelGGL((k_bsweep<P, 0>), dim3(grid), dim3(kWG), 0, B.stream, bi, bc, B.dirs, n, B.chunk_cap, q, B.strided);
    }
    const int32_t d_rows = kMaxBatchClasses, d_dual = kMaxBatchClasses + 1;
    hipLaunchKernelGGL((k_bepoch<P>), dim3(cdiv(win, kWG)), dim3(kWG), 0, B.stream, bi, (const int32_t *)B.alist,
                       (const int32_t *)B.ctl, B.rows_wg, B.dual_wg);
    hipLaunchKernelGGL(k_bdir, dim3(1), dim3(kWG), 0, B.stream, (const int32_t *)B.rows_wg, (const int32_t *)B.alist,
                       (const int32_t *)B.ctl, n, B.dirs, B.chunk_cap, d_rows);
    hipLaunchKernelGGL(k_bdir, dim3(1), dim3(kWG), 0, B.stream, (const int32_t *)B.dual_wg, (const int32_t *)B.alist,
                       (const int32_t *)B.ctl, n, B.dirs, B.chunk_cap, d_dual);
    hipLaunchKernelGGL((k_brows<P>), dim3(grid), dim3(kWG), 0, B.stream, (const BInst<P> *)bi, B.dirs, n, B.chunk_cap, d_rows, B.strided);
    if (B.vals) hipLaunchKernelGGL((k_bdual<P, true>), dim3(grid), dim3(kWG), 0, B.stream, (const BInst<P> *)bi, B.dirs, n, B.chunk_cap, d_dual, B.strided);
    else hipLaunchKernelGGL((k_bdual<P, false>), dim3(grid), dim3(kWG), 0, B.stream, (const BInst<P> *)bi, B.dirs, n, B.chunk_cap, d_dual, B.strided);
    hipLaunchKernelGGL((k_bfinal<P>), dim3(std::min<int64_t>(win, 1024)), dim3(kWG), 0, B.stream, bi,
                       (const int32_t *)B.alist, (const int32_t *)B.ctl);
    hipLaunchKernelGGL((k_bwindow<P>), dim3(1), dim3(kWG), 0, B.stream, bi, n, win, B.alist, B.ctl);
}

template <class P>
thetis_status batch_capture(thetis_batch &B) {
    batch_drop_graph(B);
    HIP_TRY(hipStreamBeginCapture(B.stream, hipStreamCaptureModeThreadLocal));
    for (int32_t k = 0; k < B.graph_epochs; ++k) batch_epoch_launches<P>(B);
    hipError_t e = hipStreamEndCapture(B.stream, &B.graph);
    if (e != hipSuccess) { B.graph = nullptr; return fail(THETIS_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e)); }
    HIP_TRY(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
    B.captured_widen = B.widen;
    B.captured_grid = B.grid_mult;
    B.captured_most = B.most_items;
    B.captured_strided = B.strided;
    B.captured_cols = B.cols;
    B.captured_window = B.window;
    B.captured_epochs = B.graph_epochs;
    return THETIS_OK;
}

template <class P>
thetis_status batch_run_impl(thetis_batch &B, int32_t max_epochs, double gap_tol, int32_t *done, int32_t *status,
                             double *ms_out) {
    for (thetis_solver *S : B.solvers) if (S) HIP_TRY(hipStreamSynchronize(S->stream));
    thetis_status st = batch_upload<P>(B, max_epochs, gap_tol);
    if (st) return st;
    int32_t refresh_min = 1 << 30, occupied = 0;
    for (thetis_solver *S : B.solvers)
        if (S) { refresh_min = std::min(refresh_min, S->p.refresh_every); ++occupied; }
    if (refresh_min == (1 << 30)) refresh_min = 1;
    // with a window, instances run in turns: enough epochs for every turn
    const bool windowed = B.window > 0 && B.window < occupied;
    const int64_t epochs = windowed ? (int64_t)max_epochs * (cdiv(occupied, B.window) + 1) : max_epochs;
    // One graph launch runs K epochs: the shortest refresh period (an
    // instance can only stop at a refresh), at most kGraphEpochs.  An
    // instance past its epoch cap or its stop is retired on the device, so
    // the epochs of the last launch beyond what it needs leave it unchanged.
    // A call that one launch would cover (a serving tick) replays a
    // one-epoch graph instead: there is nothing to overlap with the host's
    // check, and a K-epoch graph costs K times the capture whenever the slot
    // contents change.
    int64_t K = std::max<int64_t>(1, std::min<int64_t>((int64_t)refresh_min, kGraphEpochs));
    if (epochs <= K) K = 1;
    B.graph_epochs = (int32_t)K;
    if (!B.exec || B.captured_widen != B.widen || B.captured_grid != B.grid_mult || B.captured_strided != B.strided ||
        (B.grid_mult == 0 && B.captured_most != B.most_items) ||
        B.captured_cols != B.cols || B.captured_window != B.window || B.captured_epochs != B.graph_epochs) {
        st = batch_capture<P>(B);
        if (st) return st;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ms_out) {
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        HIP_TRY(hipEventRecord(e0, B.stream));
    }
    const int64_t launches = cdiv(epochs, K);
    const bool poll = gap_tol > 0.0 || windowed;
    // After each launch that passes a refresh epoch the count of instances
    // left is copied to pinned memory; the host reads it one launch later,
    // while the next launch runs, and stops once none is left.
    int64_t pending = -1;   // launch whose count is in flight
    for (int64_t g = 0; g < launches; ++g) {
        HIP_TRY(hipGraphLaunch(B.exec, B.stream));
        if (!poll || g + 1 >= launches) continue;
        if ((g + 1) * K / refresh_min == g * K / refresh_min) continue;   // no refresh in this launch
        if (pending >= 0) {
            HIP_TRY(hipEventSynchronize(B.poll_ev[pending & 1]));
            if (B.poll[pending & 1] == 0) break;
        }
        HIP_TRY(hipMemcpyAsync(B.poll + (g & 1), B.ctl + CTL_LEFT, 4, hipMemcpyDeviceToHost, B.stream));
        HIP_TRY(hipEventRecord(B.poll_ev[g & 1], B.stream));
        pending = g;
    }
    if (ms_out) {
        HIP_TRY(hipEventRecord(e1, B.stream));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        *ms_out = ms;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    std::vector<BInst<P>> bi(B.count);
    HIP_TRY(hipMemcpyAsync(bi.data(), B.bi, sizeof(BInst<P>) * B.count, hipMemcpyDeviceToHost, B.stream));
    HIP_TRY(hipStreamSynchronize(B.stream));
    bool diverged = false;
    for (int32_t i = 0; i < B.count; ++i) {
        if (status) status[i] = B.solvers[i] ? (bi[i].active ? 0 : bi[i].reason) : -1;
        if (!B.solvers[i]) { if (done) done[i] = 0; continue; }
        thetis_solver &S = *B.solvers[i];
        S.epoch = bi[i].epoch;
        const bool fresh = bi[i].epochs_done > 0 && (bi[i].epoch % S.p.refresh_every) == 0;
        if (bi[i].epochs_done > 0) {
            S.metrics_fresh = fresh;
            S.metrics_dual = fresh && gap_tol > 0.0;
            S.have_round = false;
        }
        if (done) done[i] = bi[i].epochs_done;
        diverged = diverged || bi[i].diverged;
    }
    if (diverged) return fail(THETIS_EDIVERGED, "NaN or Inf in an instance's refresh");
    return THETIS_OK;
}

#define BDISPATCH(B, CALL) \
    ((B).precision == THETIS_PREC_FP64 ? CALL<PF64> : ((B).precision == THETIS_PREC_BF16X ? CALL<PB16> : CALL<PF32>))

size_t binst_bytes(int32_t precision) {
    return precision == THETIS_PREC_FP64 ? sizeof(BInst<PF64>)
                                         : (precision == THETIS_PREC_BF16X ? sizeof(BInst<PB16>) : sizeof(BInst<PF32>));
}

}  // namespace

namespace {
thetis_status batch_check_solver(thetis_batch &B, const thetis_solver *S) {
    if (S->p.schedule != THETIS_SCHED_DET) return fail(THETIS_EINVAL, "batches run the DET schedule");
    if (S->p.precision != B.precision || (!S->unit_vals) != B.vals)
        return fail(THETIS_EINVAL, "batch solvers must share precision and matrix value kind");
    const int32_t vm = det_vmode(*S);
    if (B.vmode >= 0 && B.vmode != vm)
        return fail(THETIS_EINVAL, "batch solvers must share how their values are stored (all +-1 or general)");
    if (S->nclasses > kMaxBatchClasses) return fail(THETIS_EUNSUPPORTED, "batched instances need at most 64 colour classes");
    return THETIS_OK;
}

// shape signature for the tuner cache: slot count, entries and largest
// degree on a log2 scale, precision
void batch_signature(thetis_batch &B) {
    uint64_t sig = 1469598103934665603ULL;
    int64_t nnz_total = 0, maxdeg = 0;
    for (thetis_solver *S : B.solvers)
        if (S) { nnz_total += S->nnz; maxdeg = std::max<int64_t>(maxdeg, S->max_degree); }
    auto mix = [&](uint64_t v) { sig = (sig ^ v) * 1099511628211ULL; };
    mix((uint64_t)B.count);
    mix((uint64_t)(nnz_total > 0 ? 64 - __builtin_clzll((uint64_t)nnz_total) : 0));
    mix((uint64_t)(maxdeg > 0 ? 64 - __builtin_clzll((uint64_t)maxdeg) : 0));
    mix((uint64_t)B.precision);
    B.signature = sig;
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    auto it = tuned_choices().find(sig);
    if (it != tuned_choices().end()) {
        B.widen = it->second.widen;
        B.grid_mult = it->second.grid_mult;
        B.strided = it->second.strided;
        B.cols = it->second.cols;
    }
}
}  // namespace

extern "C" thetis_status thetis_batch_create(int32_t capacity, thetis_solver *const *solvers, int32_t precision,
                                             int32_t unit_values, void *stream, thetis_batch **out) {
    thetis_batch *Bp = nullptr;   // released by the handler below if the host side throws
    try {
        clear_error();
        if (!out || capacity < 1) return fail(THETIS_EINVAL, "need a capacity of at least one slot");
        *out = nullptr;
        if (precision != THETIS_PREC_FP32 && precision != THETIS_PREC_FP64 && precision != THETIS_PREC_BF16X)
            return fail(THETIS_EINVAL, "unknown precision");
        Bp = new (std::nothrow) thetis_batch;
        if (!Bp) return fail(THETIS_ENOMEM, "host allocation failed");
        thetis_batch &B = *Bp;
        B.count = capacity;
        B.precision = precision;
        B.vals = unit_values == 0;
        B.solvers.assign(capacity, nullptr);
        for (int32_t i = 0; solvers && i < capacity; ++i) {
            thetis_solver *S = solvers[i];
            if (!S) continue;
            thetis_status st = batch_check_solver(B, S);
            if (st) { delete Bp; return st; }
            B.solvers[i] = S;
            B.vmode = det_vmode(*S);
        }
        if (!B.vals) B.vmode = 0;
        B.stream = (hipStream_t)stream;
        if (!B.stream) {
            // stream capture needs a stream other than the null stream
            if (hipStreamCreateWithFlags(&B.stream, hipStreamNonBlocking) != hipSuccess) {
                delete Bp;
                return fail(THETIS_EDEVICE, "could not create the batch stream");
            }
            B.own_stream = true;
        }
        batch_signature(B);
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0) cus = prop.multiProcessorCount;
        }
        B.resident_wg = (int64_t)cus * 8;    // 8 workgroups of 256 threads per CU
        const int32_t count = capacity;
        const size_t nb = binst_bytes(B.precision);
        hipError_t e = hipMalloc(&B.bi, nb * count);
        if (e == hipSuccess) e = hipMalloc((void **)&B.rows_wg, 4 * count);
        if (e == hipSuccess) e = hipMalloc((void **)&B.dual_wg, 4 * count);
        if (e == hipSuccess) e = hipMalloc((void **)&B.alist, 4 * (size_t)count);
        if (e == hipSuccess) e = hipMalloc((void **)&B.ctl, 4 * CTL_N);
        if (e == hipSuccess) e = hipMalloc((void **)&B.order, (size_t)kMaxBatchClasses * count);
        if (e == hipSuccess) e = hipHostMalloc((void **)&B.poll, 8, hipHostMallocDefault);
        for (hipEvent_t &ev : B.poll_ev)
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            thetis_batch_destroy(Bp);
            return fail(THETIS_ENOMEM, "device allocation of the batch tables failed");
        }
        for (thetis_solver *S : B.solvers)
            if (S) S->batch_slots++;
        B.slots_counted = true;
        *out = Bp;
        return THETIS_OK;
    } catch (...) {
        const thetis_status st = exception_status();
        if (Bp) thetis_batch_destroy(Bp);
        return st;
    }
}

extern "C" thetis_status thetis_batch_set(thetis_batch *b, int32_t slot, thetis_solver *s) {
    try {
        clear_error();
        if (!b) return fail(THETIS_EINVAL, "batch is NULL");
        if (slot < 0 || slot >= b->count) return fail(THETIS_EINVAL, "slot out of range");
        if (s) {
            thetis_status st = batch_check_solver(*b, s);
            if (st) return st;
        }
        if (b->solvers[slot]) b->solvers[slot]->batch_slots--;
        if (s) s->batch_slots++;
        b->solvers[slot] = s;
        // the value storage the batch's sweeps read: that of its solvers
        b->vmode = b->vals ? -1 : 0;
        for (const thetis_solver *o : b->solvers)
            if (o) { b->vmode = det_vmode(*o); break; }
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_batch_run(thetis_batch *b, int32_t max_epochs, double gap_tol, int32_t *done,
                                          int32_t *status) {
    try {
        clear_error();
        if (!b) return fail(THETIS_EINVAL, "batch is NULL");
        if (max_epochs < 0) return fail(THETIS_EINVAL, "max_epochs < 0");
        if (max_epochs == 0) {
            for (int32_t i = 0; i < b->count; ++i) {
                if (done) done[i] = 0;
                if (status) status[i] = b->solvers[i] ? 0 : -1;
            }
            return THETIS_OK;
        }
        return BDISPATCH(*b, batch_run_impl)(*b, max_epochs, gap_tol, done, status, nullptr);
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_batch_configure(thetis_batch *b, int32_t widen, int32_t grid_mult, int32_t strided,
                                                int32_t cols) {
    try {
        clear_error();
        if (!b) return fail(THETIS_EINVAL, "batch is NULL");
        if (widen != 1 && widen != 2 && widen != 4) return fail(THETIS_EINVAL, "widen must be 1, 2 or 4");
        if (grid_mult != 0 && grid_mult != 1 && grid_mult != 2 && grid_mult != 4 && grid_mult != 8)
            return fail(THETIS_EINVAL, "grid multiplier must be 0 (one workgroup per item), 1, 2, 4 or 8");
        if (strided != 0 && strided != 1) return fail(THETIS_EINVAL, "strided must be 0 or 1");
        if (cols != 1 && cols != 2 && cols != 4) return fail(THETIS_EINVAL, "cols must be 1, 2 or 4");
        b->widen = widen;
        b->grid_mult = grid_mult;
        b->strided = strided;
        b->cols = cols;
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

namespace {
// one timed candidate: the first run after a capture includes the capture,
// so a second run is timed
thetis_status tune_time(thetis_batch &B, const Choice &c, int32_t epochs, double *ms) {
    B.widen = c.widen;
    B.grid_mult = c.grid_mult;
    B.strided = c.strided;
    B.cols = c.cols;
    thetis_status rc = BDISPATCH(B, batch_run_impl)(B, 1, 0.0, nullptr, nullptr, nullptr);
    if (rc) return rc;
    return BDISPATCH(B, batch_run_impl)(B, epochs, 0.0, nullptr, nullptr, ms);
}
}  // namespace

extern "C" thetis_status thetis_batch_autotune(thetis_batch *b, int32_t epochs_per_candidate, int32_t *choice) {
    try {
        clear_error();
        if (!b) return fail(THETIS_EINVAL, "batch is NULL");
        if (epochs_per_candidate < 1) return fail(THETIS_EINVAL, "epochs_per_candidate < 1");
        // two stages: the per-column shape (lanes and columns per group) at the
        // current grid, then the grid size and walk with the best shape
        const Choice shapes[4] = {{1, 0, 0, 1}, {2, 0, 0, 1}, {1, 0, 0, 2}, {1, 0, 0, 4}};
        Choice best{b->widen, b->grid_mult, b->strided, b->cols};
        double best_ms = 1e300;
        for (const Choice &sh : shapes) {
            const Choice c{sh.widen, best.grid_mult, best.strided, sh.cols};
            double ms = 0;
            thetis_status rc = tune_time(*b, c, epochs_per_candidate, &ms);
            if (rc) return rc;
            if (ms < best_ms) { best_ms = ms; best = c; }
        }
        const Choice base = best;
        for (int st = 0; st < 2; ++st)
            for (int g : {0, 1, 2, 4}) {
                const Choice c{base.widen, g, st, base.cols};
                if (g == base.grid_mult && st == base.strided) continue;
                double ms = 0;
                thetis_status rc = tune_time(*b, c, epochs_per_candidate, &ms);
                if (rc) return rc;
                if (ms < best_ms) { best_ms = ms; best = c; }
            }
        b->widen = best.widen;
        b->grid_mult = best.grid_mult;
        b->strided = best.strided;
        b->cols = best.cols;
        {
            std::lock_guard<std::mutex> lock(g_tuned_mu);
            tuned_choices()[b->signature] = best;
        }
        if (choice) { choice[0] = best.widen; choice[1] = best.grid_mult; choice[2] = best.strided; choice[3] = best.cols; }
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_batch_set_window(thetis_batch *b, int32_t window) {
    try {
        clear_error();
        if (!b) return fail(THETIS_EINVAL, "batch is NULL");
        if (window < 0) return fail(THETIS_EINVAL, "window must be >= 0");
        b->window = window;
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_batch_destroy(thetis_batch *b) {
    try {
        if (!b) return THETIS_OK;
        (void)hipStreamSynchronize(b->stream);
        if (b->slots_counted)
            for (thetis_solver *S : b->solvers)
                if (S) S->batch_slots--;
        batch_drop_graph(*b);
        for (hipEvent_t &ev : b->poll_ev)
            if (ev) (void)hipEventDestroy(ev);
        if (b->poll) (void)hipHostFree(b->poll);
        (void)hipFree(b->bi);
        if (b->bc) (void)hipFree(b->bc);
        (void)hipFree(b->rows_wg);
        (void)hipFree(b->dual_wg);
        (void)hipFree(b->alist);
        (void)hipFree(b->ctl);
        if (b->dirs) (void)hipFree(b->dirs);
        (void)hipFree(b->order);
        if (b->own_stream) (void)hipStreamDestroy(b->stream);
        delete b;
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}
