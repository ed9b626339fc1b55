// Internal declarations of libthetis shared by the host layout code
// (layout.cpp) and the HIP translation unit (thetis.hip).  Not installed.
#pragma once

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/thetis.h"

namespace thetis {

// error plumbing: every C entry point funnels failures through fail()
thetis_status fail(thetis_status code, const char *msg) noexcept;
thetis_status fail(thetis_status code, const std::string &msg) noexcept;
void clear_error();
// C++ exceptions never cross the C ABI: every entry point catches them and
// returns this (called inside a handler): THETIS_ENOMEM for a failed host
// allocation, THETIS_EINVAL with the message for anything else
thetis_status exception_status();

// Work kinds of the class sweep.  Plain columns are grouped by degree into
// lane groups of G lanes per column (G divides the 64-lane wavefront);
// columns above 64 entries get a whole 256-thread workgroup with the
// residual entries staged in LDS; simplex blocks get one wavefront each;
// slacks one lane each.
enum SegKind : int32_t {
    SEG_G2 = 0, SEG_G4, SEG_G8, SEG_G16, SEG_G32, SEG_G64,   // lane groups
    SEG_HUB,                                        // workgroup per column
    SEG_BLOCK,                                      // wavefront per simplex block
    SEG_SLACK,                                      // lane per slack row
    SEG_NKIND
};
constexpr int kGroupKinds = 6;
constexpr int kGroupLanes[kGroupKinds] = {2, 4, 8, 16, 32, 64};
constexpr int kWG = 256;              // threads per workgroup, every kernel
constexpr int kHubMinDegree = 65;     // columns with more entries go to SEG_HUB

// A solo class sweep splits every segment of its launch into kXcds
// contiguous parts, part x = [count x / kXcds, count (x + 1) / kXcds), and
// runs part x on workgroups b with b % kXcds == x, which the hardware
// dispatches round-robin to XCD x (each XCD has its own L2).  The row layout
// uses the same split to give each XCD the rows its columns reach at random.
constexpr int kXcds = 8;
inline int32_t xcd_part(int64_t i, int64_t count) {
    int32_t x = (int32_t)(i * kXcds / count);
    while (x + 1 < kXcds && count * (x + 1) / kXcds <= i) ++x;
    while (x > 0 && count * x / kXcds > i) --x;
    return x;
}

struct Segment {
    int32_t kind;
    int64_t first;   // offset into Inst::sched
    int64_t count;   // units in this segment
    int64_t pb_first = -1;   // SEG_BLOCK of the DET plan: first block in Inst::pb_det
    // lane-group segment of the DET plan: its columns' entries sit at a fixed
    // stride (the group width), entry l of the segment's i-th column at
    // ebase + i * stride + l, unused slots holding kNoRow; stride 0 = packed
    int64_t ebase = 0;
    int32_t stride = 0;
};
// an unused slot of a fixed-stride column (no row has this index)
constexpr int32_t kNoRow = 0x7fffffff;

struct ClassPlan {
    std::vector<Segment> segs;   // at most one segment per kind
};

// Column entries packed in schedule order: entry q of a schedule (a plain
// column of a hub or lane-group segment) owns row[ptr[q] .. ptr[q+1]);
// block and slack entries own empty ranges.  A class's columns are thus
// contiguous in memory and a lane group reads its indices coalesced.
struct Packed {
    std::vector<int32_t> ptr, row;
    std::vector<double> val;   // empty when every entry is 1
};

// The simplex blocks of the DET plan packed in plan order: block t is block
// id[t] with first column j0[t]; the entries of its column i are
// [ptr[t k + i], ptr[t k + i + 1]) of row / val, in column order.
struct PackedBlocks {
    std::vector<int32_t> id, j0, ptr, row;
    std::vector<double> val;   // empty when every entry is 1
};

// Host copy of an instance plus everything derived from it once.
struct Inst {
    int64_t m = 0, n = 0, nnz = 0;
    // CSR of A (structural columns only)
    std::vector<int32_t> row_ptr, col_idx;
    std::vector<double> val;            // empty: all entries are 1
    std::vector<double> b, c, u;
    std::vector<int8_t> sense;
    bool unit_vals = true;
    bool uniform_ub = true;             // every structural u_j equal
    double ub_value = 1.0;
    bool all_rows_slack = true;         // every row is an inequality
    // CSC of A
    std::vector<int32_t> col_ptr, row_idx;
    std::vector<double> cval;           // empty when unit_vals
    // simplex blocks
    int64_t nblocks = 0;
    int32_t k = 0;
    std::vector<int32_t> bfirst, fixed, col_block;   // col_block[j] = block or -1
    // update units, in unit order: free blocks and free columns (by first
    // column), then slack rows
    int64_t nunits = 0, nstruct_units = 0;
    std::vector<int8_t> ukind;          // 0 column, 1 block, 2 slack
    std::vector<int32_t> uid;           // column / block / row
    std::vector<int32_t> ucolour;
    int32_t nclasses = 0, nstruct_classes = 0;
    // DET schedule: units of each class, grouped by segment kind
    std::vector<int32_t> sched;
    std::vector<ClassPlan> classes;
    // ASYNC schedule: every structural unit (one "class"), then the slacks
    std::vector<int32_t> async_sched;
    ClassPlan async_struct, async_slack;
    Packed pk_det, pk_async;
    PackedBlocks pb_det;
    bool planned = false;
    bool has_solver = false;
    int64_t max_col_degree = 0;
    // shapes the general roundings need (binary columns, no blocks): every
    // row '>=' with non-negative integer entries and right-hand side
    // (covering), additionally all entries and right-hand sides 1 (set
    // cover), or every row '<=' with non-negative entries and b > 0
    // (packing); q(P) of the covering lemma; the longest row
    // pairwise factors of a MAP-inference LP (npw = -1: none declared):
    // factor e joins blocks pw_ends[2e], pw_ends[2e+1], its k*k columns
    // start at pw_first[e] (row-major in the two labels)
    int64_t npw = -1;
    std::vector<int32_t> pw_ends, pw_first;
    bool cover_int = false, set_cover = false, packing = false;
    double cover_q = 0.0;
    // every matrix value is +1 or -1 (and not all +1): the DET copies keep
    // the sign in the row index's top bit instead of a value array
    bool sign_vals = false;
    int64_t max_row_len = 0;
    // Internal row order: rows are renumbered so that every row's owner (its
    // first column in DET schedule order) sees its rows contiguously, class
    // by class.  row_orig[r] = caller's index of internal row r.
    std::vector<int32_t> row_orig;
    // Internal column order: without simplex blocks the columns are
    // renumbered into DET plan order (class by class, segment by segment),
    // so a class sweep reads its columns' data in order and a plain column's
    // id is its plan position.  col_orig[j] = caller's index of internal
    // column j (empty: the caller's order).
    std::vector<int32_t> col_orig;
    // 64-bit digest of the LP as given (sizes, matrix, b, c, u, senses) and
    // of the simplex blocks; a checkpoint records it and a load compares it
    uint64_t lp_digest = 0, digest = 0;
};

thetis_status build_layout(Inst &in);   // CSC, units, colouring, plans
uint64_t layout_digest(const Inst &in);  // digest of the internal row and column orders

// Philox4x64-10 (Salmon et al., SC'11), host and device.
struct Philox4x64 {
    static constexpr uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    static constexpr uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
};
enum : uint64_t { RNG_CLASS_ORDER = 1, RNG_ROUND = 4 };

void philox_host(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
uint64_t philox_word_host(uint64_t seed, uint64_t stream, uint64_t c0, uint64_t c1, uint64_t c2);
inline double unit53(uint64_t w) { return (double)(w >> 11) * (1.0 / 9007199254740992.0); }
// order of the classes in epoch e: sorted by (Philox word, class id)
void class_order(int32_t nclasses, uint64_t seed, int64_t epoch, int32_t *order);

}  // namespace thetis

struct thetis_inst {
    thetis::Inst in;
    std::mutex layout_mu;    // the layout is built once, on first use
};

namespace thetis {
// builds the instance's layout if it is not built yet (thread-safe)
thetis_status ensure_layout(const thetis_inst *h);
}
