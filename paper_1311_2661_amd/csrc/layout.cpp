// Host-side instance layout of libthetis: validation, slack augmentation,
// the column-compressed copy of A, the update units and their greedy
// colouring into conflict-free classes, and the per-class work plan that
// the class-sweep kernels execute.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>

#include "thetis_internal.h"

namespace thetis {

static thread_local std::string g_last_error;

// recording the message never throws: if it cannot be stored it is dropped
thetis_status fail(thetis_status code, const char *msg) noexcept {
    try {
        g_last_error.assign(msg);
    } catch (...) {
        g_last_error.clear();
    }
    return code;
}
thetis_status fail(thetis_status code, const std::string &msg) noexcept { return fail(code, msg.c_str()); }
void clear_error() { g_last_error.clear(); }

thetis_status exception_status() {
    try {
        throw;
    } catch (const std::bad_alloc &) {
        return fail(THETIS_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        try {
            return fail(THETIS_EINVAL, std::string("host error: ") + e.what());
        } catch (...) {
            return fail(THETIS_EINVAL, "host error");
        }
    } catch (...) {
        return fail(THETIS_EINVAL, "unknown host error");
    }
}

// ------------------------------------------------------------------ Philox
void philox_host(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round) { k0 += Philox4x64::W0; k1 += Philox4x64::W1; }
        const unsigned __int128 p0 = (unsigned __int128)Philox4x64::M0 * x0;
        const unsigned __int128 p1 = (unsigned __int128)Philox4x64::M1 * x2;
        const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        x0 = hi1 ^ x1 ^ k0; x1 = lo1; x2 = hi0 ^ x3 ^ k1; x3 = lo0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

uint64_t philox_word_host(uint64_t seed, uint64_t stream, uint64_t c0, uint64_t c1, uint64_t c2) {
    const uint64_t ctr[4] = {c0, c1, c2, 0}, key[2] = {seed, stream};
    uint64_t out[4];
    philox_host(ctr, key, out);
    return out[0];
}

void class_order(int32_t nclasses, uint64_t seed, int64_t epoch, int32_t *order) {
    std::vector<std::pair<uint64_t, int32_t>> k(nclasses);
    for (int32_t c = 0; c < nclasses; ++c)
        k[c] = {philox_word_host(seed, RNG_CLASS_ORDER, (uint64_t)epoch, (uint64_t)c, 0), c};
    std::sort(k.begin(), k.end());
    for (int32_t c = 0; c < nclasses; ++c) order[c] = k[c].second;
}

// ------------------------------------------------------------------ layout

static void build_csc(Inst &in) {
    in.col_ptr.assign(in.n + 1, 0);
    for (int64_t e = 0; e < in.nnz; ++e) in.col_ptr[in.col_idx[e] + 1]++;
    for (int64_t j = 0; j < in.n; ++j) in.col_ptr[j + 1] += in.col_ptr[j];
    in.row_idx.resize(in.nnz);
    if (!in.unit_vals) in.cval.resize(in.nnz);
    std::vector<int32_t> fill(in.col_ptr.begin(), in.col_ptr.end() - 1);
    for (int64_t i = 0; i < in.m; ++i)
        for (int32_t e = in.row_ptr[i]; e < in.row_ptr[i + 1]; ++e) {
            const int32_t j = in.col_idx[e];
            in.row_idx[fill[j]] = (int32_t)i;
            if (!in.unit_vals) in.cval[fill[j]] = in.val[e];
            fill[j]++;
        }
    in.max_col_degree = 0;
    for (int64_t j = 0; j < in.n; ++j)
        in.max_col_degree = std::max<int64_t>(in.max_col_degree, in.col_ptr[j + 1] - in.col_ptr[j]);
}

// The slack units, one per inequality row in row order, after the
// structural units: all in one class after the structural classes.
static void list_slack_units(Inst &in) {
    in.ukind.resize(in.nstruct_units);
    in.uid.resize(in.nstruct_units);
    in.ucolour.resize(in.nstruct_units);
    bool any_slack = false;
    in.all_rows_slack = true;
    for (int64_t i = 0; i < in.m; ++i) {
        if (in.sense[i] != 0) {
            in.ukind.push_back(2); in.uid.push_back((int32_t)i); in.ucolour.push_back(in.nstruct_classes);
            any_slack = true;
        } else {
            in.all_rows_slack = false;
        }
    }
    in.nunits = (int64_t)in.ukind.size();
    in.nclasses = in.nstruct_classes + (any_slack ? 1 : 0);
}

// Units in unit order and a greedy colouring: unit t takes the smallest
// colour not held by an earlier unit that shares a row with it.  Slack
// units (one per inequality row) all go to one extra, last class: they
// touch one row each, all different.
static void colour_units(Inst &in) {
    const int64_t n = in.n;
    in.ukind.clear(); in.uid.clear(); in.ucolour.clear();
    std::vector<int32_t> unit_of_col(n, -1);
    for (int64_t j = 0; j < n; ++j) {
        const int32_t bl = in.nblocks ? in.col_block[j] : -1;
        if (bl >= 0) {
            if (in.fixed[bl] >= 0) continue;
            if (j == in.bfirst[bl]) { in.ukind.push_back(1); in.uid.push_back(bl); }
            unit_of_col[j] = (int32_t)in.ukind.size() - 1;
        } else {
            in.ukind.push_back(0); in.uid.push_back((int32_t)j);
            unit_of_col[j] = (int32_t)in.ukind.size() - 1;
        }
    }
    in.nstruct_units = (int64_t)in.ukind.size();
    in.ucolour.assign(in.nstruct_units, 0);
    std::vector<int64_t> stamp(64, -1);
    int32_t ncol = 0;
    for (int64_t t = 0; t < in.nstruct_units; ++t) {
        int64_t j0, j1;
        if (in.ukind[t] == 1) { j0 = in.bfirst[in.uid[t]]; j1 = j0 + in.k; }
        else { j0 = in.uid[t]; j1 = j0 + 1; }
        for (int64_t j = j0; j < j1; ++j)
            for (int32_t e = in.col_ptr[j]; e < in.col_ptr[j + 1]; ++e) {
                const int32_t i = in.row_idx[e];
                for (int32_t q = in.row_ptr[i]; q < in.row_ptr[i + 1]; ++q) {
                    const int32_t o = unit_of_col[in.col_idx[q]];
                    if (o >= 0 && o < t) stamp[in.ucolour[o]] = t;
                }
            }
        int32_t cc = 0;
        while (cc < (int32_t)stamp.size() && stamp[cc] == t) ++cc;
        if (cc == (int32_t)stamp.size()) stamp.resize(stamp.size() * 2, -1);
        in.ucolour[t] = cc;
        ncol = std::max(ncol, cc + 1);
    }
    in.nstruct_classes = ncol;
    list_slack_units(in);
}

static int32_t column_kind(int64_t d) {
    if (d >= kHubMinDegree) return SEG_HUB;
    for (int g = 0; g < kGroupKinds; ++g)
        if (d <= kGroupLanes[g]) return g;
    return SEG_HUB;
}

// Splits a list of units into per-kind segments (unit order kept inside
// each kind) appended to `sched`.
static ClassPlan plan_units(const Inst &in, const std::vector<int64_t> &units,
                            std::vector<int32_t> &sched) {
    ClassPlan cp;
    std::vector<std::vector<int32_t>> by(SEG_NKIND);
    for (int64_t t : units) {
        const int8_t kd = in.ukind[t];
        const int32_t id = in.uid[t];
        int32_t sk;
        if (kd == 2) sk = SEG_SLACK;
        else if (kd == 1) sk = SEG_BLOCK;
        else sk = column_kind(in.col_ptr[id + 1] - in.col_ptr[id]);
        by[sk].push_back(id);
    }
    for (int32_t sk = 0; sk < SEG_NKIND; ++sk) {
        if (by[sk].empty()) continue;
        Segment s;
        s.kind = sk;
        s.first = (int64_t)sched.size();
        s.count = (int64_t)by[sk].size();
        sched.insert(sched.end(), by[sk].begin(), by[sk].end());
        cp.segs.push_back(s);
    }
    return cp;
}

// the sign bit of a packed row index (values +-1, rows below 2^31)
static int32_t signed_row(int32_t row, double val) { return val < 0 ? (int32_t)((uint32_t)row | 0x80000000u) : row; }

static void pack_blocks(Inst &in) {
    PackedBlocks &pb = in.pb_det;
    pb = PackedBlocks();
    if (!in.nblocks) return;
    pb.ptr.push_back(0);
    for (ClassPlan &cp : in.classes)
        for (Segment &sg : cp.segs) {
            if (sg.kind != SEG_BLOCK) continue;
            sg.pb_first = (int64_t)pb.id.size();
            for (int64_t q = 0; q < sg.count; ++q) {
                const int32_t bl = in.sched[sg.first + q];
                pb.id.push_back(bl);
                pb.j0.push_back(in.bfirst[bl]);
                for (int32_t i = 0; i < in.k; ++i) {
                    const int32_t j = in.bfirst[bl] + i;
                    for (int32_t e = in.col_ptr[j]; e < in.col_ptr[j + 1]; ++e) {
                        if (in.sign_vals) pb.row.push_back(signed_row(in.row_idx[e], in.cval[e]));
                        else {
                            pb.row.push_back(in.row_idx[e]);
                            if (!in.unit_vals) pb.val.push_back(in.cval[e]);
                        }
                    }
                    pb.ptr.push_back((int32_t)pb.row.size());
                }
            }
        }
}

// Packs the plain columns' entries in schedule order.  With `pad`, every
// column of a lane-group segment takes exactly its group width of slots
// (the unused ones hold kNoRow), so a lane finds its entry from the
// column's plan position alone, and the segment records its base and stride.
static void pack(const Inst &in, const std::vector<int32_t> &sched,
                 const std::vector<ClassPlan *> &plans, Packed &pk, bool signs, bool pad) {
    std::vector<int32_t> slots(sched.size(), -1);   // -1: not a plain column; else slots taken
    for (const ClassPlan *cp : plans)
        for (const Segment &sg : cp->segs)
            if (sg.kind < kGroupKinds || sg.kind == SEG_HUB)
                for (int64_t q = 0; q < sg.count; ++q)
                    slots[sg.first + q] = pad && sg.kind < kGroupKinds ? kGroupLanes[sg.kind] : 0;
    pk.ptr.assign(sched.size() + 1, 0);
    for (size_t q = 0; q < sched.size(); ++q) {
        const int32_t j = sched[q];
        const int32_t d = slots[q] < 0 ? 0 : in.col_ptr[j + 1] - in.col_ptr[j];
        pk.ptr[q + 1] = pk.ptr[q] + std::max(d, slots[q]);
    }
    pk.row.assign(pk.ptr.back(), kNoRow);
    pk.val.clear();
    const bool vals = !in.unit_vals && !signs;
    if (vals) pk.val.assign(pk.ptr.back(), 0.0);
    for (size_t q = 0; q < sched.size(); ++q) {
        if (slots[q] < 0) continue;
        const int32_t j = sched[q];
        int32_t w = pk.ptr[q];
        for (int32_t e = in.col_ptr[j]; e < in.col_ptr[j + 1]; ++e, ++w) {
            pk.row[w] = signs ? signed_row(in.row_idx[e], in.cval[e]) : in.row_idx[e];
            if (vals) pk.val[w] = in.cval[e];
        }
    }
    for (ClassPlan *cp : plans)
        for (Segment &sg : cp->segs) {
            sg.ebase = 0;
            sg.stride = 0;
            if (pad && sg.kind < kGroupKinds && sg.count) {
                sg.ebase = pk.ptr[sg.first];
                sg.stride = kGroupLanes[sg.kind];
            }
        }
}

// Orders the plain columns inside every (class, segment, XCD part) of the
// DET plan, class by class, by the owner position of their first foreign
// row (a row's owner is its first unit in schedule order, its foreign unit
// the second).  The row layout keeps a window's rows in owner order, so
// columns next to each other in a wavefront then reach neighbouring rows of
// their window: their random accesses share cache lines.  Ties -- above all
// the columns with no foreign row, such as the whole first class -- go by
// the windows their owned rows fall in (the smallest three window ids), so
// neighbouring owners write into the same few windows.  Only the order
// inside a part changes (not the classes, not the parts), and a DET class's
// result does not depend on the order of its columns.
static void order_parts_by_window(Inst &in) {
    if (in.nblocks) return;
    const int64_t n = in.n, m = in.m;
    const int32_t none = INT32_MAX;
    std::vector<int32_t> pos(n, none), win(n, 0);   // win: 1 + class * kXcds + XCD part
    for (int32_t c = 0; c < (int32_t)in.classes.size(); ++c)
        for (const Segment &sg : in.classes[c].segs) {
            if (sg.kind == SEG_SLACK || sg.kind == SEG_BLOCK) continue;
            for (int64_t q = 0; q < sg.count; ++q) {
                const int32_t j = in.sched[sg.first + q];
                pos[j] = (int32_t)(sg.first + q);
                win[j] = 1 + c * kXcds + xcd_part(q, sg.count);
            }
        }
    // the row's second unit in schedule order stays its second: classes come
    // in schedule order and reordering inside a class keeps the class
    std::vector<int32_t> first_of(m, -1), second_of(m, -1);
    for (int64_t i = 0; i < m; ++i) {
        int32_t b = none, s2 = none, bj = -1, sj = -1;
        for (int32_t e = in.row_ptr[i]; e < in.row_ptr[i + 1]; ++e) {
            const int32_t j = in.col_idx[e], pj = pos[j];
            if (pj < b) { s2 = b; sj = bj; b = pj; bj = j; }
            else if (pj < s2) { s2 = pj; sj = j; }
        }
        first_of[i] = bj;
        second_of[i] = s2 < none ? sj : -1;
    }
    // the windows a column's owned rows fall in: the smallest three ids
    // (10 bits each), a key that groups owners writing to the same windows
    std::vector<int64_t> own_key(n, 0);
    for (int64_t j = 0; j < n; ++j) {
        int32_t w3[3] = {INT32_MAX, INT32_MAX, INT32_MAX};
        for (int32_t e = in.col_ptr[j]; e < in.col_ptr[j + 1]; ++e) {
            const int32_t i = in.row_idx[e];
            if (first_of[i] != j || second_of[i] < 0) continue;
            int32_t w = std::min<int32_t>(win[second_of[i]], 1023);
            for (int t = 0; t < 3; ++t)
                if (w < w3[t]) std::swap(w, w3[t]);
        }
        int64_t k = 0;
        for (int t = 0; t < 3; ++t) k = (k << 10) | (w3[t] == INT32_MAX ? 1023 : w3[t]);
        own_key[j] = k;
    }
    std::vector<int64_t> key(n, INT64_MAX);
    std::vector<std::pair<std::pair<int64_t, int64_t>, int32_t>> buf;
    for (ClassPlan &cp : in.classes) {
        // owners of this class's foreign rows are in earlier classes: final
        for (const Segment &sg : cp.segs)
            if (sg.kind != SEG_SLACK && sg.kind != SEG_BLOCK)
                for (int64_t q = 0; q < sg.count; ++q) key[in.sched[sg.first + q]] = INT64_MAX;
        for (const Segment &sg : cp.segs) {
            if (sg.kind == SEG_SLACK || sg.kind == SEG_BLOCK) continue;
            for (int64_t q = 0; q < sg.count; ++q) {
                const int32_t v = in.sched[sg.first + q];
                for (int32_t e = in.col_ptr[v]; e < in.col_ptr[v + 1]; ++e) {
                    const int32_t i = in.row_idx[e];
                    if (second_of[i] == v) key[v] = std::min<int64_t>(key[v], pos[first_of[i]]);
                }
            }
        }
        for (const Segment &sg : cp.segs) {
            if (sg.kind == SEG_SLACK || sg.kind == SEG_BLOCK) continue;
            for (int32_t x = 0; x < kXcds; ++x) {
                const int64_t lo = sg.count * x / kXcds, hi = sg.count * (x + 1) / kXcds;
                buf.clear();
                for (int64_t q = lo; q < hi; ++q) {
                    const int32_t v = in.sched[sg.first + q];
                    buf.push_back({{key[v], own_key[v]}, v});
                }
                std::stable_sort(buf.begin(), buf.end(),
                                 [](const std::pair<std::pair<int64_t, int64_t>, int32_t> &a,
                                    const std::pair<std::pair<int64_t, int64_t>, int32_t> &b) {
                                     return a.first < b.first;
                                 });
                for (int64_t q = lo; q < hi; ++q) {
                    const int32_t v = buf[q - lo].second;
                    in.sched[sg.first + q] = v;
                    pos[v] = (int32_t)(sg.first + q);
                }
            }
        }
    }
}

// Renumbers the plain columns into DET plan order (instances without
// simplex blocks): the column at plan position q becomes column q, so the
// plan's ids are the identity and a class sweep reads x, c and the bounds of
// its columns in order.  The colouring was made in the caller's order and is
// carried over unit by unit (a plain column is its own unit), so the classes
// -- and every result -- do not change; entries keep their order inside each
// row.  Returns false when the order is already that one.
static bool renumber_cols(Inst &in) {
    const int64_t n = in.n;
    if (in.nblocks || in.nstruct_units != n) return false;
    std::vector<int32_t> nid(n, -1);
    int32_t next = 0;
    for (const ClassPlan &cp : in.classes)
        for (const Segment &sg : cp.segs) {
            if (sg.kind == SEG_SLACK) continue;
            if (sg.kind == SEG_BLOCK) return false;
            for (int64_t q = 0; q < sg.count; ++q) nid[in.sched[sg.first + q]] = next++;
        }
    if (next != n) return false;
    bool same = true;
    for (int64_t j = 0; j < n && same; ++j) same = nid[j] == j;
    if (same) return false;
    for (int32_t &j : in.col_idx) j = nid[j];
    std::vector<double> cc(n), uu(in.u.size());
    std::vector<int32_t> orig(n), colour(n);
    for (int64_t j = 0; j < n; ++j) {
        cc[nid[j]] = in.c[j];
        if (!uu.empty()) uu[nid[j]] = in.u[j];
        orig[nid[j]] = in.col_orig[j];
        colour[nid[j]] = in.ucolour[j];   // unit j is column j
    }
    in.c.swap(cc);
    if (!uu.empty()) in.u.swap(uu);
    in.col_orig.swap(orig);
    std::copy(colour.begin(), colour.end(), in.ucolour.begin());
    return true;
}

// Puts the columns back into the caller's order (before simplex blocks,
// which name columns by the caller's index, are set on an instance whose
// layout was built without them); a layout built on the renumbered columns
// is dropped and rebuilt on next use.
static void restore_cols(Inst &in) {
    if (in.col_orig.empty()) return;
    const int64_t n = in.n;
    bool ident = true;
    for (int64_t j = 0; j < n && ident; ++j) ident = in.col_orig[j] == j;
    if (!ident) {
        in.planned = false;
        for (int32_t &j : in.col_idx) j = in.col_orig[j];
        std::vector<double> cc(n), uu(in.u.size());
        for (int64_t j = 0; j < n; ++j) {
            cc[in.col_orig[j]] = in.c[j];
            if (!uu.empty()) uu[in.col_orig[j]] = in.u[j];
        }
        in.c.swap(cc);
        if (!uu.empty()) in.u.swap(uu);
    }
    for (int64_t j = 0; j < n; ++j) in.col_orig[j] = (int32_t)j;
}

// Renumbers the rows: every row goes to its owner, the structural unit of
// the row that comes first in the DET schedule (class by class, in plan
// order); rows are then numbered owner by owner, so the rows a class owns
// are one contiguous range walked in the order the class sweep visits its
// columns.  Rows without a free structural column go last.
//
// Without simplex blocks the rows are further grouped by their first
// foreign unit (the row's second unit in schedule order): first by its
// class, then by the XCD part of its segment that runs it (xcd_part), owner
// order kept inside each group.  A class launch then reaches its foreign
// rows at random only inside the group of each XCD, a window of about
// (rows of the class) / 8 that stays in that XCD's L2 for the whole launch,
// while the owners still walk their rows in order (one sequential stream
// per group).  Results do not depend on the row order.  Returns false when
// the order is already the chosen one.
static bool renumber_rows(Inst &in) {
    const int64_t n = in.n, m = in.m;
    const int32_t none = (int32_t)in.sched.size();  // positions are below n + m < 2^31
    std::vector<int32_t> pos(n, none);          // schedule position of a column's unit
    const bool windows = in.nblocks == 0;
    std::vector<int32_t> grp(windows ? n : 0, 0);   // 1 + class * kXcds + XCD part
    for (int32_t c = 0; c < (int32_t)in.classes.size(); ++c)
        for (const Segment &sg : in.classes[c].segs) {
            if (sg.kind == SEG_SLACK) continue;
            for (int64_t q = 0; q < sg.count; ++q) {
                const int32_t id = in.sched[sg.first + q];
                const int64_t at = sg.first + q;
                if (sg.kind == SEG_BLOCK)
                    for (int32_t i = 0; i < in.k; ++i) pos[in.bfirst[id] + i] = (int32_t)at;
                else {
                    pos[id] = (int32_t)at;
                    if (windows) grp[id] = 1 + c * kXcds + xcd_part(q, sg.count);
                }
            }
        }
    // owner position of every row, then a stable counting sort by it
    std::vector<int32_t> key(m), at((size_t)none + 2, 0), order(m);
    std::vector<int32_t> fgrp(windows ? m : 0, 0);
    for (int64_t i = 0; i < m; ++i) {
        int32_t best = none, second = none;
        int32_t bcol = -1, scol = -1;
        for (int32_t e = in.row_ptr[i]; e < in.row_ptr[i + 1]; ++e) {
            const int32_t j = in.col_idx[e], pj = pos[j];
            if (pj < best) { second = best; scol = bcol; best = pj; bcol = j; }
            else if (pj < second) { second = pj; scol = j; }
        }
        key[i] = best;
        at[(size_t)best + 1]++;
        if (windows && second < none) fgrp[i] = grp[scol];
    }
    for (size_t q = 1; q < at.size(); ++q) at[q] += at[q - 1];
    for (int64_t i = 0; i < m; ++i) order[at[key[i]]++] = (int32_t)i;
    if (windows) {
        // stable by group: owner order kept inside every group
        const size_t ng = 1 + (size_t)in.classes.size() * kXcds;
        std::vector<int64_t> cnt(ng + 1, 0);
        for (int64_t i = 0; i < m; ++i) cnt[(size_t)fgrp[i] + 1]++;
        for (size_t g = 1; g <= ng; ++g) cnt[g] += cnt[g - 1];
        std::vector<int32_t> by(m);
        for (int64_t r = 0; r < m; ++r) by[cnt[fgrp[order[r]]]++] = order[r];
        order.swap(by);
    }
    bool same = true;
    for (int64_t r = 0; r < m && same; ++r) same = order[r] == r;
    if (same) return false;
    std::vector<int32_t> rp(m + 1, 0), ci(in.nnz);
    std::vector<double> vv(in.unit_vals ? 0 : in.nnz), bb(m);
    std::vector<int8_t> ss(m);
    std::vector<int32_t> orig(m);
    for (int64_t r = 0; r < m; ++r) {
        const int32_t o = order[r];
        const int32_t len = in.row_ptr[o + 1] - in.row_ptr[o];
        rp[r + 1] = rp[r] + len;
        std::copy(in.col_idx.begin() + in.row_ptr[o], in.col_idx.begin() + in.row_ptr[o + 1], ci.begin() + rp[r]);
        if (!in.unit_vals) std::copy(in.val.begin() + in.row_ptr[o], in.val.begin() + in.row_ptr[o + 1], vv.begin() + rp[r]);
        bb[r] = in.b[o];
        ss[r] = in.sense[o];
        orig[r] = in.row_orig.empty() ? o : in.row_orig[o];
    }
    in.row_ptr.swap(rp);
    in.col_idx.swap(ci);
    if (!in.unit_vals) in.val.swap(vv);
    in.b.swap(bb);
    in.sense.swap(ss);
    in.row_orig.swap(orig);
    return true;
}

// The DET sweeps update the residual with plain read-modify-writes, which is
// race-free only because the units of one class touch pairwise-disjoint
// rows.  Checked here on the final plans, independently of how the colouring
// was made: every row is touched at most once per class.
static bool classes_row_disjoint(const Inst &in) {
    std::vector<int32_t> stamp(in.m, -1);
    for (int32_t c = 0; c < in.nclasses; ++c)
        for (const Segment &sg : in.classes[c].segs)
            for (int64_t q = 0; q < sg.count; ++q) {
                const int32_t id = in.sched[sg.first + q];
                if (sg.kind == SEG_SLACK) {
                    if (stamp[id] == c) return false;
                    stamp[id] = c;
                    continue;
                }
                const int32_t j0 = sg.kind == SEG_BLOCK ? in.bfirst[id] : id;
                const int32_t j1 = sg.kind == SEG_BLOCK ? j0 + in.k : j0 + 1;
                for (int32_t j = j0; j < j1; ++j)
                    for (int32_t e = in.col_ptr[j]; e < in.col_ptr[j + 1]; ++e) {
                        const int32_t i = in.row_idx[e];
                        if (stamp[i] == c) return false;
                        stamp[i] = c;
                    }
            }
    return true;
}

// the DET plan: the units of every class split into segment kinds
static void plan_classes(Inst &in) {
    in.sched.clear();
    in.classes.assign(in.nclasses, ClassPlan());
    std::vector<std::vector<int64_t>> members(in.nclasses);
    for (int64_t t = 0; t < in.nunits; ++t) members[in.ucolour[t]].push_back(t);
    for (int32_t c = 0; c < in.nclasses; ++c) in.classes[c] = plan_units(in, members[c], in.sched);
}

// Shapes for the general roundings and q(P) of the covering lemma
// (Appendix C): over the rows with b_j > 0, the least b_j - A_j x among
// binary x with A_j x < b_j, i.e. b_j minus the largest subset sum of the
// row's entries below b_j, found with a bitset of the reachable sums.  Rows
// with b_j above 2^24 take the lower bound 1 (valid for integer data).
static void rounding_facts(Inst &in) {
    in.max_row_len = 0;
    for (int64_t i = 0; i < in.m; ++i)
        in.max_row_len = std::max<int64_t>(in.max_row_len, in.row_ptr[i + 1] - in.row_ptr[i]);
    bool binary = in.nblocks == 0;
    for (int64_t j = 0; j < in.n && binary; ++j) binary = in.u[j] == 1.0;
    auto entry = [&](int64_t e) { return in.unit_vals ? 1.0 : in.val[e]; };
    bool cover = binary, setc = binary, pack = binary;
    for (int64_t i = 0; i < in.m; ++i) {
        const double bi = in.b[i];
        if (in.sense[i] != 1 || bi != std::floor(bi)) cover = false;
        if (in.sense[i] != 1 || bi != 1.0) setc = false;
        if (in.sense[i] != -1 || !(bi > 0.0)) pack = false;
        for (int32_t e = in.row_ptr[i]; e < in.row_ptr[i + 1]; ++e) {
            const double v = entry(e);
            if (v < 0.0) { cover = false; setc = false; pack = false; }
            if (v != std::floor(v)) cover = false;
            if (v != 1.0) setc = false;
        }
    }
    in.cover_int = cover;
    in.set_cover = cover && setc;
    in.packing = pack;
    in.cover_q = INFINITY;
    if (!cover) return;
    std::vector<uint64_t> bits;
    for (int64_t i = 0; i < in.m; ++i) {
        const double bi = in.b[i];
        if (bi <= 0.0) continue;
        if (bi > 16777216.0) { in.cover_q = std::min(in.cover_q, 1.0); continue; }
        const int64_t B = (int64_t)bi, W = (B + 63) / 64;
        bits.assign(W, 0);
        bits[0] = 1;
        for (int32_t e = in.row_ptr[i]; e < in.row_ptr[i + 1]; ++e) {
            const int64_t a = (int64_t)entry(e);
            if (a <= 0 || a >= B) continue;
            // bits |= bits << a, high words first so every source word is old
            const int64_t ws = a / 64, bs = a % 64;
            for (int64_t w = W - 1; w >= ws; --w) {
                uint64_t v = bits[w - ws] << bs;
                if (bs && w - ws - 1 >= 0) v |= bits[w - ws - 1] >> (64 - bs);
                bits[w] |= v;
            }
            if (B % 64) bits[W - 1] &= (uint64_t(1) << (B % 64)) - 1;
        }
        int64_t top = 0;
        for (int64_t w = W - 1; w >= 0; --w)
            if (bits[w]) { top = 64 * w + 63 - __builtin_clzll(bits[w]); break; }
        in.cover_q = std::min(in.cover_q, bi - (double)top);
    }
}

thetis_status build_layout(Inst &in) {
    try {
        rounding_facts(in);
        in.sign_vals = !in.unit_vals;
        for (size_t e = 0; e < in.val.size() && in.sign_vals; ++e) in.sign_vals = in.val[e] == 1.0 || in.val[e] == -1.0;
        if (in.row_orig.empty()) {
            in.row_orig.resize(in.m);
            for (int64_t i = 0; i < in.m; ++i) in.row_orig[i] = (int32_t)i;
        }
        if (in.col_orig.empty()) {
            in.col_orig.resize(in.n);
            for (int64_t j = 0; j < in.n; ++j) in.col_orig[j] = (int32_t)j;
        }
        // colour in the caller's column order (the classes are part of the
        // method's schedule), then lay the columns out in plan order
        restore_cols(in);
        build_csc(in);
        colour_units(in);
        plan_classes(in);
        order_parts_by_window(in);
        if (renumber_cols(in)) {
            build_csc(in);
            plan_classes(in);
        }
        // the colouring does not depend on the row order: after the
        // renumbering only the column copy, the slack units (listed in row
        // order) and the plans are redone
        if (renumber_rows(in)) {
            build_csc(in);
            list_slack_units(in);
            plan_classes(in);
        }
        in.async_sched.clear();
        std::vector<int64_t> st, sl;
        for (int64_t t = 0; t < in.nunits; ++t) (in.ukind[t] == 2 ? sl : st).push_back(t);
        in.async_struct = plan_units(in, st, in.async_sched);
        in.async_slack = plan_units(in, sl, in.async_sched);
        pack_blocks(in);
        std::vector<ClassPlan *> det;
        for (ClassPlan &cp : in.classes) det.push_back(&cp);
        pack(in, in.sched, det, in.pk_det, in.sign_vals, true);
        pack(in, in.async_sched, {&in.async_struct, &in.async_slack}, in.pk_async, false, false);
        if (!classes_row_disjoint(in))
            return fail(THETIS_EINVAL, "internal: two units of one colour class share a row");
        in.planned = true;
    } catch (const std::bad_alloc &) {
        return fail(THETIS_ENOMEM, "host allocation failed while building the layout");
    }
    return THETIS_OK;
}

}  // namespace thetis

using namespace thetis;

thetis_status thetis::ensure_layout(const thetis_inst *hc) {
    thetis_inst *h = const_cast<thetis_inst *>(hc);
    std::lock_guard<std::mutex> lock(h->layout_mu);
    return h->in.planned ? THETIS_OK : build_layout(h->in);
}

// ------------------------------------------------------------------ C ABI

namespace {

// Word-wise multiply-xorshift digest (not cryptographic): it tells one
// instance from another, so a checkpoint cannot be loaded into a solver of a
// different LP with the same sizes.
uint64_t digest_bytes(uint64_t h, const void *p, size_t bytes) {
    const unsigned char *q = (const unsigned char *)p;
    auto step = [&h](uint64_t w) {
        h ^= w;
        h *= 0x9E3779B97F4A7C15ULL;
        h ^= h >> 29;
    };
    size_t i = 0;
    for (; i + 8 <= bytes; i += 8) {
        uint64_t w;
        std::memcpy(&w, q + i, 8);
        step(w);
    }
    uint64_t tail = 0;
    std::memcpy(&tail, q + i, bytes - i);
    step(tail ^ ((uint64_t)bytes << 56));
    return h;
}

template <class T>
uint64_t digest_vec(uint64_t h, const std::vector<T> &v) {
    const uint64_t len = v.size();
    h = digest_bytes(h, &len, sizeof(len));
    return v.empty() ? h : digest_bytes(h, v.data(), v.size() * sizeof(T));
}

uint64_t block_digest(const Inst &in) {
    uint64_t h = digest_bytes(in.lp_digest, &in.nblocks, sizeof(in.nblocks));
    h = digest_bytes(h, &in.k, sizeof(in.k));
    h = digest_vec(h, in.bfirst);
    return digest_vec(h, in.fixed);
}

}  // namespace

// the internal row and column orders: a checkpoint stores y and r in them,
// so it records this digest and is loaded only into the same layout
uint64_t thetis::layout_digest(const Inst &in) {
    uint64_t h = digest_vec(0x4C41594F55544F52ULL, in.row_orig);
    return digest_vec(h, in.col_orig);
}

extern "C" const char *thetis_last_error(void) { return g_last_error.c_str(); }

extern "C" thetis_status thetis_params_default(thetis_params *p) {
    try {
        if (!p) return fail(THETIS_EINVAL, "params is NULL");
        std::memset(p, 0, sizeof(*p));
        p->beta = 10.0;
        p->step_rule = THETIS_STEP_PER_COORD;
        p->step_scale = 1.0;
        p->prox = 0;
        p->schedule = THETIS_SCHED_DET;
        p->precision = THETIS_PREC_FP32;
        p->refresh_every = 5;
        p->seed = 0;
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_inst_create_csr(int64_t m, int64_t n, int64_t nnz,
                                                const int64_t *row_ptr, const int32_t *col_idx,
                                                const double *val, const double *b,
                                                const double *c, const double *u,
                                                const int8_t *sense, thetis_inst **out) {
    try {
        clear_error();
        if (!out) return fail(THETIS_EINVAL, "out is NULL");
        *out = nullptr;
        if (m < 0 || n < 0 || nnz < 0) return fail(THETIS_EINVAL, "negative size");
        if (nnz >= (int64_t(1) << 31) || n + m >= (int64_t(1) << 31))
            return fail(THETIS_EUNSUPPORTED, "nnz and n+m must stay below 2^31");
        if (!row_ptr || (nnz && !col_idx) || (m && !b) || (n && !c))
            return fail(THETIS_EINVAL, "missing array");
        if (row_ptr[0] != 0 || row_ptr[m] != nnz) return fail(THETIS_EINVAL, "row_ptr must run from 0 to nnz");
        thetis_inst *h = new (std::nothrow) thetis_inst;
        if (!h) return fail(THETIS_ENOMEM, "host allocation failed");
        Inst &in = h->in;
        try {
            in.m = m; in.n = n; in.nnz = nnz;
            in.row_ptr.resize(m + 1);
            for (int64_t i = 0; i <= m; ++i) {
                if (i && row_ptr[i] < row_ptr[i - 1]) { delete h; return fail(THETIS_EINVAL, "row_ptr decreases"); }
                in.row_ptr[i] = (int32_t)row_ptr[i];
            }
            in.col_idx.assign(col_idx, col_idx + nnz);
            std::vector<int64_t> seen(n, -1);
            for (int64_t i = 0; i < m; ++i)
                for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                    const int32_t j = col_idx[e];
                    if (j < 0 || j >= n) { delete h; return fail(THETIS_EINVAL, "column index out of range"); }
                    if (seen[j] == i) { delete h; return fail(THETIS_EINVAL, "column repeated inside a row"); }
                    seen[j] = i;
                }
            in.unit_vals = true;
            if (val) {
                for (int64_t e = 0; e < nnz; ++e) {
                    if (!std::isfinite(val[e])) { delete h; return fail(THETIS_EINVAL, "non-finite matrix entry"); }
                    if (val[e] != 1.0) in.unit_vals = false;
                }
                if (!in.unit_vals) in.val.assign(val, val + nnz);
            }
            in.b.assign(b, b + m);
            in.c.assign(c, c + n);
            for (int64_t i = 0; i < m; ++i)
                if (!std::isfinite(b[i])) { delete h; return fail(THETIS_EINVAL, "non-finite b"); }
            for (int64_t j = 0; j < n; ++j)
                if (!std::isfinite(c[j])) { delete h; return fail(THETIS_EINVAL, "non-finite c"); }
            in.u.assign(n, INFINITY);
            if (u) {
                for (int64_t j = 0; j < n; ++j) {
                    if (std::isnan(u[j]) || u[j] < 0) { delete h; return fail(THETIS_EINVAL, "upper bounds must be >= 0 or +inf"); }
                    in.u[j] = u[j];
                }
            }
            in.uniform_ub = true;
            in.ub_value = n ? in.u[0] : 1.0;
            for (int64_t j = 1; j < n; ++j) if (in.u[j] != in.ub_value) in.uniform_ub = false;
            in.sense.assign(m, 0);
            if (sense)
                for (int64_t i = 0; i < m; ++i) {
                    if (sense[i] < -1 || sense[i] > 1) { delete h; return fail(THETIS_EINVAL, "sense must be -1, 0 or +1"); }
                    in.sense[i] = sense[i];
                }
        } catch (const std::bad_alloc &) {
            delete h;
            return fail(THETIS_ENOMEM, "host allocation failed");
        }
        {
            const int64_t sizes[3] = {m, n, nnz};
            uint64_t d = digest_bytes(0x5448455449534C50ULL, sizes, sizeof(sizes));
            for (const auto *v : {&in.row_ptr, &in.col_idx}) d = digest_vec(d, *v);
            for (const auto *v : {&in.val, &in.b, &in.c, &in.u}) d = digest_vec(d, *v);
            in.lp_digest = digest_vec(d, in.sense);
            in.digest = block_digest(in);
        }
        in.planned = false;          // built on first use (blocks may still be set)
        *out = h;
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_inst_set_simplex_blocks(thetis_inst *h, int64_t nblocks, int32_t k,
                                                        const int64_t *first,
                                                        const int32_t *fixed_label) {
    try {
        clear_error();
        if (!h) return fail(THETIS_EINVAL, "instance is NULL");
        Inst &in = h->in;
        if (in.has_solver) return fail(THETIS_EBUSY, "blocks must be set before any solver is created");
        if (k < 1 || k > 64) return fail(THETIS_EUNSUPPORTED, "block size k must be in [1, 64]");
        // blocks name columns in the caller's order
        std::lock_guard<std::mutex> lock(h->layout_mu);
        restore_cols(in);
        if (nblocks < 0 || (nblocks && !first)) return fail(THETIS_EINVAL, "bad block list");
        std::vector<int32_t> cb(in.n, -1), bf(nblocks), fx(nblocks, -1);
        for (int64_t t = 0; t < nblocks; ++t) {
            if (first[t] < 0 || first[t] + k > in.n) return fail(THETIS_EINVAL, "block out of range");
            bf[t] = (int32_t)first[t];
            if (fixed_label) {
                if (fixed_label[t] < -1 || fixed_label[t] >= k) return fail(THETIS_EINVAL, "fixed label out of range");
                fx[t] = fixed_label[t];
            }
            for (int32_t i = 0; i < k; ++i) {
                if (cb[first[t] + i] != -1) return fail(THETIS_EINVAL, "blocks overlap");
                cb[first[t] + i] = (int32_t)t;
            }
        }
        for (int64_t t = 0; t < nblocks; ++t)
            for (int32_t i = 0; i < k; ++i)
                if (in.u[bf[t] + i] < 1.0)
                    return fail(THETIS_EINVAL, "simplex block columns need an upper bound of at least 1");
        // The columns of one block must not share a row.  Then the block of
        // A^T A is diagonal, its curvature bound is exact, and the block's
        // lanes scatter into distinct rows (a DET class writes each row once).
        std::vector<int64_t> stamp(nblocks, -1);
        for (int64_t i = 0; i < in.m; ++i)
            for (int32_t e = in.row_ptr[i]; e < in.row_ptr[i + 1]; ++e) {
                const int32_t t = cb[in.col_idx[e]];
                if (t < 0) continue;
                if (stamp[t] == i) return fail(THETIS_EINVAL, "two columns of one simplex block share a row");
                stamp[t] = i;
            }
        in.nblocks = nblocks; in.k = k;
        in.bfirst.swap(bf); in.fixed.swap(fx); in.col_block.swap(cb);
        in.digest = block_digest(in);
        in.planned = false;
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_inst_set_pairwise(thetis_inst *h, int64_t nfactors, const int32_t *ends,
                                                  const int64_t *first_col) {
    try {
        clear_error();
        if (!h) return fail(THETIS_EINVAL, "instance is NULL");
        Inst &in = h->in;
        if (in.has_solver) return fail(THETIS_EBUSY, "pairwise factors must be set before any solver is created");
        if (in.nblocks <= 0) return fail(THETIS_EINVAL, "pairwise factors need simplex blocks");
        if (nfactors < 0 || (nfactors && (!ends || !first_col))) return fail(THETIS_EINVAL, "bad factor list");
        const int64_t kk = (int64_t)in.k * in.k;
        std::vector<int32_t> pe(2 * nfactors), pf(nfactors);
        for (int64_t e = 0; e < nfactors; ++e) {
            for (int q = 0; q < 2; ++q) {
                if (ends[2 * e + q] < 0 || ends[2 * e + q] >= in.nblocks) return fail(THETIS_EINVAL, "factor end out of range");
                pe[2 * e + q] = ends[2 * e + q];
            }
            if (first_col[e] < 0 || first_col[e] + kk > in.n) return fail(THETIS_EINVAL, "factor columns out of range");
            for (int64_t j = first_col[e]; j < first_col[e] + kk; ++j)
                if (in.col_block[j] >= 0) return fail(THETIS_EINVAL, "factor columns inside a simplex block");
            pf[e] = (int32_t)first_col[e];
        }
        std::lock_guard<std::mutex> lock(h->layout_mu);
        in.npw = nfactors;
        in.pw_ends.swap(pe);
        in.pw_first.swap(pf);
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_inst_classes(const thetis_inst *h, int32_t *nclasses, int64_t *nunits,
                                             int32_t *class_host) {
    try {
        clear_error();
        if (!h) return fail(THETIS_EINVAL, "instance is NULL");
        thetis_status st = ensure_layout(h);
        if (st) return st;
        if (nclasses) *nclasses = h->in.nclasses;
        if (nunits) *nunits = h->in.nunits;
        if (class_host) {
            const Inst &in = h->in;
            std::copy(in.ucolour.begin(), in.ucolour.end(), class_host);
            // plain columns are their own units: back to the caller's order
            if (!in.nblocks && in.nstruct_units == in.n)
                for (int64_t j = 0; j < in.n; ++j) class_host[in.col_orig[j]] = in.ucolour[j];
        }
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_inst_rounding_shape(const thetis_inst *h, int32_t *flags, double *cover_q) {
    try {
        clear_error();
        if (!h) return fail(THETIS_EINVAL, "instance is NULL");
        thetis_status st = ensure_layout(h);
        if (st) return st;
        const Inst &in = h->in;
        if (flags)
            *flags = (in.cover_int ? THETIS_SHAPE_COVER : 0) | (in.set_cover ? THETIS_SHAPE_SET_COVER : 0) |
                     (in.packing ? THETIS_SHAPE_PACK : 0);
        if (cover_q) *cover_q = in.cover_int ? in.cover_q : 0.0;
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}

extern "C" thetis_status thetis_inst_destroy(thetis_inst *h) {
    try {
        delete h;
        return THETIS_OK;
    } catch (...) {
        return exception_status();
    }
}
