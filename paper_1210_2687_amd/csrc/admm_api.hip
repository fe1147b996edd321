// admm_api.hip — host implementation of the C ABI declared in include/admm_deconv.h.
//
// A plan owns one device arena per batch holding, for every problem, the
// transposed half-spectrum ping-pong buffers, the kernel spectrum Lambda,
// the working duals, the mask and scratch planes (layout in admm_internal.h),
// plus shared twiddle tables, problem descriptors and work-item lists.
// solve/batch drive the iteration on the plan's stream: per iteration one
// column launch and the row launches of each regulariser family; every
// check_every iterations a reduction launch fills the per-problem residuals
// and the host reads the active flags to stop early.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/admm_deconv.h"
#include "admm_host.h"
#include "admm_internal.h"
#include "admm_launch.h"

using namespace admm;
using admm_host::fail;
using admm_host::make_key;
using admm_host::read_cache;
using admm_host::smooth7;
using admm_host::TuneEntry;
using admm_host::validate;
using admm_host::write_cache;
static_assert(admm_host::kRowClasses == ADMM_ROW_CLASSES, "tuning cache fields: one per row size class");

namespace {

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) {                                                                     \
            return fail(e_ == hipErrorOutOfMemory ? ADMM_E_NOMEM : ADMM_E_DEVICE, "%s failed: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                          \
        }                                                                                           \
    } while (0)

// Radix schedule: powers of two as radix 8 with a tail of 4 or 2, then 7, 5, 3
// (variant 0), or one of the alternatives of fft_schedule_variant.
int radices(int n, int* out, int cap, int variant = 0) {
    if (!smooth7(n)) return -1;
    return fft_schedule_variant(n, variant, out, cap);
}

// The variant a plan uses for a length-n transform: the requested one, unless
// it gives the same schedule as variant 0 or none at all (then 0, whose
// compile-time transforms serve the common lengths); radix 16 only in the row
// passes (wave-level column stages hold at most 8 operands per butterfly).
int effective_variant(int n, int variant, bool column) {
    if (variant <= 0 || variant >= FFT_VARIANTS || (column && variant == 3)) return 0;
    int a[ADMM_MAX_STAGES] = {}, b[ADMM_MAX_STAGES] = {};
    const int na = radices(n, a, ADMM_MAX_STAGES, variant);
    const int nb = radices(n, b, ADMM_MAX_STAGES, 0);
    if (na < 1) return 0;
    if (na == nb && std::equal(a, a + na, b)) return 0;
    return variant;
}

// Does a block of NT threads with MAXE registers per thread fit `ntrans`
// length-N transforms for every radix of the schedule?
bool fits(int ntrans, const FftPlanDev& f, int maxe, int nt = block_threads()) {
    for (int s = 0; s < f.nst; ++s) {
        const int R = f.rad[s];
        const long long bf = (long long)ntrans * (f.N / R);
        if ((bf + nt - 1) / nt > maxe / R) return false;
    }
    return true;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// The narrower-block launch of fused TV row class c (0..2) that takes problem
// d, or ADMM_RTV_SUBS for 512-thread blocks: the first whose threads cover the
// row at 2^c columns each and whose row transforms fit them at the class's
// most rows per block (so that the choice, and the rounding of the transforms,
// does not depend on the tile shape).
int rtv_sub_of(const ProbDesc& d, int c) {
    for (int t = 0; t < ADMM_RTV_SUBS; ++t) {
        const int nt = row_tv_sub_threads(c, t);
        if (nt > 0 && d.W <= (1 << c) * nt && fits(row_tv_max_rows(d.W) + 2, d.fr, row_maxe(d.W), nt)) return t;
    }
    return ADMM_RTV_SUBS;
}

// Plain row passes (frame problems, the CG and blur passes of TV problems) run
// rows of at most row_sub_threads() columns in blocks of that many threads
// when every stage of the row's schedule fits them at the class's most rows
// per block (again independent of the tile shape).
bool plain_narrow(const ProbDesc& d) {
    const int nt = row_sub_threads();
    return size_class(d.W) == 0 && d.W <= nt && fits(row_max_rows(d.W), d.fr, row_maxe(d.W), nt);
}

// tw_off: the length's slot in the table arrays (2 N entries: the natural
// twiddles exp(-2 pi i k / N), then the stage table)
void fill_plan(FftPlanDev& f, int N, int tw_off, int variant) {
    f.N = N;
    f.tw_off = tw_off;
    f.variant = variant;
    f.nst = radices(N, f.rad, ADMM_MAX_STAGES, variant);
    f.ends8 = f.nst >= 1 && f.rad[0] == 8 && f.rad[f.nst - 1] == 8;
    int Ns = 1, off = 0;
    for (int s = 0; s < f.nst; ++s) {
        const int R = f.rad[s];
        f.ns[s] = Ns;
        f.nbf[s] = N / R;
        f.tso[s] = off;
        f.mnbf[s] = div_magic((unsigned)f.nbf[s]);
        f.mns[s] = div_magic((unsigned)Ns);
        off += Ns * (R - 1);
        Ns *= R;
    }
}

// The stage table of length N (N - 1 entries) for a schedule variant, in
// double then rounded once.
void stage_twiddles(int N, int variant, float2* out) {
    int rad[ADMM_MAX_STAGES] = {};
    const int nst = radices(N, rad, ADMM_MAX_STAGES, variant);
    int Ns = 1, off = 0;
    for (int s = 0; s < nst; ++s) {
        const int R = rad[s];
        for (int k = 0; k < Ns; ++k)
            for (int r = 1; r < R; ++r) {
                const double ang = 2.0 * M_PI * (double)k * r / ((double)Ns * R);
                out[off + k * (R - 1) + r - 1] = make_float2((float)std::cos(ang), (float)-std::sin(ang));
            }
        off += Ns * (R - 1);
        Ns *= R;
    }
}

}  // namespace

// Tile shape forced on every problem of a plan (0 = the planner's heuristic):
// columns per column-pass block and rows per row-pass block.
struct TileChoice {
    int tc = 0, b = 0;
    int bc[ADMM_ROW_CLASSES] = {};   // rows per row block by size class of the row length (0: use b)
    int rsched = 0, csched = 0;   // radix schedule variants of the row and column transforms
};

constexpr int kPeriodsInFlight = 2;      // period graphs queued ahead of the host's stop test
constexpr int kPeriodIters = 40;         // iterations per period graph (whole check periods)
constexpr int kProfClasses = 7;          // kernel classes of the profiling totals

struct admm_plan {
    hipStream_t stream = nullptr;
    TileChoice tile;                      // what the plan was built with
    int count = 0;
    int method = METHOD_MD;               // shared by every problem of the plan
    std::vector<admm_problem> probs;      // copies (host pointers cleared)
    std::vector<ProbDesc> hd;             // host copy of the descriptors
    std::vector<int> col_beg, col_end, row_beg, row_end, frm_beg, frm_end;   // item ranges per problem
    int ncol = 0, nrowtv = 0, nrowfa = 0, nfrm = 0;
    int nrowtvs = 0;                      // TV row items of rows longer than 2048 (three-pass schedule)
    int ntv = 0, nfa = 0;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    // allocation-free plans (admm_deconv_solve_static): the arena is a region
    // the plan does not own, infos are staged in ordinary host memory, and
    // solves launch eagerly (no graphs, no events, no host-mapped flags)
    bool no_alloc = false;
    std::vector<InfoDev> h_info_host;
    ProbDesc* d_desc = nullptr;
    WorkItem* d_items = nullptr;
    InfoDev* d_info = nullptr;
    InfoDev* h_info = nullptr;            // pinned
    double* d_partials = nullptr;
    float2* d_tw = nullptr;
    float* d_s2 = nullptr;
    LaunchCtx all, tv, fa;
    LaunchCtx tvs;                        // TV rows longer than 2048 (three-pass schedule)
    // graph replay of plain iterations: executable per chunk length (even)
    hipStream_t cap_stream = nullptr;
    std::map<int, hipGraphExec_t> graphs;
    // graph replay of whole check periods (tolerance solves): executable per
    // (period, periods per graph, state export, tolerance bits of both rules); the iteration
    // counter they advance; active flags mirrored into host-mapped memory; one
    // event per graph in flight
    std::map<std::tuple<int, int, int, uint64_t, uint64_t>, hipGraphExec_t> pgraphs;
    int* d_kbase = nullptr;
    int* h_active = nullptr;
    int* h_active_dev = nullptr;
    hipEvent_t pev[kPeriodsInFlight] = {};
    // profiling: per-class totals of the last profiled run
    double prof_ms[kProfClasses] = {};
    int prof_n[kProfClasses] = {};
};

static const char* const kProfNames[kProfClasses] = {"col", "row_tv", "row_inv", "frame", "row_fwd", "reduce", "cg"};

namespace {

void penalties(const admm_problem& p, double* mu1, double* mu2) {
    double m2 = p.mu2 > 0 ? p.mu2 : 10.0 * p.lambda;
    double m1 = p.mu1 > 0 ? p.mu1 : std::min(1.0, 5000.0 * (p.mu2 > 0 ? p.mu2 : 10.0 * p.lambda));
    if (m2 <= 0) m2 = 1e-3;   // lambda == 0 with the heuristic: any positive penalty converges
    if (m1 <= 0) m1 = 1e-3;
    *mu1 = m1;
    *mu2 = m2;
}

}  // namespace

extern "C" const char* admm_last_error(void) { return admm_host::last_error(); }

extern "C" int32_t admm_fft_radices(int32_t n, int32_t* out, int32_t cap) {
    if (!out || cap <= 0) return -1;
    return radices(n, out, cap);
}

extern "C" int32_t admm_fft_schedule(int32_t n, int32_t variant, int32_t* out, int32_t cap) {
    if (!out || cap <= 0) return -1;
    return radices(n, out, cap, variant);
}

extern "C" admm_status admm_validate_problem(const admm_problem* prob) {
    if (!prob) return fail(ADMM_E_INVALID, "null problem");
    return validate(*prob);
}

extern "C" void admm_plan_destroy(admm_plan* P) {
    if (!P) return;
    for (auto& kv : P->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& kv : P->pgraphs) (void)hipGraphExecDestroy(kv.second);
    for (hipEvent_t e : P->pev)
        if (e) (void)hipEventDestroy(e);
    if (P->h_active) (void)hipHostFree(P->h_active);
    if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
    if (P->arena && !P->no_alloc) (void)hipFree(P->arena);
    if (P->h_info && !P->no_alloc) (void)hipHostFree(P->h_info);
    delete P;
}

static admm_status build_plan(admm_plan* P, const admm_problem* probs, int32_t count, void* hip_stream,
                              TileChoice tile, void* ext_arena = nullptr, size_t ext_cap = 0);

extern "C" admm_status admm_deconv_plan(const admm_problem* probs, int32_t count, void* hip_stream, admm_plan** out) {
    if (!out) return fail(ADMM_E_INVALID, "null output pointer");
    *out = nullptr;
    if (!probs || count < 1) return fail(ADMM_E_INVALID, "need at least one problem");
    for (int i = 0; i < count; ++i) {
        admm_status s = validate(probs[i]);
        if (s != ADMM_OK) {
            admm_host::prefix_error("problem " + std::to_string(i) + ": ");
            return s;
        }
    }
    admm_plan* P = new admm_plan();
    admm_status s = build_plan(P, probs, count, hip_stream, TileChoice{});
    if (s != ADMM_OK) {
        admm_plan_destroy(P);
        return s;
    }
    *out = P;
    return ADMM_OK;
}

// ext_arena (device memory of ext_cap bytes, not owned) replaces the plan's
// own allocation; the plan then allocates nothing on the device or pinned in
// host memory.
extern "C" admm_status admm_deconv_plan_with(const admm_problem* probs, int32_t count, void* hip_stream,
                                             const admm_tiles* tiles, admm_plan** out) {
    if (!out) return fail(ADMM_E_INVALID, "null output pointer");
    *out = nullptr;
    if (!probs || count < 1) return fail(ADMM_E_INVALID, "need at least one problem");
    if (!tiles) return fail(ADMM_E_INVALID, "null tile description");
    if (tiles->cols_per_block < 0 || tiles->rows_per_block < 0 || tiles->row_schedule < 0 ||
        tiles->row_schedule >= FFT_VARIANTS || tiles->col_schedule < 0 || tiles->col_schedule >= FFT_VARIANTS - 1)
        return fail(ADMM_E_INVALID, "tile counts must be >= 0, row schedule 0..%d, column schedule 0..%d",
                    FFT_VARIANTS - 1, FFT_VARIANTS - 2);
    for (int i = 0; i < count; ++i) {
        admm_status s = validate(probs[i]);
        if (s != ADMM_OK) {
            admm_host::prefix_error("problem " + std::to_string(i) + ": ");
            return s;
        }
    }
    TileChoice t;
    t.tc = tiles->cols_per_block;
    t.b = tiles->rows_per_block;
    t.rsched = tiles->row_schedule;
    t.csched = tiles->col_schedule;
    admm_plan* P = new admm_plan();
    admm_status s = build_plan(P, probs, count, hip_stream, t);
    if (s != ADMM_OK) {
        admm_plan_destroy(P);
        return s;
    }
    *out = P;
    return ADMM_OK;
}

static admm_status build_plan(admm_plan* P, const admm_problem* probs, int32_t count, void* hip_stream,
                              TileChoice tile, void* ext_arena, size_t ext_cap) {
    auto bail = [](admm_status s) { return s; };
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int lds_cap = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds_cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // the pass kernels may use the whole LDS of a compute unit; if the runtime
    // refuses, plan within the 64 KiB every device allows
    size_t cap = std::min<size_t>((size_t)lds_cap, 65536);
    if (lds_cap > 65536) {
        if (allow_dynamic_lds(lds_cap) == hipSuccess)
            cap = (size_t)lds_cap;
        else
            (void)hipGetLastError();
    }
    for (int i = 1; i < count; ++i)
        if (probs[i].method != probs[0].method)
            return bail(fail(ADMM_E_UNSUPPORTED, "problem %d: every problem of a plan needs the same method", i));
    P->method = probs[0].method == ADMM_METHOD_CG ? METHOD_CG : METHOD_MD;
    const bool cg = P->method == METHOD_CG;
    // the TV step (method CG, and TV rows longer than 2048) holds a little static
    // LDS (its block sums) beside the dynamic part: its own limit
    constexpr size_t kTvStepStatic = 1024;
    size_t tv_cap = 65536 - kTvStepStatic;
    if (lds_cap > 65536 && cap > 65536) {
        if (allow_dynamic_lds_cg((int)((size_t)lds_cap - kTvStepStatic)) == hipSuccess)
            tv_cap = (size_t)lds_cap - kTvStepStatic;
        else
            (void)hipGetLastError();
    }
    P->stream = (hipStream_t)hip_stream;
    P->count = count;
    P->probs.assign(probs, probs + count);
    P->hd.resize(count);

    // distinct (transform length, schedule variant) pairs -> table offsets
    std::map<std::pair<int, int>, int> tab_off;
    int tab_len = 0;
    auto slot = [&](int N, int v) {
        const auto key = std::make_pair(N, v);
        if (!tab_off.count(key)) {
            tab_off[key] = tab_len;
            tab_len += 2 * N;
        }
        return tab_off[key];
    };
    for (int i = 0; i < count; ++i) {
        slot(probs[i].W, effective_variant(probs[i].W, tile.rsched, false));
        slot(probs[i].H, effective_variant(probs[i].H, tile.csched, true));
        const int hs = probs[i].H / col_split_factor(probs[i].H);   // sub-transforms of split columns
        if (hs != probs[i].H) slot(hs, effective_variant(hs, tile.csched, true));
    }

    // about two blocks per compute unit per pass (measured best on 8 x 512^2: TC = 4,
    // B = 8; on one 512^2 problem: TC = 1, B = 2)
    const int target_blocks = 512;
    long long cols_total = 0;   // column transforms per pass over the batch
    for (int i = 0; i < count; ++i) cols_total += probs[i].W / 2 + 1;
    const int tc_batch = (int)std::max(1LL, std::min<long long>(col_max_tiles(), cols_total / target_blocks));
    for (int i = 0; i < count; ++i) {
        const admm_problem& q = probs[i];
        ProbDesc& d = P->hd[i];
        std::memset(&d, 0, sizeof d);
        d.H = q.H;
        d.W = q.W;
        d.P = q.W / 2 + 1;
        d.reg = q.reg;
        // both frame formulations plan as frame problems; fs selects the synthesis steps
        d.fs = q.reg == ADMM_REG_FRAME_SYNTHESIS;
        if (d.fs) d.reg = REG_FRAME;
        d.J = d.reg == REG_FRAME ? q.levels : 0;
        d.nb = d.reg == REG_FRAME ? 3 * q.levels + 1 : 2;
        double mu1, mu2;
        penalties(q, &mu1, &mu2);
        d.mu1 = (float)mu1;
        d.mu2 = (float)mu2;
        d.lam = (float)q.lambda;
        d.tau = (float)(q.lambda / mu2);
        d.inv_hw = (float)(1.0 / ((double)q.H * q.W));
        d.inv1pmu1 = (float)(1.0 / (1.0 + mu1));
        d.method = P->method;
        d.mut = q.reg == ADMM_REG_TV ? (float)mu1 : 1.0f;
        const int rv = effective_variant(q.W, tile.rsched, false), cv = effective_variant(q.H, tile.csched, true);
        fill_plan(d.fr, q.W, slot(q.W, rv), rv);
        fill_plan(d.fc, q.H, slot(q.H, cv), cv);
        d.csp = col_split_factor(q.H);
        if (d.csp > 1) {
            const int hs = q.H / d.csp, sv = effective_variant(hs, tile.csched, true);
            fill_plan(d.fc2, hs, slot(hs, sv), sv);
        }
        const int per = std::max(1, (target_blocks + count - 1) / count);
        // column tile: one column per wave of the column-pass block, as many as LDS holds
        int tcmax = 0;
        while (tcmax + 1 <= col_max_tiles() && lds_col_bytes(q.H, tcmax + 1) <= cap) ++tcmax;
        if (tcmax < 1)
            return bail(fail(ADMM_E_UNSUPPORTED, "problem %d: column length %d does not fit a block", i, q.H));
        d.TC = std::min(std::min(tcmax, tc_batch), d.P);
        if (tile.tc > 0) d.TC = std::min(d.TC, tile.tc);
        if (const char* e = std::getenv("ADMM_TC")) d.TC = std::max(1, std::min(d.TC, std::atoi(e)));
        if (q.H > 2048) {   // the block-level column pass: one column (or sub-transform) per block
            d.TC = 1;
            if (!fits(1, d.csp > 1 ? d.fc2 : d.fc, COL_BIG_MAXE, col_big_threads(q.H)))
                return bail(fail(ADMM_E_UNSUPPORTED, "problem %d: column schedule of length %d does not fit a block", i,
                                 q.H));
        }
        // rows per row-pass block
        int bmax = 0;
        const bool tv_split = q.reg == ADMM_REG_TV && q.W > 2048;   // three-pass TV schedule
        if (q.reg == ADMM_REG_TV && !tv_split) {
            while (bmax + 1 <= std::min(q.H, row_tv_max_rows(q.W)) && fits(bmax + 3, d.fr, row_maxe(q.W)) &&
                   lds_rowtv_bytes(q.W, bmax + 1) <= cap && (!cg || lds_tvstep_bytes(q.W, bmax + 1) <= tv_cap))
                ++bmax;
        } else if (tv_split) {
            while (bmax + 1 <= std::min(q.H, row_max_rows(q.W)) &&
                   fits(bmax + 1, d.fr, row_maxe(q.W), row_threads(q.W)) && lds_row_bytes(q.W, bmax + 1) <= cap &&
                   lds_tvstep_bytes(q.W, bmax + 1) <= tv_cap)
                ++bmax;
        } else {
            while (bmax + 1 <= std::min(q.H, row_max_rows(q.W)) &&
                   fits(bmax + 1, d.fr, row_maxe(q.W), row_threads(q.W)) && lds_row_bytes(q.W, bmax + 1) <= cap)
                ++bmax;
        }
        if (bmax < 1) return bail(fail(ADMM_E_UNSUPPORTED, "problem %d: row length %d does not fit a block", i, q.W));
        const int bmin = q.reg == ADMM_REG_TV && !tv_split ? std::min(bmax, 2) : 1;   // fused TV: halo rows cost (B + 2) / B
        d.B = std::max(bmin, std::min(bmax, (q.H + per - 1) / per));
        const int breq = tile.bc[size_class(q.W)] > 0 ? tile.bc[size_class(q.W)] : tile.b;
        if (breq > 0) d.B = std::min(bmax, breq);
        if (const char* e = std::getenv("ADMM_ROWS")) d.B = std::max(1, std::min(bmax, std::atoi(e)));
        d.nrowblk = (q.H + d.B - 1) / d.B;
        d.ncolblk = d.csp > 1 ? d.P * d.csp : (d.P + d.TC - 1) / d.TC;
        if (d.reg == REG_FRAME) {
            d.frm_tile = frame_tile(q.levels);
            d.nfrmblk = ((q.H + d.frm_tile - 1) / d.frm_tile) * ((q.W + d.frm_tile - 1) / d.frm_tile);
        }
    }

    // work items: problems in order of decreasing size (largest first), each problem's items contiguous
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (long long)P->hd[a].H * P->hd[a].W > (long long)P->hd[b].H * P->hd[b].W;
    });
    std::vector<WorkItem> col, rowtv, rowfa, frm;
    P->col_beg.assign(count, 0);
    P->col_end.assign(count, 0);
    P->row_beg.assign(count, 0);
    P->row_end.assign(count, 0);
    P->frm_beg.assign(count, 0);
    P->frm_end.assign(count, 0);
    // column items grouped by column class and TV row items by size class (each
    // class is one launch of its own instantiation), largest problems first
    // within a class
    int col_cb[ADMM_COL_CLASSES], col_cc[ADMM_COL_CLASSES], rtv_cb[ADMM_ROW_CLASSES], rtv_cc[ADMM_ROW_CLASSES];
    size_t lds_col_c[ADMM_COL_CLASSES] = {}, lds_rtv_c[ADMM_ROW_CLASSES] = {};
    for (int c = 0; c < ADMM_COL_CLASSES; ++c) {
        col_cb[c] = (int)col.size();
        for (int i : order) {
            ProbDesc& d = P->hd[i];
            if (col_class(d) != c) continue;
            P->col_beg[i] = (int)col.size();
            for (int b = 0; b < d.ncolblk; ++b)   // split columns: one item per (column, sub-transform)
                col.push_back(d.csp > 1 ? WorkItem{i, b / d.csp, b, b % d.csp} : WorkItem{i, b * d.TC, b, 0});
            P->col_end[i] = (int)col.size();
            lds_col_c[c] = std::max(lds_col_c[c], lds_col_bytes(d.H, d.TC));
        }
        col_cc[c] = (int)col.size() - col_cb[c];
    }
    // (classes 3 to 5, rows longer than 2048, take the three-pass TV schedule: no fused pass)
    // Within a fused class the problems of its narrower-block launches come first.
    int rtv_sub[3][ADMM_RTV_SUBS] = {};
    size_t lds_rtv_sub[3][ADMM_RTV_SUBS] = {};
    int tv_sub0 = 0, fa_sub0 = 0;   // leading class-0 items of the plain passes' narrower blocks
    size_t lds_tv_sub0 = 0, lds_fa_sub0 = 0;
    for (int c = 0; c < ADMM_ROW_CLASSES; ++c) {
        rtv_cb[c] = (int)rowtv.size();
        for (int t = 0; t <= ADMM_RTV_SUBS; ++t)
            for (int pass = 0; pass < 2; ++pass)   // the plain passes' narrower blocks first (a subset of t = 0)
            for (int i : order) {
                ProbDesc& d = P->hd[i];
                if (d.reg != REG_TV || size_class(d.W) != c || (c < 3 ? rtv_sub_of(d, c) : 0) != t) continue;
                const bool late = c == 0 && t == 0 && !plain_narrow(d);
                if (late != (pass == 1)) continue;
                if (c == 0 && t == 0 && !late) {
                    tv_sub0 += d.nrowblk;
                    lds_tv_sub0 = std::max(lds_tv_sub0, lds_row_bytes(d.W, d.B));
                }
                P->row_beg[i] = (int)rowtv.size();
                for (int b = 0; b < d.nrowblk; ++b) rowtv.push_back({i, b * d.B, b, 0});
                P->row_end[i] = (int)rowtv.size();
                if (c < 3 && t < ADMM_RTV_SUBS) {
                    rtv_sub[c][t] += d.nrowblk;
                    lds_rtv_sub[c][t] = std::max(lds_rtv_sub[c][t], lds_rowtv_bytes(d.W, d.B));
                } else if (c < 3) {
                    lds_rtv_c[c] = std::max(lds_rtv_c[c], lds_rowtv_bytes(d.W, d.B));
                }
            }
        rtv_cc[c] = (int)rowtv.size() - rtv_cb[c];
    }
    int part = 0;
    for (int i : order) {
        ProbDesc& d = P->hd[i];
        d.part_base = part;
        part += d.nrowblk + d.nfrmblk;
        if (d.reg == REG_TV)
            ++P->ntv;
        else
            ++P->nfa;
    }
    // frame items grouped by class (levels, small image), one launch per class
    int frm_cb[ADMM_FRAME_CLASSES], frm_cc[ADMM_FRAME_CLASSES];
    size_t lds_frm_c[ADMM_FRAME_CLASSES];
    for (int c = 0; c < ADMM_FRAME_CLASSES; ++c) {
        frm_cb[c] = (int)frm.size();
        lds_frm_c[c] = 0;
        for (int i : order) {
            const ProbDesc& d = P->hd[i];
            if (d.reg != REG_FRAME || frame_class(d.H, d.W, d.J, d.fs) != c) continue;
            P->frm_beg[i] = (int)frm.size();
            for (int b = 0; b < d.nfrmblk; ++b) frm.push_back({i, b, b, 0});
            P->frm_end[i] = (int)frm.size();
            lds_frm_c[c] = lds_frame_bytes(d.J);
        }
        frm_cc[c] = (int)frm.size() - frm_cb[c];
    }
    // FA row items grouped by size class of the row length, like the TV rows; the
    // plain row passes of each context use the classes of its own row items
    int rfa_cb[ADMM_ROW_CLASSES], rfa_cc[ADMM_ROW_CLASSES];
    size_t lds_rfa_c[ADMM_ROW_CLASSES] = {}, lds_rtvp_c[ADMM_ROW_CLASSES] = {};
    for (int c = 0; c < ADMM_ROW_CLASSES; ++c) {
        rfa_cb[c] = (int)rowfa.size();
        for (int pass = 0; pass < 2; ++pass)   // the narrower blocks' problems first
        for (int i : order) {
            const ProbDesc& d = P->hd[i];
            if (size_class(d.W) != c) continue;
            if ((c == 0 && !plain_narrow(d)) != (pass == 1)) continue;
            if (d.reg == REG_FRAME) {
                if (c == 0 && pass == 0) {
                    fa_sub0 += d.nrowblk;
                    lds_fa_sub0 = std::max(lds_fa_sub0, lds_row_bytes(d.W, d.B));
                }
                P->row_beg[i] = (int)rowfa.size();
                for (int b = 0; b < d.nrowblk; ++b) rowfa.push_back({i, b * d.B, b, 0});
                P->row_end[i] = (int)rowfa.size();
                lds_rfa_c[c] = std::max(lds_rfa_c[c], lds_row_bytes(d.W, d.B));
            } else {
                lds_rtvp_c[c] = std::max(lds_rtvp_c[c], lds_row_bytes(d.W, d.B));
            }
        }
        rfa_cc[c] = (int)rowfa.size() - rfa_cb[c];
    }
    P->ncol = (int)col.size();
    P->nrowtv = (int)rowtv.size();
    P->nrowtvs = 0;
    for (int c = 3; c < ADMM_ROW_CLASSES; ++c) P->nrowtvs += rtv_cc[c];
    P->nrowfa = (int)rowfa.size();
    P->nfrm = (int)frm.size();

    // arena layout
    std::vector<size_t> base(count);
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off += align256(b);
        return o;
    };
    const size_t o_desc = take(sizeof(ProbDesc) * count);
    const size_t nitems = col.size() + rowtv.size() + rowfa.size() + frm.size();
    const size_t o_items = take(sizeof(WorkItem) * nitems);
    const size_t o_info = take(sizeof(InfoDev) * count);
    const size_t o_kbase = take(sizeof(int));
    const size_t o_part = take(sizeof(double) * ADMM_NSUM * std::max(part, 1));
    const size_t o_cgpart = cg ? take(sizeof(double) * 2 * std::max(part, 1)) : 0;
    const size_t o_tw = take(sizeof(float2) * tab_len);
    const size_t o_s2 = take(sizeof(float) * tab_len);
    // row sums of the kernel spectrum (host-computed, consumed at plan time):
    // part of the arena when it is external, else a temporary allocation
    size_t t_bytes = 0;
    for (int i = 0; i < count; ++i)
        t_bytes = std::max(t_bytes, sizeof(float2) * (size_t)probs[i].ksize * (size_t)P->hd[i].P);
    const size_t o_T = ext_arena ? take(t_bytes) : 0;
    struct Offs {
        size_t spec0, spec1, lam, d1, dreg0, dreg1, u1p, uregp, tmpA, tmpB, zpl, mask;
        size_t cg[7];   // v, e, A e, O1, A O1, O2, A O2 (method CG)
    };
    std::vector<Offs> po(count);
    for (int i = 0; i < count; ++i) {
        const ProbDesc& d = P->hd[i];
        const size_t n = (size_t)d.H * d.W, hp = (size_t)d.H * d.P;
        Offs& o = po[i];
        o.spec0 = take(hp * sizeof(float4));
        const bool split = d.reg == REG_TV && d.W > 2048;   // three-pass TV: one spectrum, a z plane
        o.spec1 = d.reg == REG_TV && !split ? take(hp * sizeof(float4)) : o.spec0;
        o.lam = take(hp * sizeof(float2));
        o.d1 = take(n * sizeof(float));
        o.dreg0 = take(n * d.nb * sizeof(float));
        o.dreg1 = take(n * d.nb * sizeof(float));
        o.u1p = take(n * sizeof(float));
        o.uregp = take(n * d.nb * sizeof(float));
        o.tmpA = take(n * sizeof(float));
        o.tmpB = take(n * sizeof(float));
        o.zpl = d.reg == REG_FRAME || cg || split ? take(n * sizeof(float)) : o.tmpA;
        o.mask = take(n);
        for (int j = 0; j < 7; ++j) o.cg[j] = cg ? take(n * sizeof(float)) : 0;
    }
    P->arena_bytes = off;
    if (ext_arena) {
        if (off > ext_cap)
            return bail(fail(ADMM_E_UNSUPPORTED,
                             "the allocation-free solve holds at most %zu bytes of workspace; this problem needs %zu",
                             ext_cap, off));
        P->no_alloc = true;
        P->arena = (char*)ext_arena;
        P->h_info_host.assign(count, InfoDev{});
        P->h_info = P->h_info_host.data();
    } else {
        hipError_t e = hipMalloc((void**)&P->arena, off);
        if (e != hipSuccess) {
            P->arena = nullptr;
            (void)hipGetLastError();
            return bail(fail(e == hipErrorOutOfMemory ? ADMM_E_NOMEM : ADMM_E_DEVICE,
                             "device allocation of %zu bytes failed: %s", off, hipGetErrorString(e)));
        }
    }
    if (!P->no_alloc) {
        hipError_t e = hipHostMalloc((void**)&P->h_info, sizeof(InfoDev) * count, hipHostMallocDefault);
        if (e != hipSuccess) {
            P->h_info = nullptr;
            return bail(fail(ADMM_E_NOMEM, "pinned host allocation failed: %s", hipGetErrorString(e)));
        }
        e = hipHostMalloc((void**)&P->h_active, sizeof(int) * count, hipHostMallocMapped);
        if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&P->h_active_dev, P->h_active, 0);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return bail(fail(ADMM_E_NOMEM, "mapped host allocation failed: %s", hipGetErrorString(e)));
        }
    }
    char* A = P->arena;
    P->d_desc = (ProbDesc*)(A + o_desc);
    P->d_items = (WorkItem*)(A + o_items);
    P->d_info = (InfoDev*)(A + o_info);
    P->d_kbase = (int*)(A + o_kbase);
    P->d_partials = (double*)(A + o_part);
    P->d_tw = (float2*)(A + o_tw);
    P->d_s2 = (float*)(A + o_s2);
    for (int i = 0; i < count; ++i) {
        ProbDesc& d = P->hd[i];
        const Offs& o = po[i];
        d.spec0 = (float4*)(A + o.spec0);
        d.spec1 = (float4*)(A + o.spec1);
        d.lamhat = (float2*)(A + o.lam);
        d.d1 = (float*)(A + o.d1);
        d.dreg0 = (float*)(A + o.dreg0);
        d.dreg1 = (float*)(A + o.dreg1);
        d.u1p = (float*)(A + o.u1p);
        d.uregp = (float*)(A + o.uregp);
        d.tmpA = (float*)(A + o.tmpA);
        d.tmpB = (float*)(A + o.tmpB);
        d.zpl = (float*)(A + o.zpl);
        d.mask = (const uint8_t*)(A + o.mask);
        if (cg) {
            float** planes[7] = {&d.cgv, &d.cge, &d.cgae, &d.cgo1, &d.cgao1, &d.cgo2, &d.cgao2};
            for (int j = 0; j < 7; ++j) *planes[j] = (float*)(A + o.cg[j]);
        }
    }

    // twiddle and |Delta|^2 tables, in double then rounded once
    {
        std::vector<float2> tw(tab_len);
        std::vector<float> s2(tab_len);
        for (auto& kv : tab_off) {
            const int N = kv.first.first, v = kv.first.second, b = kv.second;
            for (int k = 0; k < N; ++k) {
                const double ang = 2.0 * M_PI * (double)k / (double)N;
                tw[b + k] = make_float2((float)std::cos(ang), (float)-std::sin(ang));
                const double sn = std::sin(M_PI * (double)k / (double)N);
                s2[b + k] = (float)(4.0 * sn * sn);
            }
            stage_twiddles(N, v, tw.data() + b + N);
        }
        HIP_TRY(hipMemcpy(P->d_tw, tw.data(), sizeof(float2) * tab_len, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(P->d_s2, s2.data(), sizeof(float) * tab_len, hipMemcpyHostToDevice));
    }
    // items and descriptors
    std::vector<WorkItem> all;
    all.insert(all.end(), col.begin(), col.end());
    all.insert(all.end(), rowtv.begin(), rowtv.end());
    all.insert(all.end(), rowfa.begin(), rowfa.end());
    all.insert(all.end(), frm.begin(), frm.end());
    if (!all.empty()) HIP_TRY(hipMemcpy(P->d_items, all.data(), sizeof(WorkItem) * all.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(P->d_desc, P->hd.data(), sizeof(ProbDesc) * count, hipMemcpyHostToDevice));
    for (int i = 0; i < count; ++i) {
        const size_t n = (size_t)P->hd[i].H * P->hd[i].W;
        HIP_TRY(hipMemcpy((void*)P->hd[i].mask, probs[i].mask, n, hipMemcpyHostToDevice));
    }

    // launch contexts
    LaunchCtx base_ctx;
    base_ctx.stream = P->stream;
    base_ctx.desc = P->d_desc;
    base_ctx.info = P->d_info;
    base_ctx.partials = P->d_partials;
    base_ctx.tw = P->d_tw;
    base_ctx.s2 = P->d_s2;
    if (cg) base_ctx.cgpart = (double*)(A + o_cgpart);
    for (int i = 0; i < count; ++i)   // the TV step: every TV problem of a CG plan, long TV rows of an MD plan
        if (P->hd[i].reg == REG_TV && (cg || P->hd[i].W > 2048))
            base_ctx.lds_tvstep = std::max(base_ctx.lds_tvstep, lds_tvstep_bytes(P->hd[i].W, P->hd[i].B));
    for (int i = 0; i < count; ++i)
        if (P->hd[i].reg == REG_TV)
            base_ctx.tv_cpt = std::max(base_ctx.tv_cpt, P->hd[i].W > 8192 ? 32 : (P->hd[i].W > 4096 ? 16 : 8));
    for (int c = 0; c < ADMM_COL_CLASSES; ++c) {
        base_ctx.col_beg[c] = col_cb[c];
        base_ctx.col_cnt[c] = col_cc[c];
        base_ctx.lds_col_c[c] = lds_col_c[c];
    }
    for (int c = 0; c < 3; ++c) {   // the fused TV row pass: classes 0..2
        base_ctx.rtv_beg[c] = rtv_cb[c];
        base_ctx.rtv_cnt[c] = rtv_cc[c];
        base_ctx.lds_rtv_c[c] = lds_rtv_c[c];
        if (c < 3)
            for (int t = 0; t < ADMM_RTV_SUBS; ++t) {
                base_ctx.rtv_sub[c][t] = rtv_sub[c][t];
                base_ctx.lds_rtv_sub[c][t] = lds_rtv_sub[c][t];
            }
    }
    for (int c = 0; c < ADMM_FRAME_CLASSES; ++c) {
        base_ctx.frm_beg[c] = frm_cb[c];
        base_ctx.frm_cnt[c] = frm_cc[c];
        base_ctx.lds_frm_c[c] = lds_frm_c[c];
    }
    base_ctx.col_items = P->d_items;
    base_ctx.ncol = P->ncol;
    P->all = base_ctx;
    P->tv = base_ctx;
    P->tv.row_items = P->d_items + col.size();
    P->tv.nrow = P->nrowtv;
    P->fa = base_ctx;
    P->fa.row_items = P->d_items + col.size() + rowtv.size();
    P->fa.nrow = P->nrowfa;
    for (int c = 0; c < ADMM_ROW_CLASSES; ++c) {
        P->tv.rrow_beg[c] = rtv_cb[c];
        P->tv.rrow_cnt[c] = rtv_cc[c];
        P->tv.lds_rrow_c[c] = lds_rtvp_c[c];
        P->fa.rrow_beg[c] = rfa_cb[c];
        P->fa.rrow_cnt[c] = rfa_cc[c];
        P->fa.lds_rrow_c[c] = lds_rfa_c[c];
    }
    P->tv.rrow_sub0 = tv_sub0;
    P->tv.lds_rrow_sub0 = lds_tv_sub0;
    P->fa.rrow_sub0 = fa_sub0;
    P->fa.lds_rrow_sub0 = lds_fa_sub0;
    P->fa.frm_items = P->d_items + col.size() + rowtv.size() + rowfa.size();
    P->fa.nfrm = P->nfrm;
    // the TV problems with rows longer than 2048 alone (their row items are the
    // last classes of the TV list): plain row passes and the TV step
    P->tvs = base_ctx;
    P->tvs.row_items = P->d_items + col.size() + rtv_cb[3];
    P->tvs.nrow = P->nrowtvs;
    for (int c = 0; c < 3; ++c) P->tvs.rtv_cnt[c] = 0;
    for (int c = 3; c < ADMM_ROW_CLASSES; ++c) {
        P->tvs.rrow_beg[c] = rtv_cb[c] - rtv_cb[3];
        P->tvs.rrow_cnt[c] = rtv_cc[c];
        P->tvs.lds_rrow_c[c] = lds_rtvp_c[c];
    }

    // kernel spectra Lambda (eq. (19)): host computes the row sums T[a][k2] in double
    for (int i = 0; i < count; ++i) {
        const ProbDesc& d = P->hd[i];
        const int ks = probs[i].ksize, l = ks / 2;
        std::vector<float2> T((size_t)ks * d.P);
        for (int a = -l; a <= l; ++a)
            for (int k2 = 0; k2 < d.P; ++k2) {
                double re = 0, im = 0;
                for (int b = -l; b <= l; ++b) {
                    const double w = probs[i].kernel[(a + l) * ks + (b + l)];
                    const long long e = ((long long)k2 * (b < 0 ? b + d.W : b)) % d.W;
                    const double ang = -2.0 * M_PI * (double)e / (double)d.W;
                    re += w * std::cos(ang);
                    im += w * std::sin(ang);
                }
                T[(size_t)(a + l) * d.P + k2] = make_float2((float)re, (float)im);
            }
        float2* dT = nullptr;
        if (P->no_alloc)
            dT = (float2*)(A + o_T);
        else
            HIP_TRY(hipMalloc((void**)&dT, sizeof(float2) * T.size()));
        hipError_t e1 = hipMemcpy(dT, T.data(), sizeof(float2) * T.size(), hipMemcpyHostToDevice);
        hipError_t e2 = e1 == hipSuccess ? launch_lambda(P->all, i, (size_t)d.H * d.P, dT, ks) : e1;
        hipError_t e3 = e2 == hipSuccess ? hipStreamSynchronize(P->stream) : e2;
        if (!P->no_alloc) (void)hipFree(dT);
        if (e3 != hipSuccess) return bail(fail(ADMM_E_DEVICE, "kernel spectrum: %s", hipGetErrorString(e3)));
    }
    return ADMM_OK;
}

namespace {

admm_status upload_desc(admm_plan* P) {
    HIP_TRY(hipMemcpyAsync(P->d_desc, P->hd.data(), sizeof(ProbDesc) * P->count, hipMemcpyHostToDevice, P->stream));
    return ADMM_OK;
}

admm_status run(admm_plan* P, const float* const* y, float* const* x, admm_state* st, const admm_opts* o,
                admm_info* infos) {
    if (!o || !infos || !y || !x) return fail(ADMM_E_INVALID, "null argument");
    if (o->max_iters < 1 || o->check_every < 1) return fail(ADMM_E_INVALID, "max_iters and check_every must be >= 1");
    const int count = P->count;
    const bool cg = P->method == METHOD_CG;
    if (cg && st) return fail(ADMM_E_UNSUPPORTED, "method CG solves start cold: pass no state");
    for (int i = 0; i < count; ++i) {
        if (!y[i] || !x[i]) return fail(ADMM_E_INVALID, "null y/x for problem %d", i);
        if (st && (!st[i].u1 || !st[i].d1 || !st[i].ureg || !st[i].dreg))
            return fail(ADMM_E_INVALID, "null state buffer for problem %d", i);
        ProbDesc& d = P->hd[i];
        d.y = y[i];
        d.x = x[i];
        d.st_u1 = st ? st[i].u1 : nullptr;
        d.st_d1 = st ? st[i].d1 : nullptr;
        d.st_ureg = st ? st[i].ureg : nullptr;
        d.st_dreg = st ? st[i].dreg : nullptr;
    }
    admm_status s = upload_desc(P);
    if (s != ADMM_OK) return s;
    hipStream_t sm = P->stream;
    // initial state
    for (int i = 0; i < count; ++i) {
        const ProbDesc& d = P->hd[i];
        const size_t n = (size_t)d.H * d.W, hp = (size_t)d.H * d.P;
        if (!st && P->no_alloc) {
            // the shared workspace keeps the previous call's contents: clear
            // every buffer that a cold start reads before writing
            HIP_TRY(launch_zero(sm, (float*)d.spec0, hp * 4));
            HIP_TRY(launch_zero(sm, d.d1, n));
            HIP_TRY(launch_zero(sm, d.dreg0, n * d.nb));
            HIP_TRY(launch_zero(sm, d.u1p, n));
            HIP_TRY(launch_zero(sm, d.uregp, n * d.nb));
        } else if (!st) {
            HIP_TRY(hipMemsetAsync(d.spec0, 0, hp * sizeof(float4), sm));
            HIP_TRY(hipMemsetAsync(d.d1, 0, n * sizeof(float), sm));
            HIP_TRY(hipMemsetAsync(d.dreg0, 0, n * d.nb * sizeof(float), sm));
            HIP_TRY(hipMemsetAsync(d.u1p, 0, n * sizeof(float), sm));
            HIP_TRY(hipMemsetAsync(d.uregp, 0, n * d.nb * sizeof(float), sm));
        }
        if (cg) {
            // the first right-hand side (u = d = 0), the boundary estimate v and its images
            for (float* q : {d.tmpA, d.tmpB, d.cgv, d.cge, d.cgae}) HIP_TRY(launch_zero(sm, q, n));
        } else if (d.fs && !st) {
            // synthesis: the first data step reads W zeta2 = s / mu2 (zero at a cold start)
            HIP_TRY(launch_zero(sm, d.tmpB, n));
        } else if (st) {
            HIP_TRY(hipMemcpyAsync(d.u1p, st[i].u1, n * sizeof(float), hipMemcpyDeviceToDevice, sm));
            // analysis: u_reg of the previous iteration (dual residual); synthesis: the
            // coefficient dual d2 (its primal residual takes z = v + d2_{k-1}, and u2 is the state)
            HIP_TRY(hipMemcpyAsync(d.uregp, d.fs ? st[i].dreg : st[i].ureg, n * d.nb * sizeof(float),
                                   hipMemcpyDeviceToDevice, sm));
            if (d.reg == REG_TV) {
                HIP_TRY(launch_import_tv(P->all, i, n));
            } else {
                HIP_TRY(launch_import_fa(P->all, i, n));
            }
        }
    }
    if (st) {
        if (P->nfa) HIP_TRY(launch_frame(P->fa, 1, 0, 1, false));     // q, working d2 <- state
        if (P->nrowtv) {
            LaunchCtx c = P->tv;
            HIP_TRY(launch_row_fwd(c, 0, 0, false));
        }
        if (P->nrowfa) HIP_TRY(launch_row_fwd(P->fa, 0, 0, false));
    }
    {
        std::vector<InfoDev> h(count);
        for (auto& f : h) {
            std::memset(&f, 0, sizeof f);
            f.active = 1;
        }
        std::memcpy(P->h_info, h.data(), sizeof(InfoDev) * count);
        HIP_TRY(hipMemcpyAsync(P->d_info, P->h_info, sizeof(InfoDev) * count, hipMemcpyHostToDevice, sm));
    }
    const int K = o->max_iters, c = o->check_every;
    const double tol = o->tol, obj_tol = o->obj_tol > 0.0 ? o->obj_tol : 0.0;
    const bool stopping = tol > 0 || obj_tol > 0;   // a stopping rule is checked every c iterations
    const bool profile = (o->flags & ADMM_FLAG_PROFILE) != 0 && !P->no_alloc;
    const bool use_graph = (o->flags & ADMM_FLAG_GRAPH) && !profile && !P->no_alloc;
    auto is_check = [&](int k) { return k == K || (stopping && k % c == 0); };
    auto is_plain = [&](int k) { return k < K && !is_check(k) && !is_check(k + 1); };

    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
    auto timed = [&](int cls, auto&& fn) -> hipError_t {
        if (!profile) return fn();
        hipEvent_t a = nullptr, b = nullptr;
        hipError_t e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        if (e == hipSuccess) e = hipEventRecord(a, sm);
        if (e == hipSuccess) e = fn();
        if (e == hipSuccess) e = hipEventRecord(b, sm);
        ev.push_back({cls, {a, b}});
        return e;
    };
    auto release_events = [&]() {
        for (auto& x : ev) {
            if (x.second.first) (void)hipEventDestroy(x.second.first);
            if (x.second.second) (void)hipEventDestroy(x.second.second);
        }
        ev.clear();
    };
    // one iteration on contexts cA (all), cT (TV rows), cF (FA rows/frame)
    // method CG (see admm_cg.hip): both circulant solves run forward rows,
    // columns and inverse rows in place on spec0 (the first solve's inverse
    // rows also form the boundary-system direction and transform it for the
    // second); the CG and data steps run per row block, then the TV step or
    // the frame step
    auto cg_iteration = [&](const LaunchCtx& cA, const LaunchCtx& cT, const LaunchCtx& cF, int par,
                            int flags) -> hipError_t {
        hipError_t e = hipSuccess;
        const LaunchCtx* rows[2] = {&cT, &cF};
        auto each = [&](int cls, auto&& fn) {
            for (const LaunchCtx* r : rows)
                if (e == hipSuccess && r->nrow) e = timed(cls, [&] { return fn(*r); });
        };
        // the inverse rows of the first solve end with the forward rows of the second
        each(4, [&](const LaunchCtx& r) { return launch_row_fwd(r, 0, 0, true); });
        for (int solve = 0; solve < 2 && e == hipSuccess; ++solve) {
            if (e == hipSuccess) e = timed(0, [&] { return launch_col(cA, 0, COL_SOLVE); });
            each(2, [&](const LaunchCtx& r) { return launch_row_inv(r, 0, 2 + solve, 0, true); });
        }
        each(6, [&](const LaunchCtx& r) { return launch_cg_update(r, flags); });
        if (e == hipSuccess && cT.nrow) e = timed(6, [&] { return launch_tv_step(cT, par, flags); });
        if (e == hipSuccess && cF.nrow) e = timed(3, [&] { return launch_frame(cF, par, flags, 0, true); });
        return e;
    };
    // cS: the TV problems with rows longer than 2048, which run inverse rows with
    // the data step (z to the z plane), the TV step and forward rows
    auto iteration = [&](const LaunchCtx& cA, const LaunchCtx& cT, const LaunchCtx& cF, const LaunchCtx& cS, int par,
                         int flags, bool last) -> hipError_t {
        if (cg) return cg_iteration(cA, cT, cF, par, flags);
        hipError_t e = timed(0, [&] { return launch_col(cA, par, COL_SOLVE); });
        if (e == hipSuccess && P->nrowtv) e = timed(1, [&] { return launch_row_tv(cT, par, flags); });
        if (e == hipSuccess && P->nrowtvs) {
            e = timed(2, [&] { return launch_row_inv(cS, 0, 1, flags, true); });
            if (e == hipSuccess) e = timed(1, [&] { return launch_tv_step(cS, par, flags); });
            if (e == hipSuccess && !last) e = timed(4, [&] { return launch_row_fwd(cS, 0, 0, true); });
        }
        if (e == hipSuccess && P->nrowfa) {
            e = timed(2, [&] { return launch_row_inv(cF, 0, 1, flags, true); });
            if (e == hipSuccess) e = timed(3, [&] { return launch_frame(cF, par, flags, 0, true); });
            if (e == hipSuccess && !last) e = timed(4, [&] { return launch_row_fwd(cF, 0, 0, true); });
        }
        return e;
    };
    auto get_graph = [&](int G, hipGraphExec_t* exec) -> admm_status {
        auto it = P->graphs.find(G);
        if (it != P->graphs.end()) {
            *exec = it->second;
            return ADMM_OK;
        }
        if (!P->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
        LaunchCtx cA = P->all, cT = P->tv, cF = P->fa, cS = P->tvs;
        cA.stream = cT.stream = cF.stream = cS.stream = P->cap_stream;
        HIP_TRY(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int i = 0; i < G && e == hipSuccess; ++i) e = iteration(cA, cT, cF, cS, i & 1, F_FORWARD, false);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(P->cap_stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(ADMM_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
        }
        hipGraphExec_t x = nullptr;
        hipError_t e3 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) return fail(ADMM_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e3));
        P->graphs[G] = x;
        *exec = x;
        return ADMM_OK;
    };

    // Check periods replayed as graphs (solves to a tolerance): a graph holds g
    // periods of c iterations, the last two of each with the pre-check and check
    // flags and then the reduction, which takes its iteration number from a
    // device counter (base + j c for period j) and mirrors the active flags into
    // host-mapped memory; the graph ends by advancing the counter by g c. The
    // host keeps at most kPeriodsInFlight graphs queued and stops launching once
    // every flag is clear; the kernels skip finished problems, so iterations
    // launched after the end change nothing. The final iteration and a tail
    // shorter than a period take the loop below.
    auto get_period_graph = [&](int g, hipGraphExec_t* exec) -> admm_status {
        uint64_t tb = 0;
        std::memcpy(&tb, &tol, sizeof tb);
        uint64_t ob = 0;
        std::memcpy(&ob, &obj_tol, sizeof ob);
        const auto key = std::make_tuple(c, g, st ? 1 : 0, tb, ob);
        auto it = P->pgraphs.find(key);
        if (it != P->pgraphs.end()) {
            *exec = it->second;
            return ADMM_OK;
        }
        if (!P->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
        LaunchCtx cA = P->all, cT = P->tv, cF = P->fa, cS = P->tvs;
        cA.stream = cT.stream = cF.stream = cS.stream = P->cap_stream;
        HIP_TRY(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int q = 1; q <= g && e == hipSuccess; ++q) {
            for (int j = 1; j <= c && e == hipSuccess; ++j) {
                // u_k is kept on the iteration before each check (every one for period 1)
                int flags = F_FORWARD | (j == c - 1 || c == 1 ? F_WRITE_UPREV : 0);
                if (j == c) flags |= F_CHECK | F_WRITE_X | (st ? F_EXPORT : 0);
                e = iteration(cA, cT, cF, cS, ((q - 1) * c + j - 1) & 1, flags, false);
            }
            if (e == hipSuccess) e = launch_reduce(cA, count, tol, obj_tol, q * c, 0, P->d_kbase, P->h_active_dev);
        }
        if (e == hipSuccess) e = launch_tick(cA, P->d_kbase, g * c, false);
        hipGraph_t gr = nullptr;
        hipError_t e2 = hipStreamEndCapture(P->cap_stream, &gr);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (gr) (void)hipGraphDestroy(gr);
            return fail(ADMM_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
        }
        hipGraphExec_t x = nullptr;
        hipError_t e3 = hipGraphInstantiate(&x, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e3 != hipSuccess) return fail(ADMM_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e3));
        P->pgraphs[key] = x;
        *exec = x;
        return ADMM_OK;
    };

    int par = 0;
    int k = 1;
    bool all_done = false;
    // an even number of iterations per graph keeps the ping-pong parity: an even
    // period, or period 1 with an even number of periods
    if (use_graph && stopping && (c % 2 == 0 || c == 1) && c < K) {
        for (hipEvent_t& e : P->pev)
            if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        for (int i = 0; i < count; ++i) P->h_active[i] = 1;
        HIP_TRY(launch_tick(P->all, P->d_kbase, 0, true));
        const int gmax = std::max(1, kPeriodIters / c);
        for (int n = 0; k + c - 1 < K; ++n) {
            int g = std::min(gmax, (K - k) / c);   // whole periods that end before K
            if (c % 2) g &= ~1;
            if (g < 1) break;
            hipEvent_t& ev_n = P->pev[n % kPeriodsInFlight];
            if (n >= kPeriodsInFlight) {
                HIP_TRY(hipEventSynchronize(ev_n));   // graph n - kPeriodsInFlight has finished
                bool any = false;
                for (int i = 0; i < count; ++i) any = any || ((volatile int*)P->h_active)[i] != 0;
                if (!any) {
                    all_done = true;
                    break;
                }
            }
            hipGraphExec_t exec = nullptr;
            admm_status gs = get_period_graph(g, &exec);
            if (gs != ADMM_OK) return gs;
            HIP_TRY(hipGraphLaunch(exec, sm));
            HIP_TRY(hipEventRecord(ev_n, sm));
            k += g * c;
        }
    }
    while (!all_done && k <= K) {
        if (use_graph && par == 0 && is_plain(k)) {
            int run = 0;
            while (k + run <= K && is_plain(k + run)) ++run;
            int G = 64;
            while (G > run) G >>= 1;
            if (G >= 2) {
                hipGraphExec_t exec = nullptr;
                admm_status gs = get_graph(G, &exec);
                if (gs != ADMM_OK) return gs;
                HIP_TRY(hipGraphLaunch(exec, sm));
                k += G;
                continue;
            }
        }
        const bool last = k == K, check = is_check(k), next_check = !last && is_check(k + 1);
        int flags = (last ? 0 : F_FORWARD) | (next_check ? F_WRITE_UPREV : 0);
        if (check) flags |= F_CHECK | F_WRITE_X | (st ? F_EXPORT : 0);
        {
            hipError_t e = iteration(P->all, P->tv, P->fa, P->tvs, par, flags, last);
            if (e != hipSuccess) {
                release_events();
                return fail(ADMM_E_DEVICE, "iteration %d launch failed: %s", k, hipGetErrorString(e));
            }
        }
        if (check) {
            hipError_t e = timed(5, [&] { return launch_reduce(P->all, count, tol, obj_tol, k, last ? 1 : 0); });
            if (e != hipSuccess) {
                release_events();
                return fail(ADMM_E_DEVICE, "reduction launch failed: %s", hipGetErrorString(e));
            }
            if (!last && stopping) {
                HIP_TRY(hipMemcpyAsync(P->h_info, P->d_info, sizeof(InfoDev) * count, hipMemcpyDeviceToHost, sm));
                HIP_TRY(hipStreamSynchronize(sm));
                bool any = false;
                for (int i = 0; i < count; ++i) any = any || P->h_info[i].active;
                if (!any) break;
            }
        }
        par ^= 1;
        ++k;
    }
    if (profile) {
        HIP_TRY(hipStreamSynchronize(sm));
        for (int i = 0; i < kProfClasses; ++i) {
            P->prof_ms[i] = 0;
            P->prof_n[i] = 0;
        }
        for (auto& x : ev) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, x.second.first, x.second.second) == hipSuccess) {
                P->prof_ms[x.first] += ms;
                P->prof_n[x.first] += 1;
            }
        }
        release_events();
    }
    HIP_TRY(hipMemcpyAsync(P->h_info, P->d_info, sizeof(InfoDev) * count, hipMemcpyDeviceToHost, sm));
    HIP_TRY(hipStreamSynchronize(sm));
    bool diverged = false;
    for (int i = 0; i < count; ++i) {
        const InfoDev& f = P->h_info[i];
        infos[i].iters = f.iters;
        infos[i].converged = f.converged;
        infos[i].diverged = f.diverged;
        infos[i].reserved = 0;
        infos[i].r_pri = f.r_pri;
        infos[i].r_dual = f.r_dual;
        infos[i].objective = f.objective;
        diverged = diverged || f.diverged;
    }
    if (diverged) return fail(ADMM_E_DIVERGED, "non-finite iterate");
    return ADMM_OK;
}

}  // namespace

extern "C" admm_status admm_deconv_solve(admm_plan* P, const float* y, float* x, admm_state* st, const admm_opts* o,
                                         admm_info* info) {
    if (!P) return fail(ADMM_E_INVALID, "null plan");
    if (P->count != 1) return fail(ADMM_E_INVALID, "solve needs a plan with one problem (has %d); use batch", P->count);
    return run(P, &y, &x, st, o, info);
}

extern "C" admm_status admm_deconv_batch(admm_plan* P, const float* const* y, float* const* x, admm_state* st,
                                         const admm_opts* o, admm_info* infos) {
    if (!P) return fail(ADMM_E_INVALID, "null plan");
    return run(P, y, x, st, o, infos);
}

// ------------------------------------------------------------ allocation-free solve
// The workspace of admm_deconv_solve_static: one array per device, held until
// the process ends, shared by every call on that device (calls that overlap
// on one device race). Host code reaches it only through the address that
// hipGetSymbolAddress returns on the device that is current.
static __device__ __align__(256) unsigned char scratch[ADMM_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

admm_status scratch_address(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(ADMM_E_DEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ADMM_E_DEVICE, "address of the static workspace on device %d: %s", dev, hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return ADMM_OK;
}

}  // namespace

extern "C" admm_status admm_deconv_solve_static(const admm_problem* prob, const float* y, float* x, admm_state* st,
                                                const admm_opts* opts, admm_info* info, void* hip_stream) {
    if (!prob) return fail(ADMM_E_INVALID, "null problem");
    admm_status s = validate(*prob);
    if (s != ADMM_OK) return s;
    void* ws = nullptr;
    s = scratch_address(&ws);
    if (s != ADMM_OK) return s;
    admm_plan P;   // host bookkeeping only: descriptors, tables and state live in the workspace
    s = build_plan(&P, prob, 1, hip_stream, TileChoice{}, ws, (size_t)ADMM_STATIC_WORKSPACE_BYTES);
    if (s == ADMM_OK) s = run(&P, &y, &x, st, opts, info);
    return s;
}

namespace {

// Context restricted to the items of one problem.
LaunchCtx single(const admm_plan* P, int i) {
    const ProbDesc& d = P->hd[i];
    LaunchCtx c = d.reg == REG_TV ? P->tv : P->fa;
    c.col_items = P->all.col_items + P->col_beg[i];
    c.ncol = P->col_end[i] - P->col_beg[i];
    c.row_items += P->row_beg[i];
    c.nrow = P->row_end[i] - P->row_beg[i];
    c.frm_items = nullptr;
    c.nfrm = 0;
    for (int k = 0; k < ADMM_COL_CLASSES; ++k) c.col_beg[k] = c.col_cnt[k] = 0;
    for (int k = 0; k < ADMM_ROW_CLASSES; ++k) {
        c.rtv_beg[k] = c.rrow_beg[k] = 0;
        c.rtv_cnt[k] = c.rrow_cnt[k] = 0;
    }
    for (int k = 0; k < 3; ++k)
        for (int t = 0; t < ADMM_RTV_SUBS; ++t) c.rtv_sub[k][t] = 0;
    c.col_cnt[col_class(d)] = c.ncol;
    c.rrow_cnt[size_class(d.W)] = c.nrow;
    c.rrow_sub0 = plain_narrow(d) ? c.nrow : 0;   // as in the batch
    if (d.reg == REG_TV) {
        const int sc = size_class(d.W);
        c.rtv_cnt[sc] = c.nrow;
        if (sc < 3 && rtv_sub_of(d, sc) < ADMM_RTV_SUBS) c.rtv_sub[sc][rtv_sub_of(d, sc)] = c.nrow;   // as in the batch
    }
    return c;
}

admm_status blur_into_tmpB(admm_plan* P, int i, const float* x) {
    const ProbDesc& d = P->hd[i];
    const size_t n = (size_t)d.H * d.W;
    LaunchCtx c = single(P, i);
    HIP_TRY(hipMemcpyAsync(d.tmpA, x, n * sizeof(float), hipMemcpyDeviceToDevice, P->stream));
    HIP_TRY(launch_row_fwd(c, 0, 1, false));
    HIP_TRY(launch_col(c, 0, COL_BLUR));
    HIP_TRY(launch_row_inv(c, 0, 0, 0, false));
    return ADMM_OK;
}

}  // namespace

extern "C" admm_status admm_deconv_blur(admm_plan* P, int32_t index, const float* x, float* Ax) {
    if (!P || !x || !Ax) return fail(ADMM_E_INVALID, "null argument");
    if (index < 0 || index >= P->count) return fail(ADMM_E_INVALID, "index %d out of range", index);
    admm_status s = blur_into_tmpB(P, index, x);
    if (s != ADMM_OK) return s;
    const ProbDesc& d = P->hd[index];
    HIP_TRY(hipMemcpyAsync(Ax, d.tmpB, (size_t)d.H * d.W * sizeof(float), hipMemcpyDeviceToDevice, P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    return ADMM_OK;
}

extern "C" admm_status admm_warmstart_map(admm_plan* P, int32_t index, const float* x0, const float* p0, const float* y,
                                          admm_state* st) {
    if (!P || !x0 || !p0 || !y || !st || !st->u1 || !st->d1 || !st->ureg || !st->dreg)
        return fail(ADMM_E_INVALID, "null argument");
    if (index < 0 || index >= P->count) return fail(ADMM_E_INVALID, "index %d out of range", index);
    const ProbDesc& d = P->hd[index];
    if (d.reg != REG_TV) return fail(ADMM_E_INVALID, "warm-start mapping is defined for TV problems");
    admm_status s = blur_into_tmpB(P, index, x0);
    if (s != ADMM_OK) return s;
    HIP_TRY(launch_warmstart(P->all, index, (size_t)d.H * d.W, x0, p0, y, st->u1, st->d1, st->ureg, st->dreg));
    HIP_TRY(hipStreamSynchronize(P->stream));
    return ADMM_OK;
}

extern "C" admm_status admm_warmstart_dual(admm_plan* P, int32_t index, const float* dreg, float* p0) {
    if (!P || !dreg || !p0) return fail(ADMM_E_INVALID, "null argument");
    if (index < 0 || index >= P->count) return fail(ADMM_E_INVALID, "index %d out of range", index);
    const ProbDesc& d = P->hd[index];
    if (d.reg != REG_TV) return fail(ADMM_E_INVALID, "the dual field is defined for TV problems");
    const double lam = P->probs[index].lambda;
    if (!(lam > 0.0)) return fail(ADMM_E_INVALID, "lambda must be > 0 to scale the dual field (got %g)", lam);
    HIP_TRY(launch_scale(P->stream, dreg, p0, 2 * (size_t)d.H * d.W, (float)(-(double)d.mu2 / lam)));
    HIP_TRY(hipStreamSynchronize(P->stream));
    return ADMM_OK;
}

extern "C" int32_t admm_plan_kernel_times(const admm_plan* P, admm_kernel_time* out, int32_t cap) {
    if (!P) return 0;
    for (int i = 0; i < kProfClasses && out && i < cap; ++i) {
        std::memset(&out[i], 0, sizeof out[i]);
        std::snprintf(out[i].name, sizeof out[i].name, "%s", kProfNames[i]);
        out[i].launches = P->prof_n[i];
        out[i].total_ms = P->prof_ms[i];
    }
    return kProfClasses;
}

// ------------------------------------------------------------ FFT autotuner
// Chooses the tile shapes of the two pass kernels by measurement: columns per
// column-pass block (one column per wave) and rows per row-pass block. Each
// trial plan is timed on whole iterations replayed from graphs, as solves run:
// first the column tiles with the planner's row count, then the row counts
// with the best tile, then, when the batch's rows fall in several size
// classes, the row count of each class with the others held. Results are
// cached in a JSON object keyed by device architecture and the batch's shape
// multiset, with the per-launch times of the two passes under the choice for
// the record; per-class row counts appear only where they differ from "rows":
//   {"gfx950|tv512x512*8": {"tc": 4, "rows": 8, "col_us": 16.1, "row_us": 30.6}}
//   {"gfx950|h...*256": {"tc": 4, "rows": 5, "rows_512": 8, "col_us": 896, "row_us": 1597}}
// The tile shape changes which thread computes what, never the arithmetic of
// an element, so the iterates do not depend on it.
namespace {

// Time one trial plan: per-launch microseconds of the column kernel and of
// the row-side kernels (TV row pass, or FA inverse rows + frame + forward rows).
admm_status time_plan(admm_plan* P, const float* const* y, float* const* x, double* col_us, double* row_us) {
    admm_opts o{};
    o.max_iters = 10;
    o.tol = 0.0;
    o.check_every = 1 << 20;
    o.flags = ADMM_FLAG_PROFILE;
    std::vector<admm_info> infos(P->count);
    double best_c = 1e300, best_r = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
        admm_status s = run(P, y, x, nullptr, &o, infos.data());
        if (s != ADMM_OK) return s;
        if (rep == 0) continue;   // the first run warms caches and code
        const double c = P->prof_n[0] ? P->prof_ms[0] / P->prof_n[0] * 1e3 : 0.0;
        double r = 0.0;
        for (int k = 1; k < kProfClasses; ++k)   // everything but the columns and the reduction
            if (k != 5 && P->prof_n[k]) r += P->prof_ms[k] / P->prof_n[k] * 1e3;
        best_c = std::min(best_c, c);
        best_r = std::min(best_r, r);
    }
    *col_us = best_c;
    *row_us = best_r;
    return ADMM_OK;
}

// Time one trial plan the way solves run: whole iterations replayed from
// graphs, one event pair around each run on the plan's stream. Runs of K and
// 3K iterations are timed (best of three after a warm-up run of each) and the
// difference divided by 2K: the per-run work (state reset, descriptor upload,
// the final iteration and its reduction) cancels, which for large batches is
// a large share of a short run. Per-launch event pairs (time_plan) carry the
// dispatch of every launch, a few microseconds of jitter against tile
// differences below one, so they only describe the choice made.
admm_status time_iterations(admm_plan* P, const float* const* y, float* const* x, double* us) {
    size_t px = 0;
    for (int i = 0; i < P->count; ++i) px += (size_t)P->hd[i].H * P->hd[i].W;
    const int K = (int)std::max<size_t>(4, std::min<size_t>(20, (size_t)1e8 / std::max<size_t>(px, 1)));
    admm_opts o{};
    o.tol = 0.0;
    o.check_every = 1 << 20;
    o.flags = ADMM_FLAG_GRAPH;
    std::vector<admm_info> infos(P->count);
    hipEvent_t ev[2] = {nullptr, nullptr};
    admm_status s = ADMM_OK;
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
        s = fail(ADMM_E_DEVICE, "autotuner: event creation failed");
    double best[2] = {1e300, 1e300};
    for (int rep = 0; rep < 4 && s == ADMM_OK; ++rep) {
        for (int len = 0; len < 2 && s == ADMM_OK; ++len) {
            o.max_iters = len ? 3 * K : K;
            if (hipEventRecord(ev[0], P->stream) != hipSuccess) {
                s = fail(ADMM_E_DEVICE, "autotuner: event record failed");
                break;
            }
            s = run(P, y, x, nullptr, &o, infos.data());
            float ms = 0.f;
            if (s == ADMM_OK && (hipEventRecord(ev[1], P->stream) != hipSuccess ||
                                 hipEventSynchronize(ev[1]) != hipSuccess ||
                                 hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess))
                s = fail(ADMM_E_DEVICE, "autotuner: event timing failed");
            if (s == ADMM_OK && rep > 0) best[len] = std::min(best[len], 1e3 * (double)ms);
        }
    }
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    *us = best[1] > best[0] ? (best[1] - best[0]) / (2.0 * K) : best[1] / (3.0 * K);
    return s;
}

}  // namespace

extern "C" int32_t admm_tune_key(const admm_problem* probs, int32_t count, const char* arch, char* out, size_t cap) {
    if (!probs || count < 1 || !arch) return -1;
    const std::string k = make_key(probs, count, arch);
    if (out && cap > 0) std::snprintf(out, cap, "%s", k.c_str());
    return (int32_t)k.size();
}

extern "C" int32_t admm_tune_cache_lookup(const char* path, const char* key, int32_t* tc, int32_t* rows) {
    if (!path || !key) return -1;
    std::map<std::string, TuneEntry> m;
    if (read_cache(path, m) != 0) return -1;
    auto it = m.find(key);
    if (it == m.end()) return 0;
    if (tc) *tc = it->second.tc;
    if (rows) *rows = it->second.rows;
    return 1;
}

extern "C" admm_status admm_tune_cache_store(const char* path, const char* key, int32_t tc, int32_t rows,
                                             double col_us, double row_us) {
    if (!path || !key || tc < 1 || rows < 1) return fail(ADMM_E_INVALID, "bad cache entry");
    for (const char* c = key; *c; ++c)
        if (*c == '"' || *c == '\\' || (unsigned char)*c < 0x20) return fail(ADMM_E_INVALID, "bad cache key");
    std::map<std::string, TuneEntry> m;
    if (read_cache(path, m) != 0) return fail(ADMM_E_INVALID, "tuning cache %s is not a cache file", path);
    TuneEntry e;
    e.tc = tc;
    e.rows = rows;
    e.col_us = col_us;
    e.row_us = row_us;
    m[key] = e;
    if (write_cache(path, m) != 0) return fail(ADMM_E_INVALID, "cannot write tuning cache %s", path);
    return ADMM_OK;
}

extern "C" admm_status admm_deconv_plan_tuned(const admm_problem* probs, int32_t count, void* hip_stream,
                                              const char* cache_path, admm_plan** out) {
    if (!out) return fail(ADMM_E_INVALID, "null output pointer");
    *out = nullptr;
    if (!probs || count < 1) return fail(ADMM_E_INVALID, "need at least one problem");
    for (int i = 0; i < count; ++i) {
        admm_status s = validate(probs[i]);
        if (s != ADMM_OK) {
            admm_host::prefix_error("problem " + std::to_string(i) + ": ");
            return s;
        }
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    const std::string key = make_key(probs, count, arch.c_str());

    TileChoice best;
    std::map<std::string, TuneEntry> cache;
    bool have = false;
    if (cache_path) {
        if (read_cache(cache_path, cache) != 0)
            return fail(ADMM_E_INVALID, "tuning cache %s is not a cache file", cache_path);
        auto it = cache.find(key);
        if (it != cache.end() && it->second.tc > 0 && it->second.rows > 0) {
            best.tc = it->second.tc;
            best.b = it->second.rows;
            for (int c = 0; c < ADMM_ROW_CLASSES; ++c) best.bc[c] = it->second.rows_c[c];
            best.rsched = it->second.rsched;
            best.csched = it->second.csched;
            have = true;
        }
    }
    if (!have) {
        // trial data: one shared zero observation, one output per problem
        size_t nmax = 0, ntot = 0;
        for (int i = 0; i < count; ++i) {
            const size_t n = (size_t)probs[i].H * probs[i].W;
            nmax = std::max(nmax, n);
            ntot += n;
        }
        float* dy = nullptr;
        float* dx = nullptr;
        if (hipMalloc(&dy, nmax * sizeof(float)) != hipSuccess || hipMalloc(&dx, ntot * sizeof(float)) != hipSuccess) {
            (void)hipFree(dy);
            return fail(ADMM_E_NOMEM, "autotuner: no device memory for trial data");
        }
        std::vector<const float*> yv(count, dy);
        std::vector<float*> xv(count);
        size_t off = 0;
        for (int i = 0; i < count; ++i) {
            xv[i] = dx + off;
            off += (size_t)probs[i].H * probs[i].W;
        }
        admm_status st = hipMemsetAsync(dy, 0, nmax * sizeof(float), (hipStream_t)hip_stream) == hipSuccess
                             ? ADMM_OK
                             : fail(ADMM_E_DEVICE, "autotuner: memset failed");
        // searches on the time per whole iteration: the column tile with the
        // planner's row count, then the row count with that tile, then (batches
        // whose rows fall in several size classes) the row count of each class
        // with the others held
        const int tcs[] = {1, 2, 3, 4};
        const int bs[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16};
        const int ntc = 4, nb = 10;
        TuneEntry rec;
        // trials are keyed by the tile shapes the planner actually uses (a
        // request beyond a problem's limit is clamped): a shape already timed
        // is not timed again, so a repeat cannot win on measurement noise
        std::map<std::vector<int>, double> timed;
        auto trial = [&](TileChoice t, double* us) -> admm_status {
            admm_plan* P = new admm_plan();
            admm_status s = build_plan(P, probs, count, hip_stream, t);
            if (s == ADMM_OK) {
                std::vector<int> shape;
                for (const ProbDesc& d : P->hd) {
                    shape.push_back(d.TC);
                    shape.push_back(d.B);
                    shape.push_back(d.fr.variant);
                    shape.push_back(d.fc.variant);
                }
                auto it = timed.find(shape);
                if (it != timed.end()) {
                    *us = it->second;
                } else {
                    s = time_iterations(P, yv.data(), xv.data(), us);
                    if (s == ADMM_OK) timed[shape] = *us;
                }
            }
            admm_plan_destroy(P);
            return s;
        };
        double best_t = 1e300;
        for (int k = 0; k < ntc + nb && st == ADMM_OK; ++k) {
            TileChoice t;
            t.tc = k < ntc ? tcs[k] : best.tc;
            t.b = k < ntc ? 0 : bs[k - ntc];
            if (k == ntc) best_t = 1e300;   // row counts compete among themselves
            if (k >= ntc && best.tc < 1) break;
            double us = 0.0;
            const admm_status s = trial(t, &us);
            // the requested shapes are recorded: planning with them again
            // reproduces this trial (the planner clamps them the same way)
            if (s == ADMM_OK && us < best_t) {
                best_t = us;
                if (k < ntc)
                    best.tc = t.tc;
                else
                    best.b = t.b;
            }
            if (s == ADMM_E_DEVICE || s == ADMM_E_NOMEM) st = s;
        }
        bool cls[ADMM_ROW_CLASSES] = {};
        int ncls = 0;
        for (int i = 0; i < count; ++i) cls[size_class(probs[i].W)] = true;
        for (int c = 0; c < ADMM_ROW_CLASSES; ++c) ncls += cls[c];
        if (ncls > 1 && best.tc >= 1 && best.b >= 1) {
            for (int c = 0; c < ADMM_ROW_CLASSES && st == ADMM_OK; ++c) {
                if (!cls[c]) continue;
                for (int k = 0; k < nb && st == ADMM_OK; ++k) {
                    if (bs[k] == best.b) continue;   // the common count is the incumbent
                    TileChoice t = best;
                    t.bc[c] = bs[k];
                    double us = 0.0;
                    const admm_status s = trial(t, &us);
                    if (s == ADMM_OK && us < 0.995 * best_t) {   // a clear gain over the common count
                        best_t = us;
                        best.bc[c] = bs[k];
                    }
                    if (s == ADMM_E_DEVICE || s == ADMM_E_NOMEM) st = s;
                }
            }
        }
        // radix schedules (the tile shape fixed): each alternative of the column
        // transforms, then of the row transforms, kept on a clear gain. A
        // schedule changes the rounding of the transforms, not what they
        // compute (every variant is checked against the oracle by the tests).
        if (best.tc >= 1 && best.b >= 1) {
            for (int pass = 0; pass < 2 && st == ADMM_OK; ++pass) {
                const int nv = pass == 0 ? FFT_VARIANTS - 1 : FFT_VARIANTS;   // no radix 16 in columns
                for (int v = 1; v < nv && st == ADMM_OK; ++v) {
                    TileChoice t = best;
                    (pass == 0 ? t.csched : t.rsched) = v;
                    double us = 0.0;
                    const admm_status s = trial(t, &us);
                    if (s == ADMM_OK && us < 0.995 * best_t) {
                        best_t = us;
                        best = t;
                    }
                    if (s == ADMM_E_DEVICE || s == ADMM_E_NOMEM) st = s;
                }
            }
        }
        double best_c = 0.0, best_r = 0.0;   // per-pass figures of the choice, for the record
        if (st == ADMM_OK && best.tc >= 1 && best.b >= 1) {
            admm_plan* P = new admm_plan();
            admm_status s = build_plan(P, probs, count, hip_stream, best);
            if (s == ADMM_OK) s = time_plan(P, yv.data(), xv.data(), &best_c, &best_r);
            admm_plan_destroy(P);
            if (s == ADMM_E_DEVICE || s == ADMM_E_NOMEM) st = s;
        }
        (void)hipStreamSynchronize((hipStream_t)hip_stream);
        (void)hipFree(dy);
        (void)hipFree(dx);
        if (st != ADMM_OK) return st;
        if (best.tc < 1 || best.b < 1) return fail(ADMM_E_UNSUPPORTED, "autotuner: no tile shape could be planned");
        rec.tc = best.tc;
        rec.rows = best.b;
        for (int c = 0; c < ADMM_ROW_CLASSES; ++c) rec.rows_c[c] = best.bc[c];
        rec.rsched = best.rsched;
        rec.csched = best.csched;
        rec.col_us = best_c;
        rec.row_us = best_r;
        if (cache_path) {
            cache[key] = rec;
            if (write_cache(cache_path, cache) != 0)
                return fail(ADMM_E_INVALID, "cannot write tuning cache %s", cache_path);
        }
    }
    admm_plan* P = new admm_plan();
    admm_status s = build_plan(P, probs, count, hip_stream, best);
    if (s != ADMM_OK) {
        admm_plan_destroy(P);
        return s;
    }
    *out = P;
    return ADMM_OK;
}

extern "C" admm_status admm_plan_tiles(const admm_plan* P, int32_t index, int32_t* tc, int32_t* rows) {
    if (!P || index < 0 || index >= P->count) return fail(ADMM_E_INVALID, "bad plan or index");
    if (tc) *tc = P->hd[index].TC;
    if (rows) *rows = P->hd[index].B;
    return ADMM_OK;
}

extern "C" admm_status admm_plan_schedules(const admm_plan* P, int32_t index, int32_t* row_schedule,
                                           int32_t* col_schedule) {
    if (!P || index < 0 || index >= P->count) return fail(ADMM_E_INVALID, "bad plan or index");
    if (row_schedule) *row_schedule = P->hd[index].fr.variant;
    if (col_schedule) *col_schedule = P->hd[index].fc.variant;
    return ADMM_OK;
}

extern "C" admm_status admm_plan_time_pass(admm_plan* P, const char* kernel, int32_t reps, double* avg_ms) {
    if (!P || !kernel || !avg_ms || reps < 1) return fail(ADMM_E_INVALID, "bad argument");
    std::string k = kernel;
    int cls = -1;   // "col:c", "row_tv:c": size class c alone
    const size_t colon = k.find(':');
    if (colon != std::string::npos) {
        const std::string num = k.substr(colon + 1);
        k = k.substr(0, colon);
        const int ncls = k == "col" ? ADMM_COL_CLASSES : 3;
        if ((k != "col" && k != "row_tv") || num.empty() || num.size() > 1 || num[0] < '0' || num[0] - '0' >= ncls)
            return fail(ADMM_E_INVALID, "unknown pass kernel %s", kernel);
        cls = num[0] - '0';
    }
    const bool fa = k == "frame" || k == "row_inv" || k == "row_fwd";
    if (k != "col" && k != "row_tv" && !fa) return fail(ADMM_E_INVALID, "unknown pass kernel %s", kernel);
    LaunchCtx ccol = P->all, crow = P->tv;   // with cls >= 0: that class's launches only
    if (cls >= 0) {
        for (int c = 0; c < ADMM_COL_CLASSES; ++c)
            if (c != cls) ccol.col_cnt[c] = 0;
        for (int c = 0; c < ADMM_ROW_CLASSES; ++c)
            if (c != cls) crow.rtv_cnt[c] = 0;
        if ((k == "col" && !ccol.col_cnt[cls]) || (k == "row_tv" && !crow.rtv_cnt[cls]))
            return fail(ADMM_E_INVALID, "the plan has no %s launches", kernel);
    }
    // "row_tv": the fused TV row pass and the TV step of long TV rows; "row_inv",
    // "row_fwd": the plain row passes of the frame problems and of long TV rows
    if ((k == "row_tv" && !P->nrowtv) || (k == "frame" && !P->nfa) ||
        ((k == "row_inv" || k == "row_fwd") && !P->nrowfa && !P->nrowtvs))
        return fail(ADMM_E_INVALID, "the plan has no %s launches", kernel);
    // every problem active, as in a running solve (a finished solve leaves them inactive)
    for (int i = 0; i < P->count; ++i) {
        std::memset(&P->h_info[i], 0, sizeof(InfoDev));
        P->h_info[i].active = 1;
    }
    HIP_TRY(hipMemcpyAsync(P->d_info, P->h_info, sizeof(InfoDev) * P->count, hipMemcpyHostToDevice, P->stream));
    auto launch = [&]() -> hipError_t {
        if (k == "col") return launch_col(ccol, 0, COL_SOLVE);
        if (k == "frame") return launch_frame(P->fa, 0, 0, 0, true);
        hipError_t e = hipSuccess;
        if (k == "row_tv") {
            e = launch_row_tv(crow, 0, F_FORWARD);
            if (e == hipSuccess && P->nrowtvs && cls < 0) e = launch_tv_step(P->tvs, 0, 0);
            return e;
        }
        const bool inv = k == "row_inv";
        for (const LaunchCtx* c : {&P->fa, &P->tvs})
            if (e == hipSuccess && c->nrow)
                e = inv ? launch_row_inv(*c, 0, 1, 0, true) : launch_row_fwd(*c, 0, 0, true);
        return e;
    };
    HIP_TRY(launch());   // warm
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ADMM_E_DEVICE, "hipEventCreate failed");
    }
    hipError_t e = hipEventRecord(e0, P->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, P->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(ADMM_E_DEVICE, "timing %s failed: %s", kernel, hipGetErrorString(e));
    *avg_ms = (double)ms / reps;
    return ADMM_OK;
}
