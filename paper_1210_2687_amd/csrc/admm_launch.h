// admm_launch.h — host-side launchers of the gfx950 kernels (internal interface).
#pragma once
#include <hip/hip_runtime.h>
#include "admm_internal.h"

namespace admm {

constexpr int ADMM_FRAME_CLASSES = 16;   // (analysis, synthesis) x levels 1..4 x (small image)
// column classes: 2 x (size class of the column length) + 1 for a general
// schedule (first or last stage not radix 8: the column cannot stay in
// registers around the solve), each launched with its own instantiation,
// classes 6 and 7 for columns of 2049..4096 and 4097..8192 (block-level
// transforms, any schedule), and class 8 for longer columns (split into
// sub-transforms of at most 8192 around a radix pass through HBM)
constexpr int ADMM_COL_CLASSES = 9;
// size classes of the row length: <= 512, <= 1024, <= 2048, <= 4096, <= 8192,
// <= 16384 (rows longer than 2048 run the plain row passes only; a TV problem
// with such rows takes the three-pass schedule: inverse rows with the data
// step, the TV step, forward rows)
constexpr int ADMM_ROW_CLASSES = 6;
constexpr int ADMM_RTV_SUBS = 2;   // narrower-block launches per fused TV row class

// Everything a launch needs; item lists are device arrays, counts are the grid sizes.
struct LaunchCtx {
    hipStream_t stream = nullptr;
    const ProbDesc* desc = nullptr;
    const WorkItem* col_items = nullptr;
    int ncol = 0;
    const WorkItem* row_items = nullptr;   // rows of TV problems (fused pass) or of FA problems
    int nrow = 0;
    const WorkItem* frm_items = nullptr;
    int nfrm = 0;
    InfoDev* info = nullptr;
    double* partials = nullptr;
    const float2* tw = nullptr;
    const float* s2 = nullptr;
    // classes of the column pass (col_class) and size classes of the TV row pass
    // (0: length <= 512, 1: <= 1024, 2: <= 2048), each launched with its own
    // instantiation: the items of class c are [beg[c], beg[c] + cnt[c]) of
    // col_items / row_items
    int col_beg[ADMM_COL_CLASSES] = {}, col_cnt[ADMM_COL_CLASSES] = {};
    size_t lds_col_c[ADMM_COL_CLASSES] = {};
    int rtv_beg[ADMM_ROW_CLASSES] = {}, rtv_cnt[ADMM_ROW_CLASSES] = {};
    size_t lds_rtv_c[ADMM_ROW_CLASSES] = {};
    // fused TV row classes 0..2: their first rtv_sub[c][0], then rtv_sub[c][1]
    // items run in blocks of row_tv_sub_threads(c, t) threads (LDS lds_rtv_sub)
    int rtv_sub[3][ADMM_RTV_SUBS] = {};
    size_t lds_rtv_sub[3][ADMM_RTV_SUBS] = {};
    // size classes of the plain row passes (FA rows, blur, state import) over row_items
    int rrow_beg[ADMM_ROW_CLASSES] = {}, rrow_cnt[ADMM_ROW_CLASSES] = {};
    size_t lds_rrow_c[ADMM_ROW_CLASSES] = {};
    // the first rrow_sub0 items of class 0 run in blocks of row_sub_threads() threads
    int rrow_sub0 = 0;
    size_t lds_rrow_sub0 = 0;
    // frame classes (levels 1..4, image smaller than a window or not): items of
    // class c are [frm_beg[c], frm_beg[c] + frm_cnt[c]) of frm_items
    int frm_beg[ADMM_FRAME_CLASSES] = {}, frm_cnt[ADMM_FRAME_CLASSES] = {};
    size_t lds_frm_c[ADMM_FRAME_CLASSES] = {};
    // method CG: two sums per row block (p^T p, p^T S p; written by the inverse
    // row pass, modes 2 and 3); the TV step's LDS (method CG, and TV-MD rows
    // longer than 2048)
    double* cgpart = nullptr;
    size_t lds_tvstep = 0;
    int tv_cpt = 8;   // columns per thread the TV step's row walk needs (8: rows <= 4096, 16: <= 8192, 32)
};

hipError_t launch_col(const LaunchCtx& L, int par, int mode);
hipError_t launch_row_tv(const LaunchCtx& L, int par, int flags);
hipError_t launch_row_fwd(const LaunchCtx& L, int par, int src, bool gated);
hipError_t launch_row_inv(const LaunchCtx& L, int par, int mode, int flags, bool gated);
hipError_t launch_frame(const LaunchCtx& L, int par, int flags, int import_mode, bool gated);
hipError_t launch_reduce(const LaunchCtx& L, int count, double tol, double obj_tol, int iter, int final_iter,
                         const int* iter_dev = nullptr, int* host_active = nullptr);
hipError_t launch_tick(const LaunchCtx& L, int* counter, int c, bool set);   // counter = set ? c : counter + c
hipError_t launch_zero(hipStream_t stream, float* p, size_t n);
hipError_t launch_scale(hipStream_t stream, const float* d, float* p, size_t n, float s);
hipError_t launch_import_tv(const LaunchCtx& L, int prob, size_t n);
hipError_t launch_import_fa(const LaunchCtx& L, int prob, size_t n);
hipError_t launch_lambda(const LaunchCtx& L, int prob, size_t HP, const float2* T, int ks);
hipError_t launch_warmstart(const LaunchCtx& L, int prob, size_t n, const float* x0, const float* p0,
                            const float* y, float* u1, float* d1, float* ureg, float* dreg);

// Reeves-Sorel variants (method CG), over the row items of the context
hipError_t launch_cg_update(const LaunchCtx& L, int flags);
// the TV step over a z plane (TV-CG; TV-MD rows longer than 2048)
hipError_t launch_tv_step(const LaunchCtx& L, int par, int flags);
size_t lds_tvstep_bytes(int W, int B);
hipError_t allow_dynamic_lds_cg(int bytes);

hipError_t allow_dynamic_lds(int bytes);
size_t lds_col_bytes(int H, int TC);
size_t lds_rowtv_bytes(int W, int B);
size_t lds_row_bytes(int W, int B);
size_t lds_frame_bytes(int J);
int frame_class(int H, int W, int J, bool fs);   // 8 fs + 2 (J - 1) + (image smaller than a window)
int col_max_tiles();                       // columns per column-pass block (one per wave)
int row_tv_max_rows(int w);                  // rows per block of the TV row pass for width w
int row_tv_sub_threads(int c, int t);        // threads of narrower-block launch t of fused TV class c (0: none)
int row_sub_threads();                       // threads of the plain row passes' narrower blocks (rows <= that)
int row_max_rows(int w);                     // rows per block of the plain row passes for width w
int size_class(int n);                      // 0: n <= 512, 1: <= 1024, 2: <= 2048, 3: <= 4096, 4: <= 8192, 5: larger
int col_class(const ProbDesc& d);           // 2 size_class(H) + (general column schedule); 6, 7, 8 above 2048
int col_split_factor(int h);                // radix of the HBM pass of a split column transform (1: none)
int col_big_threads(int h);                 // threads per block of the block-level column pass
constexpr int COL_BIG_MAXE = 16;            // its operands per thread in a stage
int row_maxe(int w);                        // operands per thread in a stage of the row passes for width w
int row_threads(int w);                     // threads per block of the plain row passes for width w
int block_threads();

}  // namespace admm
