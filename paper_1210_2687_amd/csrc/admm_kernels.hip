// admm_kernels.hip — gfx950 kernels of the mask-decoupled ADMM iteration.
//
// One TV-MD iteration (Alg. 3 with the data step of eq. (49)) is two launches:
//
//   k_col     column pass, one work item = TC columns of the transposed half
//             spectrum: forward column DFT of (zeta1^, s^), the circulant solve
//             z^ = K (mu1 conj(Lambda) zeta1^ + s^) with
//             K = 1 / (mu1 |Lambda|^2 + mu2 (|Delta^h|^2 + |Delta^v|^2))   (eq. (33)),
//             A z^ = Lambda z^, inverse column DFT; in place.
//   k_row_tv  row pass, one work item = B rows plus a one-row halo on each side:
//             inverse row DFT of (z^ + i A z^) -> z, A z; mask prox and data
//             dual (eq. (49)); vector soft threshold and TV duals (Sec. III-C);
//             zeta1 = u1 + d1 and s = mu2 D^T (u_TV + d_TV) for the next
//             iteration; forward row DFT of (mu1 zeta1 + i s) -> next half spectra.
//             Residual partial sums on check iterations.
//
// FA-MD (Sec. IV-C) uses k_col with K = 1 / (mu1 |Lambda|^2 + mu2) (eq. (25)),
// then k_row_inv (inverse rows + data step), k_frame (frame analysis, soft
// threshold, frame duals and synthesis q = mu2 P^T (u2 + d2)) and k_row_fwd.
//
// Long sides: columns longer than 2048 take k_col_big (one block per column),
// those longer than 8192 split into sub-transforms around k_col_split's radix
// pass through HBM; TV rows longer than 2048 run k_row_inv (data step),
// k_tv_step and k_row_fwd in place of k_row_tv.
#include <algorithm>

#include "admm_internal.h"
#include "fft_lds.h"
#include "admm_launch.h"

namespace admm {

constexpr int NT = 512;            // threads per block of the FFT passes
constexpr int MAXE_ROW = 16;       // float2 elements per thread in the row passes
constexpr int ROW_BURST = 8;       // plane elements per thread fetched together by the FA row passes
// rows of the TV row pass's epilogue inputs requested before its inverse
// transforms, per size class (as many as keep the kernel at 128 VGPRs or fewer,
// two blocks per compute unit)
constexpr int RTV_EARLY[3] = {5, 3, 1};
// Narrower blocks of the TV row pass, per fused size class: rows of at most
// CPT x RTV_SUB_NT[c][t] take blocks of that many threads (the first such t),
// so that fewer lanes idle past the row's end; the others 512 (0: unused).
constexpr int RTV_SUB_NT[3][ADMM_RTV_SUBS] = {{256, 384}, {384, 0}, {0, 0}};
// The plain row passes likewise run rows of at most RROW_SUB_NT columns (size
// class 0) in blocks of that many threads.
constexpr int RROW_SUB_NT = 256;
// most rows per block of the plain row passes, per size class (W <= 512, 1024, 2048, 4096, 8192, 16384)
constexpr int ROW_RB[ADMM_ROW_CLASSES] = {16, 8, 4, 4, 2, 1};
// Rows longer than 2048: the plain row passes run NTL threads per block up to
// rows of 8192 (the padded rows fill the LDS of a compute unit, so one block
// per unit, and 16 waves hide more latency than 8; one row of 16384 keeps 512
// threads, whose 32 entries each would not fit the 128 registers of a
// 1024-thread block) and read the stage table from global memory
// through the caches, so that four padded rows fit the LDS (two rows would
// write 32-byte pieces of the transposed spectrum, which the caches do not
// merge at this size: measured at 2.4x the spectrum's bytes).
constexpr int NTL = 1024;
template <int CPT, int NTR = NT> constexpr bool row_twg() { return CPT * NTR > 2048; }
template <int CPT, int NTR = NT> constexpr int row_maxe_c() { return row_twg<CPT, NTR>() && NTR < 1024 ? 32 : MAXE_ROW; }

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// ------------------------------------------------------------ block reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sum ADMM_NSUM per-thread values over each wave into wsum[wave][0..NSUM) (LDS).
__device__ __forceinline__ void wave_sums_to_lds(const double* v, double* wsum) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < ADMM_NSUM; ++i) {
        const double s = wave_sum(v[i]);
        if (lane == 0) wsum[wave * ADMM_NSUM + i] = s;
    }
}

// Sum ADMM_NSUM per-thread values over the block (NTH threads) and write them
// to out[0..NSUM). scratch: >= (NTH/64) * ADMM_NSUM doubles of LDS.
template <int NTH = NT>
__device__ __forceinline__ void block_sums_write(const double* v, double* scratch, double* out) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ADMM_NSUM; ++i) {
        double s = wave_sum(v[i]);
        if (lane == 0) scratch[wave * ADMM_NSUM + i] = s;
    }
    __syncthreads();
    if (tid < ADMM_NSUM) {
        double s = 0.0;
        for (int w = 0; w < NTH / 64; ++w) s += scratch[w * ADMM_NSUM + tid];
        out[tid] = s;
    }
}

// ------------------------------------------------------------ column pass
// Block of NTC threads = 4 waves; wave w owns column c0 + w of the work item
// (TC <= 4 columns; with fewer columns the spare waves leave after the shared
// twiddle table is loaded). The spectral solve of one entry:
//   TV  z^ = K (conj(Lambda) (mu1 zeta1)^ + s^),
//       K = 1 / (H W (mu1 |Lambda|^2 + mu2 (|Delta^h|^2 + |Delta^v|^2)))   (eq. (33))
//   FA  the same with mu2 in place of mu2 (|Delta^h|^2 + |Delta^v|^2)      (eq. (25))
// followed by A z^ = Lambda z^; the 1/(H W) of the inverse 2-D DFT is folded in.
// The row pass transforms mu1 zeta1 (not zeta1) so that both halves of the
// packed complex transform have comparable magnitude: the rounding of the
// larger half leaks into the other one when they are separated, and s is
// O(mu) while zeta1 is O(1).
constexpr int NTC = 256;

__device__ __forceinline__ float4 col_solve(float4 f, float2 lam, float w, float mu1, float mu2, float ihw, int mode) {
    if (mode == COL_SOLVE) {
        const float l2 = fmaf(lam.x, lam.x, lam.y * lam.y);
        // hardware reciprocal (about 1 ulp) instead of a correctly rounded
        // division: the denominator is positive and far from the range limits
        const float K = ihw * __builtin_amdgcn_rcpf(fmaf(mu1, l2, mu2 * w));
        const float rx = fmaf(lam.x, f.x, lam.y * f.y) + f.z;
        const float ry = fmaf(lam.x, f.y, -(lam.y * f.x)) + f.w;
        const float zx = K * rx, zy = K * ry;
        return make_float4(zx, zy, fmaf(lam.x, zx, -(lam.y * zy)), fmaf(lam.x, zy, lam.y * zx));
    }
    // COL_BLUR: (x^, 0) -> (Lambda x^ / (H W), 0)
    const float ax = fmaf(lam.x, f.x, -(lam.y * f.y)), ay = fmaf(lam.x, f.y, lam.y * f.x);
    return make_float4(ax * ihw, ay * ihw, 0.f, 0.f);
}

// EPL: most column entries per lane (H <= 64 EPL). GEN: the instantiation for
// general schedules (first or last stage not radix 8); the other one takes the
// columns whose schedule starts and ends with radix 8. Separate instantiations
// keep the registers of the fused path out of the general one (which needs
// fewer, so more waves fit a SIMD).
template <int EPL, bool GEN>
__global__ __launch_bounds__(NTC) void k_col(const ProbDesc* __restrict__ pd, const WorkItem* __restrict__ items,
                                             int nitems, int par, int mode, const InfoDev* __restrict__ info,
                                             const float2* __restrict__ tw, const float* __restrict__ s2tab) {
    extern __shared__ float4 cl[];
    const int wi = xcd_remap(blockIdx.x, gridDim.x);
    const WorkItem it = items[wi];
    if (info && !info[it.prob].active) return;
    const ProbDesc& p = pd[it.prob];
    const int H = p.H, c0 = it.start;
    const int nc = min(p.TC, p.P - c0);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr bool fused = !GEN;   // the host puts each column in the class of its schedule
    const int nbf = H >> 3;
    const int col = c0 + wave;
    const bool live = wave < nc;
    float4* S = ((p.reg == REG_TV && par) ? p.spec1 : p.spec0) + (size_t)col * H;
    const float2* L = p.lamhat + (size_t)col * H;
    const float* s2H = s2tab + p.fc.tw_off;
    const float mu1 = p.mu1, mu2 = p.mu2, ihw = p.inv_hw;
    const float w2 = (p.reg == REG_TV && live) ? s2tab[p.fr.tw_off + col] : 0.0f;

    // first radix-8 stage operands, Lambda and |Delta^v|^2 of the entries this
    // lane holds after the last forward stage (both sets are j + r H / 8)
    constexpr int NB8 = (EPL + 7) / 8;
    constexpr bool PF = EPL <= 16;
    float4 v[NB8][8];
    float2 lam[PF ? NB8 : 1][8];
    float wv[PF ? NB8 : 1][8];
    if (fused && live) {
#pragma unroll
        for (int i = 0; i < NB8; ++i) {
            const int j = lane + 64 * i;
            if (j < nbf) {
#pragma unroll
                for (int r = 0; r < 8; ++r) v[i][r] = gld(S, j + r * nbf);
                if (PF) {
#pragma unroll
                    for (int r = 0; r < 8; ++r) {
                        lam[PF ? i : 0][r] = gld(L, j + r * nbf);
                        wv[PF ? i : 0][r] = s2H[j + r * nbf];
                    }
                }
            }
        }
    }
    float2* twg = reinterpret_cast<float2*>(cl);
    load_twiddles<(64 * EPL + NTC - 1) / NTC>(twg, tw + p.fc.tw_off + H, H, tid, NTC);   // the stage table
    __syncthreads();
    if (!live) return;
    const ADMM_LDS float2* stw = (const ADMM_LDS float2*)twg;
    ADMM_LDS float4* buf = (ADMM_LDS float4*)(cl + (H + 1) / 2 + wave * pidx_len(H));
    const int nst = p.fc.nst;
    // the fixed-length transform when the column length is the instantiation's maximum
    constexpr int NF = 64 * EPL;
    constexpr int NST = CSched<NF>::nst();
    static_assert(CSched<NF>::rad(0) == 8 && CSched<NF>::rad(NST - 1) == 8 && CSt<NF, 0>::NB == NB8,
                  "fixed column length must start and end with radix 8");
    const bool fixed = H == NF && p.fc.variant == 0;
    // and half that length (256 in the 512 instantiation: columns of 256^2 problems)
    constexpr int NH = NF / 2;
    constexpr bool HALF = NF == 512;
    const bool fixedh = HALF && H == NH && p.fc.variant == 0;

    if (fused) {
        // forward: stage 0 (radix 8, no twiddles) from registers
#pragma unroll
        for (int i = 0; i < NB8; ++i) {
            const int j = lane + 64 * i;
            if (j < nbf) {
                dft<8, false>(v[i]);
                if (nst > 1) {
#pragma unroll
                    for (int r = 0; r < 8; ++r) lds_st(buf + 9 * j + r, v[i][r]);   // pidx(8 j + r)
                }
            }
        }
        if (nst > 1) {
            lane_exchange_fence();
            if (fixed) {
                c_stages<NF, 1, NST - 1, false>(buf, stw, lane);
                c_load<NF, NST - 1>(buf, v, lane);
                c_bfly<NF, NST - 1, false>(stw, v, lane);
            } else if (HALF && fixedh) {
                if constexpr (HALF) {
                    constexpr int NSH = CSched<NH>::nst();
                    c_stages<NH, 1, NSH - 1, false>(buf, stw, lane);
                    c_load<NH, NSH - 1>(buf, v, lane);
                    c_bfly<NH, NSH - 1, false>(stw, v, lane);
                }
            } else {
                wave_stages<EPL, false>(buf, stw, p.fc, 1, nst - 1, lane);
                // last stage (radix 8, Ns = H / 8): output r of butterfly j is entry j + r H / 8
                const ADMM_LDS float2* tl = stw + p.fc.tso[nst - 1];
#pragma unroll
                for (int i = 0; i < NB8; ++i) {
                    const int j = lane + 64 * i;
                    if (j < nbf) {
#pragma unroll
                        for (int r = 0; r < 8; ++r) v[i][r] = lds_ld(buf + pidx(j + r * nbf));
#pragma unroll
                        for (int r = 1; r < 8; ++r) v[i][r] = cmul(v[i][r], lds_ld(tl + 7 * j + r - 1));
                        dft<8, false>(v[i]);
                    }
                }
            }
            lane_exchange_fence();
        }
        // solve, then the first inverse stage (radix 8, no twiddles) on the same entries
#pragma unroll
        for (int i = 0; i < NB8; ++i) {
            const int j = lane + 64 * i;
            if (j < nbf) {
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int k1 = j + r * nbf;
                    const float2 lm = PF ? lam[PF ? i : 0][r] : gld(L, k1);
                    const float w = p.reg == REG_TV ? (PF ? wv[PF ? i : 0][r] : s2H[k1]) + w2 : 1.0f;
                    v[i][r] = col_solve(v[i][r], lm, w, mu1, mu2, ihw, mode);
                }
                dft<8, true>(v[i]);
                if (nst > 1) {
#pragma unroll
                    for (int r = 0; r < 8; ++r) lds_st(buf + 9 * j + r, v[i][r]);
                }
            }
        }
        if (nst > 1) {
            lane_exchange_fence();
            if (fixed) {
                c_stages<NF, 1, NST - 1, true>(buf, stw, lane);
                c_load<NF, NST - 1>(buf, v, lane);
                c_bfly<NF, NST - 1, true>(stw, v, lane);
            } else if (HALF && fixedh) {
                if constexpr (HALF) {
                    constexpr int NSH = CSched<NH>::nst();
                    c_stages<NH, 1, NSH - 1, true>(buf, stw, lane);
                    c_load<NH, NSH - 1>(buf, v, lane);
                    c_bfly<NH, NSH - 1, true>(stw, v, lane);
                }
            } else {
                wave_stages<EPL, true>(buf, stw, p.fc, 1, nst - 1, lane);
                const ADMM_LDS float2* tl = stw + p.fc.tso[nst - 1];
#pragma unroll
                for (int i = 0; i < NB8; ++i) {
                    const int j = lane + 64 * i;
                    if (j < nbf) {
#pragma unroll
                        for (int r = 0; r < 8; ++r) v[i][r] = lds_ld(buf + pidx(j + r * nbf));
#pragma unroll
                        for (int r = 1; r < 8; ++r) {
                            float2 w = lds_ld(tl + 7 * j + r - 1);
                            w.y = -w.y;
                            v[i][r] = cmul(v[i][r], w);
                        }
                        dft<8, true>(v[i]);
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < NB8; ++i) {
            const int j = lane + 64 * i;
            if (j < nbf) {
#pragma unroll
                for (int r = 0; r < 8; ++r) gst(S, j + r * nbf, v[i][r]);
            }
        }
        return;
    }

    // general schedule: the whole column goes through LDS. Its entries (GC per
    // lane at a time), and Lambda and |Delta^v|^2 for the solve (GS at a time),
    // are fetched in bursts of unconditional loads (indices clamped), not one
    // round trip each.
    constexpr int GC = 8;
#pragma unroll
    for (int c0 = 0; c0 < EPL; c0 += GC) {
        float4 t[GC];
#pragma unroll
        for (int u = 0; u < GC; ++u) t[u] = gld(S, min(lane + 64 * (c0 + u), H - 1));
#pragma unroll
        for (int u = 0; u < GC; ++u) {
            const int e = lane + 64 * (c0 + u);
            if (e < H) lds_st(buf + pidx(e), t[u]);
        }
        lane_exchange_fence();   // one chunk in registers at a time
    }
    lane_exchange_fence();
    wave_stages<EPL, false>(buf, stw, p.fc, 0, nst, lane);
    lane_exchange_fence();
    constexpr int GS = 4;   // solve entries per lane per burst (each solve holds a division's temporaries)
#pragma unroll 1
    for (int c0 = 0; c0 < EPL; c0 += GS) {
        float2 lm[GS];
        float wq[GS];
#pragma unroll
        for (int u = 0; u < GS; ++u) {
            const int e = min(lane + 64 * (c0 + u), H - 1);
            lm[u] = gld(L, e);
            wq[u] = p.reg == REG_TV ? s2H[e] + w2 : 1.0f;
        }
#pragma unroll
        for (int u = 0; u < GS; ++u) {
            const int e = lane + 64 * (c0 + u);
            if (e < H) lds_st(buf + pidx(e), col_solve(lds_ld(buf + pidx(e)), lm[u], wq[u], mu1, mu2, ihw, mode));
        }
        lane_exchange_fence();
    }
    lane_exchange_fence();
    wave_stages<EPL, true>(buf, stw, p.fc, 0, nst, lane);
    lane_exchange_fence();
    for (int e = lane; e < H; e += 64) gst(S, e, lds_ld(buf + pidx(e)));
}

// Column pass for columns longer than 2048: one block of NTB threads per
// column, or, for columns longer than 8192, per sub-transform of a split column
// (work item sub = k1: the csp-th part of the column at k1 H / csp, whose
// entry e holds the spectrum at frequency k1 + csp e after the forward
// transform; k_col_split runs before and after). The column (float4 entries:
// the two packed complex sequences) sits in LDS and every stage runs
// block-wide (fft_lds over float4 elements, any schedule of the plan); the
// stage table is read from global memory through the caches (it is shared by
// every column of the length). The solve between the transforms is the one of
// k_col, entry by entry.
// Columns of up to 4096 take 512 threads (two blocks share a compute unit),
// longer ones 1024 (the column's LDS allows one block per compute unit, and
// 16 waves hide more latency than 8). Every thread holds up to 8 column
// entries (H <= 8 NTB) and up to 16 float4 operands in a stage.
constexpr int NLB = 8;
constexpr int MAXE_BIG = 16;
template <int NTB>
__global__ __launch_bounds__(NTB) void k_col_big(const ProbDesc* __restrict__ pd, const WorkItem* __restrict__ items,
                                                 int nitems, int par, int mode, const InfoDev* __restrict__ info,
                                                 const float2* __restrict__ tw, const float* __restrict__ s2tab) {
    extern __shared__ float4 cl[];
    const WorkItem it = items[xcd_remap(blockIdx.x, gridDim.x)];
    if (info && !info[it.prob].active) return;
    const ProbDesc& p = pd[it.prob];
    const int H = p.H, col = it.start;   // one column (or sub-transform) per work item
    const int tid = threadIdx.x;
    const int csp = p.csp > 1 ? p.csp : 1, k1 = it.sub;
    const FftPlanDev& f = csp > 1 ? p.fc2 : p.fc;
    const int Hs = H / csp;                                        // this transform's length
    float4* S = ((p.reg == REG_TV && par) ? p.spec1 : p.spec0) + (size_t)col * H + (size_t)k1 * Hs;
    const float2* L = p.lamhat + (size_t)col * H;                  // indexed by frequency k1 + csp e
    const float* s2H = s2tab + p.fc.tw_off;
    const float mu1 = p.mu1, mu2 = p.mu2, ihw = p.inv_hw;
    const float w2 = p.reg == REG_TV ? s2tab[p.fr.tw_off + col] : 0.0f;
    float4* buf = cl;                                              // the column, padded (pidx)
    ADMM_LDS float4* const bl = (ADMM_LDS float4*)buf;
    const float2* tws = tw + f.tw_off + Hs;                        // stage table: Hs - 1 entries
    // the column, then the solve's coefficients, each in one burst of
    // unconditional loads (indices clamped), so that the block waits for one
    // memory latency instead of one per element
    {
        float4 v[NLB];
#pragma unroll
        for (int u = 0; u < NLB; ++u) v[u] = gld(S, (unsigned)min(tid + u * NTB, Hs - 1));
#pragma unroll
        for (int u = 0; u < NLB; ++u) {
            const int e = tid + u * NTB;
            if (e < Hs) lds_st(bl + pidx(e), v[u]);
        }
    }
    __syncthreads();
    fft_lds<MAXE_BIG, false, true, true, false>(buf, f, tws, 1, 0, tid, NTB);
    // (fetched after the transform: held across it, they would cost the
    // registers that let two blocks share a compute unit)
    float2 lm[NLB];
    float wq[NLB];
#pragma unroll
    for (int u = 0; u < NLB; ++u) {
        const unsigned k = (unsigned)(k1 + csp * min(tid + u * NTB, Hs - 1));
        lm[u] = gld(L, k);
        wq[u] = p.reg == REG_TV ? gld(s2H, k) + w2 : 1.0f;
    }
#pragma unroll
    for (int u = 0; u < NLB; ++u) {   // computed on clamped entries too, so that the loads above stay in their burst
        const int e = tid + u * NTB;
        const float4 z = col_solve(lds_ld(bl + pidx(min(e, Hs - 1))), lm[u], wq[u], mu1, mu2, ihw, mode);
        if (e < Hs) lds_st(bl + pidx(e), z);
    }
    __syncthreads();
    fft_lds<MAXE_BIG, true, true, true, false>(buf, f, tws, 1, 0, tid, NTB);
    for (int e = tid; e < Hs; e += NTB) gst(S, (unsigned)e, lds_ld(bl + pidx(e)));
}

// The radix-csp pass of a split column transform (columns longer than 8192,
// H = csp Hs): the column is taken as csp interleaved sequences. Forward
// (decimation in frequency), for each n2 < Hs:
//   y_k1[n2] = w_H^(n2 k1) sum_n1 x[n2 + Hs n1] w_csp^(n1 k1),   w_N = exp(-2 pi i / N),
// stored at k1 Hs + n2, so that the length-Hs transform of y_k1 holds the
// column's spectrum at the frequencies k1 + csp k2. Inverse: the same steps
// undone in reverse order (conjugate twiddles, then the inverse csp-point DFT
// back to n2 + Hs n1). Both are in place: the csp entries a thread reads are
// the ones it writes. Work item (column, sub = s): the s-th of csp slices of
// the n2 range of that column.
constexpr int NTS = 256;
template <int R, bool INV>
__device__ __forceinline__ void col_split_one(float4* __restrict__ S, const float2* __restrict__ twH, int Hs, int n2) {
    float4 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = gld(S, (unsigned)(n2 + Hs * r));
    if (INV) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
            float2 w = gld(twH, (unsigned)(n2 * r));
            w.y = -w.y;
            v[r] = cmul(v[r], w);
        }
        dft<R, true>(v);
    } else {
        dft<R, false>(v);
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], gld(twH, (unsigned)(n2 * r)));
    }
#pragma unroll
    for (int r = 0; r < R; ++r) gst(S, (unsigned)(n2 + Hs * r), v[r]);
}

template <bool INV>
__global__ __launch_bounds__(NTS) void k_col_split(const ProbDesc* __restrict__ pd, const WorkItem* __restrict__ items,
                                                   int nitems, int par, const InfoDev* __restrict__ info,
                                                   const float2* __restrict__ tw) {
    const WorkItem it = items[xcd_remap(blockIdx.x, gridDim.x)];
    if (info && !info[it.prob].active) return;
    const ProbDesc& p = pd[it.prob];
    const int H = p.H, csp = p.csp, Hs = H / csp;
    float4* S = ((p.reg == REG_TV && par) ? p.spec1 : p.spec0) + (size_t)it.start * H;
    const float2* twH = tw + p.fc.tw_off;   // w_H^k, k < H (n2 k1 < H)
    const int per = (Hs + csp - 1) / csp;
    const int n0 = it.sub * per, n1 = min(n0 + per, Hs);
    for (int n2 = n0 + (int)threadIdx.x; n2 < n1; n2 += NTS) {
        switch (csp) {
            case 2: col_split_one<2, INV>(S, twH, Hs, n2); break;
            case 3: col_split_one<3, INV>(S, twH, Hs, n2); break;
            case 5: col_split_one<5, INV>(S, twH, Hs, n2); break;
            default: col_split_one<7, INV>(S, twH, Hs, n2); break;
        }
    }
}

// ------------------------------------------------------------ row helpers
// Load transposed half-spectrum rows [rbeg, rbeg + nrows) (wrapping mod H) as
// full complex rows Y = z^ + i A z^ (Hermitian completion of both halves), row
// rr at X + rr pitch, padded (pidx) if PAD. The first NLD entries of each
// thread are fetched in one burst of unconditional loads (indices past the
// end clamped to the last entry) so that one memory latency covers them; the
// loop after it takes any remainder (none when P nrows <= NLD NT, which the
// launch configurations guarantee). The stage table of the row transforms
// (n entries, when twl is given) is fetched behind the burst.
template <bool PAD>
__device__ __forceinline__ void store_hermitian(float2* X, int pitch, int W, int P, int k2, int rr, float4 f) {
    float2* row = X + rr * pitch;
    if (k2 == 0 || 2 * k2 == W) {
        row[PAD ? pidx(k2) : k2] = make_float2(f.x, f.z);  // real parts only at DC / Nyquist
    } else {
        row[PAD ? pidx(k2) : k2] = make_float2(f.x - f.w, f.y + f.z);
        if (k2 <= W - P) row[PAD ? pidx(W - k2) : W - k2] = make_float2(f.x + f.w, f.z - f.y);
    }
}

template <bool PAD, int NLD, int NTW = 1, int NTH = NT>
__device__ __forceinline__ void load_rows_hermitian(float2* X, int pitch, const float4* __restrict__ S, int H, int W,
                                                    int P, int rbeg, int nrows, int tid, float2* twl = nullptr,
                                                    const float2* __restrict__ tw = nullptr, int ntw = 0) {
    const int tot = P * nrows;
    const unsigned mr = div_magic((unsigned)nrows);
    float4 f[NLD];
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
        const int i = min(tid + u * NTH, tot - 1);
        const int k2 = (int)udiv16((unsigned)i, (unsigned)nrows, mr);
        const int r = wrapi(rbeg + i - k2 * nrows, H);
        f[u] = gld(S, (unsigned)(k2 * H + r));
    }
    if (twl) load_twiddles<NTW>(twl, tw, ntw, tid, NTH);
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
        const int i = tid + u * NTH;
        if (i < tot) {
            const int k2 = (int)udiv16((unsigned)i, (unsigned)nrows, mr);
            store_hermitian<PAD>(X, pitch, W, P, k2, i - k2 * nrows, f[u]);
        }
    }
    for (int i = tid + NLD * NTH; i < tot; i += NTH) {
        const int k2 = (int)udiv16((unsigned)i, (unsigned)nrows, mr);
        const int rr = i - k2 * nrows;
        store_hermitian<PAD>(X, pitch, W, P, k2, rr, gld(S, (unsigned)(k2 * H + wrapi(rbeg + rr, H))));
    }
}

// Split the row DFTs C of (a + i b) in X rows [0, nrows) into the half spectra of
// a and b and store them transposed at rows [r0, r0 + nrows).
template <bool PAD, int NTH = NT>
__device__ __forceinline__ void store_rows_split(const float2* X, int pitch, float4* __restrict__ S, int H, int W,
                                                 int P, int r0, int nrows, int tid) {
    const int tot = P * nrows;
    const unsigned mr = div_magic((unsigned)nrows);
    for (int i = tid; i < tot; i += NTH) {
        const int k2 = (int)udiv16((unsigned)i, (unsigned)nrows, mr);
        const int rr = i - k2 * nrows;
        const float2* row = X + rr * pitch;
        const int km = k2 == 0 ? 0 : W - k2;
        const float2 c = row[PAD ? pidx(k2) : k2];
        const float2 m = row[PAD ? pidx(km) : km];
        // A^ = (C + conj(Cm)) / 2 ; B^ = (C - conj(Cm)) / (2 i)
        gst(S, (unsigned)(k2 * H + r0 + rr),
            make_float4(0.5f * (c.x + m.x), 0.5f * (c.y - m.y), 0.5f * (c.y + m.y), 0.5f * (m.x - c.x)));
    }
}

// ------------------------------------------------------------ fused TV row pass
// CPT: columns per thread (W <= CPT * NTR); RB: most rows per block; NTR: threads
// (512, or fewer for rows that leave most of a 512-thread block idle). All global
// inputs of the epilogue are loaded in one burst after the inverse transform
// (register arrays indexed by the unrolled row loop), so the row steps, which
// exchange delta^h through LDS, wait on memory once rather than once per row.
template <int MAXE, int CPT, int RB, int EARLY, bool CHK, int NTR = NT>
__global__ __launch_bounds__(NTR) void k_row_tv(const ProbDesc* __restrict__ pd, const WorkItem* __restrict__ items,
                                               int nitems, int par, int flags, const InfoDev* __restrict__ info,
                                               const float2* __restrict__ tw, double* __restrict__ partials) {
    extern __shared__ float2 X[];
    const int wi = xcd_remap(blockIdx.x, gridDim.x);
    const WorkItem it = items[wi];
    if (!info[it.prob].active) return;
    const ProbDesc& p = pd[it.prob];
    const int H = p.H, W = p.W, P = p.P, r0 = it.start;
    const int nr = min(p.B, H - r0);
    __builtin_assume(nr >= 1);
    const int nrh = nr + 2;
    const int tid = threadIdx.x;
    const unsigned n = (unsigned)(H * W);   // planes hold at most 16384^2 values (1 GiB): 32-bit offsets
    const int pitch = row_pitch(W);                                        // padded rows (pidx)
    float* dl = reinterpret_cast<float*>(X + (size_t)(p.B + 2) * pitch);   // 2 x W: delta^h of the row (ping-pong)
    float2* twl = reinterpret_cast<float2*>(dl + 2 * W);                 // row twiddles

    const float4* Sin = par ? p.spec1 : p.spec0;
    float4* Sout = par ? p.spec0 : p.spec1;
    // Descriptor fields used after the epilogue's global stores, read once: the
    // compiler cannot tell that those stores leave the descriptor unchanged and
    // would reload each field (and wait for it) on every row.
    float* const D1 = p.d1;
    float* const XO = p.x;
    float* const U1P = p.u1p;
    float* const UREGP = p.uregp;
    float* const SU1 = p.st_u1;
    float* const SD1 = p.st_d1;
    float* const SUREG = p.st_ureg;
    float* const SDREG = p.st_dreg;
    const uint8_t* const MK = p.mask;
    const float* const YV = p.y;
    const float mu1 = p.mu1;
    const float* dh_in = par ? p.dreg1 : p.dreg0;
    const float* dv_in = dh_in + n;
    float* dh_out = par ? p.dreg0 : p.dreg1;
    float* dv_out = dh_out + n;

    // spectrum rows r0 - 1 .. r0 + nr (P <= NTR CPT / 2 + 1 entries each), then the stage table
    constexpr int NLD = ((NTR * CPT / 2 + 1) * (RB + 2) + NTR - 1) / NTR;
    load_rows_hermitian<true, NLD, CPT, NTR>(X, pitch, Sin, H, W, P, r0 - 1, nrh, tid, twl, tw + p.fr.tw_off + W, W);

    // Epilogue inputs: duals of rows r0-1 .. r0+nr-1, data of rows r0 .. r0+nr-1,
    // fetched unconditionally (rows past nr and columns past W are clamped to
    // valid ones and never used), so that no load waits for another. The first
    // EARLY rows are requested before the inverse transforms, whose arithmetic
    // then covers their latency; the rest after them (register budget).
    // A check iteration (CHK) also fetches u of the previous iteration (dual residual).
    float pdh[CPT][RB + 1], pdv[CPT][RB + 1], pd1[CPT][RB], py[CPT][RB];
    float pq1[CPT][CHK ? RB : 1], pqh[CPT][CHK ? RB : 1], pqv[CPT][CHK ? RB : 1];
    uint8_t pmk[CPT][RB];
    auto fetch_row = [&](int rr) {
        const int r = wrapi(r0 - 1 + min(rr, nr), H);
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const unsigned g = (unsigned)(r * W + min(tid + j * NTR, W - 1));
            pdh[j][rr] = gld(dh_in, g);
            pdv[j][rr] = gld(dv_in, g);
            if (rr > 0) {
                pd1[j][rr - 1] = gld(D1, g);
                pmk[j][rr - 1] = gld(MK, g);
                py[j][rr - 1] = gld(YV, g);
                if (CHK) {
                    pq1[j][CHK ? rr - 1 : 0] = gld(U1P, g);
                    pqh[j][CHK ? rr - 1 : 0] = gld(UREGP, g);
                    pqv[j][CHK ? rr - 1 : 0] = gld(UREGP, n + g);
                }
            }
        }
    };
#pragma unroll
    for (int rr = 0; rr < EARLY; ++rr) fetch_row(rr);
    __syncthreads();
    rows_fft<NTR * CPT, NTR, RB + 2, MAXE, true>(X, pitch, p.fr, twl, nrh, tid);
    // X[rr][c] = z + i A z for row r0 - 1 + rr

    const float tau = p.tau, mu2 = p.mu2, c1 = p.inv1pmu1;
    constexpr bool chk = CHK;                 // the launch picks the instantiation from F_CHECK
    double acc[ADMM_NSUM];
#pragma unroll
    for (int i = 0; i < ADMM_NSUM; ++i) acc[i] = 0.0;

#pragma unroll
    for (int rr = EARLY; rr <= RB; ++rr) fetch_row(rr);   // the rest of the epilogue burst
    float dvp[CPT], zet[CPT], dvc[CPT];

#pragma unroll
    for (int rr = 0; rr <= RB; ++rr) {
        if (rr > nr) break;
        const int r = wrapi(r0 - 1 + rr, H);
        const float2* Xr = X + rr * pitch;
        const float2* Xn = Xr + pitch;
        float* dlr = dl + (rr & 1) * W;
        // every lane computes (lanes past W on the last column, identical values),
        // only the global stores and the sums are guarded: the loaded values are
        // then used outside any branch and stay in the burst
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const bool live = tid + j * NTR < W;
            const int c = live ? tid + j * NTR : W - 1;
            {
                const float2 xc = Xr[pidx(c)];
                const float zc = xc.x;
                const float zh = Xr[pidx(c + 1 == W ? 0 : c + 1)].x - zc;
                const float zv = Xn[pidx(c)].x - zc;
                const unsigned g = (unsigned)(r * W + c);
                const float dh = pdh[j][rr], dv = pdv[j][rr];
                const float vh = zh - dh, vv = zv - dv;
                // hardware square root and reciprocal (about 1 ulp): the prox only
                // needs them when rho > tau > 0
                const float rho = __builtin_amdgcn_sqrtf(fmaf(vh, vh, vv * vv));
                const float sc = rho > tau ? (rho - tau) * __builtin_amdgcn_rcpf(rho) : 0.0f;
                const float uh = vh * sc, uv = vv * sc;
                const float dhn = uh - vh, dvn = uv - vv;      // d - (D z - u)
                dlr[c] = uh + dhn;
                dvc[j] = uv + dvn;
                if (rr > 0) {
                    const float Az = xc.y;
                    const float d1o = pd1[j][rr - 1];
                    const bool obs = pmk[j][rr - 1] != 0;
                    const float yv = obs ? py[j][rr - 1] : 0.0f;
                    const float v1 = Az - d1o;
                    const float u1 = obs ? fmaf(yv - v1, c1, v1) : v1;   // (y + mu1 v)/(1 + mu1) or v
                    const float d1n = u1 - v1;                           // d1 - (A z - u1)
                    zet[j] = u1 + d1n;
                  if (live) {
                    gst(D1, g, d1n);
                    gst(dh_out, g, dhn);
                    gst(dv_out, g, dvn);
                    if (flags & F_WRITE_X) gst(XO, g, zc);
                    if (chk) {
                        const float u1q = pq1[j][CHK ? rr - 1 : 0], uhq = pqh[j][CHK ? rr - 1 : 0],
                                    uvq = pqv[j][CHK ? rr - 1 : 0];
                        const float e0 = Az - u1, e1h = zh - uh, e1v = zv - uv;
                        const float f6 = u1 - u1q, f7h = uh - uhq, f7v = uv - uvq;
                        const float ry = yv - Az;
                        acc[0] += (double)(e0 * e0);
                        acc[1] += (double)fmaf(e1h, e1h, e1v * e1v);
                        acc[2] += (double)(Az * Az);
                        acc[3] += (double)fmaf(zh, zh, zv * zv);
                        acc[4] += (double)(u1 * u1);
                        acc[5] += (double)fmaf(uh, uh, uv * uv);
                        acc[6] += (double)(f6 * f6);
                        acc[7] += (double)fmaf(f7h, f7h, f7v * f7v);
                        acc[8] += (double)(d1n * d1n);
                        acc[9] += (double)fmaf(dhn, dhn, dvn * dvn);
                        acc[10] += obs ? (double)(ry * ry) : 0.0;
                        acc[11] += (double)sqrtf(fmaf(zh, zh, zv * zv));
                    }
                    if (flags & F_WRITE_UPREV) {
                        gst(U1P, g, u1);
                        gst(UREGP, g, uh);
                        gst(UREGP, n + g, uv);
                    }
                    if (flags & F_EXPORT) {
                        gst(SU1, g, u1);
                        gst(SD1, g, d1n);
                        gst(SUREG, g, uh);
                        gst(SUREG, n + g, uv);
                        gst(SDREG, g, dhn);
                        gst(SDREG, n + g, dvn);
                    }
                  }
                }
            }
        }
        __syncthreads();
        if (rr > 0) {
            float2* Xw = X + rr * pitch;
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int c = min(tid + j * NTR, W - 1);
                const float s = mu2 * ((dlr[c == 0 ? W - 1 : c - 1] - dlr[c]) + (dvp[j] - dvc[j]));
                Xw[pidx(c)] = make_float2(mu1 * zet[j], s);
            }
        }
#pragma unroll
        for (int j = 0; j < CPT; ++j) dvp[j] = dvc[j];
    }
    __syncthreads();
    if (flags & F_FORWARD) {
        rows_fft<NTR * CPT, NTR, RB, MAXE, false>(X + pitch, pitch, p.fr, twl, nr, tid);
        store_rows_split<true, NTR>(X + pitch, pitch, Sout, H, W, P, r0, nr, tid);
    }
    if (chk) block_sums_write<NTR>(acc, reinterpret_cast<double*>(X), partials + (size_t)(p.part_base + it.blk) * ADMM_NSUM);
}

// ------------------------------------------------------------ plane -> spectrum rows
// Forward row DFT of (a + i b) for rows [r0, r0 + nr) of two planes. NTR
// threads, CPT columns per thread (W <= CPT NTR), at most RB rows, rows padded
// (pidx) at row_pitch(W).
template <int CPT, int RB, int NTR = NT>
__global__ __launch_bounds__(NTR) void k_row_fwd(const ProbDesc* __restrict__ pd, const WorkItem* __restrict__ items,
                                                int nitems, int par, int src, const InfoDev* __restrict__ info,
                                                const float2* __restrict__ tw) {
    extern __shared__ float2 X[];
    const int wi = xcd_remap(blockIdx.x, gridDim.x);
    const WorkItem it = items[wi];
    if (info && !info[it.prob].active) return;
    const ProbDesc& p = pd[it.prob];
    const int H = p.H, W = p.W, P = p.P, r0 = it.start;
    const int nr = min(p.B, H - r0);
    const int tid = threadIdx.x;
    const int pitch = row_pitch(W);                           // padded rows (pidx)
    float2* twl = X + (size_t)p.B * pitch;                    // the stage table
    // src 0: (mu1 * zeta1, s) from (tmpA, tmpB); src 1: (x, 0) from tmpA (blur)
    const float* a = p.tmpA + (size_t)r0 * W;
    const float* b = p.tmpB + (size_t)r0 * W;
    const float mu1 = p.mu1;
    constexpr bool TWG = row_twg<CPT, NTR>();
    // the stage table, then bursts of RCH rows of both planes per thread
    // (unconditional loads, rows and columns clamped; the second plane is read
    // but not used for src 1), so that each burst costs one memory latency
    constexpr int RCH = CPT >= ROW_BURST ? 1 : ROW_BURST / CPT;
    const float2* tws = tw + p.fr.tw_off + W;
    float2 tv[CPT];
    if constexpr (!TWG) {
#pragma unroll
        for (int u = 0; u < CPT; ++u) tv[u] = gld(tws, (unsigned)min(tid + u * NTR, W - 1));
    }
    for (int rb = 0; rb < nr; rb += RCH) {
        float va[RCH][CPT], vb[RCH][CPT];
#pragma unroll
        for (int k = 0; k < RCH; ++k) {
            const int rr = min(rb + k, nr - 1);
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const unsigned g = (unsigned)(rr * W + min(tid + j * NTR, W - 1));
                va[k][j] = gld(a, g);
                vb[k][j] = gld(b, g);
            }
        }
        if (!TWG && rb == 0) {
#pragma unroll
            for (int u = 0; u < CPT; ++u)
                if (tid + u * NTR < W) twl[tid + u * NTR] = tv[u];
        }
#pragma unroll
        for (int k = 0; k < RCH; ++k) {
            const int rr = rb + k;
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int c = tid + j * NTR;
                if (rr < nr && c < W)
                    X[rr * pitch + pidx(c)] = src == 0 ? make_float2(mu1 * va[k][j], vb[k][j]) : make_float2(va[k][j], 0.0f);
            }
        }
    }
    __syncthreads();
    rows_fft<NTR * CPT, NTR, RB, row_maxe_c<CPT, NTR>(), false, TWG>(X, pitch, p.fr, TWG ? tws : twl, nr, tid);
    store_rows_split<true, NTR>(X, pitch, par ? p.spec1 : p.spec0, H, W, P, r0, nr, tid);
}

// ------------------------------------------------------------ spectrum rows -> planes
// Inverse row DFT of (z^ + i A z^) for rows [r0, r0 + nr).
//   mode 0 (blur): write z (the real part) to tmpB.
//   mode 1 (FA data step): z -> zpl, mask prox and data dual (eq. (40)), zeta1 -> tmpA;
//          for a synthesis problem (FS-MD) zpl receives x - s / mu2 = x - W zeta2 instead
//          (tmpB holds s = mu2 W zeta2 of the previous frame step).
//   mode 2, 3 (method CG): the two parts to (cgo1, cgao1), (cgo2, cgao2), and the
//          boundary-system direction and its sums (below).
// Rows padded as in k_row_fwd.
template <int CPT, int RB, int NTR = NT>
__global__ __launch_bounds__(NTR) void k_row_inv(const ProbDesc* __restrict__ pd, const WorkItem* __restrict__ items,
                                                int nitems, int par, int mode, int flags,
                                                const InfoDev* __restrict__ info, const float2* __restrict__ tw,
                                                double* __restrict__ partials) {
    extern __shared__ float2 X[];
    const int wi = xcd_remap(blockIdx.x, gridDim.x);
    const WorkItem it = items[wi];
    if (info && !info[it.prob].active) return;
    const ProbDesc& p = pd[it.prob];
    const int H = p.H, W = p.W, P = p.P, r0 = it.start;
    const int nr = min(p.B, H - r0);
    const int tid = threadIdx.x;
    const int pitch = row_pitch(W);
    constexpr bool TWG = row_twg<CPT, NTR>();
    const float2* const tws = tw + p.fr.tw_off + W;
    float2* const twl = TWG ? nullptr : X + (size_t)p.B * pitch;
    const float2* const stab = TWG ? tws : twl;
    // spectrum rows r0 .. r0 + nr - 1 (P <= NTR CPT / 2 + 1 entries each), then the stage table
    constexpr int NLD = ((NTR * CPT / 2 + 1) * RB + NTR - 1) / NTR;
    load_rows_hermitian<true, NLD, CPT, NTR>(X, pitch, par ? p.spec1 : p.spec0, H, W, P, r0, nr, tid, twl, tws, W);
    __syncthreads();
    rows_fft<NTR * CPT, NTR, RB, row_maxe_c<CPT, NTR>(), true, TWG>(X, pitch, p.fr, stab, nr, tid);
    const unsigned off = (unsigned)(r0 * W);
    if (mode == 0) {
        float* const TB = p.tmpB;   // read once: the stores below would make the compiler reload it
        for (int rr = 0; rr < nr; ++rr) {
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int c = tid + j * NTR;
                if (c < W) gst(TB, off + (unsigned)(rr * W + c), X[rr * pitch + pidx(c)].x);
            }
        }
        return;
    }
    if (mode >= 2) {
        // method CG: the two parts of the solve to (O, A O), and the boundary-system
        // step on the unobserved pixels. Mode 2 (first solve, O1 = C r / mu_t):
        // the direction p = B (C r + C B^T v) - v = mu_t A O1 + A e - v into
        // tmpA, p^T p, and the forward row DFT of (mu1 p, 0) into spec0, the
        // input of the second solve (as the forward row pass would compute it
        // from tmpA and a zero plane); mode 3 (second solve, O2 = C B^T p):
        // p^T (I - B C B^T) p = p^T (p - A O2). The block's sum goes to slot 0
        // or 1 of its pair in `partials` (the launcher passes the CG sums there).
        const bool first = mode == 2;
        float* const O = first ? p.cgo1 : p.cgo2;
        float* const AO = first ? p.cgao1 : p.cgao2;
        float* const TA = p.tmpA;
        const float* const AE = p.cgae;
        const float* const V = p.cgv;
        const uint8_t* const MK = p.mask;
        const float mut = p.mut, mu1 = p.mu1;
        double acc = 0.0;
        for (int rr = 0; rr < nr; ++rr) {
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int c = tid + j * NTR;
                if (c >= W) continue;
                const float2 xv = X[rr * pitch + pidx(c)];
                const unsigned g = off + (unsigned)(rr * W + c);
                gst(O, g, xv.x);
                gst(AO, g, xv.y);
                const bool obs = gld(MK, g) != 0;
                if (first) {
                    const float r = fmaf(mut, xv.y, gld(AE, g)) - gld(V, g);
                    const float pv = obs ? 0.0f : r;
                    gst(TA, g, pv);
                    X[rr * pitch + pidx(c)] = make_float2(mu1 * pv, 0.0f);   // the entry this thread read
                    acc += (double)pv * (double)pv;
                } else {
                    const float pv = gld(TA, g);
                    const float q = obs ? 0.0f : pv - xv.y;
                    acc += (double)pv * (double)q;
                }
            }
        }
        if (first) {
            __syncthreads();
            rows_fft<NTR * CPT, NTR, RB, row_maxe_c<CPT, NTR>(), false, TWG>(X, pitch, p.fr, stab, nr, tid);
            store_rows_split<true, NTR>(X, pitch, p.spec0, H, W, P, r0, nr, tid);
        }
        __syncthreads();   // X becomes the reduction scratch
        double* const red = reinterpret_cast<double*>(X);
        const double sw = wave_sum(acc);
        if ((tid & 63) == 0) red[tid >> 6] = sw;
        __syncthreads();
        if (tid == 0) {
            double sum = 0.0;
            for (int w = 0; w < NTR / 64; ++w) sum += red[w];
            partials[(size_t)(p.part_base + it.blk) * 2 + (first ? 0 : 1)] = sum;
        }
        return;
    }
    const float c1 = p.inv1pmu1;
    const bool chk = flags & F_CHECK;
    const bool fs = p.fs != 0;
    const float inv_mu2 = 1.0f / p.mu2;
    // descriptor fields read once (the row loop's global stores would make the
    // compiler reload each of them, and wait for it, on every row)
    float* const D1 = p.d1;
    float* const TA = p.tmpA;
    float* const ZP = p.zpl;
    float* const XO = p.x;
    float* const U1P = p.u1p;
    float* const SU1 = p.st_u1;
    float* const SD1 = p.st_d1;
    const uint8_t* const MK = p.mask;
    const float* const YV = p.y;
    const float* const SB = p.tmpB;
    double acc[ADMM_NSUM];
#pragma unroll
    for (int i = 0; i < ADMM_NSUM; ++i) acc[i] = 0.0;
    constexpr int RCH = CPT >= ROW_BURST ? 1 : ROW_BURST / CPT;
    for (int rb = 0; rb < nr; rb += RCH) {
        // one burst of unconditional loads (rows and columns clamped) per RCH rows
        float d1b[RCH][CPT], yb[RCH][CPT];
        uint8_t mb[RCH][CPT];
#pragma unroll
        for (int k = 0; k < RCH; ++k) {
            const int rr = min(rb + k, nr - 1);
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const unsigned g = off + (unsigned)(rr * W + min(tid + j * NTR, W - 1));
                d1b[k][j] = gld(D1, g);
                mb[k][j] = gld(MK, g);
                yb[k][j] = gld(YV, g);
            }
        }
#pragma unroll
        for (int k = 0; k < RCH; ++k) {
            const int rr = rb + k;
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int c = tid + j * NTR;
                if (rr >= nr || c >= W) continue;
                const unsigned g = off + (unsigned)(rr * W + c);
                const float2 xv = X[rr * pitch + pidx(c)];
                const float z = xv.x, Az = xv.y;
                const float d1o = d1b[k][j];
                const bool obs = mb[k][j] != 0;
                const float yv = obs ? yb[k][j] : 0.0f;
                const float v1 = Az - d1o;
                const float u1 = obs ? fmaf(yv - v1, c1, v1) : v1;
                const float d1n = u1 - v1;
                gst(D1, g, d1n);
                gst(TA, g, u1 + d1n);
                gst(ZP, g, fs ? fmaf(-inv_mu2, gld(SB, g), z) : z);
                if (flags & F_WRITE_X) gst(XO, g, z);
                if (chk) {
                    const float e0 = Az - u1, f6 = u1 - gld(U1P, g), ry = yv - Az;
                    acc[0] += (double)(e0 * e0);
                    acc[2] += (double)(Az * Az);
                    acc[4] += (double)(u1 * u1);
                    acc[6] += (double)(f6 * f6);
                    acc[8] += (double)(d1n * d1n);
                    acc[10] += obs ? (double)(ry * ry) : 0.0;
                }
                if (flags & F_WRITE_UPREV) gst(U1P, g, u1);
                if (flags & F_EXPORT) {
                    gst(SU1, g, u1);
                    gst(SD1, g, d1n);
                }
            }
        }
    }
    if (chk) block_sums_write<NTR>(acc, reinterpret_cast<double*>(X), partials + (size_t)(p.part_base + it.blk) * ADMM_NSUM);
}

// ------------------------------------------------------------ TV state import
// From a caller state (u, d): working duals, zeta1 = u1 + d1 -> tmpA and
// s = mu2 D^T (u_TV + d_TV) -> tmpB, with the same expressions (and rounding)
// as the fused row pass so that a resumed solve continues bit for bit.
__global__ void k_import_tv(const ProbDesc* __restrict__ pd, int prob) {
    const ProbDesc& p = pd[prob];
    const int H = p.H, W = p.W;
    const size_t n = (size_t)H * W;
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int r = (int)(g / W), c = (int)(g - (size_t)r * W);
    const float* uh = p.st_ureg;
    const float* uv = p.st_ureg + n;
    const float* dh = p.st_dreg;
    const float* dv = p.st_dreg + n;
    const size_t gl = (size_t)r * W + (c == 0 ? W - 1 : c - 1);
    const size_t gu = (size_t)(r == 0 ? H - 1 : r - 1) * W + c;
    const float dlc = uh[g] + dh[g], dll = uh[gl] + dh[gl];
    const float dvc = uv[g] + dv[g], dvu = uv[gu] + dv[gu];
    p.tmpB[g] = p.mu2 * ((dll - dlc) + (dvu - dvc));
    p.tmpA[g] = p.st_u1[g] + p.st_d1[g];
    p.d1[g] = p.st_d1[g];
    p.dreg0[g] = dh[g];
    p.dreg0[n + g] = dv[g];
}

// ------------------------------------------------------------ second-stage reduction
// One block per problem: sum the block partials in a fixed order (deterministic),
// form the residuals and objective, update the problem's info and active flag.
// iter_dev (if given): the iteration number is iter_dev[0] + iter (graph
// replays of whole check periods); host_active (if given, host-mapped memory)
// receives each problem's active flag so that the host can see the end of a
// solve without synchronising.
__global__ __launch_bounds__(NT) void k_reduce(const ProbDesc* __restrict__ pd, const double* __restrict__ partials,
                                               InfoDev* __restrict__ info, double tol, double obj_tol, int iter,
                                               int final_iter, const int* __restrict__ iter_dev,
                                               int* __restrict__ host_active) {
    __shared__ double sm[NT / 64][ADMM_NSUM];
    const int prob = blockIdx.x;
    if (!info[prob].active) return;
    const ProbDesc& p = pd[prob];
    const int nblk = p.nrowblk + p.nfrmblk;
    const int tid = threadIdx.x;
    double v[ADMM_NSUM];
#pragma unroll
    for (int i = 0; i < ADMM_NSUM; ++i) v[i] = 0.0;
    for (int b = tid; b < nblk; b += NT) {
        const double* q = partials + (size_t)(p.part_base + b) * ADMM_NSUM;
#pragma unroll
        for (int i = 0; i < ADMM_NSUM; ++i) v[i] += q[i];
    }
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int i = 0; i < ADMM_NSUM; ++i) {
        double s = wave_sum(v[i]);
        if (lane == 0) sm[wave][i] = s;
    }
    __syncthreads();
    if (tid == 0) {
        double s[ADMM_NSUM];
        for (int i = 0; i < ADMM_NSUM; ++i) {
            s[i] = 0.0;
            for (int w = 0; w < NT / 64; ++w) s[i] += sm[w][i];
        }
        const double mu1 = p.mu1, mu2 = p.mu2;
        const double pri = sqrt(s[0] + s[1]);
        const double den = fmax(fmax(sqrt(s[2] + s[3]), sqrt(s[4] + s[5])), 1e-30);
        const double dual = sqrt(mu1 * mu1 * s[6] + mu2 * mu2 * s[7]);
        const double dden = fmax(sqrt(mu1 * mu1 * s[8] + mu2 * mu2 * s[9]), 1e-30);
        InfoDev f = info[prob];
        const bool had_check = f.iters > 0;   // a previous check iteration left its objective
        const double f_prev = f.objective;
        f.iters = iter_dev ? iter_dev[0] + iter : iter;
        f.r_pri = pri / den;
        f.r_dual = dual / dden;
        f.objective = 0.5 * s[10] + (double)p.lam * s[11];
        bool finite = true;
        for (int i = 0; i < ADMM_NSUM; ++i) finite = finite && isfinite(s[i]);
        if (!finite) {
            f.diverged = 1;
            f.active = 0;
        } else if ((tol > 0.0 && f.r_pri <= tol && f.r_dual <= tol) ||
                   (obj_tol > 0.0 && had_check && fabs(f.objective - f_prev) <= obj_tol * fabs(f_prev))) {
            f.converged = 1;
            f.active = 0;
        }
        if (final_iter) f.active = 0;
        info[prob] = f;
        if (host_active) host_active[prob] = f.active;
    }
}

// Zero n floats (the allocation-free solve clears its state with a kernel
// rather than a memset node, so that a caller may capture the stream).
__global__ void k_zero(float* __restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// Iteration counter of graph-replayed check periods: counter[0] += c (one
// lane; an ordinary vector store).
__global__ void k_tick(int* __restrict__ counter, int c, int set) {
    const int t = threadIdx.x;
    if (t == 0) counter[t] = set ? c : counter[t] + c;
}

// ------------------------------------------------------------ kernel spectrum
// Lambda[k2][k1] = sum_a exp(-2 pi i k1 a / H) T[a][k2], T[a][k2] = sum_b h[a, b]
// exp(-2 pi i k2 b / W) (eq. (19) for the centred kernel), T precomputed on the host.
__global__ void k_lambda(const ProbDesc* __restrict__ pd, int prob, const float2* __restrict__ T, int ks,
                         const float2* __restrict__ tw) {
    const ProbDesc& p = pd[prob];
    const int H = p.H, P = p.P;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)H * P) return;
    const int k2 = (int)(i / H), k1 = (int)(i - (size_t)k2 * H);
    const float2* twH = tw + p.fc.tw_off;
    const int l = ks / 2;
    float2 acc = make_float2(0.f, 0.f);
    for (int a = -l; a <= l; ++a) {
        int e = (int)(((long long)k1 * (a < 0 ? a + H : a)) % H);
        const float2 w = twH[e];
        const float2 t = T[(size_t)(a + l) * P + k2];
        acc.x = fmaf(w.x, t.x, fmaf(-w.y, t.y, acc.x));
        acc.y = fmaf(w.x, t.y, fmaf(w.y, t.x, acc.y));
    }
    p.lamhat[i] = acc;
}

// ------------------------------------------------------------ warm-start mapping
// u1 = A x0 (already in tmpB), d1 = m (y - A x0) / mu1, u_TV = D x0,
// d_TV = -(lambda / mu2) p0 / max(1, |p0|).
__global__ void k_warmstart(const ProbDesc* __restrict__ pd, int prob, const float* __restrict__ x0,
                            const float* __restrict__ p0, const float* __restrict__ y, float* u1, float* d1,
                            float* ureg, float* dreg) {
    const ProbDesc& p = pd[prob];
    const int H = p.H, W = p.W;
    const size_t n = (size_t)H * W;
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int r = (int)(g / W), c = (int)(g - (size_t)r * W);
    const float Ax = p.tmpB[g];
    const float xc = x0[g];
    u1[g] = Ax;
    d1[g] = p.mask[g] ? (y[g] - Ax) / p.mu1 : 0.0f;
    ureg[g] = x0[(size_t)r * W + (c + 1 == W ? 0 : c + 1)] - xc;
    ureg[n + g] = x0[(size_t)(r + 1 == H ? 0 : r + 1) * W + c] - xc;
    const float ph = p0[g], pv = p0[n + g];
    const float nrm = fmaxf(1.0f, sqrtf(fmaf(ph, ph, pv * pv)));
    const float sc = -(p.lam / p.mu2) / nrm;
    dreg[g] = sc * ph;
    dreg[n + g] = sc * pv;
}

// p = s d for the 2 n entries of a TV dual pair (s = -mu2 / lambda: the dual
// field whose warm-start mapping reproduces d_TV)
__global__ void k_scale2(const float* __restrict__ d, float* __restrict__ p, size_t n2, float s) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (size_t)gridDim.x * blockDim.x)
        p[i] = s * d[i];
}

// ------------------------------------------------------------ host launchers
static size_t col_lds(int H, int TC) {
    // the block-level column pass: the column (or sub-transform) alone
    if (H > 2048) return (size_t)pidx_len(H / col_split_factor(H)) * sizeof(float4);
    return (size_t)((H + 1) / 2) * sizeof(float4) + (size_t)TC * pidx_len(H) * sizeof(float4);
}
static size_t rowtv_lds(int W, int B) {
    const size_t b = (size_t)(B + 2) * row_pitch(W) * sizeof(float2) + 2 * (size_t)W * sizeof(float) +
                     (size_t)W * sizeof(float2);
    const size_t scratch = NT / 64 * ADMM_NSUM * sizeof(double);   // block partial sums reuse the buffer
    return b > scratch ? b : scratch;
}
static size_t row_lds(int W, int B) {
    // padded rows + the stage table (in global memory for rows longer than 2048)
    const size_t b = ((size_t)B * row_pitch(W) + (W > 2048 ? 0 : W)) * sizeof(float2);
    const size_t scratch = NT / 64 * ADMM_NSUM * sizeof(double);    // block sums reuse the rows
    return b > scratch ? b : scratch;
}

int size_class(int n) {
    return n <= 512 ? 0 : (n <= 1024 ? 1 : (n <= 2048 ? 2 : (n <= 4096 ? 3 : (n <= 8192 ? 4 : 5))));
}

int col_class(const ProbDesc& d) {
    if (d.H > 8192) return 8;
    return d.H > 4096 ? 7 : (d.H > 2048 ? 6 : 2 * size_class(d.H) + (d.fc.ends8 ? 0 : 1));
}

// The smallest prime factor of a 7-smooth length above 8192 (its HBM pass's
// radix: the sub-transforms are then at most 8192 long up to 16384).
int col_split_factor(int h) {
    if (h <= 8192) return 1;
    for (int p : {2, 3, 5, 7})
        if (h % p == 0) return p;
    return 1;
}

int col_big_threads(int h) { return h > 4096 ? 1024 : 512; }

namespace {
template <int EPL, bool GEN>
void launch_col_class(const LaunchCtx& L, int c, int par, int mode, const InfoDev* info) {
    const int n = L.col_cnt[c];
    hipLaunchKernelGGL((k_col<EPL, GEN>), dim3(n), dim3(NTC), L.lds_col_c[c], L.stream, L.desc,
                       L.col_items + L.col_beg[c], n, par, mode, info, L.tw, L.s2);
}
}  // namespace

hipError_t launch_col(const LaunchCtx& L, int par, int mode) {
    const InfoDev* info = mode == COL_SOLVE ? L.info : nullptr;
    for (int c = 0; c < ADMM_COL_CLASSES; ++c) {
        if (!L.col_cnt[c]) continue;
        switch (c) {
            case 0: launch_col_class<8, false>(L, c, par, mode, info); break;
            case 1: launch_col_class<8, true>(L, c, par, mode, info); break;
            case 2: launch_col_class<16, false>(L, c, par, mode, info); break;
            case 3: launch_col_class<16, true>(L, c, par, mode, info); break;
            case 4: launch_col_class<32, false>(L, c, par, mode, info); break;
            case 5: launch_col_class<32, true>(L, c, par, mode, info); break;
            case 6:
                hipLaunchKernelGGL(k_col_big<512>, dim3(L.col_cnt[c]), dim3(512), L.lds_col_c[c], L.stream, L.desc,
                                   L.col_items + L.col_beg[c], L.col_cnt[c], par, mode, info, L.tw, L.s2);
                break;
            case 7:
                hipLaunchKernelGGL(k_col_big<1024>, dim3(L.col_cnt[c]), dim3(1024), L.lds_col_c[c], L.stream, L.desc,
                                   L.col_items + L.col_beg[c], L.col_cnt[c], par, mode, info, L.tw, L.s2);
                break;
            default: {   // split columns: radix pass, sub-transforms with the solve, inverse radix pass
                const WorkItem* it = L.col_items + L.col_beg[c];
                const int n = L.col_cnt[c];
                hipLaunchKernelGGL(k_col_split<false>, dim3(n), dim3(NTS), 0, L.stream, L.desc, it, n, par, info, L.tw);
                hipLaunchKernelGGL(k_col_big<1024>, dim3(n), dim3(1024), L.lds_col_c[c], L.stream, L.desc, it, n, par,
                                   mode, info, L.tw, L.s2);
                hipLaunchKernelGGL(k_col_split<true>, dim3(n), dim3(NTS), 0, L.stream, L.desc, it, n, par, info, L.tw);
                break;
            }
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

namespace {
template <int CPT, int RB, int EARLY, int NTR>
void launch_row_tv_part(const LaunchCtx& L, const WorkItem* it, int n, size_t lds, int par, int flags) {
    if (n <= 0) return;
    if (flags & F_CHECK)
        hipLaunchKernelGGL((k_row_tv<MAXE_ROW, CPT, RB, EARLY, true, NTR>), dim3(n), dim3(NTR), lds, L.stream, L.desc,
                           it, n, par, flags, L.info, L.tw, L.partials);
    else
        hipLaunchKernelGGL((k_row_tv<MAXE_ROW, CPT, RB, EARLY, false, NTR>), dim3(n), dim3(NTR), lds, L.stream, L.desc,
                           it, n, par, flags, L.info, L.tw, L.partials);
}

// The class's items start with those of its narrower blocks (rtv_sub[c][t]
// items for RTV_SUB_NT[c][t] threads, in order); the rest take 512 threads.
template <int CPT, int RB, int EARLY, int NT0, int NT1>
void launch_row_tv_class(const LaunchCtx& L, int c, int par, int flags) {
    const WorkItem* it = L.row_items + L.rtv_beg[c];
    const int n = L.rtv_cnt[c];
    int off = 0;
    if constexpr (NT0 > 0) {
        const int m = std::min(L.rtv_sub[c][0], n - off);
        launch_row_tv_part<CPT, RB, EARLY, NT0>(L, it + off, m, L.lds_rtv_sub[c][0], par, flags);
        off += m;
    }
    if constexpr (NT1 > 0) {
        const int m = std::min(L.rtv_sub[c][1], n - off);
        launch_row_tv_part<CPT, RB, EARLY, NT1>(L, it + off, m, L.lds_rtv_sub[c][1], par, flags);
        off += m;
    }
    launch_row_tv_part<CPT, RB, EARLY, NT>(L, it + off, n - off, L.lds_rtv_c[c], par, flags);
}
}  // namespace

hipError_t launch_row_tv(const LaunchCtx& L, int par, int flags) {
    for (int c = 0; c < 3; ++c) {   // rows longer than 2048 take the three-pass schedule (no fused class)
        if (!L.rtv_cnt[c]) continue;
        if (c == 0)
            launch_row_tv_class<1, 8, RTV_EARLY[0], RTV_SUB_NT[0][0], RTV_SUB_NT[0][1]>(L, c, par, flags);
        else if (c == 1)
            launch_row_tv_class<2, 6, RTV_EARLY[1], RTV_SUB_NT[1][0], RTV_SUB_NT[1][1]>(L, c, par, flags);
        else
            launch_row_tv_class<4, 2, RTV_EARLY[2], RTV_SUB_NT[2][0], RTV_SUB_NT[2][1]>(L, c, par, flags);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int row_tv_max_rows(int w) { return w <= NT ? 8 : (w <= 2 * NT ? 6 : 2); }
int row_tv_sub_threads(int c, int t) { return c >= 0 && c < 3 && t >= 0 && t < ADMM_RTV_SUBS ? RTV_SUB_NT[c][t] : 0; }
int row_sub_threads() { return RROW_SUB_NT; }

// The plain row passes (FA rows, blur, state import) per size class of the row
// length: CPT columns per thread, at most ROW_RB[c] rows per block; NT threads
// per block, NTL for rows of 2049..8192, RROW_SUB_NT for the first rrow_sub0
// items of class 0.
hipError_t launch_row_fwd(const LaunchCtx& L, int par, int src, bool gated) {
    const InfoDev* info = gated ? L.info : nullptr;
    for (int c = 0; c < ADMM_ROW_CLASSES; ++c) {
        int n = L.rrow_cnt[c];
        if (!n) continue;
        const WorkItem* it = L.row_items + L.rrow_beg[c];
        if (c == 0 && L.rrow_sub0 > 0) {
            const int m = std::min(L.rrow_sub0, n);
            hipLaunchKernelGGL((k_row_fwd<1, ROW_RB[0], RROW_SUB_NT>), dim3(m), dim3(RROW_SUB_NT), L.lds_rrow_sub0,
                               L.stream, L.desc, it, m, par, src, info, L.tw);
            it += m;
            n -= m;
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            if (!n) continue;
        }
        if (c == 0)
            hipLaunchKernelGGL((k_row_fwd<1, ROW_RB[0]>), dim3(n), dim3(NT), L.lds_rrow_c[0], L.stream, L.desc, it, n,
                               par, src, info, L.tw);
        else if (c == 1)
            hipLaunchKernelGGL((k_row_fwd<2, ROW_RB[1]>), dim3(n), dim3(NT), L.lds_rrow_c[1], L.stream, L.desc, it, n,
                               par, src, info, L.tw);
        else if (c == 2)
            hipLaunchKernelGGL((k_row_fwd<4, ROW_RB[2]>), dim3(n), dim3(NT), L.lds_rrow_c[2], L.stream, L.desc, it, n,
                               par, src, info, L.tw);
        else if (c == 3)
            hipLaunchKernelGGL((k_row_fwd<4, ROW_RB[3], NTL>), dim3(n), dim3(NTL), L.lds_rrow_c[3], L.stream, L.desc, it,
                               n, par, src, info, L.tw);
        else if (c == 4)
            hipLaunchKernelGGL((k_row_fwd<8, ROW_RB[4], NTL>), dim3(n), dim3(NTL), L.lds_rrow_c[4], L.stream, L.desc, it,
                               n, par, src, info, L.tw);
        else
            hipLaunchKernelGGL((k_row_fwd<32, ROW_RB[5]>), dim3(n), dim3(NT), L.lds_rrow_c[5], L.stream, L.desc, it, n,
                               par, src, info, L.tw);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_row_inv(const LaunchCtx& L, int par, int mode, int flags, bool gated) {
    const InfoDev* info = gated ? L.info : nullptr;
    double* const part = mode >= 2 ? L.cgpart : L.partials;   // modes 2, 3: the CG sums
    for (int c = 0; c < ADMM_ROW_CLASSES; ++c) {
        int n = L.rrow_cnt[c];
        if (!n) continue;
        const WorkItem* it = L.row_items + L.rrow_beg[c];
        if (c == 0 && L.rrow_sub0 > 0) {
            const int m = std::min(L.rrow_sub0, n);
            hipLaunchKernelGGL((k_row_inv<1, ROW_RB[0], RROW_SUB_NT>), dim3(m), dim3(RROW_SUB_NT), L.lds_rrow_sub0,
                               L.stream, L.desc, it, m, par, mode, flags, info, L.tw, part);
            it += m;
            n -= m;
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            if (!n) continue;
        }
        if (c == 0)
            hipLaunchKernelGGL((k_row_inv<1, ROW_RB[0]>), dim3(n), dim3(NT), L.lds_rrow_c[0], L.stream, L.desc, it, n,
                               par, mode, flags, info, L.tw, part);
        else if (c == 1)
            hipLaunchKernelGGL((k_row_inv<2, ROW_RB[1]>), dim3(n), dim3(NT), L.lds_rrow_c[1], L.stream, L.desc, it, n,
                               par, mode, flags, info, L.tw, part);
        else if (c == 2)
            hipLaunchKernelGGL((k_row_inv<4, ROW_RB[2]>), dim3(n), dim3(NT), L.lds_rrow_c[2], L.stream, L.desc, it, n,
                               par, mode, flags, info, L.tw, part);
        else if (c == 3)
            hipLaunchKernelGGL((k_row_inv<4, ROW_RB[3], NTL>), dim3(n), dim3(NTL), L.lds_rrow_c[3], L.stream, L.desc, it,
                               n, par, mode, flags, info, L.tw, part);
        else if (c == 4)
            hipLaunchKernelGGL((k_row_inv<8, ROW_RB[4], NTL>), dim3(n), dim3(NTL), L.lds_rrow_c[4], L.stream, L.desc, it,
                               n, par, mode, flags, info, L.tw, part);
        else
            hipLaunchKernelGGL((k_row_inv<32, ROW_RB[5]>), dim3(n), dim3(NT), L.lds_rrow_c[5], L.stream, L.desc, it, n,
                               par, mode, flags, info, L.tw, part);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int row_max_rows(int w) { return ROW_RB[size_class(w)]; }

hipError_t launch_reduce(const LaunchCtx& L, int count, double tol, double obj_tol, int iter, int final_iter,
                         const int* iter_dev, int* host_active) {
    hipLaunchKernelGGL(k_reduce, dim3(count), dim3(NT), 0, L.stream, L.desc, L.partials, L.info, tol, obj_tol, iter,
                       final_iter, iter_dev, host_active);
    return hipGetLastError();
}

hipError_t launch_tick(const LaunchCtx& L, int* counter, int c, bool set) {
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, L.stream, counter, c, set ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_zero(hipStream_t stream, float* p, size_t n) {
    if (!n) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_scale(hipStream_t stream, const float* d, float* p, size_t n, float s) {
    if (!n) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_scale2, dim3((unsigned)blocks), dim3(256), 0, stream, d, p, n, s);
    return hipGetLastError();
}

hipError_t launch_import_tv(const LaunchCtx& L, int prob, size_t n) {
    hipLaunchKernelGGL(k_import_tv, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L.stream, L.desc, prob);
    return hipGetLastError();
}

hipError_t launch_lambda(const LaunchCtx& L, int prob, size_t HP, const float2* T, int ks) {
    hipLaunchKernelGGL(k_lambda, dim3((unsigned)((HP + 255) / 256)), dim3(256), 0, L.stream, L.desc, prob, T, ks,
                       L.tw);
    return hipGetLastError();
}

hipError_t launch_warmstart(const LaunchCtx& L, int prob, size_t n, const float* x0, const float* p0,
                            const float* y, float* u1, float* d1, float* ureg, float* dreg) {
    hipLaunchKernelGGL(k_warmstart, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L.stream, L.desc, prob, x0, p0,
                       y, u1, d1, ureg, dreg);
    return hipGetLastError();
}

// Allow dynamic LDS beyond the 64 KiB default on every pass kernel (gfx950 has
// 160 KiB per compute unit). Returns the first error, if any.
hipError_t allow_dynamic_lds(int bytes) {
    const void* fns[] = {
        reinterpret_cast<const void*>(&k_col<8, false>),  reinterpret_cast<const void*>(&k_col<8, true>),
        reinterpret_cast<const void*>(&k_col<16, false>), reinterpret_cast<const void*>(&k_col<16, true>),
        reinterpret_cast<const void*>(&k_col<32, false>), reinterpret_cast<const void*>(&k_col<32, true>),
        reinterpret_cast<const void*>(&k_row_tv<MAXE_ROW, 1, 8, RTV_EARLY[0], false>),
        reinterpret_cast<const void*>(&k_row_tv<MAXE_ROW, 2, 6, RTV_EARLY[1], false>),
        reinterpret_cast<const void*>(&k_row_tv<MAXE_ROW, 4, 2, RTV_EARLY[2], false>),
        reinterpret_cast<const void*>(&k_row_tv<MAXE_ROW, 1, 8, RTV_EARLY[0], true>),
        reinterpret_cast<const void*>(&k_row_tv<MAXE_ROW, 2, 6, RTV_EARLY[1], true>),
        reinterpret_cast<const void*>(&k_row_tv<MAXE_ROW, 4, 2, RTV_EARLY[2], true>),
        reinterpret_cast<const void*>(&k_row_tv<MAXE_ROW, 1, 8, RTV_EARLY[0], false, RTV_SUB_NT[0][0]>),
        reinterpret_cast<const void*>(&k_row_tv<MAXE_ROW, 1, 8, RTV_EARLY[0], true, RTV_SUB_NT[0][0]>),
        reinterpret_cast<const void*>(&k_row_tv<MAXE_ROW, 1, 8, RTV_EARLY[0], false, RTV_SUB_NT[0][1]>),
        reinterpret_cast<const void*>(&k_row_tv<MAXE_ROW, 1, 8, RTV_EARLY[0], true, RTV_SUB_NT[0][1]>),
        reinterpret_cast<const void*>(&k_row_tv<MAXE_ROW, 2, 6, RTV_EARLY[1], false, RTV_SUB_NT[1][0]>),
        reinterpret_cast<const void*>(&k_row_tv<MAXE_ROW, 2, 6, RTV_EARLY[1], true, RTV_SUB_NT[1][0]>),
        reinterpret_cast<const void*>(&k_row_fwd<1, ROW_RB[0]>),
        reinterpret_cast<const void*>(&k_row_fwd<1, ROW_RB[0], RROW_SUB_NT>),
        reinterpret_cast<const void*>(&k_row_inv<1, ROW_RB[0], RROW_SUB_NT>),
        reinterpret_cast<const void*>(&k_row_fwd<2, ROW_RB[1]>),
        reinterpret_cast<const void*>(&k_row_fwd<4, ROW_RB[2]>),
        reinterpret_cast<const void*>(&k_row_fwd<4, ROW_RB[3], NTL>),
        reinterpret_cast<const void*>(&k_row_inv<4, ROW_RB[3], NTL>),
        reinterpret_cast<const void*>(&k_row_fwd<8, ROW_RB[4], NTL>),
        reinterpret_cast<const void*>(&k_row_inv<8, ROW_RB[4], NTL>),
        reinterpret_cast<const void*>(&k_row_fwd<32, ROW_RB[5]>),
        reinterpret_cast<const void*>(&k_row_inv<32, ROW_RB[5]>),
        reinterpret_cast<const void*>(&k_col_big<512>),
        reinterpret_cast<const void*>(&k_col_big<1024>),
        reinterpret_cast<const void*>(&k_row_inv<1, ROW_RB[0]>),
        reinterpret_cast<const void*>(&k_row_inv<2, ROW_RB[1]>),
        reinterpret_cast<const void*>(&k_row_inv<4, ROW_RB[2]>)};
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t lds_col_bytes(int H, int TC) { return col_lds(H, TC); }
size_t lds_rowtv_bytes(int W, int B) { return rowtv_lds(W, B); }
size_t lds_row_bytes(int W, int B) { return row_lds(W, B); }
int col_max_tiles() { return NTC / 64; }
int row_maxe(int w) { return w > 8192 ? row_maxe_c<32>() : (w > 2048 ? row_maxe_c<4, NTL>() : MAXE_ROW); }
int row_threads(int w) { return w > 2048 && w <= 8192 ? NTL : NT; }
int block_threads() { return NT; }

}  // namespace admm
