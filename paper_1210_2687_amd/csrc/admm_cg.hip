// admm_cg.hip — gfx950 kernels of the Reeves-Sorel variants TV-CG and FA-CG
// (Sec. IV-B..IV-D): H1 = M A, the z-step by the Sherman-Morrison-Woodbury
// split z = (C r + C B^T v) / mu_t, C the circulant inverse, B the rows of A at
// the unobserved pixels, v from one conjugate-gradient iteration on the
// boundary system (I - B C B^T) v = B C r started at the previous v.
//
// One iteration, with the circulant solves done by the FFT passes (row DFT,
// column DFT + solve + inverse, inverse row DFT into a pair of planes):
//   solve 1   (M (u1 + d1), s)   -> O1 = C r / mu_t, AO1 = A O1; the inverse
//             row pass also forms p = res = B (C r + C B^T v) - v on the
//             unobserved pixels (C B^T v and A C B^T v held as the images e,
//             Ae), the row block's sum p^T p and the forward row DFT of
//             (mu1 p, 0), which starts the second solve
//   solve 2   (p, 0)             -> O2 = C B^T p, AO2 = A O2, and the row
//             block's p^T (I - B C B^T) p = p^T (p - (1 - m) AO2)
//   k_cg_update  a = sum p^T p / sum p^T S p over the problem's row blocks (0
//             unless both are positive), v += a p, e += a O2, Ae += a AO2
//             (linearity of C B^T and A), z = O1 + e / mu_t,
//             A z = AO1 + Ae / mu_t, data step on the observed pixels
//             u1 = (y + mu1 (A z - d1)) / (1 + mu1), d1 <- d1 - (A z - u1),
//             next M (u1 + d1)
//   k_tv_step (TV) vector soft threshold, TV duals, next s = mu2 D^T (u + d);
//             the frame variant runs the FA frame step on z instead.
// k_tv_step is also the TV step of TV-MD for rows longer than 2048, which run
// the three-pass schedule (inverse rows with the data step into z, this step,
// forward rows) instead of the fused TV row pass.
// Every kernel takes the rows of one row item of a problem (the work items of
// the row passes) and skips finished problems.
#include "admm_internal.h"
#include "admm_launch.h"
#include "fft_lds.h"

namespace admm {

constexpr int NTG = 512;
constexpr int TVS_BAND_MAX_W = 2048;   // longer rows take the row-walking TV step

namespace {

__device__ __forceinline__ double cg_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sum K per-thread values over the block into out[0..K) (thread 0 writes).
template <int K>
__device__ __forceinline__ void cg_block_sums(const double* v, double* out) {
    __shared__ double sm[NTG / 64][K];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const double s = cg_wave_sum(v[i]);
        if (lane == 0) sm[wave][i] = s;
    }
    __syncthreads();
    if (tid < K) {
        double s = 0.0;
        for (int w = 0; w < NTG / 64; ++w) s += sm[w][tid];
        out[tid] = s;
    }
}

// The block's residual sums into its slot: every entry (odd == false; the data
// step, whose regulariser entries are zero) or the odd entries only (the TV
// step, which runs after the data step on the same row block).
__device__ __forceinline__ void cg_write_sums(const double* acc, double* slot, bool odd) {
    __shared__ double out[ADMM_NSUM];
    cg_block_sums<ADMM_NSUM>(acc, out);
    __syncthreads();
    const int t = threadIdx.x;
    if (t < ADMM_NSUM && (!odd || (t & 1))) slot[t] = out[t];
}

}  // namespace

// CG update, z, A z and the data step (observed pixels), the data block's
// residual sums on check iterations (the regulariser entries written as zero).
template <bool CHK>
__global__ __launch_bounds__(NTG) void k_cg_update(const ProbDesc* __restrict__ pd, const WorkItem* __restrict__ items,
                                                  const InfoDev* __restrict__ info, int flags,
                                                  const double* __restrict__ cgpart, double* __restrict__ partials) {
    const WorkItem it = items[xcd_remap(blockIdx.x, gridDim.x)];
    if (!info[it.prob].active) return;
    const ProbDesc& p = pd[it.prob];
    const int W = p.W, nr = min(p.B, p.H - it.start);
    const unsigned base = (unsigned)(it.start * W), cnt = (unsigned)(nr * W);
    // the step length from the row blocks' sums; every block of the problem
    // adds them in the same order, so all of them use the same a
    __shared__ float a_sh;
    {
        double two[2] = {0.0, 0.0};
        for (int b = threadIdx.x; b < p.nrowblk; b += NTG) {
            two[0] += cgpart[(size_t)(p.part_base + b) * 2];
            two[1] += cgpart[(size_t)(p.part_base + b) * 2 + 1];
        }
        __shared__ double sums[2];
        cg_block_sums<2>(two, sums);
        __syncthreads();
        if (threadIdx.x == 0) {
            const double q = (sums[0] > 0.0 && sums[1] > 0.0) ? sums[0] / sums[1] : 0.0;
            a_sh = isfinite(q) ? (float)q : 0.0f;
        }
        __syncthreads();
    }
    const float a = a_sh, inv_mut = 1.0f / p.mut, mu1 = p.mu1, c1 = p.inv1pmu1;
    const uint8_t* const MK = p.mask;
    const float* const YV = p.y;
    const float* const TA = p.tmpA;   // p of this iteration
    const float* const O1 = p.cgo1;
    const float* const AO1 = p.cgao1;
    const float* const O2 = p.cgo2;
    const float* const AO2 = p.cgao2;
    float* const V = p.cgv;
    float* const E = p.cge;
    float* const AE = p.cgae;
    float* const D1 = p.d1;
    float* const ZP = p.zpl;
    float* const XO = p.x;
    float* const U1P = p.u1p;
    float* const ZETA = p.tmpA;       // next M (u1 + d1), written after p is read
    double acc[ADMM_NSUM];
#pragma unroll
    for (int i = 0; i < ADMM_NSUM; ++i) acc[i] = 0.0;
    for (unsigned i = threadIdx.x; i < cnt; i += NTG) {
        const unsigned g = base + i;
        const bool obs = gld(MK, g) != 0;
        const float pv = gld(TA, g);
        const float e = fmaf(a, gld(O2, g), gld(E, g));
        const float ae = fmaf(a, gld(AO2, g), gld(AE, g));
        gst(V, g, fmaf(a, pv, gld(V, g)));
        gst(E, g, e);
        gst(AE, g, ae);
        const float z = fmaf(e, inv_mut, gld(O1, g));
        const float Az = fmaf(ae, inv_mut, gld(AO1, g));
        const float MAz = obs ? Az : 0.0f;
        const float d1o = gld(D1, g);
        const float yv = obs ? gld(YV, g) : 0.0f;
        const float v1 = MAz - d1o;
        const float u1 = obs ? fmaf(yv - v1, c1, v1) : 0.0f;   // (y + mu1 v) / (1 + mu1) on the observed pixels
        const float d1n = d1o - (MAz - u1);
        gst(D1, g, d1n);
        gst(ZP, g, z);
        gst(ZETA, g, u1 + d1n);
        if (flags & F_WRITE_X) gst(XO, g, z);
        if (CHK) {
            const float e0 = MAz - u1, f6 = u1 - gld(U1P, g), ry = obs ? yv - Az : 0.0f;
            acc[0] += (double)(e0 * e0);
            acc[2] += (double)(MAz * MAz);
            acc[4] += (double)(u1 * u1);
            acc[6] += (double)(f6 * f6);
            acc[8] += (double)(d1n * d1n);
            acc[10] += (double)(ry * ry);
        }
        if (flags & F_WRITE_UPREV) gst(U1P, g, u1);
    }
    if (CHK) cg_write_sums(acc, partials + (size_t)(p.part_base + it.blk) * ADMM_NSUM, false);
}

// TV step on z (the plane k_cg_update or the inverse row pass wrote): vector
// soft threshold and TV duals for the block's rows and the row above (whose
// u + d enters the adjoint difference), then s = mu2 D^T (u + d) for the
// block's rows; the TV block's residual sums on check iterations (odd
// entries). One element of a row at (r, c):
//   v = D z - d, u = vector soft threshold of v at tau, d' = u - v (= d - (D z - u)),
// with D z the periodic forward differences (z(r, c + 1) - z, z(r + 1, c) - z).
struct TvElem {
    float zh, zv, uh, uv, dhn, dvn;
};
__device__ __forceinline__ TvElem tv_elem(float zc, float zr, float zd, float dh, float dv, float tau) {
    TvElem t;
    t.zh = zr - zc;
    t.zv = zd - zc;
    const float vh = t.zh - dh, vv = t.zv - dv;
    const float rho = __builtin_amdgcn_sqrtf(fmaf(vh, vh, vv * vv));
    const float sc = rho > tau ? (rho - tau) * __builtin_amdgcn_rcpf(rho) : 0.0f;
    t.uh = vh * sc;
    t.uv = vv * sc;
    t.dhn = t.uh - vh;
    t.dvn = t.uv - vv;
    return t;
}

// Outputs of one element of the block's own rows: the new duals, the check
// sums, u of this iteration (for the next check) and the exported state.
template <bool CHK>
__device__ __forceinline__ void tv_elem_out(const TvElem& t, unsigned g, unsigned n, float uph, float upv, int flags,
                                            float* dh_out, float* dv_out, float* UREGP, float* SUREG, float* SDREG,
                                            double* acc) {
    gst(dh_out, g, t.dhn);
    gst(dv_out, g, t.dvn);
    if (CHK) {   // u_{k-1} was read before a check iteration that also keeps u_k (period 1) overwrites it
        const float e1h = t.zh - t.uh, e1v = t.zv - t.uv;
        const float f7h = t.uh - uph, f7v = t.uv - upv;
        acc[1] += (double)fmaf(e1h, e1h, e1v * e1v);
        acc[3] += (double)fmaf(t.zh, t.zh, t.zv * t.zv);
        acc[5] += (double)fmaf(t.uh, t.uh, t.uv * t.uv);
        acc[7] += (double)fmaf(f7h, f7h, f7v * f7v);
        acc[9] += (double)fmaf(t.dhn, t.dhn, t.dvn * t.dvn);
        acc[11] += (double)sqrtf(fmaf(t.zh, t.zh, t.zv * t.zv));
    }
    if (flags & F_WRITE_UPREV) {
        gst(UREGP, g, t.uh);
        gst(UREGP, n + g, t.uv);
    }
    if (flags & F_EXPORT) {
        gst(SUREG, g, t.uh);
        gst(SUREG, n + g, t.uv);
        gst(SDREG, g, t.dhn);
        gst(SDREG, n + g, t.dvn);
    }
}

// Rows of up to 2048: the block's (nr + 1) x W elements are spread over all
// threads; u + d of every row (both components) goes to LDS, then s.
// LDS: (nr + 1) x W of each component of u + d.
template <bool CHK>
__device__ __forceinline__ void tv_step_band(const ProbDesc& p, int r0, int nr, int par, int flags, float* ud,
                                             double* acc) {
    const int H = p.H, W = p.W;
    const unsigned n = (unsigned)(H * W);
    const float tau = p.tau, mu2 = p.mu2;
    const float* const Z = p.zpl;
    const float* const dh_in = par ? p.dreg1 : p.dreg0;
    const float* const dv_in = dh_in + n;
    float* const dh_out = par ? p.dreg0 : p.dreg1;
    float* const dv_out = dh_out + n;
    float* const UREGP = p.uregp;
    float* const SUREG = p.st_ureg;
    float* const SDREG = p.st_dreg;
    float* const TB = p.tmpB;
    float* udh = ud;
    float* udv = ud + (size_t)(nr + 1) * W;
    const int tot = (nr + 1) * W;
    for (int i = threadIdx.x; i < tot; i += NTG) {
        const int rr = i / W, c = i - rr * W;
        const int r = rr == 0 ? (r0 == 0 ? H - 1 : r0 - 1) : r0 + rr - 1;   // row r0 - 1 + rr (wrapped)
        const int rn = r + 1 == H ? 0 : r + 1, cn = c + 1 == W ? 0 : c + 1;
        const unsigned g = (unsigned)(r * W + c);
        const TvElem t = tv_elem(gld(Z, g), gld(Z, (unsigned)(r * W + cn)), gld(Z, (unsigned)(rn * W + c)),
                                 gld(dh_in, g), gld(dv_in, g), tau);
        udh[i] = t.uh + t.dhn;
        udv[i] = t.uv + t.dvn;
        if (rr > 0) {
            const float uph = CHK ? gld(UREGP, g) : 0.0f, upv = CHK ? gld(UREGP, n + g) : 0.0f;
            tv_elem_out<CHK>(t, g, n, uph, upv, flags, dh_out, dv_out, UREGP, SUREG, SDREG, acc);
        }
    }
    __syncthreads();
    const int own = nr * W;
    for (int i = threadIdx.x; i < own; i += NTG) {
        const int rr = i / W + 1, c = i - (rr - 1) * W;
        const int k = rr * W + c, kl = rr * W + (c == 0 ? W - 1 : c - 1), ku = k - W;
        const float s = mu2 * ((udh[kl] - udh[k]) + (udv[ku] - udv[k]));
        gst(TB, (unsigned)((r0 + rr - 1) * W + c), s);
    }
}

// Rows of 2049..16384: thread t owns columns t, t + NTG, ... (CPT of them,
// clamped to the row; 8 up to 4096, 16 up to 8192, 32 above) and walks the
// rows from the one above the block's first row down. A row's inputs are fetched in bursts of
// unconditional loads of TVW_BURST columns each; the vertical component of
// u + d of the row above stays in registers, the horizontal one of the current
// row goes through LDS (two row buffers, so one barrier per row).
// LDS: 2 x W floats.
constexpr int TVW_BURST = 8;
template <bool CHK, int CPT>
__device__ __forceinline__ void tv_step_walk(const ProbDesc& p, int r0, int nr, int par, int flags, float* ud,
                                             double* acc) {
    const int H = p.H, W = p.W, tid = threadIdx.x;
    const unsigned n = (unsigned)(H * W);
    const float tau = p.tau, mu2 = p.mu2;
    const float* const Z = p.zpl;
    const float* const dh_in = par ? p.dreg1 : p.dreg0;
    const float* const dv_in = dh_in + n;
    float* const dh_out = par ? p.dreg0 : p.dreg1;
    float* const dv_out = dh_out + n;
    float* const UREGP = p.uregp;
    float* const SUREG = p.st_ureg;
    float* const SDREG = p.st_dreg;
    float* const TB = p.tmpB;
    float udv_up[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) udv_up[j] = 0.0f;
    for (int rr = 0; rr <= nr; ++rr) {
        const int r = rr == 0 ? (r0 == 0 ? H - 1 : r0 - 1) : r0 + rr - 1;   // row r0 - 1 + rr (wrapped)
        const int rn = r + 1 == H ? 0 : r + 1;
        const bool own = rr > 0;
        float* const ub = ud + (rr & 1) * W;
        float udv[CPT];
#pragma unroll
        for (int j0 = 0; j0 < CPT; j0 += TVW_BURST) {
            float zc[TVW_BURST], zr[TVW_BURST], zd[TVW_BURST], dh[TVW_BURST], dv[TVW_BURST], uph[TVW_BURST],
                upv[TVW_BURST];
#pragma unroll
            for (int j = 0; j < TVW_BURST; ++j) {
                const int c = min(tid + (j0 + j) * NTG, W - 1), cn = c + 1 == W ? 0 : c + 1;
                const unsigned g = (unsigned)(r * W + c);
                zc[j] = gld(Z, g);
                zr[j] = gld(Z, (unsigned)(r * W + cn));
                zd[j] = gld(Z, (unsigned)(rn * W + c));
                dh[j] = gld(dh_in, g);
                dv[j] = gld(dv_in, g);
                uph[j] = CHK ? gld(UREGP, g) : 0.0f;
                upv[j] = CHK ? gld(UREGP, n + g) : 0.0f;
            }
#pragma unroll
            for (int j = 0; j < TVW_BURST; ++j) {
                const int c = tid + (j0 + j) * NTG;
                const TvElem t = tv_elem(zc[j], zr[j], zd[j], dh[j], dv[j], tau);
                udv[j0 + j] = t.uv + t.dvn;
                if (c < W) {
                    ub[c] = t.uh + t.dhn;
                    if (own)
                        tv_elem_out<CHK>(t, (unsigned)(r * W + c), n, uph[j], upv[j], flags, dh_out, dv_out, UREGP,
                                         SUREG, SDREG, acc);
                }
            }
        }
        __syncthreads();
        if (own) {
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int c = tid + j * NTG;
                if (c < W) {
                    const float s = mu2 * ((ub[c == 0 ? W - 1 : c - 1] - ub[c]) + (udv_up[j] - udv[j]));
                    gst(TB, (unsigned)(r * W + c), s);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < CPT; ++j) udv_up[j] = udv[j];
    }
}

// MCPT: the widest walk the instantiation takes (8, 16 or 32 columns per
// thread: rows of up to 4096, 8192, 16384); a wider walk holds more registers,
// which would cost the narrower rows occupancy, so a launch takes the
// narrowest instantiation its batch allows.
template <bool CHK, int MCPT>
__global__ __launch_bounds__(NTG) void k_tv_step(const ProbDesc* __restrict__ pd, const WorkItem* __restrict__ items,
                                              const InfoDev* __restrict__ info, int par, int flags,
                                              double* __restrict__ partials) {
    extern __shared__ float ud[];
    const WorkItem it = items[xcd_remap(blockIdx.x, gridDim.x)];
    if (!info[it.prob].active) return;
    const ProbDesc& p = pd[it.prob];
    const int r0 = it.start, nr = min(p.B, p.H - r0);
    double acc[ADMM_NSUM];
#pragma unroll
    for (int i = 0; i < ADMM_NSUM; ++i) acc[i] = 0.0;
    if (MCPT >= 32 && p.W > 8192)
        tv_step_walk<CHK, 32>(p, r0, nr, par, flags, ud, acc);
    else if (MCPT >= 16 && p.W > 4096)
        tv_step_walk<CHK, 16>(p, r0, nr, par, flags, ud, acc);
    else if (p.W > TVS_BAND_MAX_W)
        tv_step_walk<CHK, 8>(p, r0, nr, par, flags, ud, acc);
    else
        tv_step_band<CHK>(p, r0, nr, par, flags, ud, acc);
    if (CHK) cg_write_sums(acc, partials + (size_t)(p.part_base + it.blk) * ADMM_NSUM, true);
}

// ------------------------------------------------------------ launchers
hipError_t launch_cg_update(const LaunchCtx& L, int flags) {
    if (!L.nrow) return hipSuccess;
    if (flags & F_CHECK)
        hipLaunchKernelGGL(k_cg_update<true>, dim3(L.nrow), dim3(NTG), 0, L.stream, L.desc, L.row_items, L.info, flags,
                           L.cgpart, L.partials);
    else
        hipLaunchKernelGGL(k_cg_update<false>, dim3(L.nrow), dim3(NTG), 0, L.stream, L.desc, L.row_items, L.info,
                           flags, L.cgpart, L.partials);
    return hipGetLastError();
}

namespace {
template <int MCPT>
void launch_tv_step_w(const LaunchCtx& L, int par, int flags) {
    if (flags & F_CHECK)
        hipLaunchKernelGGL((k_tv_step<true, MCPT>), dim3(L.nrow), dim3(NTG), L.lds_tvstep, L.stream, L.desc,
                           L.row_items, L.info, par, flags, L.partials);
    else
        hipLaunchKernelGGL((k_tv_step<false, MCPT>), dim3(L.nrow), dim3(NTG), L.lds_tvstep, L.stream, L.desc,
                           L.row_items, L.info, par, flags, L.partials);
}
}  // namespace

hipError_t launch_tv_step(const LaunchCtx& L, int par, int flags) {
    if (!L.nrow) return hipSuccess;
    if (L.tv_cpt > 16)
        launch_tv_step_w<32>(L, par, flags);
    else if (L.tv_cpt > 8)
        launch_tv_step_w<16>(L, par, flags);
    else
        launch_tv_step_w<8>(L, par, flags);
    return hipGetLastError();
}

size_t lds_tvstep_bytes(int W, int B) {
    return W > TVS_BAND_MAX_W ? (size_t)2 * W * sizeof(float) : (size_t)2 * (B + 1) * W * sizeof(float);
}

hipError_t allow_dynamic_lds_cg(int bytes) {
    const void* fns[] = {reinterpret_cast<const void*>(&k_tv_step<false, 8>),
                         reinterpret_cast<const void*>(&k_tv_step<true, 8>),
                         reinterpret_cast<const void*>(&k_tv_step<false, 16>),
                         reinterpret_cast<const void*>(&k_tv_step<true, 16>),
                         reinterpret_cast<const void*>(&k_tv_step<false, 32>),
                         reinterpret_cast<const void*>(&k_tv_step<true, 32>)};
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace admm
