// admm_frame.hip — frame step of FA-MD and FS-MD (Sec. IV-C) on gfx950.
//
// For each FT x FT tile of the image this kernel computes, from z (written by
// the row pass) and the frame duals d2:
//   P z                       undecimated Haar analysis, J levels, 3J+1 bands
//                             (Parseval: P^T P = I, as eq. (25) requires);
//   u2 = soft(P z - d2, lambda / mu2)                          (eqs. (8), (16));
//   d2' = d2 - (P z - u2);                                     (Alg. 2)
//   q  = mu2 P^T (u2 + d2')   the frame part of the next right-hand side
//                             (eq. (24) with zeta2 = u2 + d2').
// Level j uses dilation s = 2^(j-1) and the periodic filters
// (x[i] + x[i+s]) / 2 and (x[i] - x[i+s]) / 2; the adjoint looks backward by s.
// The analysis at a pixel reads z up to h = 2^J - 1 pixels ahead and the
// synthesis reads coefficients up to h pixels behind, so a tile works on a
// (FT + 2h)^2 window of z and an (FT + h)^2 window of coefficients, all in LDS:
//   a_0 = z, a_j = low-low band of level j     (window shrinks by s at the far side)
//   omega bands of level j on [-(2^j - 1), FT)^2, synthesised level by level
//   from j = J down to 1 into a'_{j-1} on [-(2^(j-1) - 1), FT)^2; q = mu2 a'_0.
// The duals are ping-pong buffers: halo reads see only the previous iteration.
//
// FS-MD (template FS): the unknowns are the coefficients z of x = W z, W = P^T.
// With W W^T = I the z-step of eq. (17) (its matrix inverted by eq. (18))
// has the closed form
//   x = W z = (mu1 A^T A + mu2 I)^{-1} (mu1 A^T zeta1 + mu2 W zeta2),
//   z = zeta2 + P (x - W zeta2),
// (substitute z = zeta2 + W^T q into eq. (17): q = x - W zeta2 solves it, and
// the solution is unique), so the spectral pass solves for x as FA-MD does,
// with s = mu2 W zeta2, and the row pass hands this kernel e = x - s / mu2.
// With zeta2 = u2 + d2 the thresholded argument is v = z - d2 = u2 + P e, and
//   u2' = soft(v, lambda / mu2),  d2' = u2' - v,  zeta2' = u2' + d2',
//   s'  = mu2 P^T zeta2'.
// The working state is u2 (ping-pong); z = v + d2 is needed only for the
// residual sums, so d2 is kept (in the u_prev planes) on the iteration before
// a check, while the dual residual reads u2 of the previous iteration from the
// state itself.
#include "admm_internal.h"
#include "admm_launch.h"
#include "fft_lds.h"

namespace admm {

constexpr int NTF = 512;

__device__ __forceinline__ int wrapm(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}
// i in [-n, 2n): one conditional add or subtract
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ double fwave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

__device__ __forceinline__ float softf(float v, float t) {
    const float a = fabsf(v) - t;
    return a > 0.0f ? copysignf(a, v) : 0.0f;
}

// Window edge of a_j (j = 0 .. J) and the LDS offset of a_j, in floats.
__host__ __device__ constexpr int fr_la(int J, int j) { return frame_tile(J) + 2 * ((1 << J) - 1) - ((1 << j) - 1); }
__host__ __device__ constexpr int fr_aoff(int J, int j) {
    int o = 0;
    for (int l = 0; l < j; ++l) o += fr_la(J, l) * fr_la(J, l);
    return o;
}
__host__ __device__ constexpr int fr_cdiv(int a, int b) { return (a + b - 1) / b; }

// J levels and the tile size are compile-time, so every window size, LDS offset
// and loop trip count is a constant. SMALL: the image is smaller than a window
// and indices wrap by a full modulo. MODE: FR_PLAIN iteration, FR_CHECK
// iteration that also accumulates the residual sums, or FR_IMPORT: omega =
// u2 + d2 from the caller's state (no analysis) and the working duals are
// initialised from it; used to start or resume a solve.
enum { FR_PLAIN = 0, FR_CHECK = 1, FR_IMPORT = 2 };

template <int J, bool SMALL, int MODE, bool FS>
__global__ __launch_bounds__(NTF) void k_frame(const ProbDesc* __restrict__ pd, const WorkItem* __restrict__ items,
                                               int nitems, int par, int flags, const InfoDev* __restrict__ info,
                                               double* __restrict__ partials) {
    constexpr bool IMPORT = MODE == FR_IMPORT, chk = MODE == FR_CHECK;
    constexpr int FT = frame_tile(J);
    constexpr int h = (1 << J) - 1;
    constexpr int L0 = FT + 2 * h, LE = FT + h;
    constexpr int NZ = fr_cdiv(L0 * L0, NTF);       // z window values per thread
    constexpr int NC = fr_cdiv(LE * LE, NTF);       // coefficients per thread and band (largest window)
    // the z window is stored to LDS unconditionally (positions past it are
    // overwritten by the analysis after the next barrier)
    static_assert(fr_aoff(J, J + 1) + 5 * LE * LE >= NZ * NTF, "LDS smaller than the z prefetch");
    extern __shared__ float sm[];
    const int wi = xcd_remap(blockIdx.x, gridDim.x);
    const WorkItem it = items[wi];
    if (info && !info[it.prob].active) return;
    const ProbDesc& p = pd[it.prob];
    const int H = p.H, W = p.W;
    const int ntx = (W + FT - 1) / FT;
    const int ty = it.start / ntx, tx = it.start - ty * ntx;
    const int r0 = ty * FT, c0 = tx * FT;
    const unsigned hlim = (unsigned)min(FT, H - r0), wlim = (unsigned)min(FT, W - c0);   // owned part of the tile
    const unsigned n = (unsigned)(H * W);   // 32-bit offsets: the plan keeps the 3J+1 bands within 4 GiB
    const int tid = threadIdx.x;
    auto wrap = [&](int i, int m) { return SMALL ? wrapm(i, m) : wrap1(i, m); };
    const float tau = p.tau, mu2 = p.mu2;

    // LDS: a_0 .. a_J, three omega planes and two a' planes of LE^2
    ADMM_LDS float* const smem = (ADMM_LDS float*)sm;
    constexpr int WB0 = fr_aoff(J, J + 1);
    ADMM_LDS float* const wb0 = smem + WB0;
    ADMM_LDS float* const wb1 = wb0 + LE * LE;
    ADMM_LDS float* const wb2 = wb1 + LE * LE;
    ADMM_LDS float* const ap[2] = {wb2 + LE * LE, wb2 + 2 * LE * LE};

    const float* din = par ? p.dreg1 : p.dreg0;
    float* dout = par ? p.dreg0 : p.dreg1;
    // descriptor fields read once (the coefficient stores would make the
    // compiler reload each of them, and wait for it, after every store)
    float* const UREGP = p.uregp;
    float* const SUREG = p.st_ureg;
    float* const SDREG = p.st_dreg;
    float* const TB = p.tmpB;

    double acc[ADMM_NSUM];
#pragma unroll
    for (int i = 0; i < ADMM_NSUM; ++i) acc[i] = 0.0;

    auto cidx = [&](int band, int i, int k) -> unsigned {
        return (unsigned)band * n + (unsigned)(wrap(r0 + i, H) * W + wrap(c0 + k, W));
    };

    // Every global input of the tile is requested before any of it is used: the
    // z window, then the duals of the coarsest band and of levels J .. 1 over
    // their coefficient windows, in the order they are consumed. The loads are
    // unconditional (indices past a window are clamped to its last element), so
    // each use waits only for the loads issued before it. A check iteration also
    // fetches u2 of the previous iteration for the dual residual.
    float zr[NZ], dcv[NC], dlv[J][3][NC], ucv[NC], ulv[J][3][NC];
    // plane offsets of the coefficients this thread loads, kept for their stores
    // in plain iterations (the check instantiation recomputes them: it holds
    // the previous u2 as well, and the offsets would cost it occupancy)
    constexpr bool KEEP = MODE == FR_PLAIN;
    unsigned gcs[NC], gls[J][NC];
    if (!IMPORT) {
#pragma unroll
        for (int u = 0; u < NZ; ++u) {
            const int idx = min(tid + u * NTF, L0 * L0 - 1);
            const int i = idx / L0, k = idx - i * L0;
            zr[u] = gld(p.zpl, (unsigned)(wrap(r0 - h + i, H) * W + wrap(c0 - h + k, W)));
        }
#pragma unroll
        for (int u = 0; u < NC; ++u) {
            const int idx = min(tid + u * NTF, LE * LE - 1);
            const int ie = idx / LE;
            const unsigned g = cidx(3 * J, ie - h, idx - ie * LE - h);
            if (KEEP) gcs[u] = g;
            dcv[u] = gld(din, g);
            if (chk) ucv[u] = gld(UREGP, g);
        }
#pragma unroll
        for (int jj = J - 1; jj >= 0; --jj) {
            const int e = (2 << jj) - 1, Lb = FT + e;     // level jj + 1
#pragma unroll
            for (int u = 0; u < NC; ++u) {
                if (u * NTF < Lb * Lb) {
                    const int idx = min(tid + u * NTF, Lb * Lb - 1);
                    const int ii = idx / Lb;
                    const unsigned g = cidx(3 * jj, ii - e, idx - ii * Lb - e);
                    if (KEEP) gls[jj][u] = g;
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        dlv[jj][b][u] = gld(din, g + (unsigned)b * n);
                        if (chk) ulv[jj][b][u] = gld(UREGP, g + (unsigned)b * n);
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < NZ; ++u) smem[tid + u * NTF] = zr[u];
        __syncthreads();
#pragma unroll
        for (int j = 1; j <= J; ++j) {
            const int s = 1 << (j - 1), Lp = fr_la(J, j - 1), Lc = fr_la(J, j);
            const ADMM_LDS float* A = smem + fr_aoff(J, j - 1);
            ADMM_LDS float* An = smem + fr_aoff(J, j);
#pragma unroll
            for (int u = 0; u < fr_cdiv(Lc * Lc, NTF); ++u) {
                const int idx = tid + u * NTF;
                if (idx < Lc * Lc) {
                    const int i = idx / Lc, k = idx - i * Lc;
                    const float x00 = A[i * Lp + k], x10 = A[(i + s) * Lp + k];
                    const float x01 = A[i * Lp + k + s], x11 = A[(i + s) * Lp + k + s];
                    // the two filter halvings as one quarter (exact: powers of two)
                    An[idx] = 0.25f * ((x00 + x10) + (x01 + x11));
                }
            }
            __syncthreads();
        }
    }

    // One coefficient at tile-relative (i, k), plane offset g, with its dual:
    // prox, dual update and omega = u2 + d2'. Only the owner of a coefficient
    // (its tile) writes it back and counts it in the residual sums.
    auto coef = [&](float Pz, float dl, float uprev, unsigned g, bool own) -> float {
        if (FS) {
            // Pz = P e, dl = u2 of the previous iteration, uprev = d2_{k-1} (check iterations)
            const float v = dl + Pz;
            const float u = softf(v, tau);
            const float dn = u - v;              // d2' = d2 - (z - u2')
            if (own) {
                gst(dout, g, u);
                if (chk) {
                    const float z = v + uprev, e = z - u, f = u - dl;
                    acc[1] += (double)(e * e);
                    acc[3] += (double)(z * z);
                    acc[5] += (double)(u * u);
                    acc[7] += (double)(f * f);
                    acc[9] += (double)(dn * dn);
                    acc[11] += (double)fabsf(z);
                }
                if (flags & F_WRITE_UPREV) gst(UREGP, g, dn);
                if (flags & F_EXPORT) {
                    gst(SUREG, g, u);
                    gst(SDREG, g, dn);
                }
            }
            return u + dn;
        }
        const float v = Pz - dl;
        const float u = softf(v, tau);
        const float dn = u - v;                  // d2 - (P z - u2)
        if (own) {
            gst(dout, g, dn);
            if (chk) {
                const float e = Pz - u, f = u - uprev;
                acc[1] += (double)(e * e);
                acc[3] += (double)(Pz * Pz);
                acc[5] += (double)(u * u);
                acc[7] += (double)(f * f);
                acc[9] += (double)(dn * dn);
                acc[11] += (double)fabsf(Pz);
            }
            if (flags & F_WRITE_UPREV) gst(UREGP, g, u);
            if (flags & F_EXPORT) {
                gst(SUREG, g, u);
                gst(SDREG, g, dn);
            }
        }
        return u + dn;
    };
    auto coef_import = [&](unsigned g, bool own) -> float {
        const float d = gld(SDREG, g), u = gld(SUREG, g);
        if (own) gst(dout, g, FS ? u : d);   // the working state: d2 (analysis) or u2 (synthesis)
        return u + d;
    };
    auto owns = [&](int i, int k) { return (unsigned)i < hlim && (unsigned)k < wlim; };

    // coarsest low-low band on [-h, FT)^2 -> a'_J
#pragma unroll
    for (int u = 0; u < NC; ++u) {
        const int idx = tid + u * NTF;
        if (idx < LE * LE) {
            const int ie = idx / LE;
            const int i = ie - h, k = idx - ie * LE - h;
            const unsigned g = KEEP ? gcs[u] : cidx(3 * J, i, k);   // the loaded offset (same element)
            ap[0][idx] = IMPORT ? coef_import(g, owns(i, k)) : coef(smem[fr_aoff(J, J) + idx], dcv[u], chk ? ucv[u] : 0.0f, g, owns(i, k));
        }
    }
    __syncthreads();
#pragma unroll
    for (int jj = J - 1; jj >= 0; --jj) {
        const int s = 1 << jj, e = (2 << jj) - 1, Lb = FT + e;   // level j = jj + 1
        const ADMM_LDS float* A = smem + fr_aoff(J, jj);
        const int Lp = fr_la(J, jj);
        const ADMM_LDS float* Ap = ap[(J - 1 - jj) & 1];
        ADMM_LDS float* An = ap[(J - jj) & 1];
#pragma unroll
        for (int u = 0; u < NC; ++u) {
            const int idx = tid + u * NTF;
            if (idx < Lb * Lb) {
                const int ii = idx / Lb;
                const int i = ii - e, k = idx - ii * Lb - e;
                const unsigned g0 = KEEP ? gls[jj][u] : cidx(3 * jj, i, k), g1 = g0 + n, g2 = g1 + n;
                const bool own = owns(i, k);
                if (IMPORT) {
                    wb0[idx] = coef_import(g0, own);
                    wb1[idx] = coef_import(g1, own);
                    wb2[idx] = coef_import(g2, own);
                } else {
                    const int pi = i + h, pk = k + h;     // position in the a_{j-1} window
                    const float x00 = A[pi * Lp + pk], x10 = A[(pi + s) * Lp + pk];
                    const float x01 = A[pi * Lp + pk + s], x11 = A[(pi + s) * Lp + pk + s];
                    const float lv0 = x00 + x10, lv1 = x01 + x11;   // vertical filters, halvings deferred
                    const float hv0 = x00 - x10, hv1 = x01 - x11;
                    wb0[idx] = coef(0.25f * (lv0 - lv1), dlv[jj][0][u], chk ? ulv[jj][0][u] : 0.0f, g0, own);
                    wb1[idx] = coef(0.25f * (hv0 + hv1), dlv[jj][1][u], chk ? ulv[jj][1][u] : 0.0f, g1, own);
                    wb2[idx] = coef(0.25f * (hv0 - hv1), dlv[jj][2][u], chk ? ulv[jj][2][u] : 0.0f, g2, own);
                }
            }
        }
        __syncthreads();
        // synthesis a'_{j-1} on [-(s-1), FT)^2 from level-j planes on [-e, FT)^2 (stride Lb)
        const int Lc = FT + s - 1;
#pragma unroll
        for (int u = 0; u < fr_cdiv(Lc * Lc, NTF); ++u) {
            const int idx = tid + u * NTF;
            if (idx < Lc * Lc) {
                const int ci = idx / Lc, ck = idx - ci * Lc;
                const int ii = ci - (s - 1) + e, kk = ck - (s - 1) + e;     // >= s by construction
                const int q0 = ii * Lb + kk, q1 = ii * Lb + kk - s, q2 = (ii - s) * Lb + kk, q3 = (ii - s) * Lb + kk - s;
                // horizontal adjoints of the rows ii and ii - s
                const float lvA = (Ap[q0] + Ap[q1]) + (wb0[q0] - wb0[q1]);   // halvings deferred
                const float hvA = (wb1[q0] + wb1[q1]) + (wb2[q0] - wb2[q1]);
                const float lvB = (Ap[q2] + Ap[q3]) + (wb0[q2] - wb0[q3]);
                const float hvB = (wb1[q2] + wb1[q3]) + (wb2[q2] - wb2[q3]);
                An[idx] = 0.25f * ((lvA + lvB) + (hvA - hvB));
            }
        }
        __syncthreads();
    }
    // q = mu2 P^T omega on the tile (a'_0 is ap[J & 1])
    const ADMM_LDS float* Af = ap[J & 1];
#pragma unroll
    for (int u = 0; u < fr_cdiv(FT * FT, NTF); ++u) {
        const int idx = tid + u * NTF;
        const int i = idx / FT, k = idx - i * FT;
        if ((unsigned)i < hlim && (unsigned)k < wlim) gst(TB, (unsigned)((r0 + i) * W + c0 + k), mu2 * Af[idx]);
    }
    if (chk) {
        const int lane = tid & 63, wave = tid >> 6;
        __syncthreads();
        double* scratch = reinterpret_cast<double*>(sm);
#pragma unroll
        for (int i = 0; i < ADMM_NSUM; ++i) {
            double v = fwave_sum(acc[i]);
            if (lane == 0) scratch[wave * ADMM_NSUM + i] = v;
        }
        __syncthreads();
        if (tid < ADMM_NSUM) {
            double v = 0.0;
            for (int w = 0; w < NTF / 64; ++w) v += scratch[w * ADMM_NSUM + tid];
            partials[(size_t)(p.part_base + p.nrowblk + it.blk) * ADMM_NSUM + tid] = v;
        }
    }
}

// zeta1 = u1 + d1 and the working data dual, from a caller state (FA import).
__global__ void k_import_fa(const ProbDesc* __restrict__ pd, int prob) {
    const ProbDesc& p = pd[prob];
    const unsigned n = (unsigned)(p.H * p.W);
    const unsigned g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    gst(p.tmpA, g, gld(p.st_u1, g) + gld(p.st_d1, g));
    gst(p.d1, g, gld(p.st_d1, g));
}

int frame_class(int H, int W, int J, bool fs) {
    const int w = frame_tile(J) + 2 * ((1 << J) - 1);
    return (fs ? 8 : 0) + 2 * (J - 1) + ((H < w || W < w) ? 1 : 0);
}

size_t lds_frame_bytes(int J) {
    const int LE = frame_tile(J) + (1 << J) - 1;
    const size_t b = (size_t)(fr_aoff(J, J + 1) + 5 * LE * LE) * sizeof(float);
    const size_t need = NTF / 64 * ADMM_NSUM * sizeof(double);
    return b > need ? b : need;
}

namespace {
template <int J, bool SMALL, bool FS>
void launch_frame_class(const LaunchCtx& L, int c, int par, int flags, int import_mode, bool gated) {
    const WorkItem* it = L.frm_items + L.frm_beg[c];
    const int n = L.frm_cnt[c];
    const InfoDev* info = gated ? L.info : nullptr;
    if (import_mode)
        hipLaunchKernelGGL((k_frame<J, SMALL, FR_IMPORT, FS>), dim3(n), dim3(NTF), L.lds_frm_c[c], L.stream, L.desc,
                           it, n, par, flags, info, L.partials);
    else if (flags & F_CHECK)
        hipLaunchKernelGGL((k_frame<J, SMALL, FR_CHECK, FS>), dim3(n), dim3(NTF), L.lds_frm_c[c], L.stream, L.desc,
                           it, n, par, flags, info, L.partials);
    else
        hipLaunchKernelGGL((k_frame<J, SMALL, FR_PLAIN, FS>), dim3(n), dim3(NTF), L.lds_frm_c[c], L.stream, L.desc,
                           it, n, par, flags, info, L.partials);
}

template <bool FS>
void launch_frame_kind(const LaunchCtx& L, int c, int par, int flags, int import_mode, bool gated) {
    switch (c & 7) {
        case 0: launch_frame_class<1, false, FS>(L, c, par, flags, import_mode, gated); break;
        case 1: launch_frame_class<1, true, FS>(L, c, par, flags, import_mode, gated); break;
        case 2: launch_frame_class<2, false, FS>(L, c, par, flags, import_mode, gated); break;
        case 3: launch_frame_class<2, true, FS>(L, c, par, flags, import_mode, gated); break;
        case 4: launch_frame_class<3, false, FS>(L, c, par, flags, import_mode, gated); break;
        case 5: launch_frame_class<3, true, FS>(L, c, par, flags, import_mode, gated); break;
        case 6: launch_frame_class<4, false, FS>(L, c, par, flags, import_mode, gated); break;
        default: launch_frame_class<4, true, FS>(L, c, par, flags, import_mode, gated); break;
    }
}
}  // namespace

// One launch per frame class (levels, small image) that has items.
hipError_t launch_frame(const LaunchCtx& L, int par, int flags, int import_mode, bool gated) {
    for (int c = 0; c < ADMM_FRAME_CLASSES; ++c) {
        if (!L.frm_items || L.frm_cnt[c] == 0) continue;
        if (c < 8)
            launch_frame_kind<false>(L, c, par, flags, import_mode, gated);
        else
            launch_frame_kind<true>(L, c, par, flags, import_mode, gated);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_import_fa(const LaunchCtx& L, int prob, size_t n) {
    hipLaunchKernelGGL(k_import_fa, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L.stream, L.desc, prob);
    return hipGetLastError();
}

}  // namespace admm
