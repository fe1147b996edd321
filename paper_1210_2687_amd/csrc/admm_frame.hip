// admm_frame.hip — frame-analysis step of FA-MD (Sec. IV-C) on gfx950.
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

// import_mode: omega = u2 + d2 from the caller's state (no analysis), the
// working duals are initialised from it; used to start or resume a solve.
__global__ __launch_bounds__(NTF) void k_frame(const ProbDesc* __restrict__ pd, const WorkItem* __restrict__ items,
                                               int nitems, int par, int flags, int import_mode,
                                               const InfoDev* __restrict__ info, double* __restrict__ partials) {
    extern __shared__ float sm[];
    const int wi = xcd_remap(blockIdx.x, gridDim.x);
    const WorkItem it = items[wi];
    if (info && !info[it.prob].active) return;
    const ProbDesc& p = pd[it.prob];
    const int H = p.H, W = p.W, J = p.J, FT = p.frm_tile;
    const int h = (1 << J) - 1;
    const int ntx = (W + FT - 1) / FT;
    const int ty = it.start / ntx, tx = it.start - ty * ntx;
    const int r0 = ty * FT, c0 = tx * FT;
    const unsigned n = (unsigned)(H * W);   // planes hold at most 2048^2 values: 32-bit offsets
    const int tid = threadIdx.x;
    // windows reach h pixels beyond the tile; a single wrap suffices unless the
    // image is smaller than a window
    const bool small = H < FT + 2 * h || W < FT + 2 * h;
    auto wrap = [&](int i, int m) { return small ? wrapm(i, m) : wrap1(i, m); };
    const float tau = p.tau, mu2 = p.mu2;
    const bool chk = (flags & F_CHECK) && !import_mode;

    // LDS carve-up: a_0..a_J, three omega planes, two a' planes
    // (explicit LDS pointers: indexed arrays of generic pointers would become flat accesses)
    const int L0 = FT + 2 * h, LE = FT + h;
    ADMM_LDS float* const smem = (ADMM_LDS float*)sm;
    ADMM_LDS float* a[5];
    int La[5];
    int off = 0;
    for (int j = 0; j <= J; ++j) {
        La[j] = L0 - ((1 << j) - 1);
        a[j] = smem + off;
        off += La[j] * La[j];
    }
    ADMM_LDS float* wb[3];
    for (int b = 0; b < 3; ++b) {
        wb[b] = smem + off;
        off += LE * LE;
    }
    ADMM_LDS float* ap[2] = {smem + off, smem + off + LE * LE};

    const float* din = par ? p.dreg1 : p.dreg0;
    float* dout = par ? p.dreg0 : p.dreg1;

    double acc[ADMM_NSUM];
#pragma unroll
    for (int i = 0; i < ADMM_NSUM; ++i) acc[i] = 0.0;

    if (!import_mode) {
        const unsigned m0 = div_magic((unsigned)L0);
        for (int idx = tid; idx < L0 * L0; idx += NTF) {
            const int i = (int)udiv16((unsigned)idx, (unsigned)L0, m0), k = idx - i * L0;
            a[0][idx] = gld(p.zpl, (unsigned)(wrap(r0 - h + i, H) * W + wrap(c0 - h + k, W)));
        }
        __syncthreads();
        for (int j = 1; j <= J; ++j) {
            const int s = 1 << (j - 1), Lp = La[j - 1], Lc = La[j];
            const ADMM_LDS float* A = a[j - 1];
            const unsigned mc = div_magic((unsigned)Lc);
            for (int idx = tid; idx < Lc * Lc; idx += NTF) {
                const int i = (int)udiv16((unsigned)idx, (unsigned)Lc, mc), k = idx - i * Lc;
                const float x00 = A[i * Lp + k], x10 = A[(i + s) * Lp + k];
                const float x01 = A[i * Lp + k + s], x11 = A[(i + s) * Lp + k + s];
                const float lv0 = 0.5f * (x00 + x10), lv1 = 0.5f * (x01 + x11);
                a[j][idx] = 0.5f * (lv0 + lv1);
            }
            __syncthreads();
        }
    }

    // One coefficient of band `band` at tile-relative (i, k): its plane offset,
    // its dual (the loads of up to CH coefficients per thread are issued
    // together), then prox, dual update and omega = u2 + d2'.
    auto cidx = [&](int band, int i, int k) -> unsigned {
        return (unsigned)band * n + (unsigned)(wrap(r0 + i, H) * W + wrap(c0 + k, W));
    };
    auto cload = [&](unsigned g) -> float2 {
        return import_mode ? make_float2(gld(p.st_dreg, g), gld(p.st_ureg, g)) : make_float2(gld(din, g), 0.0f);
    };
    auto coef = [&](float Pz, float2 dl, unsigned g, int i, int k) -> float {
        const bool own = i >= 0 && k >= 0 && i < FT && k < FT && r0 + i < H && c0 + k < W;
        if (import_mode) {
            if (own) gst(dout, g, dl.x);
            return dl.y + dl.x;
        }
        const float v = Pz - dl.x;
        const float u = softf(v, tau);
        const float dn = u - v;                  // d2 - (P z - u2)
        if (own) {
            gst(dout, g, dn);
            if (chk) {
                const float e = Pz - u, f = u - gld(p.uregp, g);
                acc[1] += (double)(e * e);
                acc[3] += (double)(Pz * Pz);
                acc[5] += (double)(u * u);
                acc[7] += (double)(f * f);
                acc[9] += (double)(dn * dn);
                acc[11] += (double)fabsf(Pz);
            }
            if (flags & F_WRITE_UPREV) gst(p.uregp, g, u);
            if (flags & F_EXPORT) {
                gst(p.st_ureg, g, u);
                gst(p.st_dreg, g, dn);
            }
        }
        return u + dn;
    };
    constexpr int CH = 4;

    // coarsest low-low band on [-h, FT)^2 -> a'_J
    const unsigned mE = div_magic((unsigned)LE);
    for (int base = tid; base < LE * LE; base += CH * NTF) {
        unsigned g[CH];
        float2 dl[CH];
        int iv[CH], kv[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int idx = min(base + u * NTF, LE * LE - 1);
            const int ie = (int)udiv16((unsigned)idx, (unsigned)LE, mE);
            iv[u] = ie - h;
            kv[u] = idx - ie * LE - h;
            g[u] = cidx(3 * J, iv[u], kv[u]);
            if (base + u * NTF < LE * LE) dl[u] = cload(g[u]);
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int idx = base + u * NTF;
            if (idx < LE * LE) ap[0][idx] = coef(import_mode ? 0.0f : a[J][idx], dl[u], g[u], iv[u], kv[u]);
        }
    }
    __syncthreads();
    int cur = 0;
    for (int j = J; j >= 1; --j) {
        const int s = 1 << (j - 1), e = (1 << j) - 1, Lb = FT + e;
        const ADMM_LDS float* A = a[j - 1];
        const int Lp = La[j - 1];
        const unsigned mb = div_magic((unsigned)Lb);
        const int b0 = 3 * (j - 1);
        for (int base = tid; base < Lb * Lb; base += CH * NTF) {
            unsigned g[CH][3];
            float2 dl[CH][3];
            int iv[CH], kv[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int idx = min(base + u * NTF, Lb * Lb - 1);
                const int ii = (int)udiv16((unsigned)idx, (unsigned)Lb, mb), kk = idx - ii * Lb;
                iv[u] = ii - e;
                kv[u] = kk - e;
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    g[u][b] = cidx(b0 + b, iv[u], kv[u]);
                    if (base + u * NTF < Lb * Lb) dl[u][b] = cload(g[u][b]);
                }
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int idx = base + u * NTF;
                if (idx >= Lb * Lb) break;
                const int i = iv[u], k = kv[u];
                float lh = 0.f, hl = 0.f, hh = 0.f;
                if (!import_mode) {
                    const int pi = i + h, pk = k + h;     // position in the a_{j-1} window
                    const float x00 = A[pi * Lp + pk], x10 = A[(pi + s) * Lp + pk];
                    const float x01 = A[pi * Lp + pk + s], x11 = A[(pi + s) * Lp + pk + s];
                    const float lv0 = 0.5f * (x00 + x10), lv1 = 0.5f * (x01 + x11);
                    const float hv0 = 0.5f * (x00 - x10), hv1 = 0.5f * (x01 - x11);
                    lh = 0.5f * (lv0 - lv1);
                    hl = 0.5f * (hv0 + hv1);
                    hh = 0.5f * (hv0 - hv1);
                }
                wb[0][idx] = coef(lh, dl[u][0], g[u][0], i, k);
                wb[1][idx] = coef(hl, dl[u][1], g[u][1], i, k);
                wb[2][idx] = coef(hh, dl[u][2], g[u][2], i, k);
            }
        }
        __syncthreads();
        // synthesis a'_{j-1} on [-(s-1), FT)^2 from level-j planes on [-e, FT)^2 (stride Lb)
        const int Lc = FT + s - 1;
        const ADMM_LDS float* Ap = ap[cur];
        ADMM_LDS float* An = ap[cur ^ 1];
        const unsigned mc = div_magic((unsigned)Lc);
        for (int idx = tid; idx < Lc * Lc; idx += NTF) {
            const int ci = (int)udiv16((unsigned)idx, (unsigned)Lc, mc), ck = idx - ci * Lc;
            const int ii = ci - (s - 1) + e, kk = ck - (s - 1) + e;     // >= s by construction
            const int q0 = ii * Lb + kk, q1 = ii * Lb + kk - s, q2 = (ii - s) * Lb + kk, q3 = (ii - s) * Lb + kk - s;
            // horizontal adjoints of the rows ii and ii - s
            const float lvA = 0.5f * ((Ap[q0] + Ap[q1]) + (wb[0][q0] - wb[0][q1]));
            const float hvA = 0.5f * ((wb[1][q0] + wb[1][q1]) + (wb[2][q0] - wb[2][q1]));
            const float lvB = 0.5f * ((Ap[q2] + Ap[q3]) + (wb[0][q2] - wb[0][q3]));
            const float hvB = 0.5f * ((wb[1][q2] + wb[1][q3]) + (wb[2][q2] - wb[2][q3]));
            An[idx] = 0.5f * ((lvA + lvB) + (hvA - hvB));
        }
        __syncthreads();
        cur ^= 1;
    }
    // q = mu2 P^T omega on the tile
    const ADMM_LDS float* Af = ap[cur];
    const unsigned mf = div_magic((unsigned)FT);
    for (int idx = tid; idx < FT * FT; idx += NTF) {
        const int i = (int)udiv16((unsigned)idx, (unsigned)FT, mf), k = idx - i * FT;
        const int gr = r0 + i, gc = c0 + k;
        if (gr < H && gc < W) gst(p.tmpB, (unsigned)(gr * W + gc), mu2 * Af[idx]);
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

size_t lds_frame_bytes(int FT, int J) {
    const int h = (1 << J) - 1, L0 = FT + 2 * h, LE = FT + h;
    size_t f = 0;
    for (int j = 0; j <= J; ++j) {
        const size_t L = L0 - ((1 << j) - 1);
        f += L * L;
    }
    f += 5 * (size_t)LE * LE;
    size_t b = f * sizeof(float);
    const size_t need = NTF / 64 * ADMM_NSUM * sizeof(double);
    return b > need ? b : need;
}

hipError_t launch_frame(const LaunchCtx& L, int par, int flags, int import_mode, bool gated) {
    hipLaunchKernelGGL(k_frame, dim3(L.nfrm), dim3(NTF), L.lds_frm, L.stream, L.desc, L.frm_items, L.nfrm, par,
                       flags, import_mode, gated ? L.info : nullptr, L.partials);
    return hipGetLastError();
}

hipError_t launch_import_fa(const LaunchCtx& L, int prob, size_t n) {
    hipLaunchKernelGGL(k_import_fa, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L.stream, L.desc, prob);
    return hipGetLastError();
}

}  // namespace admm
