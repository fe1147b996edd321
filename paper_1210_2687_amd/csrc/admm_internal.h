// admm_internal.h — descriptors shared by the host library and the gfx950 kernels.
//
// Data layout in HBM, per problem (H x W unknown domain, P = W/2 + 1):
//   planes      row-major H x W float32 (pitch W): duals d1, d^h, d^v (TV) or
//               d1 and 3J+1 frame bands (FA), the observation y and mask m;
//   spectra     two ping-pong buffers of P x H float4, stored TRANSPOSED
//               ([k2][k1], k1 fastest) so the column pass reads contiguous
//               columns; each float4 holds two complex values: after the row
//               pass the row-DFT half spectra of (zeta1, s); after the column
//               pass the row-DFT half spectra of (z, A z);
//   lamhat      P x H float2 ([k2][k1]): the kernel spectrum Lambda of eq. (19).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define ADMM_MAX_STAGES 12
#define ADMM_NSUM 12
#define ADMM_MAX_SIDE 16384
#define ADMM_MAX_BANDS 16

namespace admm {

enum { REG_TV = 0, REG_FRAME = 1 };

// Row-kernel flags (per launch).
enum {
    F_WRITE_X = 1,      // write z into the output image
    F_WRITE_UPREV = 2,  // keep u_k for the next iteration's dual residual
    F_CHECK = 4,        // accumulate the residual / objective sums
    F_EXPORT = 8,       // write (u, d) to the caller's state buffers
    F_FORWARD = 16,     // finish with the next iteration's forward row DFT
};

// Column-kernel modes.
enum { COL_SOLVE = 0, COL_BLUR = 1 };

// Radix schedule of a 7-smooth length n >= 2, written to out[0..nst) (returns
// nst, or -1 if n is not 7-smooth or needs more than cap stages). Radix 8 as
// far as the power of two allows (a leftover 2^4 as 4 x 4 rather than 8 x 2),
// then 7, 5, 3. With at least two factors of 8 the schedule starts and ends
// with radix 8 and the other radices go in between: the column pass then keeps
// the last forward and the first inverse stage in registers. The host plans
// and the compile-time transforms of the kernels share this one definition.
__host__ __device__ constexpr int fft_schedule(int n, int* out, int cap) {
    if (n < 2) return -1;
    int a = 0;
    while (n % 2 == 0) {
        n /= 2;
        ++a;
    }
    int r[40] = {};
    int m = 0;
    const bool ends = a >= 6;
    if (ends) a -= 6;
    int n8 = a / 3;
    const int rem = a % 3;
    const bool split = rem == 1 && n8 > 0;
    if (split) --n8;
    for (int i = 0; i < n8; ++i) r[m++] = 8;
    if (split) {
        r[m++] = 4;
        r[m++] = 4;
    } else if (rem == 1) {
        r[m++] = 2;
    } else if (rem == 2) {
        r[m++] = 4;
    }
    for (int p = 7; p >= 3; p -= 2)
        while (n % p == 0) {
            n /= p;
            r[m++] = p;
        }
    if (n != 1) return -1;
    const int nst = m + (ends ? 2 : 0);
    if (nst > cap) return -1;
    int o = 0;
    if (ends) out[o++] = 8;
    for (int i = 0; i < m; ++i) out[o++] = r[i];
    if (ends) out[o++] = 8;
    return nst;
}

// Alternative radix schedules (the autotuner's radix dimension). Variant 0 is
// fft_schedule; the others reorder or regroup the same factorisation:
//   1  powers of two as radix 4 (one radix 2 for an odd exponent), then 7, 5, 3;
//   2  the odd radices first, then radix 8 with a 4 or 2 tail;
//   3  powers of two as radix 16 with one 8, 4 or 2 for the rest, then 7, 5, 3
//      (block-level row transforms only: a wave-level column stage does not
//      hold 16 operands per butterfly).
// Returns the number of stages written to out, or -1 (not 7-smooth, too many
// stages, unknown variant).
constexpr int FFT_VARIANTS = 4;
__host__ __device__ constexpr int fft_schedule_variant(int n, int variant, int* out, int cap) {
    if (variant == 0) return fft_schedule(n, out, cap);
    if (n < 2 || variant < 0 || variant >= FFT_VARIANTS) return -1;
    int a = 0;
    while (n % 2 == 0) {
        n /= 2;
        ++a;
    }
    int odd[40] = {};
    int no = 0;
    for (int p = 7; p >= 3; p -= 2)
        while (n % p == 0) {
            n /= p;
            odd[no++] = p;
        }
    if (n != 1) return -1;
    int r[40] = {};
    int m = 0;
    if (variant == 1) {
        for (int i = 0; i < a / 2; ++i) r[m++] = 4;
        if (a % 2) r[m++] = 2;
        for (int i = 0; i < no; ++i) r[m++] = odd[i];
    } else if (variant == 2) {
        for (int i = 0; i < no; ++i) r[m++] = odd[i];
        for (int i = 0; i < a / 3; ++i) r[m++] = 8;
        if (a % 3 == 1) r[m++] = 2;
        else if (a % 3 == 2) r[m++] = 4;
    } else {
        for (int i = 0; i < a / 4; ++i) r[m++] = 16;
        if (a % 4 == 1) r[m++] = 2;
        else if (a % 4 == 2) r[m++] = 4;
        else if (a % 4 == 3) r[m++] = 8;
        for (int i = 0; i < no; ++i) r[m++] = odd[i];
    }
    if (m < 1 || m > cap) return -1;
    for (int i = 0; i < m; ++i) out[i] = r[i];
    return m;
}

// Per-stage constants of one transform length: for stage s of radix R after
// Ns = product of the earlier radices, nbf = N / R butterflies, the exact
// reciprocal multipliers of nbf and Ns (x / d == umulhi(x, ceil(2^32 / d)) for x, d <
// 2^16; d == 1 is handled apart) and tso, the offset of the stage's twiddles
// in the length's stage table. The stage table holds, for each stage, entries
// [k][r - 1] = exp(-2 pi i k r / (Ns R)) for k < Ns, 1 <= r < R (N - 1
// entries over all stages), so that a butterfly's R - 1 twiddles are adjacent.
struct FftPlanDev {
    int N;
    int nst;
    int ends8;                  // first and last stage are radix 8 (register-fused column pass)
    int variant;                // schedule variant (0: fft_schedule, which the compile-time paths follow)
    int tw_off;                 // offset of this length's tables in the shared table arrays
    int rad[ADMM_MAX_STAGES];
    int ns[ADMM_MAX_STAGES];
    int nbf[ADMM_MAX_STAGES];
    int tso[ADMM_MAX_STAGES];
    unsigned mnbf[ADMM_MAX_STAGES];
    unsigned mns[ADMM_MAX_STAGES];
};

// Frame tiles: 32 x 32 up to three levels, 16 x 16 at four (the windows reach
// 2^J - 1 pixels beyond the tile on each side).
__host__ __device__ constexpr int frame_tile(int J) { return J >= 4 ? 16 : 32; }

// exact division for operands below 2^16 by a divisor with multiplier m = ceil(2^32 / d)
__host__ __device__ inline unsigned div_magic(unsigned d) { return d <= 1 ? 0u : (unsigned)((0x100000000ull + d - 1) / d); }
__device__ __forceinline__ unsigned udiv16(unsigned x, unsigned d, unsigned m) { return d == 1 ? x : __umulhi(x, m); }

// Residual sums (index into the per-block partial vector):
//  0 |A z - u1|^2   1 |G_reg z - u_reg|^2   2 |A z|^2   3 |G_reg z|^2
//  4 |u1|^2         5 |u_reg|^2             6 |u1 - u1_prev|^2
//  7 |u_reg - u_reg_prev|^2   8 |d1|^2      9 |d_reg|^2
// 10 sum m (y - A z)^2       11 regulariser value (TV sum of |D_i z|, or |P z|_1)
struct ProbDesc {
    int H, W, P, reg, J, nb;
    int B, TC;                  // rows per row block, columns per column tile
    int nrowblk, ncolblk, nfrmblk, frm_tile;
    int part_base;              // first partial-vector slot of this problem
    float mu1, mu2, tau, lam, inv_hw, inv1pmu1;
    FftPlanDev fr, fc;          // row (length W) and column (length H) transforms
    // columns longer than 8192: the column transform splits into csp
    // sub-transforms of length H / csp (plan fc2) around a radix-csp pass
    // through HBM (csp = 1: no split)
    int csp;
    FftPlanDev fc2;
    float4* spec0;
    float4* spec1;
    float2* lamhat;
    float* d1;
    float* dreg0;               // regulariser duals, ping: TV [d^h, d^v]; FA 3J+1 bands
    float* dreg1;               // pong (neighbouring blocks read halos of the old values)
    float* u1p;                 // u1 of the previous iteration (dual residual)
    float* uregp;               // u_reg of the previous iteration (2 or nb planes)
    float* tmpA;                // zeta1 plane (FA per iteration; TV at initialisation)
    float* tmpB;                // s / q plane
    float* zpl;                 // z plane (FA)
    const float* y;             // caller's observation (read where mask == 1)
    const uint8_t* mask;
    float* x;                   // caller's output
    float* st_u1;               // caller's state buffers (export / import), may be null
    float* st_d1;
    float* st_ureg;
    float* st_dreg;
    // Reeves-Sorel variants (method CG): the boundary-system estimate v, the
    // images C B^T v and A C B^T v, the outputs (z part, A z part) of the two
    // circulant solves of an iteration, and mu_t (mu1 for TV, where the solve
    // returns t / mu1; 1 for the frame)
    int method;
    int fs;                     // frame synthesis (FS-MD): the frame pass works on coefficients
    float mut;
    float* cgv;
    float* cge;
    float* cgae;
    float* cgo1;
    float* cgao1;
    float* cgo2;
    float* cgao2;
};

enum { METHOD_MD = 0, METHOD_CG = 1 };

struct WorkItem {
    int prob;
    int start;                  // first row (row pass), first column (column pass) or tile index
    int blk;                    // block index within the problem (partial-sum slot)
    int sub;                    // split column transforms: the sub-transform (0 otherwise)
};

struct InfoDev {
    int iters, converged, diverged, active;
    double r_pri, r_dual, objective;
};

// Map a linear block id so that consecutive work items land on the same XCD
// (workgroups are dispatched round-robin over the 8 XCDs of an MI355X, each
// with its own L2; neighbouring items share halo rows and cache lines).
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
    const int xcd = bid & 7, slot = bid >> 3;
    const int per = nblk >> 3, rem = nblk & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + slot;
}

}  // namespace admm
