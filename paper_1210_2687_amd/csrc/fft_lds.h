// fft_lds.h — radix-staged in-LDS FFT for gfx950 (device code only).
//
// The z-step of the splitting is a circulant solve diagonalised by the 2-D DFT
// (eqs. (19), (25), (33)); this header provides the 1-D transforms from which
// the row and column passes are built.
//
// Algorithm: Stockham auto-sort, mixed radix {2,3,4,5,7,8,16} (16 in the
// block-level transforms only). At a stage of
// radix R with Ns = product of the radices already applied, butterfly j of a
// length-N transform reads x[j + r N/R] (r < R), multiplies input r by the
// twiddle w_N^{r (j mod Ns) N/(Ns R)}, takes an R-point DFT and writes output r
// to position (j / Ns) Ns R + (j mod Ns) + r Ns. After the last stage the data
// is in natural order. Each lane holds its butterflies' operands in registers
// between the loads and the stores of a stage, so the transform is in place.
//
// Twiddles come from a per-length table tw[k] = exp(-2 pi i k / N) computed in
// double precision on the host and rounded once, copied to LDS by each block;
// the inverse uses conj(tw).
// Arithmetic uses explicit fmaf where a fused multiply-add is wanted and the
// library is compiled with -ffp-contract=off, so every instantiation rounds
// identically (a requirement for bit-exact checkpoint/resume).
#pragma once
#include <hip/hip_runtime.h>
#include "admm_internal.h"

namespace admm {

// Pointers into LDS (address space 3) and global memory (address space 1). The
// radix stages are separate functions (keeping the register allocation of each
// radix independent), so the LDS address space is spelled out to keep ds_*
// instructions instead of flat ones.
#define ADMM_LDS __attribute__((address_space(3)))
#define ADMM_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ ADMM_GLOBAL T* gptr(T* p) { return (ADMM_GLOBAL T*)p; }
template <typename T> __device__ __forceinline__ const ADMM_GLOBAL T* gptr(const T* p) { return (const ADMM_GLOBAL T*)p; }

typedef float vf2 __attribute__((ext_vector_type(2)));
typedef float vf4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float2 lds_ld(const ADMM_LDS float2* p) {
    const vf2 v = *(const ADMM_LDS vf2*)p;
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ float4 lds_ld(const ADMM_LDS float4* p) {
    const vf4 v = *(const ADMM_LDS vf4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void lds_st(ADMM_LDS float2* p, float2 a) { *(ADMM_LDS vf2*)p = vf2{a.x, a.y}; }

// Global-memory accesses through pointers held in the problem descriptors: the
// compiler cannot tell where a pointer loaded from memory points, so without
// the address space it emits flat instructions, which also count against the
// LDS wait counter and so stall the LDS traffic of the same wave.
__device__ __forceinline__ float4 gld(const float4* p) {
    const vf4 v = *(const ADMM_GLOBAL vf4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 gld(const float2* p) {
    const vf2 v = *(const ADMM_GLOBAL vf2*)p;
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ float gld(const float* p) { return *(const ADMM_GLOBAL float*)p; }
__device__ __forceinline__ uint8_t gld(const uint8_t* p) { return *(const ADMM_GLOBAL uint8_t*)p; }
__device__ __forceinline__ void gst(float4* p, float4 a) { *(ADMM_GLOBAL vf4*)p = vf4{a.x, a.y, a.z, a.w}; }
__device__ __forceinline__ void gst(float2* p, float2 a) { *(ADMM_GLOBAL vf2*)p = vf2{a.x, a.y}; }
__device__ __forceinline__ void gst(float* p, float a) { *(ADMM_GLOBAL float*)p = a; }
// A twiddle of a stage table that sits in LDS, or in global memory (read
// through the caches) when a block's data leaves no room for it.
__device__ __forceinline__ float2 tw_ld(const ADMM_LDS float2* p) { return lds_ld(p); }
__device__ __forceinline__ float2 tw_ld(const float2* p) { return gld(p); }
// base[i] with a 32-bit byte offset (every plane and spectrum is far below
// 4 GiB), so the access takes a scalar base plus one 32-bit vector offset
// instead of a 64-bit vector address per element
template <typename T> __device__ __forceinline__ ADMM_GLOBAL T* gat(T* base, unsigned i) {
    return (ADMM_GLOBAL T*)((ADMM_GLOBAL char*)base + i * (unsigned)sizeof(T));
}
template <typename T> __device__ __forceinline__ const ADMM_GLOBAL T* gat(const T* base, unsigned i) {
    return (const ADMM_GLOBAL T*)((const ADMM_GLOBAL char*)base + i * (unsigned)sizeof(T));
}
__device__ __forceinline__ float4 gld(const float4* base, unsigned i) {
    const vf4 v = *(const ADMM_GLOBAL vf4*)gat(base, i);
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 gld(const float2* base, unsigned i) {
    const vf2 v = *(const ADMM_GLOBAL vf2*)gat(base, i);
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ float gld(const float* base, unsigned i) { return *gat(base, i); }
__device__ __forceinline__ uint8_t gld(const uint8_t* base, unsigned i) { return *gat(base, i); }
__device__ __forceinline__ void gst(float4* base, unsigned i, float4 a) {
    *(ADMM_GLOBAL vf4*)gat(base, i) = vf4{a.x, a.y, a.z, a.w};
}
__device__ __forceinline__ void gst(float2* base, unsigned i, float2 a) { *(ADMM_GLOBAL vf2*)gat(base, i) = vf2{a.x, a.y}; }
__device__ __forceinline__ void gst(float* base, unsigned i, float a) { *gat(base, i) = a; }
__device__ __forceinline__ void lds_st(ADMM_LDS float4* p, float4 a) { *(ADMM_LDS vf4*)p = vf4{a.x, a.y, a.z, a.w}; }

// ----------------------------------------------------------- complex helpers
// float2 = one complex value; float4 = a pair of complex values (x,y) and (z,w)
// that are transformed together with the same twiddles.

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float4 cadd(float4 a, float4 b) { return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }
__device__ __forceinline__ float4 csub(float4 a, float4 b) { return make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w); }

__device__ __forceinline__ float2 cmul(float2 a, float2 w) {
    return make_float2(fmaf(a.x, w.x, -(a.y * w.y)), fmaf(a.x, w.y, a.y * w.x));
}
__device__ __forceinline__ float4 cmul(float4 a, float2 w) {
    return make_float4(fmaf(a.x, w.x, -(a.y * w.y)), fmaf(a.x, w.y, a.y * w.x),
                       fmaf(a.z, w.x, -(a.w * w.y)), fmaf(a.z, w.y, a.w * w.x));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float4 cscale(float4 a, float s) { return make_float4(a.x * s, a.y * s, a.z * s, a.w * s); }

// multiply by -i (forward direction) or +i (inverse direction)
template <bool INV> __device__ __forceinline__ float2 cmuli(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
template <bool INV> __device__ __forceinline__ float4 cmuli(float4 a) {
    return INV ? make_float4(-a.y, a.x, -a.w, a.z) : make_float4(a.y, -a.x, a.w, -a.z);
}

// a + s * b for a real scalar s (fused)
__device__ __forceinline__ float2 caxpy(float s, float2 b, float2 a) { return make_float2(fmaf(s, b.x, a.x), fmaf(s, b.y, a.y)); }
__device__ __forceinline__ float4 caxpy(float s, float4 b, float4 a) {
    return make_float4(fmaf(s, b.x, a.x), fmaf(s, b.y, a.y), fmaf(s, b.z, a.z), fmaf(s, b.w, a.w));
}

// ----------------------------------------------------------- small DFTs
// X_k = sum_m v_m exp(s 2 pi i k m / R), s = -1 forward, +1 inverse.

template <bool INV, typename E> __device__ __forceinline__ void dft2(E* v) {
    E a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <bool INV, typename E> __device__ __forceinline__ void dft4(E* v) {
    E t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    E t2 = cadd(v[1], v[3]), t3 = cmuli<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}

template <bool INV, typename E> __device__ __forceinline__ void dft8(E* v) {
    constexpr float H = 0.70710678118654752f;   // sqrt(1/2)
    E e[4] = {v[0], v[2], v[4], v[6]};
    E o[4] = {v[1], v[3], v[5], v[7]};
    dft4<INV>(e);
    dft4<INV>(o);
    // o_k *= w8^k, w8 = exp(s 2 pi i / 8)
    o[1] = cmul(o[1], make_float2(H, INV ? H : -H));
    o[2] = cmuli<INV>(o[2]);
    o[3] = cmul(o[3], make_float2(-H, INV ? H : -H));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        E a = e[k], b = o[k];
        v[k] = cadd(a, b);
        v[k + 4] = csub(a, b);
    }
}

// Odd radix R = 2h+1: X_k = v0 + sum_m (v_m + v_{R-m}) cos(2 pi k m / R)
//                         + s i sum_m (v_m - v_{R-m}) sin(2 pi k m / R),
// and X_{R-k} is the same with the sine part negated.
template <int R> struct OddTab;
template <> struct OddTab<3> {
    static __device__ __forceinline__ float c(int j) { return -0.5f; }
    static __device__ __forceinline__ float s(int j) { return 0.86602540378443865f; }
};
template <> struct OddTab<5> {
    static __device__ __forceinline__ float c(int j) { return j == 1 ? 0.30901699437494742f : -0.80901699437494742f; }
    static __device__ __forceinline__ float s(int j) { return j == 1 ? 0.95105651629515357f : 0.58778525229247313f; }
};
template <> struct OddTab<7> {
    static __device__ __forceinline__ float c(int j) {
        return j == 1 ? 0.62348980185873353f : (j == 2 ? -0.22252093395631440f : -0.90096886790241913f);
    }
    static __device__ __forceinline__ float s(int j) {
        return j == 1 ? 0.78183148246802981f : (j == 2 ? 0.97492791218182361f : 0.43388373911755812f);
    }
};

// cos / sin of 2 pi j / R for any integer j (reduced with the symmetries)
template <int R> __device__ __forceinline__ float oddcos(int j) {
    j %= R;
    if (j > R / 2) j = R - j;
    return OddTab<R>::c(j);
}
template <int R> __device__ __forceinline__ float oddsin(int j) {
    j %= R;
    return j > R / 2 ? -OddTab<R>::s(R - j) : OddTab<R>::s(j);
}

template <int R, bool INV, typename E> __device__ __forceinline__ void dft_odd(E* v) {
    constexpr int h = R / 2;
    E A[h], B[h];
#pragma unroll
    for (int m = 1; m <= h; ++m) {
        A[m - 1] = cadd(v[m], v[R - m]);
        B[m - 1] = csub(v[m], v[R - m]);
    }
    E x0 = v[0];
    E sum = v[0];
#pragma unroll
    for (int m = 0; m < h; ++m) sum = cadd(sum, A[m]);
#pragma unroll
    for (int k = 1; k <= h; ++k) {
        E P = x0, Q;
#pragma unroll
        for (int m = 1; m <= h; ++m) P = caxpy(oddcos<R>(k * m), A[m - 1], P);
        Q = cscale(B[0], oddsin<R>(k));
#pragma unroll
        for (int m = 2; m <= h; ++m) Q = caxpy(oddsin<R>(k * m), B[m - 1], Q);
        // s i Q with s = -1 (forward) -> -i Q ; s = +1 (inverse) -> +i Q
        E iQ = cmuli<INV>(Q);
        v[k] = cadd(P, iQ);
        v[R - k] = csub(P, iQ);
    }
    v[0] = sum;
}

// 16 points as two 8-point DFTs of the even and odd inputs, the odd ones
// rotated by w16^k = exp(s 2 pi i k / 16), then 8 sums and 8 differences
template <bool INV, typename E> __device__ __forceinline__ void dft16(E* v) {
    constexpr float C1 = 0.92387953251128676f, S1 = 0.38268343236508977f, H = 0.70710678118654752f;
    E e[8], o[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        e[m] = v[2 * m];
        o[m] = v[2 * m + 1];
    }
    dft8<INV>(e);
    dft8<INV>(o);
    constexpr float sg = INV ? 1.0f : -1.0f;
    o[1] = cmul(o[1], make_float2(C1, sg * S1));
    o[2] = cmul(o[2], make_float2(H, sg * H));
    o[3] = cmul(o[3], make_float2(S1, sg * C1));
    o[4] = cmuli<INV>(o[4]);
    o[5] = cmul(o[5], make_float2(-S1, sg * C1));
    o[6] = cmul(o[6], make_float2(-H, sg * H));
    o[7] = cmul(o[7], make_float2(-C1, sg * S1));
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        E a = e[k], b = o[k];
        v[k] = cadd(a, b);
        v[k + 8] = csub(a, b);
    }
}

template <int R, bool INV, typename E> __device__ __forceinline__ void dft(E* v) {
    if constexpr (R == 2) dft2<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v);
    else if constexpr (R == 8) dft8<INV>(v);
    else if constexpr (R == 16) dft16<INV>(v);
    else dft_odd<R, INV>(v);
}

// Padded layout of a sequence in LDS: element e at pidx(e) = e + e / 8, so
// that the stride-8 element accesses of a first radix-8 stage fall in
// distinct banks.
__host__ __device__ constexpr int pidx_len(int n) { return n + (n >> 3) + 1; }
__device__ __forceinline__ int pidx(int e) { return e + (e >> 3); }
// Pitch of padded rows that several lanes visit at one column (a transposing
// load or store): pidx_len rounded up to 2 modulo 32 complex values, so that
// consecutive rows start four banks apart (measured against 1, 4 and 8 modulo
// 32 on the TV row pass: 4% fewer bank-conflict cycles than 4, 1% faster).
__host__ __device__ constexpr int row_pitch(int n) { return pidx_len(n) + ((34 - pidx_len(n) % 32) % 32); }

// ----------------------------------------------------------- block-level transforms
// Used by the row passes: the `ntrans` transforms of length N of one block, at
// stride `tstride` (elements) in LDS, share the stages; every thread takes
// butterflies q = tid, tid + nthr, ... over all transforms, and the block
// synchronises between the loads and the stores of a stage. Requirement
// (checked on the host): ntrans * N / R <= (MAXE / R) * nthr. stw: the stage's
// twiddle block (entries [k][r - 1]).
template <int R, int MAXE, bool INV, bool PAD, typename E, typename TWP>
__device__ __forceinline__ void stockham_stage(ADMM_LDS E* buf, TWP stw, int ntrans, int tstride,
                                            int Ns, int nbf, unsigned mnbf, unsigned mns, int tid, int nthr) {
    constexpr int NB = MAXE / R;
    const int total = ntrans * nbf;
    E v[NB][R];
    int dst[NB], row[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int q = tid + i * nthr;
        dst[i] = -1;
        row[i] = 0;
        if (q < total) {
            const int t = (int)udiv16((unsigned)q, (unsigned)nbf, mnbf);
            const int j = q - t * nbf;
            const int jq = (int)udiv16((unsigned)j, (unsigned)Ns, mns);
            const int k = j - jq * Ns;
            const ADMM_LDS E* b = buf + t * tstride;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = lds_ld(b + (PAD ? pidx(j + r * nbf) : j + r * nbf));
            if (Ns > 1) {
                const TWP tk = stw + k * (R - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = tw_ld(tk + r - 1);
                    if (INV) w.y = -w.y;
                    v[i][r] = cmul(v[i][r], w);
                }
            }
            dft<R, INV>(v[i]);
            dst[i] = jq * Ns * R + k;
            row[i] = t * tstride;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if (dst[i] >= 0) {
            ADMM_LDS E* o = buf + row[i];
#pragma unroll
            for (int r = 0; r < R; ++r) lds_st(o + (PAD ? pidx(dst[i] + r * Ns) : dst[i] + r * Ns), v[i][r]);
        }
    }
    __syncthreads();
}

// Full transform of `ntrans` length-N sequences in LDS at stride `tstride`
// (natural order in and out, unnormalised); PAD: each sequence in the padded
// layout (pidx); stw: the length's stage table, in LDS (or, with TWG, in
// global memory). R16: whether radix-16 stages are compiled (the column
// schedules have none, and their code would set the kernel's register count).
template <int MAXE, bool INV, bool PAD, bool R16, typename E, typename TWP>
__device__ __forceinline__ void fft_lds_stages(ADMM_LDS E* buf, const FftPlanDev& f, TWP stw, int ntrans, int tstride,
                                               int tid, int nthr) {
    const int nst = f.nst;
    for (int s = 0; s < nst; ++s) {
        const int R = f.rad[s], Ns = f.ns[s], nbf = f.nbf[s];
        const unsigned mnbf = f.mnbf[s], mns = f.mns[s];
        const TWP t = stw + f.tso[s];
        switch (R) {
            case 16:
                if constexpr (R16) stockham_stage<16, MAXE, INV, PAD>(buf, t, ntrans, tstride, Ns, nbf, mnbf, mns, tid, nthr);
                break;
            case 8: stockham_stage<8, MAXE, INV, PAD>(buf, t, ntrans, tstride, Ns, nbf, mnbf, mns, tid, nthr); break;
            case 4: stockham_stage<4, MAXE, INV, PAD>(buf, t, ntrans, tstride, Ns, nbf, mnbf, mns, tid, nthr); break;
            case 2: stockham_stage<2, MAXE, INV, PAD>(buf, t, ntrans, tstride, Ns, nbf, mnbf, mns, tid, nthr); break;
            case 3: stockham_stage<3, MAXE, INV, PAD>(buf, t, ntrans, tstride, Ns, nbf, mnbf, mns, tid, nthr); break;
            case 5: stockham_stage<5, MAXE, INV, PAD>(buf, t, ntrans, tstride, Ns, nbf, mnbf, mns, tid, nthr); break;
            case 7: stockham_stage<7, MAXE, INV, PAD>(buf, t, ntrans, tstride, Ns, nbf, mnbf, mns, tid, nthr); break;
            default: break;
        }
    }
}
template <int MAXE, bool INV, bool PAD, bool TWG = false, bool R16 = true, typename E>
__device__ __forceinline__ void fft_lds(E* gbuf, const FftPlanDev& f, const float2* gstw, int ntrans, int tstride,
                                        int tid, int nthr) {
    if constexpr (TWG)
        fft_lds_stages<MAXE, INV, PAD, R16>((ADMM_LDS E*)gbuf, f, gstw, ntrans, tstride, tid, nthr);
    else
        fft_lds_stages<MAXE, INV, PAD, R16>((ADMM_LDS E*)gbuf, f, (const ADMM_LDS float2*)gstw, ntrans, tstride, tid,
                                            nthr);
}

// ----------------------------------------------------------- wave-level transforms
// One 64-lane wave owns one length-N sequence in LDS
// and transforms it alone (lane l takes butterflies j = l, l + 64, ... of every
// stage). A wave's LDS instructions are executed in issue order, so a stage
// needs no block barrier: all of a wave's loads of a stage are issued before
// its stores, and the next stage's loads after those stores. Waves therefore
// run their columns independently and overlap one another's memory phases.
// The sequence is stored padded (pidx).

// Keeps the compiler from moving LDS accesses across a stage boundary: the
// stages of a wave-owned transform exchange data between lanes, which the
// per-lane alias analysis cannot see.
__device__ __forceinline__ void lane_exchange_fence() { asm volatile("" ::: "memory"); }

// ---- general lengths: schedule read from the plan at run time
// One radix-R stage; NB bounds the butterflies per lane. stw: the stage's
// twiddle block (entries [k][r - 1]).
template <int R, int NB, bool INV, typename E>
__device__ __forceinline__ void wave_stage(ADMM_LDS E* buf, const ADMM_LDS float2* stw, int Ns, int nbf, unsigned mns,
                                        int lane) {
    E v[NB][R];
    int dst[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = lane + 64 * i;
        dst[i] = -1;
        if (j < nbf) {
            const int jq = (int)udiv16((unsigned)j, (unsigned)Ns, mns);
            const int k = j - jq * Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = lds_ld(buf + pidx(j + r * nbf));
            if (Ns > 1) {
                const ADMM_LDS float2* tk = stw + k * (R - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = lds_ld(tk + r - 1);
                    if (INV) w.y = -w.y;
                    v[i][r] = cmul(v[i][r], w);
                }
            }
            dft<R, INV>(v[i]);
            dst[i] = jq * Ns * R + k;
        }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if (dst[i] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) lds_st(buf + pidx(dst[i] + r * Ns), v[i][r]);
        }
    }
}

// Stages [s0, s1) of plan f on the wave-owned sequence buf; EPL bounds N / 64;
// stw: the length's stage table.
template <int EPL, bool INV, typename E>
__device__ __forceinline__ void wave_stages(ADMM_LDS E* buf, const ADMM_LDS float2* stw, const FftPlanDev& f, int s0,
                                            int s1, int lane) {
    for (int s = s0; s < s1; ++s) {
        const int Ns = f.ns[s], nbf = f.nbf[s];
        const unsigned mns = f.mns[s];
        const ADMM_LDS float2* t = stw + f.tso[s];
        switch (f.rad[s]) {
            case 8: wave_stage<8, (EPL + 7) / 8, INV>(buf, t, Ns, nbf, mns, lane); break;
            case 4: wave_stage<4, (EPL + 3) / 4, INV>(buf, t, Ns, nbf, mns, lane); break;
            case 2: wave_stage<2, (EPL + 1) / 2, INV>(buf, t, Ns, nbf, mns, lane); break;
            case 3: wave_stage<3, (EPL + 2) / 3, INV>(buf, t, Ns, nbf, mns, lane); break;
            case 5: wave_stage<5, (EPL + 4) / 5, INV>(buf, t, Ns, nbf, mns, lane); break;
            case 7: wave_stage<7, (EPL + 6) / 7, INV>(buf, t, Ns, nbf, mns, lane); break;
            default: break;
        }
    }
}

// ---- fixed lengths: the schedule is a compile-time constant, so every index,
// stride and twiddle offset folds into the instruction immediates
template <int N> struct CSched {
    static constexpr int nst() {
        int r[ADMM_MAX_STAGES] = {};
        return fft_schedule(N, r, ADMM_MAX_STAGES);
    }
    static constexpr int rad(int s) {
        int r[ADMM_MAX_STAGES] = {};
        fft_schedule(N, r, ADMM_MAX_STAGES);
        return r[s];
    }
    static constexpr int ns(int s) {
        int p = 1;
        for (int t = 0; t < s; ++t) p *= rad(t);
        return p;
    }
    static constexpr int tso(int s) {
        int o = 0;
        for (int t = 0; t < s; ++t) o += ns(t) * (rad(t) - 1);
        return o;
    }
};

template <int N, int S> struct CSt {
    static constexpr int R = CSched<N>::rad(S);
    static constexpr int Ns = CSched<N>::ns(S);
    static constexpr int nbf = N / R;
    static constexpr int NB = (nbf + 63) / 64;
    static constexpr int TSO = CSched<N>::tso(S);
    static constexpr bool full = nbf % 64 == 0;   // every lane has NB butterflies
};

// Operands of stage S: v[i][r] = x[j + r nbf], j = lane + 64 i.
template <int N, int S, typename E>
__device__ __forceinline__ void c_load(const ADMM_LDS E* buf, E (&v)[CSt<N, S>::NB][CSt<N, S>::R], int lane) {
    using T = CSt<N, S>;
#pragma unroll
    for (int i = 0; i < T::NB; ++i) {
        const int j = lane + 64 * i;
        if (T::full || j < T::nbf) {
            if constexpr (T::nbf % 8 == 0) {
                const ADMM_LDS E* b = buf + pidx(j);
#pragma unroll
                for (int r = 0; r < T::R; ++r) v[i][r] = lds_ld(b + r * (T::nbf + T::nbf / 8));
            } else {
#pragma unroll
                for (int r = 0; r < T::R; ++r) v[i][r] = lds_ld(buf + pidx(j + r * T::nbf));
            }
        }
    }
}

// Twiddles and the R-point DFTs of stage S (stw: the length's stage table).
template <int N, int S, bool INV, typename E>
__device__ __forceinline__ void c_bfly(const ADMM_LDS float2* stw, E (&v)[CSt<N, S>::NB][CSt<N, S>::R], int lane) {
    using T = CSt<N, S>;
#pragma unroll
    for (int i = 0; i < T::NB; ++i) {
        const int j = lane + 64 * i;
        if (T::full || j < T::nbf) {
            if constexpr (T::Ns > 1) {
                const ADMM_LDS float2* tk = stw + T::TSO + (j % T::Ns) * (T::R - 1);
#pragma unroll
                for (int r = 1; r < T::R; ++r) {
                    float2 w = lds_ld(tk + r - 1);
                    if (INV) w.y = -w.y;
                    v[i][r] = cmul(v[i][r], w);
                }
            }
            dft<T::R, INV>(v[i]);
        }
    }
}

// Results of stage S: x'[(j / Ns) Ns R + j mod Ns + r Ns] = v[i][r].
template <int N, int S, typename E>
__device__ __forceinline__ void c_store(ADMM_LDS E* buf, const E (&v)[CSt<N, S>::NB][CSt<N, S>::R], int lane) {
    using T = CSt<N, S>;
#pragma unroll
    for (int i = 0; i < T::NB; ++i) {
        const int j = lane + 64 * i;
        if (T::full || j < T::nbf) {
            const int d = (j / T::Ns) * T::Ns * T::R + j % T::Ns;
            if constexpr (T::Ns % 8 == 0) {
                ADMM_LDS E* b = buf + pidx(d);
#pragma unroll
                for (int r = 0; r < T::R; ++r) lds_st(b + r * (T::Ns + T::Ns / 8), v[i][r]);
            } else if constexpr (T::Ns == 1 && T::R == 8) {
                ADMM_LDS E* b = buf + 9 * j;   // pidx(8 j + r) = 9 j + r
#pragma unroll
                for (int r = 0; r < T::R; ++r) lds_st(b + r, v[i][r]);
            } else {
#pragma unroll
                for (int r = 0; r < T::R; ++r) lds_st(buf + pidx(d + r * T::Ns), v[i][r]);
            }
        }
    }
}

template <int N, int S, bool INV, typename E>
__device__ __forceinline__ void c_stage(ADMM_LDS E* buf, const ADMM_LDS float2* stw, int lane) {
    E v[CSt<N, S>::NB][CSt<N, S>::R];
    lane_exchange_fence();
    c_load<N, S>(buf, v, lane);
    c_bfly<N, S, INV>(stw, v, lane);
    c_store<N, S>(buf, v, lane);
    lane_exchange_fence();
}

// Stages [S0, S1) of the fixed-length transform on a wave-owned sequence.
template <int N, int S0, int S1, bool INV, typename E>
__device__ __forceinline__ void c_stages(ADMM_LDS E* buf, const ADMM_LDS float2* stw, int lane) {
    if constexpr (S0 < S1) {
        c_stage<N, S0, INV>(buf, stw, lane);
        c_stages<N, S0 + 1, S1, INV>(buf, stw, lane);
    }
}

// A whole transform of a wave-owned row of length N: the fixed-length code
// when N == NF, else the general stages.
template <int NF, int EPL, bool INV, typename E>
__device__ __forceinline__ void wave_fft(ADMM_LDS E* buf, const ADMM_LDS float2* stw, const FftPlanDev& f, int lane) {
    if (f.N == NF && f.variant == 0)
        c_stages<NF, 0, CSched<NF>::nst(), INV>(buf, stw, lane);
    else
        wave_stages<EPL, INV>(buf, stw, f, 0, f.nst, lane);
}

// ---- fixed-length block-level transforms (row passes): up to MAXT padded
// rows at `pitch` in LDS share the stages; butterfly q = tid + i NTHR of a
// stage belongs to row q / nbf and is butterfly q mod nbf of that row, and
// with the length fixed every such division is a shift or a constant multiply.
template <int N, int S, int NTHR, int MAXT, bool INV, typename E, typename TWP>
__device__ __forceinline__ void b_stage(ADMM_LDS E* buf, int pitch, TWP stw, int ntrans, int tid) {
    using T = CSt<N, S>;
    constexpr int NBT = (MAXT * T::nbf + NTHR - 1) / NTHR;
    E v[NBT][T::R];
    lane_exchange_fence();
#pragma unroll
    for (int i = 0; i < NBT; ++i) {
        const int q = tid + i * NTHR;
        const int t = q / T::nbf, j = q % T::nbf;
        if (t < ntrans) {
            const ADMM_LDS E* b = buf + t * pitch;
            if constexpr (T::nbf % 8 == 0) {
                b += pidx(j);
#pragma unroll
                for (int r = 0; r < T::R; ++r) v[i][r] = lds_ld(b + r * (T::nbf + T::nbf / 8));
            } else {
#pragma unroll
                for (int r = 0; r < T::R; ++r) v[i][r] = lds_ld(b + pidx(j + r * T::nbf));
            }
            if constexpr (T::Ns > 1) {
                const TWP tk = stw + T::TSO + (j % T::Ns) * (T::R - 1);
#pragma unroll
                for (int r = 1; r < T::R; ++r) {
                    float2 w = tw_ld(tk + r - 1);
                    if (INV) w.y = -w.y;
                    v[i][r] = cmul(v[i][r], w);
                }
            }
            dft<T::R, INV>(v[i]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NBT; ++i) {
        const int q = tid + i * NTHR;
        const int t = q / T::nbf, j = q % T::nbf;
        if (t < ntrans) {
            ADMM_LDS E* b = buf + t * pitch;
            const int d = (j / T::Ns) * T::Ns * T::R + j % T::Ns;
            if constexpr (T::Ns % 8 == 0) {
                b += pidx(d);
#pragma unroll
                for (int r = 0; r < T::R; ++r) lds_st(b + r * (T::Ns + T::Ns / 8), v[i][r]);
            } else if constexpr (T::Ns == 1 && T::R == 8) {
                b += 9 * j;   // pidx(8 j + r) = 9 j + r
#pragma unroll
                for (int r = 0; r < T::R; ++r) lds_st(b + r, v[i][r]);
            } else {
#pragma unroll
                for (int r = 0; r < T::R; ++r) lds_st(b + pidx(d + r * T::Ns), v[i][r]);
            }
        }
    }
    __syncthreads();
}

template <int N, int S0, int S1, int NTHR, int MAXT, bool INV, typename E, typename TWP>
__device__ __forceinline__ void b_stages(ADMM_LDS E* buf, int pitch, TWP stw, int ntrans, int tid) {
    if constexpr (S0 < S1) {
        b_stage<N, S0, NTHR, MAXT, INV>(buf, pitch, stw, ntrans, tid);
        b_stages<N, S0 + 1, S1, NTHR, MAXT, INV>(buf, pitch, stw, ntrans, tid);
    }
}

// Transform `ntrans` <= MAXT padded rows at `pitch`: the fixed-length code when
// the length is NF, else the run-time schedule (same layout). TWG: the stage
// table gstw is in global memory (else in LDS).
template <int NF, int NTHR, int MAXT, int MAXE, bool INV, bool TWG = false, typename E>
__device__ __forceinline__ void rows_fft(E* gbuf, int pitch, const FftPlanDev& f, const float2* gstw, int ntrans,
                                         int tid) {
    if (f.N == NF && f.variant == 0) {
        if constexpr (TWG)
            b_stages<NF, 0, CSched<NF>::nst(), NTHR, MAXT, INV>((ADMM_LDS E*)gbuf, pitch, gstw, ntrans, tid);
        else
            b_stages<NF, 0, CSched<NF>::nst(), NTHR, MAXT, INV>((ADMM_LDS E*)gbuf, pitch,
                                                                (const ADMM_LDS float2*)gstw, ntrans, tid);
    } else {
        fft_lds<MAXE, INV, true, TWG>(gbuf, f, gstw, ntrans, pitch, tid, NTHR);
    }
}

// The N entries of a stage table into LDS: the first NPT per thread in one
// burst of unconditional loads (indices clamped to the last entry), any
// remainder in a loop.
template <int NPT>
__device__ __forceinline__ void load_twiddles(float2* twl, const float2* __restrict__ tw, int N, int tid, int nthr) {
    if (N <= 0) return;
    float2 t[NPT];
#pragma unroll
    for (int u = 0; u < NPT; ++u) t[u] = tw[min(tid + u * nthr, N - 1)];
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        const int i = tid + u * nthr;
        if (i < N) twl[i] = t[u];
    }
    for (int i = tid + NPT * nthr; i < N; i += nthr) twl[i] = tw[i];
}

}  // namespace admm
