// fft.hpp -- wave-level complex FFTs for gfx950 (CDNA4, wave64).
//
// The multislice/PRISM propagation (Eq. 2) is a convolution done through
// FFTs ("PRISM Probe Simulations": batched FFTs over many plane waves).  Here
// every 1D transform of length L is owned by LPT = L/E lanes of one wavefront,
// each lane holding E elements in registers in "natural" order:
//     reg[i] of lane t  <->  element t + LPT * i.
// A transform is a sequence of radix-R Stockham (autosort, decimation in
// time) stages computed in registers; consecutive stages exchange data
// through an LDS buffer private to the wavefront, so no workgroup barrier is
// needed (FftT with SPAN = 2 spreads one transform over two wavefronts and
// orders its exchanges with workgroup barriers instead).  Input and output are both in natural order, which lets callers
// load and store straight from/to coalesced global memory.
//
// Transforms are unnormalised in both directions (DIR = -1 forward
// e^{-2 pi i jk/L}, DIR = +1 inverse e^{+2 pi i jk/L}).  Stage twiddles are
// read once per kernel from an FP64-derived table W_L[m] = e^{-2 pi i m/L}
// and kept in registers for every transform the wave performs.
#pragma once
#include <hip/hip_runtime.h>

namespace prism {

// ---------------------------------------------------------------- complex --
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * w for DIR = -1, a * conj(w) for DIR = +1 (w is a forward twiddle)
template <int DIR>
__device__ __forceinline__ float2 ctw(float2 a, float2 w) { return DIR < 0 ? cmul(a, w) : cmulc(a, w); }
__device__ __forceinline__ float cnorm(float2 a) { return a.x * a.x + a.y * a.y; }

// Ordering barrier for LDS traffic among the lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------- register DFTs --
// e^{DIR 2 pi i k / R} for compile-time k, R in {2, 4, 8, 16}; multiplication
// specialised for the trivial and the 45-degree angles.
template <int R, int K, int DIR>
__device__ __forceinline__ float2 mul_root(float2 a) {
    constexpr int k = ((K % R) + R) % R;
    if constexpr (k == 0) {
        return a;
    } else if constexpr (4 * k == R) {            // DIR * i
        return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
    } else if constexpr (2 * k == R) {            // -1
        return make_float2(-a.x, -a.y);
    } else if constexpr (4 * k == 3 * R) {        // -DIR * i
        return DIR < 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
    } else {
        // general angle: cos/sin of 2 pi k / R for R = 8, 16
        constexpr double c16[16] = {1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
                                    0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
                                    -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977,
                                    0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674};
        constexpr int m = k * (16 / R);
        constexpr float c = (float)c16[m];
        constexpr float s = (float)c16[(m + 12) % 16];   // sin(x) = cos(x - pi/2)
        constexpr float sd = DIR < 0 ? -s : s;
        if constexpr (m == 2 || m == 6 || m == 10 || m == 14) {
            // (+-1 +- i) / sqrt(2)
            return make_float2(c * a.x - sd * a.y, c * a.y + sd * a.x);
        } else {
            return make_float2(c * a.x - sd * a.y, sd * a.x + c * a.y);
        }
    }
}

template <int R, int DIR>
struct Dft;

template <int DIR>
struct Dft<1, DIR> {
    __device__ __forceinline__ static void run(float2*) {}
};

template <int DIR>
struct Dft<2, DIR> {
    __device__ __forceinline__ static void run(float2* v) {
        float2 a = v[0];
        v[0] = cadd(a, v[1]);
        v[1] = csub(a, v[1]);
    }
};

// Radix-2 split of a length-R DFT into even/odd halves (natural order in/out).
template <int R, int DIR>
struct Dft {
    template <int K>
    __device__ __forceinline__ static void combine(float2* v, const float2* e, const float2* o) {
        if constexpr (K < R / 2) {
            float2 t = mul_root<R, K, DIR>(o[K]);
            v[K] = cadd(e[K], t);
            v[K + R / 2] = csub(e[K], t);
            combine<K + 1>(v, e, o);
        }
    }
    __device__ __forceinline__ static void run(float2* v) {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        Dft<R / 2, DIR>::run(e);
        Dft<R / 2, DIR>::run(o);
        combine<0>(v, e, o);
    }
};

// ------------------------------------------------------------ radix plans --
// E: elements per lane; radices applied first to last (Ns = product of the
// previous radices).  Every radix divides E.
template <int L> struct Plan;
template <> struct Plan<16>   { static constexpr int E = 4,  NST = 2; static constexpr int R[3] = {4, 4, 1}; };
template <> struct Plan<32>   { static constexpr int E = 8,  NST = 2; static constexpr int R[3] = {8, 4, 1}; };
template <> struct Plan<64>   { static constexpr int E = 8,  NST = 2; static constexpr int R[3] = {8, 8, 1}; };
template <> struct Plan<128>  { static constexpr int E = 8,  NST = 3; static constexpr int R[3] = {8, 4, 4}; };
template <> struct Plan<256>  { static constexpr int E = 8,  NST = 3; static constexpr int R[3] = {8, 8, 4}; };
template <> struct Plan<512>  { static constexpr int E = 8,  NST = 3; static constexpr int R[3] = {8, 8, 8}; };
template <> struct Plan<1024> { static constexpr int E = 16, NST = 3; static constexpr int R[3] = {16, 8, 8}; };

// Plans of transforms spread over two wavefronts of a workgroup (fewer
// registers per lane than the one-wavefront plan of the same length).
template <int L> struct Plan2;
// Radix order of the two-wavefront 1024-point plan (the 2048^2 passes):
// 8, 2, 8, 8 measured 1.446 -> 1.428 s per 1245-beam build against 8, 8, 4, 4
// (8, 8, 8, 2 / 8, 4, 8, 4 / 8, 8, 2, 8 the same as 8, 8, 4, 4; 4, 4, 8, 8 and
// 2, 8, 8, 8 slower).
#ifndef PRISM_PLAN2_1024
#define PRISM_PLAN2_1024 8, 2, 8, 8
#endif
template <> struct Plan2<1024> { static constexpr int E = 8, NST = 4; static constexpr int R[4] = {PRISM_PLAN2_1024}; };

// SPAN wavefronts own one transform: SPAN = 1 synchronises a stage exchange
// within the wavefront; SPAN = 2 uses workgroup barriers, so every wavefront
// of the workgroup must run the same sequence of transforms.
template <int L, class PL = Plan<L>, int SPAN = 1>
struct FftT {
    static constexpr int E = PL::E;
    static constexpr int NST = PL::NST;
    static constexpr int LPT = L / E;                 // lanes per transform
    static_assert(SPAN == 1 ? LPT <= 64 : LPT == 64 * SPAN, "a transform spans a whole number of wavefronts");
    // Exchange buffers insert one pad slot every 2^PADSH elements, which
    // spreads the strided stage writes over the LDS banks: one slot every 8
    // elements (measured best for the 512-point passes), or every 16 for the
    // lengths L whose bit log2(L) is set in PRISM_PAD16_MASK.
#ifndef PRISM_PAD16_MASK
#define PRISM_PAD16_MASK (128 | 1024)   // L = 128 (the 128-pixel window transforms) and L = 1024 (the
                                        // 2048^2 passes: 1.492 -> 1.468 s per 1245-beam build)
#endif
    static constexpr int PADSH = ((PRISM_PAD16_MASK) >> __builtin_ctz(L)) & 1 ? 4 : 3;
    static constexpr int LDS = L + (L >> PADSH);      // padded exchange buffer (float2)

    static constexpr int radix(int s) { return PL::R[s]; }
    static constexpr int ns(int s) { return s == 0 ? 1 : ns(s - 1) * radix(s - 1); }
    // twiddle registers per lane: for stages s >= 1, (E/R) work items x (R-1)
    static constexpr int tw_off(int s) { return s <= 1 ? 0 : tw_off(s - 1) + (E / radix(s - 1)) * (radix(s - 1) - 1); }
    static constexpr int NTW = tw_off(NST) > 0 ? tw_off(NST) : 1;

    __device__ __forceinline__ static int pad(int i) { return i + (i >> PADSH); }

    // Ordering of exchange-buffer traffic among the lanes of one transform.
    __device__ __forceinline__ static void sync() {
        if constexpr (SPAN == 1)
            wave_sync();
        else
            __syncthreads();
    }

    // Forward twiddles of this lane, read from W_L[m] = e^{-2 pi i m / L}.
    struct Twiddles {
        float2 w[NTW];
        __device__ __forceinline__ void load(const float2* __restrict__ table, int lt) {
            load_stage<1>(table, lt);
        }
        template <int S>
        __device__ __forceinline__ void load_stage(const float2* __restrict__ table, int lt) {
            if constexpr (S < NST) {
                constexpr int R = radix(S), NS = ns(S), U = E / R;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    int j = lt + LPT * u;
                    int k = j % NS;
#pragma unroll
                    for (int r = 1; r < R; ++r)
                        w[tw_off(S) + u * (R - 1) + (r - 1)] = table[(r * k * (L / (NS * R))) % L];
                }
                load_stage<S + 1>(table, lt);
            }
        }
    };

    // LDS accessor of a transform's padded exchange buffer.
    struct RowX {
        float2* p;
        __device__ __forceinline__ float2& operator()(int i) const { return p[pad(i)]; }
    };
    // The same padded buffer with a compile-time stride between consecutive
    // slots (a column of a row-major array, exchanged in place).
    template <int STRIDE>
    struct StrideX {
        float2* p;
        __device__ __forceinline__ float2& operator()(int i) const { return p[pad(i) * STRIDE]; }
    };

    template <int DIR, int S, class X>
    __device__ __forceinline__ static void stage(float2 (&v)[E], const X& lds, const Twiddles& tw, int lt) {
        constexpr int R = radix(S), NS = ns(S), U = E / R;
        float2 out[E];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            float2 w[R];
#pragma unroll
            for (int r = 0; r < R; ++r) w[r] = v[u + r * U];
            if constexpr (S > 0) {
#pragma unroll
                for (int r = 1; r < R; ++r) w[r] = ctw<DIR>(w[r], tw.w[tw_off(S) + u * (R - 1) + (r - 1)]);
            }
            Dft<R, DIR>::run(w);
#pragma unroll
            for (int r = 0; r < R; ++r) out[u * R + r] = w[r];
        }
        if constexpr (S == NST - 1) {
            // last stage: outputs j + r*NS land in natural order
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int r = 0; r < R; ++r) v[u + r * U] = out[u * R + r];
        } else {
            sync();
#pragma unroll
            for (int u = 0; u < U; ++u) {
                int j = lt + LPT * u;
                int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
                for (int r = 0; r < R; ++r) lds(base + r * NS) = out[u * R + r];
            }
            sync();
#pragma unroll
            for (int i = 0; i < E; ++i) v[i] = lds(lt + LPT * i);
            stage<DIR, S + 1>(v, lds, tw, lt);
        }
    }

    // Two independent transforms advanced stage by stage together, so the LDS
    // round trip of one overlaps the arithmetic of the other.
    template <int DIR, int S, class X>
    __device__ __forceinline__ static void stage2(float2 (&v1)[E], float2 (&v2)[E], const X& x1, const X& x2,
                                                  const Twiddles& tw, int lt) {
        constexpr int R = radix(S), NS = ns(S), U = E / R;
        float2 o1[E], o2[E];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            float2 w1[R], w2[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                w1[r] = v1[u + r * U];
                w2[r] = v2[u + r * U];
            }
            if constexpr (S > 0) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const float2 t = tw.w[tw_off(S) + u * (R - 1) + (r - 1)];
                    w1[r] = ctw<DIR>(w1[r], t);
                    w2[r] = ctw<DIR>(w2[r], t);
                }
            }
            Dft<R, DIR>::run(w1);
            Dft<R, DIR>::run(w2);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                o1[u * R + r] = w1[r];
                o2[u * R + r] = w2[r];
            }
        }
        if constexpr (S == NST - 1) {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    v1[u + r * U] = o1[u * R + r];
                    v2[u + r * U] = o2[u * R + r];
                }
        } else {
            sync();
#pragma unroll
            for (int u = 0; u < U; ++u) {
                int j = lt + LPT * u;
                int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    x1(base + r * NS) = o1[u * R + r];
                    x2(base + r * NS) = o2[u * R + r];
                }
            }
            sync();
#pragma unroll
            for (int i = 0; i < E; ++i) {
                v1[i] = x1(lt + LPT * i);
                v2[i] = x2(lt + LPT * i);
            }
            stage2<DIR, S + 1>(v1, v2, x1, x2, tw, lt);
        }
    }

    // Two transforms at once, each with its own padded exchange buffer.
    template <int DIR>
    __device__ __forceinline__ static void run2(float2 (&v1)[E], float2 (&v2)[E], float2* lds1, float2* lds2,
                                                const Twiddles& tw, int lt) {
        stage2<DIR, 0>(v1, v2, RowX{lds1}, RowX{lds2}, tw, lt);
    }

    // In-place transform of the natural-order data v of lane lt (0..LPT-1);
    // lds: this transform's private exchange buffer (LDS entries padded).
    template <int DIR>
    __device__ __forceinline__ static void run(float2 (&v)[E], float2* lds, const Twiddles& tw, int lt) {
        stage<DIR, 0>(v, RowX{lds}, tw, lt);
    }
    // The same through any exchange accessor (RowX, StrideX).
    template <int DIR, class X>
    __device__ __forceinline__ static void run_x(float2 (&v)[E], const X& x, const Twiddles& tw, int lt) {
        stage<DIR, 0>(v, x, tw, lt);
    }
};

template <int L>
using Fft = FftT<L, Plan<L>, 1>;

}  // namespace prism
