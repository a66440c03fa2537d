// propagate.hip -- transmission and band-limited Fresnel propagation passes.
//
// One multislice step is transmission by exp(i sigma V_s) in real space
// (Eq. 1) followed by the Fresnel propagator exp(-i pi lambda |q|^2 dz) in
// Fourier space (Eq. 2), restricted to |q| < 1/(4 dx).  The band limit means a
// wave never holds energy at |kx| >= n/4, so between passes only the n/2
// band columns of the x-spectrum are stored:  W[item][j][y] (8 B each).
//
//   pass A (rows):    band row -> inverse row DFT -> x T_s -> forward row DFT -> band row
//   pass B (columns): column    -> forward column DFT -> x P (mask, phase, 1/n^2)
//                               -> inverse column DFT -> column
//
// An n-point transform whose input (inverse) or output (forward) is confined
// to the band splits exactly into two n/2-point transforms over the even and
// odd samples:
//   psi(2m)   = IDFT_{n/2}[Phi_j](m)
//   psi(2m+1) = IDFT_{n/2}[Phi_j e^{+2 pi i kx(j)/n}](m)
//   Phi_j     = DFT_{n/2}[psi(2m)]_j + e^{-2 pi i kx(j)/n} DFT_{n/2}[psi(2m+1)]_j
// so all transforms here have length n/2: one wavefront per transform, or
// two for the 1024-point transforms of the row and tiled column passes at
// n = 2048 (see FftFor below).
#include "fft.hpp"
#include "kernels.hpp"

namespace prism {

constexpr int WG = 256;      // 4 wavefronts

// Tuning constants (compile-time).
#ifndef PRISM_PASSA_ROWS
#define PRISM_PASSA_ROWS 16      // rows per pass-A workgroup for n <= 1024 (half that above)
#endif
#ifndef PRISM_PASSA_PAIR
#define PRISM_PASSA_PAIR 0       // 1: the two row tiles of one 2*TR-row band segment run on one XCD together
#endif
#ifndef PRISM_PASSA_ILP
#define PRISM_PASSA_ILP 0        // 1: even/odd row transforms advanced together (extra LDS)
#endif
#ifndef PRISM_PASSB_ILP
#define PRISM_PASSB_ILP 0        // 1: even/odd column transforms advanced together
#endif
#ifndef PRISM_PASSA_WPE
#define PRISM_PASSA_WPE 1        // minimum waves per SIMD asked of the register allocator
#endif
#ifndef PRISM_PASSB_WPE
#define PRISM_PASSB_WPE 1
#endif
#ifndef PRISM_PASSA_TPREF
#define PRISM_PASSA_TPREF 1024   // largest n whose transmission row is requested before the inverse
                                 // row transforms (measured better at n = 1024; at 2048 the same
                                 // time, and holding the row there spills registers)
#endif
#ifndef PRISM_PASSB_DEPTH
#define PRISM_PASSB_DEPTH 1      // columns prefetched ahead in registers (1 or 2)
#endif
#ifndef PRISM_PASSB_COLS
#define PRISM_PASSB_COLS 8       // adjacent columns per transform group in pass B (pipelined loads)
#endif

// Non-temporal wave-buffer traffic, measured at n = 1024 (1245 beams): in the
// column pass it takes 2.08 -> 1.95 ms per launch; in the row pass it costs
// 3.23 -> 3.58 ms (the column pass then misses the copy it would find in the
// last-level cache), so it stays off there.
#ifndef PRISM_NT_A
#define PRISM_NT_A 0             // 1: row-pass wave-buffer loads and stores non-temporal
#endif
#ifndef PRISM_NT_BL
#define PRISM_NT_BL 1            // 1: column-pass wave-buffer loads non-temporal
#endif
#ifndef PRISM_NT_BS
#define PRISM_NT_BS 1            // 1: column-pass wave-buffer stores non-temporal
#endif
// Wave-buffer traffic: each element is read and written once per pass, with
// no reuse within the pass.
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ float2 wave_load(const float2* p) {
    if constexpr (NT) {
        const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
        return make_float2(v.x, v.y);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ float4 wave_load(const float4* p) {
    if constexpr (NT) {
        const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
        return make_float4(v.x, v.y, v.z, v.w);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ void wave_store(float2* p, float2 v) {
    if constexpr (NT) __builtin_nontemporal_store(nt_f2{v.x, v.y}, reinterpret_cast<nt_f2*>(p));
    else *p = v;
}
template <bool NT>
__device__ __forceinline__ void wave_store(float4* p, float4 v) {
    if constexpr (NT) __builtin_nontemporal_store(nt_f4{v.x, v.y, v.z, v.w}, reinterpret_cast<nt_f4*>(p));
    else *p = v;
}

// Columns per pass-B transform group: pipelined when the column count allows.
template <int N, int MODE>
struct PassBCols {
    static constexpr int CPB = 4 * (64 / Fft<N / 2>::LPT);
    static constexpr int value =
        (MODE != PASSB_INIT && (N / 2) % (CPB * PRISM_PASSB_COLS) == 0) ? PRISM_PASSB_COLS : 1;
};

// Transforms of length L = n/2 spread over SPAN wavefronts.  The row pass and
// the tiled column pass use two wavefronts per 1024-point transform: the
// one-wavefront plan holds 16 elements per lane and needs more than 256
// registers, i.e. one wave per SIMD.
#ifndef PRISM_SPAN2_MIN
#define PRISM_SPAN2_MIN 2048     // smallest n whose row and tiled column passes use two-wavefront transforms
#endif
template <int L, int SPAN>
struct FftFor { using type = Fft<L>; };
template <>
struct FftFor<1024, 2> { using type = FftT<1024, Plan2<1024>, 2>; };
template <int N>
constexpr int pass_span() { return (N / 2 == 1024 && N >= PRISM_SPAN2_MIN) ? 2 : 1; }

template <int N, int SPAN = 1>
struct RowCfg {
    static constexpr int L = N / 2;
    using F = typename FftFor<L, SPAN>::type;
    static constexpr int E = F::E;
    static constexpr int LPT = F::LPT;
    static constexpr int G = LPT <= 64 ? 64 / LPT : 1;       // transforms per wave at once (SPAN = 1)
    static constexpr int TPW = WG / LPT;                     // transforms per workgroup at once
    static constexpr int TR0 = (N <= 1024) ? PRISM_PASSA_ROWS : PRISM_PASSA_ROWS / 2;
    static constexpr int TR = TR0 > TPW ? TR0 : TPW;         // rows per workgroup (tile height)
    static constexpr int ROW = F::LDS + 1;                   // odd LDS row stride (float2)
    static constexpr int XO = PRISM_PASSA_ILP ? TPW * F::LDS : 1;   // odd-transform buffers
};
// Row-pass configuration.
template <int N>
using RowCfgA = RowCfg<N, pass_span<N>()>;

// ------------------------------------------------------------ transmission --
__global__ __launch_bounds__(WG) void k_transmission(const float* __restrict__ V, float2* __restrict__ T,
                                                     int64_t count, float sigma) {
    int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * WG;
    for (; i < count; i += stride) {
        float s, c;
        sincosf(sigma * V[i], &s, &c);
        T[i] = make_float2(c, s);
    }
}

hipError_t launch_transmission(const float* V, float2* T, int64_t count, float sigma, hipStream_t st) {
    int64_t blocks = (count + WG - 1) / WG;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_transmission, dim3((unsigned)blocks), dim3(WG), 0, st, V, T, count, sigma);
    return hipGetLastError();
}

// ------------------------------------------------------------------ pass A --
// LDS (float2 slots) of one row-pass workgroup.
template <int N>
constexpr int pass_a_lds() { return RowCfgA<N>::TR * RowCfgA<N>::ROW + RowCfgA<N>::XO; }

// One row-pass workgroup: logical block blk of a launch over n_items items.
template <int N>
__device__ __forceinline__ void pass_a_block(float2* __restrict__ W, const float2* __restrict__ T,
                                             const PropTables& tb, int n_items, int blk, float2* smem) {
    using C = RowCfgA<N>;
    using F = typename C::F;
    constexpr int L = C::L, E = C::E, LPT = C::LPT, TPW = C::TPW, TR = C::TR, ROW = C::ROW;
    float2* const tile = smem;
    float2* const xodd = smem + TR * ROW;

    int item, y0;
    if constexpr (PRISM_PASSA_PAIR && (N / TR) % 2 == 0) {
        // Workgroups are dealt to the 8 XCDs in turn (blk % 8), so blocks blk
        // and blk + 8 of a run of 16 share an XCD and start together: give
        // them the two row tiles whose column segments share 2*TR*8-byte
        // lines.  Units (pairs of tiles) run item-fastest, as the tiles do
        // without pairing; a tail of fewer than 16 blocks takes its units two
        // blocks at a time.
        const int grid = n_items * (N / TR), full = grid & ~15;
        int u, h;
        if (blk < full) {
            u = (blk >> 4) * 8 + (blk & 7);
            h = (blk >> 3) & 1;
        } else {
            u = (full >> 1) + ((blk - full) >> 1);
            h = (blk - full) & 1;
        }
        item = u % n_items;
        y0 = (2 * (u / n_items) + h) * TR;
    } else {
        item = blk % n_items;
        y0 = (blk / n_items) * TR;
    }
    constexpr int CS = wave_col_stride(N);
    float2* Wi = W + (size_t)item * L * CS;
    const int tid = threadIdx.x;

    // Tile element (yy, j): thread tid owns yy = tid % TR and j = tid / TR + JS k.
    // JS is a multiple of the exchange padding period, so the padded LDS slot
    // of j advances by a compile-time step: pad(j0 + JS k) = pad(j0) + JSP k.
    static_assert((L * TR) % WG == 0, "tile must split evenly over the workgroup");
    constexpr int NLD = L * TR / WG, JS = WG / TR, JSP = JS + (JS >> F::PADSH);
    constexpr bool AFFINE = JS % (1 << F::PADSH) == 0;
    const int yy0 = tid % TR, j0 = tid / TR;
    float2* const gW = Wi + (size_t)j0 * CS + y0 + yy0;
    float2* const sW = tile + yy0 * ROW + F::pad(j0);
    auto lds_slot = [&](int k) -> float2& {
        if constexpr (AFFINE) return sW[k * JSP];
        else return tile[yy0 * ROW + F::pad(j0 + JS * k)];
    };
    {
        // all loads of the tile in flight before the first LDS store
        float2 ld[NLD];
#pragma unroll
        for (int k = 0; k < NLD; ++k) ld[k] = wave_load<PRISM_NT_A>(gW + (size_t)k * JS * CS);
#pragma unroll
        for (int k = 0; k < NLD; ++k) lds_slot(k) = ld[k];
        __syncthreads();
    }

    // transform tix of the workgroup (row yy = tix, tix + TPW, ...), lane lt of it
    const int tix = tid / LPT, lt = tid % LPT;
    typename F::Twiddles tw;
    tw.load(tb.tw_half, lt);
    float2 btw[E];
#pragma unroll
    for (int i = 0; i < E; ++i) btw[i] = tb.band_tw[lt + LPT * i];

    for (int yy = tix; yy < TR; yy += TPW) {      // the same trip count for every wavefront
        const int y = y0 + yy;
        float2* row = tile + yy * ROW;
        // transmission of this row, requested before the inverse transforms
        // so the load latency hides behind them
        float4 trow[E];
        const float4* Trow = reinterpret_cast<const float4*>(T + (size_t)y * N);
        if constexpr (N <= PRISM_PASSA_TPREF) {
#pragma unroll
            for (int i = 0; i < E; ++i) trow[i] = Trow[lt + LPT * i];
        }
        float2 e[E], o[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            e[i] = row[F::pad(lt + LPT * i)];
            o[i] = cmulc(e[i], btw[i]);
        }
        if constexpr (PRISM_PASSA_ILP) {
            F::template run2<+1>(e, o, row, xodd + tix * F::LDS, tw, lt);
        } else {
            F::template run<+1>(e, row, tw, lt);
            F::template run<+1>(o, row, tw, lt);
        }
        if constexpr (N > PRISM_PASSA_TPREF) {
#pragma unroll
            for (int i = 0; i < E; ++i) trow[i] = Trow[lt + LPT * i];
        }
#pragma unroll
        for (int i = 0; i < E; ++i) {
            e[i] = cmul(e[i], make_float2(trow[i].x, trow[i].y));
            o[i] = cmul(o[i], make_float2(trow[i].z, trow[i].w));
        }
        if constexpr (PRISM_PASSA_ILP) {
            F::template run2<-1>(e, o, row, xodd + tix * F::LDS, tw, lt);
        } else {
            F::template run<-1>(e, row, tw, lt);
            F::template run<-1>(o, row, tw, lt);
        }
        F::sync();
#pragma unroll
        for (int i = 0; i < E; ++i) row[F::pad(lt + LPT * i)] = cadd(e[i], cmul(btw[i], o[i]));
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NLD; ++k) wave_store<PRISM_NT_A>(gW + (size_t)k * JS * CS, lds_slot(k));
}

// Waves per SIMD asked of the register allocator: two for the two-wavefront
// transforms (whose registers fit that budget), PRISM_PASSA_WPE otherwise.
template <int N>
constexpr int pass_a_wpe() { return pass_span<N>() == 2 ? 2 : PRISM_PASSA_WPE; }

template <int N>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(pass_a_wpe<N>()))) void k_pass_a(
    float2* __restrict__ W, const float2* __restrict__ T, PropTables tb, int n_items) {
    __shared__ float2 smem[pass_a_lds<N>()];
    pass_a_block<N>(W, T, tb, n_items, blockIdx.x, smem);
}

template <int N>
static hipError_t pass_a_n(float2* W, const float2* T, const PropTables& tb, int n_items, hipStream_t st) {
    constexpr int TR = RowCfgA<N>::TR;
    dim3 grid((unsigned)((size_t)n_items * (N / TR)));
    hipLaunchKernelGGL((k_pass_a<N>), grid, dim3(WG), 0, st, W, T, tb, n_items);
    return hipGetLastError();
}

hipError_t launch_pass_a(int n, float2* W, const float2* T, const PropTables& tb, int n_items, hipStream_t st) {
    switch (n) {
        case 64: return pass_a_n<64>(W, T, tb, n_items, st);
        case 128: return pass_a_n<128>(W, T, tb, n_items, st);
        case 256: return pass_a_n<256>(W, T, tb, n_items, st);
        case 512: return pass_a_n<512>(W, T, tb, n_items, st);
        case 1024: return pass_a_n<1024>(W, T, tb, n_items, st);
        case 2048: return pass_a_n<2048>(W, T, tb, n_items, st);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------ first slice --
// A plane wave exp(2 pi i (kx x + ky y)/n) transmitted by the first slice and
// row-transformed is the first slice's row spectrum shifted by kx and phased
// by ky:
//   sum_x e^{2 pi i (kx x + ky y)/n} T0[y][x] e^{-2 pi i k x/n} = e^{2 pi i ky y/n} R[(k - kx) mod n][y],
//   R[c][y] = sum_x T0[y][x] e^{-2 pi i c x/n},
// so the first row pass of every beam is a gather from one table R, built
// once per call: an n-point transform per row, as two n/2-point transforms
// of the even and odd frequencies (decimation in frequency).
template <int N>
__global__ __launch_bounds__(WG) void k_row_spectrum(const float2* __restrict__ T0, float2* __restrict__ R,
                                                     PropTables tb) {
    using F = Fft<N / 2>;
    constexpr int L = N / 2, E = F::E, LPT = F::LPT, TPW = WG / LPT;
    static_assert(N % TPW == 0, "whole rows per workgroup");
    __shared__ float2 xch[TPW * F::LDS];
    const int tid = threadIdx.x, tix = tid / LPT, lt = tid % LPT;
    const int y = blockIdx.x * TPW + tix;
    typename F::Twiddles tw;
    tw.load(tb.tw_half, lt);
    const float2* row = T0 + (size_t)y * N;
    float2 a[E], b[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int x = lt + LPT * i;
        const float2 u = row[x], v = row[x + L];
        a[i] = cadd(u, v);                            // even frequencies 2c
        b[i] = cmul(csub(u, v), tb.tw_full[x]);       // odd frequencies 2c + 1
    }
    float2* x = xch + tix * F::LDS;
    F::template run<-1>(a, x, tw, lt);
    F::template run<-1>(b, x, tw, lt);
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int c = lt + LPT * i;
        R[(size_t)(2 * c) * N + y] = a[i];
        R[(size_t)(2 * c + 1) * N + y] = b[i];
    }
}

// W[item][j][y] = e^{2 pi i ky y/n} R[(kx(j) - kx) mod n][y] for the item's
// beam (kx, ky): one wavefront per band column, y contiguous in R and W.
template <int N>
__global__ __launch_bounds__(WG) void k_first_from_spectrum(float2* __restrict__ W, const float2* __restrict__ R,
                                                            PropTables tb, const int2* __restrict__ beams,
                                                            int n_items) {
    constexpr int L = N / 2, CS = wave_col_stride(N);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = blockIdx.x * (WG / 64) + wave;    // item-major: item * L + j
    const int item = col / L, j = col % L;
    if (item >= n_items) return;
    const int2 k = beams[item];
    const int kxj = j < N / 4 ? j : j - L;
    const float2* src = R + (size_t)((kxj - k.x) & (N - 1)) * N;
    float2* dst = W + ((size_t)item * L + j) * CS;
#pragma unroll 4
    for (int y = lane; y < N; y += 64) {
        const float2 w = tb.tw_full[(k.y * y) & (N - 1)];
        dst[y] = cmulc(src[y], w);                    // R * conj(e^{-2 pi i ky y/n})
    }
}

template <int N>
static hipError_t row_spectrum_n(const float2* T0, float2* R, const PropTables& tb, hipStream_t st) {
    constexpr int TPW = WG / Fft<N / 2>::LPT;
    hipLaunchKernelGGL((k_row_spectrum<N>), dim3(N / TPW), dim3(WG), 0, st, T0, R, tb);
    return hipGetLastError();
}

template <int N>
static hipError_t first_n(float2* W, const float2* R, const PropTables& tb, const int2* beams, int n_items,
                          hipStream_t st) {
    constexpr int L = N / 2, CPB = WG / 64;
    static_assert(L % CPB == 0, "whole workgroups per item");
    dim3 grid((unsigned)((size_t)n_items * (L / CPB)));
    hipLaunchKernelGGL((k_first_from_spectrum<N>), grid, dim3(WG), 0, st, W, R, tb, beams, n_items);
    return hipGetLastError();
}

hipError_t launch_row_spectrum(int n, const float2* T0, float2* R, const PropTables& tb, hipStream_t st) {
    switch (n) {
        case 64: return row_spectrum_n<64>(T0, R, tb, st);
        case 128: return row_spectrum_n<128>(T0, R, tb, st);
        case 256: return row_spectrum_n<256>(T0, R, tb, st);
        case 512: return row_spectrum_n<512>(T0, R, tb, st);
        case 1024: return row_spectrum_n<1024>(T0, R, tb, st);
        case 2048: return row_spectrum_n<2048>(T0, R, tb, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_first_from_spectrum(int n, float2* W, const float2* R, const PropTables& tb, const int2* beams,
                                      int n_items, hipStream_t st) {
    switch (n) {
        case 64: return first_n<64>(W, R, tb, beams, n_items, st);
        case 128: return first_n<128>(W, R, tb, beams, n_items, st);
        case 256: return first_n<256>(W, R, tb, beams, n_items, st);
        case 512: return first_n<512>(W, R, tb, beams, n_items, st);
        case 1024: return first_n<1024>(W, R, tb, beams, n_items, st);
        case 2048: return first_n<2048>(W, R, tb, beams, n_items, st);
    }
    return hipErrorInvalidValue;
}


// ------------------------------------------------------------------ pass B --
// LDS (float2 slots) of one column-pass workgroup.
template <int N>
constexpr int pass_b_lds() { return (PRISM_PASSB_ILP ? 2 : 1) * 4 * (64 / Fft<N / 2>::LPT) * Fft<N / 2>::LDS; }

// Workgroups of a column-pass launch over n_items items.
template <int N, int MODE>
constexpr int pass_b_blocks_per_item() {
    constexpr int CPB = 4 * (64 / Fft<N / 2>::LPT) * PassBCols<N, MODE>::value;
    return (N / 2 + CPB - 1) / CPB;
}

// One column-pass workgroup: logical block blk of a launch over n_items items.
template <int N, int MODE>
__device__ __forceinline__ void pass_b_block(float2* __restrict__ W, const PropTables& tb,
                                             const float2* __restrict__ aux, float* __restrict__ inten,
                                             const int* __restrict__ ky_max, const double2* __restrict__ probe_xy,
                                             double inv_L, float amp, int n_items, int blk, float2* smem) {
    using F = Fft<N / 2>;
    constexpr int L = N / 2, E = F::E, LPT = F::LPT, G = 64 / LPT, CPB = 4 * G;
    constexpr int NB = PRISM_PASSB_ILP ? 2 : 1;
    constexpr int NC = PassBCols<N, MODE>::value;   // adjacent columns per transform group
    float2* const xch = smem;

    const int item = blk % n_items;
    const int cb = blk / n_items;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int g = lane / LPT, lt = lane % LPT;
    const int j0 = (cb * CPB + wave * G + g) * NC;
    if (j0 >= L) return;                         // whole transform groups exit together
    float2* lds = xch + (wave * G + g) * F::LDS;
    float2* lds2 = xch + ((NB - 1) * CPB + wave * G + g) * F::LDS;

    typename F::Twiddles tw;
    tw.load(tb.tw_half, lt);
    float2 btw[E];
#pragma unroll
    for (int i = 0; i < E; ++i) btw[i] = tb.band_tw[lt + LPT * i];

    float2* const Wi = W + (size_t)item * L * wave_col_stride(N);
    float2 e[E], o[E];

    if constexpr (MODE == PASSB_INIT) {
        // aperture spectrum of the probe at (x, y): amp e^{-2 pi i (kx x + ky y) / L}
        const int j = j0;
        const int kxj = j < N / 4 ? j : j - N / 2;
        float4* col4 = reinterpret_cast<float4*>(Wi + (size_t)j * wave_col_stride(N));
        const double2 p = probe_xy[item];
        const int kym = ky_max[j];
        const double ax = (double)kxj * p.x * inv_L;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            int jp = lt + LPT * i;
            int ky = jp < N / 4 ? jp : jp - N / 2;
            float2 c = make_float2(0.f, 0.f);
            if (ky <= kym && -ky <= kym) {
                double a = ax + (double)ky * p.y * inv_L;
                float fr = (float)(a - rint(a));
                float s, cs;
                sincosf(-6.283185307179586f * fr, &s, &cs);
                c = make_float2(amp * cs, amp * s);
                if (aux) c = cmul(c, aux[(size_t)j * L + jp]);
            }
            e[i] = c;
            o[i] = cmulc(c, btw[i]);
        }
        if constexpr (PRISM_PASSB_ILP) {
            F::template run2<+1>(e, o, lds, lds2, tw, lt);
        } else {
            F::template run<+1>(e, lds, tw, lt);
            F::template run<+1>(o, lds, tw, lt);
        }
#pragma unroll
        for (int i = 0; i < E; ++i) wave_store<PRISM_NT_BS>(col4 + lt + LPT * i, make_float4(e[i].x, e[i].y, o[i].x, o[i].y));
        return;
    } else {
        // software pipeline over NC columns: the next column's loads are in
        // flight while this one is transformed.  The propagator factors are
        // read before the loop: vector memory waits complete in issue order,
        // so a table load inside the loop would also wait for the prefetch.
        float2 pk[E], pjs[NC];
#pragma unroll
        for (int i = 0; i < E; ++i) pk[i] = tb.prop[lt + LPT * i];
#pragma unroll
        for (int c = 0; c < NC; ++c) pjs[c] = tb.prop[j0 + c];
        // ring of DEPTH + 1 column buffers: slot c % (DEPTH + 1) holds column c
        constexpr int DEPTH = PRISM_PASSB_DEPTH;
        float4 ring[DEPTH + 1][E];
#pragma unroll
        for (int d = 0; d < DEPTH && d < NC; ++d) {
            const float4* c4 = reinterpret_cast<const float4*>(Wi + (size_t)(j0 + d) * wave_col_stride(N));
#pragma unroll
            for (int i = 0; i < E; ++i) ring[d][i] = wave_load<PRISM_NT_BL>(c4 + lt + LPT * i);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int j = j0 + c;
            float2* col = Wi + (size_t)j * wave_col_stride(N);
            float4* col4 = reinterpret_cast<float4*>(col);
            if (c + DEPTH < NC) {
                const float4* n4 = reinterpret_cast<const float4*>(col + DEPTH * wave_col_stride(N));
#pragma unroll
                for (int i = 0; i < E; ++i) ring[(c + DEPTH) % (DEPTH + 1)][i] = wave_load<PRISM_NT_BL>(n4 + lt + LPT * i);
            }
#pragma unroll
            for (int i = 0; i < E; ++i) {
                e[i] = make_float2(ring[c % (DEPTH + 1)][i].x, ring[c % (DEPTH + 1)][i].y);
                o[i] = make_float2(ring[c % (DEPTH + 1)][i].z, ring[c % (DEPTH + 1)][i].w);
            }
            const int kxj = j < N / 4 ? j : j - N / 2;
            if constexpr (PRISM_PASSB_ILP) {
                F::template run2<-1>(e, o, lds, lds2, tw, lt);
            } else {
                F::template run<-1>(e, lds, tw, lt);
                F::template run<-1>(o, lds, tw, lt);
            }
            const float2 pj = pjs[c];
#pragma unroll
            for (int i = 0; i < E; ++i) {
                int jp = lt + LPT * i;
                int ky = jp < N / 4 ? jp : jp - N / 2;
                float2 psi = cadd(e[i], cmul(btw[i], o[i]));
                bool in = 16 * (kxj * kxj + ky * ky) < N * N;
                e[i] = in ? cmul(psi, cmul(pj, pk[i])) : make_float2(0.f, 0.f);
            }
            if constexpr (MODE == PASSB_LAST_I) {
                float* dst = inten + ((size_t)item * L + j) * L;
#pragma unroll
                for (int i = 0; i < E; ++i) dst[lt + LPT * i] = cnorm(e[i]);
            } else if constexpr (MODE == PASSB_LAST_S) {
                // even rows only: psi(2 my) for my in [0, n/2), written over the
                // first half of this (already loaded) column
                F::template run<+1>(e, lds, tw, lt);
#pragma unroll
                for (int i = 0; i < E; ++i) col[lt + LPT * i] = e[i];
            } else {
#pragma unroll
                for (int i = 0; i < E; ++i) o[i] = cmulc(e[i], btw[i]);
                if constexpr (PRISM_PASSB_ILP) {
                    F::template run2<+1>(e, o, lds, lds2, tw, lt);
                } else {
                    F::template run<+1>(e, lds, tw, lt);
                    F::template run<+1>(o, lds, tw, lt);
                }
#pragma unroll
                for (int i = 0; i < E; ++i) wave_store<PRISM_NT_BS>(col4 + lt + LPT * i, make_float4(e[i].x, e[i].y, o[i].x, o[i].y));
            }
        }
    }
}

template <int N, int MODE>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(PRISM_PASSB_WPE))) void k_pass_b(
    float2* __restrict__ W, PropTables tb, const float2* __restrict__ aux, float* __restrict__ inten,
    const int* __restrict__ ky_max, const double2* __restrict__ probe_xy, double inv_L, float amp, int n_items) {
    __shared__ float2 smem[pass_b_lds<N>()];
    pass_b_block<N, MODE>(W, tb, aux, inten, ky_max, probe_xy, inv_L, amp, n_items, blockIdx.x, smem);
}

// Tile-staged column pass for interior and last slices (used from n = 2048,
// one transform per wavefront pair there): a workgroup stages TC whole
// columns into LDS with all its loads in flight at once (as pass A stages its
// row tile), then the wavefronts transform the columns from LDS, using each
// column's own LDS slots as the two padded exchange buffers of its even and
// odd transforms, and write the result straight from registers.  The last
// slice of an S-matrix build writes the even rows only; that of a multislice
// run writes the band intensities.
#ifndef PRISM_PASSB_TILE_MIN
#define PRISM_PASSB_TILE_MIN 2048   // smallest n whose column passes (all but the first) use k_pass_b_tile
#endif
template <int N>
struct PassBTile {
    using F = typename FftFor<N / 2, pass_span<N>()>::type;
    // measured: 2.08 -> 2.23 ms at n = 1024 (slower), 24.6 -> 16.4 ms at n = 2048
    static constexpr bool ok = (F::LPT == 64 || F::LPT == 128) && N >= PRISM_PASSB_TILE_MIN;
    // columns per workgroup; at n = 2048, 2 rather than 4: 10.5 -> 9.7 ms per launch
    static constexpr int TC = N <= 1024 ? 8 : 2;
    static constexpr int CS = 2 * F::LDS;                     // LDS slots per column (e and o buffers)
    static constexpr int TPW = WG / F::LPT;                   // columns transformed at once
};

template <int N, int MODE>
__global__ __launch_bounds__(WG) void k_pass_b_tile(float2* __restrict__ W, PropTables tb, float* __restrict__ inten,
                                                    int n_items) {
    static_assert(MODE == PASSB_MID || MODE == PASSB_LAST_S || MODE == PASSB_LAST_I, "interior or last slice");
    using T = PassBTile<N>;
    using F = typename T::F;
    constexpr int L = N / 2, E = F::E, LPT = F::LPT, TC = T::TC, CS = T::CS, TPW = T::TPW;
    static_assert(LPT == 64 || LPT == 128, "one or two wavefronts per transform");
    static_assert(TC % TPW == 0, "the same column count for every wavefront");
    __shared__ float2 tile[TC * CS];
    const int item = blockIdx.x % n_items;
    const int jb = (blockIdx.x / n_items) * TC;
    const int tid = threadIdx.x, tix = tid / LPT, lt = tid % LPT;
    float2* const Wi = W + (size_t)item * L * wave_col_stride(N);
    {
        // column c, float4 m = rows (2m, 2m+1): even sample to buffer 0, odd to buffer 1
        constexpr int NLD = TC * L / WG;
        static_assert((TC * L) % WG == 0, "tile must split evenly over the workgroup");
        float4 ld[NLD];
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int idx = tid + k * WG, c = idx / L, m = idx % L;
            ld[k] = wave_load<PRISM_NT_BL>(reinterpret_cast<const float4*>(Wi + (size_t)(jb + c) * wave_col_stride(N)) + m);
        }
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int idx = tid + k * WG, c = idx / L, m = idx % L;
            tile[c * CS + F::pad(m)] = make_float2(ld[k].x, ld[k].y);
            tile[c * CS + F::LDS + F::pad(m)] = make_float2(ld[k].z, ld[k].w);
        }
    }
    typename F::Twiddles tw;
    tw.load(tb.tw_half, lt);
    float2 btw[E], pk[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        btw[i] = tb.band_tw[lt + LPT * i];
        pk[i] = tb.prop[lt + LPT * i];
    }
    __syncthreads();
#pragma unroll 1
    for (int c = tix; c < TC; c += TPW) {
        const int j = jb + c;
        float2* const xe = tile + c * CS;
        float2* const xo = xe + F::LDS;
        float2 e[E], o[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            e[i] = xe[F::pad(lt + LPT * i)];
            o[i] = xo[F::pad(lt + LPT * i)];
        }
        F::template run<-1>(e, xe, tw, lt);
        F::template run<-1>(o, xo, tw, lt);
        const int kxj = j < N / 4 ? j : j - N / 2;
        const float2 pj = tb.prop[j];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int jp = lt + LPT * i;
            const int ky = jp < N / 4 ? jp : jp - N / 2;
            const float2 psi = cadd(e[i], cmul(btw[i], o[i]));
            const bool in = 16 * (kxj * kxj + ky * ky) < N * N;
            e[i] = in ? cmul(psi, cmul(pj, pk[i])) : make_float2(0.f, 0.f);
        }
        if constexpr (MODE == PASSB_LAST_I) {
            // multislice exit: band intensities of this column
            float* dst = inten + ((size_t)item * L + j) * L;
#pragma unroll
            for (int i = 0; i < E; ++i) dst[lt + LPT * i] = cnorm(e[i]);
        } else if constexpr (MODE == PASSB_LAST_S) {
            // S-matrix exit: even rows only, psi(2 my) for my in [0, n/2),
            // over the first half of this (already staged) column
            F::template run<+1>(e, xe, tw, lt);
            float2* col = Wi + (size_t)j * wave_col_stride(N);
#pragma unroll
            for (int i = 0; i < E; ++i) col[lt + LPT * i] = e[i];
        } else {
#pragma unroll
            for (int i = 0; i < E; ++i) o[i] = cmulc(e[i], btw[i]);
            F::template run<+1>(e, xe, tw, lt);
            F::template run<+1>(o, xo, tw, lt);
            float4* col4 = reinterpret_cast<float4*>(Wi + (size_t)j * wave_col_stride(N));
#pragma unroll
            for (int i = 0; i < E; ++i)
                wave_store<PRISM_NT_BS>(col4 + lt + LPT * i, make_float4(e[i].x, e[i].y, o[i].x, o[i].y));
        }
    }
}

template <int N, int MODE>
static hipError_t pass_b_nm(float2* W, const PropTables& tb, const float2* aux, float* inten, const int* ky_max,
                            const double2* xy, double inv_L, float amp, int n_items, hipStream_t st) {
    constexpr int L = N / 2, LPT = Fft<L>::LPT, CPB = 4 * (64 / LPT) * PassBCols<N, MODE>::value;
    if constexpr (MODE != PASSB_INIT && PassBTile<N>::ok) {
        constexpr int TC = PassBTile<N>::TC;
        static_assert(L % TC == 0, "columns must split into whole tiles");
        dim3 grid((unsigned)((size_t)n_items * (L / TC)));
        hipLaunchKernelGGL((k_pass_b_tile<N, MODE>), grid, dim3(WG), 0, st, W, tb, inten, n_items);
        return hipGetLastError();
    }
    dim3 grid((unsigned)((size_t)n_items * ((L + CPB - 1) / CPB)));
    hipLaunchKernelGGL((k_pass_b<N, MODE>), grid, dim3(WG), 0, st, W, tb, aux, inten, ky_max, xy, inv_L, amp,
                       n_items);
    return hipGetLastError();
}

template <int N>
static hipError_t pass_b_n(int mode, float2* W, const PropTables& tb, const float2* aux, float* inten,
                           const int* ky_max, const double2* xy, double inv_L, float amp, int n_items,
                           hipStream_t st) {
    switch (mode) {
        case PASSB_MID: return pass_b_nm<N, PASSB_MID>(W, tb, aux, inten, ky_max, xy, inv_L, amp, n_items, st);
        case PASSB_LAST_S:
            return pass_b_nm<N, PASSB_LAST_S>(W, tb, aux, inten, ky_max, xy, inv_L, amp, n_items, st);
        case PASSB_LAST_I:
            return pass_b_nm<N, PASSB_LAST_I>(W, tb, aux, inten, ky_max, xy, inv_L, amp, n_items, st);
        case PASSB_INIT: return pass_b_nm<N, PASSB_INIT>(W, tb, aux, inten, ky_max, xy, inv_L, amp, n_items, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_pass_b(int n, int mode, float2* W, const PropTables& tb, const float2* aux, float* inten,
                         const int* ky_max, const double2* probe_xy, double inv_L, float amp, int n_items,
                         hipStream_t st) {
    switch (n) {
        case 64: return pass_b_n<64>(mode, W, tb, aux, inten, ky_max, probe_xy, inv_L, amp, n_items, st);
        case 128: return pass_b_n<128>(mode, W, tb, aux, inten, ky_max, probe_xy, inv_L, amp, n_items, st);
        case 256: return pass_b_n<256>(mode, W, tb, aux, inten, ky_max, probe_xy, inv_L, amp, n_items, st);
        case 512: return pass_b_n<512>(mode, W, tb, aux, inten, ky_max, probe_xy, inv_L, amp, n_items, st);
        case 1024: return pass_b_n<1024>(mode, W, tb, aux, inten, ky_max, probe_xy, inv_L, amp, n_items, st);
        case 2048: return pass_b_n<2048>(mode, W, tb, aux, inten, ky_max, probe_xy, inv_L, amp, n_items, st);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------------- S-matrix final pass --
// W[b][j][my], my < n/2 (band x-spectrum of the even rows, left in the wave
// buffer by the last column pass) -> S[b][my][mx] = psi(2my, 2mx).
template <int N>
__global__ __launch_bounds__(WG) void k_smatrix_final(const float2* __restrict__ half, float2* __restrict__ S,
                                                      const float2* __restrict__ tw_half, int n_items) {
    using C = RowCfg<N>;
    using F = typename C::F;
    constexpr int L = C::L, E = C::E, LPT = C::LPT, G = C::G, TR = C::TR, ROW = C::ROW;
    constexpr int TRV = TR < L ? TR : L;         // valid rows per block
    __shared__ float2 tile[TR * ROW];

    const int item = blockIdx.x % n_items;
    const int y0 = (blockIdx.x / n_items) * TRV;
    constexpr int CS = wave_col_stride(N);
    const float2* Hi = half + (size_t)item * L * CS;
    const int tid = threadIdx.x;
    {
        constexpr int NLD = (L * TRV + WG - 1) / WG;
        float2 ld[NLD];
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int idx = tid + k * WG, yy = idx % TRV, j = idx / TRV;
            if (idx < L * TRV) ld[k] = Hi[(size_t)j * CS + y0 + yy];
        }
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int idx = tid + k * WG, yy = idx % TRV, j = idx / TRV;
            if (idx < L * TRV) tile[yy * ROW + F::pad(j)] = ld[k];
        }
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63;
    const int g = lane / LPT, lt = lane % LPT;
    typename F::Twiddles tw;
    tw.load(tw_half, lt);
    for (int r0 = wave * G; r0 < TRV; r0 += 4 * G) {
        const int yy = r0 + g;
        if (yy >= TRV) break;
        float2* row = tile + yy * ROW;
        float2 v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = row[F::pad(lt + LPT * i)];
        F::template run<+1>(v, row, tw, lt);
        float2* dst = S + ((size_t)item * L + y0 + yy) * L;
#pragma unroll
        for (int i = 0; i < E; ++i) dst[lt + LPT * i] = v[i];
    }
}

template <int N>
static hipError_t final_n(const float2* half, float2* S, const float2* tw_half, int n_items, hipStream_t st) {
    constexpr int L = N / 2, TR = RowCfg<N>::TR, TRV = TR < L ? TR : L;
    dim3 grid((unsigned)((size_t)n_items * (L / TRV)));
    hipLaunchKernelGGL((k_smatrix_final<N>), grid, dim3(WG), 0, st, half, S, tw_half, n_items);
    return hipGetLastError();
}

hipError_t launch_smatrix_final(int n, const float2* half, float2* S, const float2* tw_half, int n_items,
                                hipStream_t st) {
    switch (n) {
        case 64: return final_n<64>(half, S, tw_half, n_items, st);
        case 128: return final_n<128>(half, S, tw_half, n_items, st);
        case 256: return final_n<256>(half, S, tw_half, n_items, st);
        case 512: return final_n<512>(half, S, tw_half, n_items, st);
        case 1024: return final_n<1024>(half, S, tw_half, n_items, st);
        case 2048: return final_n<2048>(half, S, tw_half, n_items, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace prism
