// kernels.hpp -- host-side launchers of the gfx950 kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace prism {

// Band-limited wave buffer layout used by the propagation passes:
//   W[item][j][y], j in [0, n/2) a band column (kx = j for j < n/4, j - n/2
//   otherwise), y in [0, n) the real-space row.  One "item" is a beam
//   (S-matrix) or a probe (multislice).  Columns are wave_col_stride(n) >= n
//   elements apart so that the column starts do not all fall on the same
//   power-of-two address stride.
#ifndef PRISM_COL_PAD
#define PRISM_COL_PAD 0
#endif
constexpr int wave_col_stride(int n) { return n + PRISM_COL_PAD; }
struct PropTables {
    const float2* tw_half;   // W_{n/2}[m] = e^{-2 pi i m/(n/2)}, n/2 entries
    const float2* tw_full;   // W_n[m]     = e^{-2 pi i m/n},     n entries
    const float2* band_tw;   // e^{-2 pi i kx(j)/n}, n/2 entries
    const float2* prop;      // (1/n) e^{-i pi lambda dz kx(j)^2 / L^2}, n/2 entries
};

enum PassBMode { PASSB_MID = 0, PASSB_LAST_S = 1, PASSB_LAST_I = 2, PASSB_INIT = 3 };

// T[s][y][x] = exp(i sigma V[s][y][x]) for count = n_slices*n*n pixels.
hipError_t launch_transmission(const float* V, float2* T, int64_t count, float sigma, hipStream_t st);

// Row pass: for each item and real-space row y, inverse row transform of the
// band, multiply by T[y][x], forward row transform, keep the band.
hipError_t launch_pass_a(int n, float2* W, const float2* T, const PropTables& tb, int n_items, hipStream_t st);

// First row pass of plane-wave items, through the row spectrum of the first
// slice's transmission: R[c][y] = sum_x T0[y][x] e^{-2 pi i c x/n} (complex64
// [n][n], frequency-major), then W[item][j][y] = e^{2 pi i ky y/n}
// R[(kx(j) - kx) mod n][y] for the item's beam (kx, ky) -- the band of the
// row transform of the plane wave times T0.
hipError_t launch_row_spectrum(int n, const float2* T0, float2* R, const PropTables& tb, hipStream_t st);
hipError_t launch_first_from_spectrum(int n, float2* W, const float2* R, const PropTables& tb, const int2* beams,
                                      int n_items, hipStream_t st);

// Column pass (see PassBMode).  inten: band intensities [item][j][j'] for
// PASSB_LAST_I.  For PASSB_INIT the spectrum is the aperture: |ky| <= ky_max[j],
// coefficient amp e^{-2 pi i (kx x + ky y)/L} times aberr[j][j'] when `aux`
// (the aberration table, complex [n/2][n/2]) is not null.
hipError_t launch_pass_b(int n, int mode, float2* W, const PropTables& tb, const float2* aux, float* inten,
                         const int* ky_max, const double2* probe_xy, double inv_L, float amp, int n_items,
                         hipStream_t st);

// Final S-matrix pass: S[b][my][mx] = inverse row transform of half[b][j][my].
hipError_t launch_smatrix_final(int n, const float2* half, float2* S, const float2* tw_half, int n_items,
                                hipStream_t st);

// ---- projected potential --------------------------------------------------
struct PotAtom { double x, y; int32_t slice, species; };
struct PotSpecies { float amp_n[4]; float inv2w2[4]; float rc2; int n_gauss; float rc; int pad; };
hipError_t launch_potential(float* V, int n, int n_slices, double L, const PotAtom* atoms,
                            const int* slice_start, const PotSpecies* species, float rc_max, hipStream_t st);

// ---- probe synthesis ----------------------------------------------------------
// C[p][b] = amp * exp(-2 pi i (kx_b x_p + ky_b y_p) / L) (FP64 argument, range
// reduced), times aberr[b] when aberr is not null.
hipError_t launch_coefficients(float2* C, const double2* xy, const int2* beams, const float2* aberr, int n_probes,
                               int n_beams, double inv_L, float amp, hipStream_t st);

// Operand records of the MFMA contraction.  A K step is 16 beams; a record
// holds, for one (pixel or probe, K step), NP parts (hi, lo) x (re, im) x two
// halves of 8 beams as bf16: NP * 64 bytes, beams past n_beams zero.
//   split S:  [K step][pixel y ns + x][record]   (pixel-major)
//   split C:  [probe][K step][record]
constexpr int KSTEP = 16;
inline int ksteps_of(int n_beams) { return (n_beams + KSTEP - 1) / KSTEP; }
// Bytes reserved for either split layout (the split-BF16 size, the larger).
inline size_t split_s_bytes(int ns, int n_beams) { return (size_t)ns * ns * ksteps_of(n_beams) * 128; }
inline size_t split_c_bytes(int64_t n_probes, int n_beams) { return (size_t)n_probes * ksteps_of(n_beams) * 128; }
// True when the MFMA contraction reads S as split records (launch_split_s
// first); false when it splits the FP32 S-matrix itself.
bool contract_reads_split_s();
// S [n_beams][ns][ns] complex64 -> split S (precision PRISM_SPLIT_BF16X3 or PRISM_BF16).
hipError_t launch_split_s(int precision, const float2* S, void* Ssplit, int n_beams, int ns, hipStream_t st);
// Coefficients as launch_coefficients, written as split C (precision
// PRISM_SPLIT_BF16X3 or PRISM_BF16).
hipError_t launch_coefficients_split(int precision, void* Csplit, const double2* xy, const int2* beams,
                                     const float2* aberr, int n_probes, int n_beams, double inv_L, float amp,
                                     hipStream_t st);

// Windowed contraction of one probe set: win[p][v][u] = sum_b C[p][b] S[b][pix]
// over the plan's work tiles (16 x 16 pixels from tile_origin, periodic).
// C and S are complex64 ([n_probes][n_beams], [n_beams][ns][ns]) for FP32;
// for the MFMA precisions C is split C, and S is split S when
// contract_reads_split_s() (else complex64).
struct ContractArgs {
    const void* C;
    const void* S;
    float2* win;
    const int* tile_start;
    const int* tile_probes;
    const int2* tile_origin;
    const int2* corner;
    int n_tiles, max_per_tile, n_beams, ns, m;
    int accumulate = 0;       // add to the windows (partial sums over beam chunks)
};
// Probes per workgroup of the MFMA contraction (the plan's work-tile cost unit).
int contract_probe_chunk();
// All jobs in as few launches as possible (one per 24 jobs).
hipError_t launch_contract_batch(int precision, const ContractArgs* jobs, int n_jobs, hipStream_t st);

// out[p][bin] = sum over the bin's pixels of |FFT_m(win[p])|^2 / m^4.  For
// m > 128 the window is transformed in place and `inten` ([p][m*m] floats)
// holds the intensities; for m <= 128 both stay untouched.
struct WindowArgs {
    float2* win;
    float* inten;
    float* out;                // binned output, or null
    float* diff;               // [p][m][m] intensities (4D output), or null
    const int* perm;
    const int* bin_start;
    const float2* tw_m;
    int n_probes, n_bins;
    float scale;               // binned output = scale * sum (+ previous value when accumulating)
    int accumulate;
};
// All jobs of one window side m (one launch per 24 jobs for m <= 128).
hipError_t launch_window_batch(int m, const WindowArgs* jobs, int n_jobs, hipStream_t st);

// out[p][bin] = sum over bin pixels of inten[p][pix] (deterministic order).
hipError_t launch_bin_reduce(const float* inten, int64_t pix_per_item, float* out, const int* perm,
                             const int* bin_start, int n_items, int n_bins, hipStream_t st, float scale = 1.f,
                             int accumulate = 0);

}  // namespace prism
