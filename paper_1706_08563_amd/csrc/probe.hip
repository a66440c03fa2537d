// probe.hip -- PRISM probe synthesis: coefficients, windowed beam contraction,
// window FFT with |Psi|^2, and deterministic annular-detector sums.
//
// "PRISM Probe Simulations": each probe is a sum over plane waves of the
// cropped S-matrix layers times per-beam phase coefficients; the modulus
// squared of the FFT of that exit wave is binned into detectors (Fig. 1i-k).
#include "fft.hpp"
#include "kernels.hpp"

namespace prism {

constexpr int WG = 256;

// ------------------------------------------------------------ coefficients --
// C[p][b] = amp e^{-2 pi i (kx x + ky y)/L}; the phase argument is formed in
// FP64 and reduced to [-1/2, 1/2] turns before the FP32 sincos.
__device__ __forceinline__ float2 coefficient(double2 r, int2 k, const float2* __restrict__ aberr, int b,
                                              double inv_L, float amp) {
    double a = ((double)k.x * r.x + (double)k.y * r.y) * inv_L;
    float fr = (float)(a - rint(a));
    float s, c;
    sincosf(-6.283185307179586f * fr, &s, &c);
    float2 v = make_float2(amp * c, amp * s);
    if (aberr) v = cmul(v, aberr[b]);
    return v;
}

__global__ __launch_bounds__(WG) void k_coefficients(float2* __restrict__ C, const double2* __restrict__ xy,
                                                     const int2* __restrict__ beams,
                                                     const float2* __restrict__ aberr, int n_probes, int n_beams,
                                                     double inv_L, float amp) {
    int64_t total = (int64_t)n_probes * n_beams;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < total; i += (int64_t)gridDim.x * WG) {
        int p = (int)(i / n_beams), b = (int)(i % n_beams);
        C[i] = coefficient(xy[p], beams[b], aberr, b, inv_L, amp);
    }
}

hipError_t launch_coefficients(float2* C, const double2* xy, const int2* beams, const float2* aberr, int n_probes,
                               int n_beams, double inv_L, float amp, hipStream_t st) {
    int64_t total = (int64_t)n_probes * n_beams;
    int64_t blocks = (total + WG - 1) / WG;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_coefficients, dim3((unsigned)blocks), dim3(WG), 0, st, C, xy, beams, aberr, n_probes,
                       n_beams, inv_L, amp);
    return hipGetLastError();
}

// --------------------------------------------------- windowed contraction --
// The contraction runs over work tiles of 16 x 16 S-grid pixels.  A probe's
// M x M window starts at its corner; the plan gives every probe a tiling
// phase (an offset of the 16-pixel tile grid, at most its corner's position
// modulo 16) and lists the probe under each tile of that phase its window
// overlaps.  When the phase equals the corner's offset (as for probes on a
// scan lattice of a few pixels' pitch) the window is exactly (M/16)^2 tiles and
// no product falls outside it.  A workgroup takes one work tile and a chunk
// of PC of its probes and forms, for every tile pixel,
//     acc[p] = sum_b C[p][b] S[b][pixel]
// then stores each (probe, pixel) that lies inside the probe's window.  The
// tiles of one phase partition the S grid, so each window element is
// produced by exactly one (tile, probe) pair: no atomics.
constexpr int TILE = 16;

// Work of one (request's) probe synthesis inside a batched contraction launch.
struct ContractJob {
    const void* C;            // coefficients: complex64 [n_probes][n_beams] (FP32) or split C
    const void* S;            // S-matrix: complex64 [n_beams][ns][ns] (FP32) or split S
    float2* win;              // [n_probes][m][m]
    const int* tile_start;    // [n_tiles + 1]
    const int* tile_probes;
    const int2* tile_origin;  // [n_tiles] first pixel (x, y) of each work tile
    const int2* corner;       // window corner per probe
    int n_beams, ns, m;
    int ksteps;               // K steps of 16 beams (split layouts)
    int accumulate;           // 1: add to the windows' contents (beam chunks of one sum)
    int chunks;               // workgroups per tile (probe chunks)
    int n_tiles;
    int block0;               // first logical workgroup of this job
};
constexpr int MAX_JOBS = 24;
struct ContractBatch {
    int n_jobs;
    int n_blocks;             // logical workgroups over all jobs
    int per_xcd;              // logical workgroups per XCD slot
    ContractJob job[MAX_JOBS];
};

// Logical workgroup of this hardware workgroup.  Hardware workgroups are
// dealt round-robin to the 8 XCDs; consecutive logical workgroups are placed
// on the same XCD, so the probe chunks and phases of neighbouring tiles (the
// plan orders work tiles by position, then phase) share that XCD's L2.
// The selected job is copied out by value: taking the address of the
// by-value kernel argument would force a private-memory copy of the table.
__device__ __forceinline__ bool locate(const ContractBatch& b, ContractJob& job, int& tile, int& chunk) {
    const int hw = blockIdx.x;
    const int l = (hw & 7) * b.per_xcd + (hw >> 3);
    if (l >= b.n_blocks) return false;
    int j = 0;
#pragma unroll
    for (int k = 1; k < MAX_JOBS; ++k)
        if (k < b.n_jobs && b.job[k].block0 <= l) j = k;
    job = b.job[j];
    const int local = l - job.block0;
    tile = local / job.chunks;
    chunk = local % job.chunks;
    return true;
}

namespace fp32c {
constexpr int PC = 32;   // probes per workgroup
constexpr int KB = 32;   // beams per LDS chunk
}

__global__ __launch_bounds__(WG) void k_contract_fp32(ContractBatch batch) {
    using namespace fp32c;
    __shared__ float2 cs[KB][PC];
    __shared__ int pidx[PC];
    int tile, chunk;
    ContractJob job;
    if (!locate(batch, job, tile, chunk)) return;
    const float2* __restrict__ C = static_cast<const float2*>(job.C);
    const float2* __restrict__ S = static_cast<const float2*>(job.S);
    float2* __restrict__ win = job.win;
    const int* __restrict__ tile_probes = job.tile_probes;
    const int2* __restrict__ corner = job.corner;
    const int n_beams = job.n_beams, ns = job.ns, m = job.m;
    const int t0 = job.tile_start[tile], t1 = job.tile_start[tile + 1];
    const int pc0 = t0 + chunk * PC;
    if (pc0 >= t1) return;
    const int np = min(PC, t1 - pc0);
    const int2 org = job.tile_origin[tile];
    const int tid = threadIdx.x;
    const int px = (org.x + tid % TILE) & (ns - 1);
    const int py = (org.y + tid / TILE) & (ns - 1);
    if (tid < PC) pidx[tid] = tid < np ? tile_probes[pc0 + tid] : -1;
    __syncthreads();

    float2 acc[PC];
#pragma unroll
    for (int p = 0; p < PC; ++p) acc[p] = make_float2(0.f, 0.f);
    const size_t plane = (size_t)ns * ns;
    const float2* Sp = S + (size_t)py * ns + px;

    for (int b0 = 0; b0 < n_beams; b0 += KB) {
        for (int e = tid; e < KB * PC; e += WG) {
            int p = e / KB, kk = e % KB;
            float2 v = make_float2(0.f, 0.f);
            if (p < np && b0 + kk < n_beams) v = C[(size_t)pidx[p] * n_beams + b0 + kk];
            cs[kk][p] = v;
        }
        __syncthreads();
        const int kb = min(KB, n_beams - b0);
        float2 s[KB];
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) s[kk] = kk < kb ? Sp[(size_t)(b0 + kk) * plane] : make_float2(0.f, 0.f);
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
#pragma unroll
            for (int p = 0; p < PC; ++p) {
                float2 c = cs[kk][p];
                acc[p].x += c.x * s[kk].x - c.y * s[kk].y;
                acc[p].y += c.x * s[kk].y + c.y * s[kk].x;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < PC; ++p) {
        if (p < np) {
            int q = pidx[p];
            int2 c0 = corner[q];
            int v = (py - c0.y) & (ns - 1);
            int u = (px - c0.x) & (ns - 1);
            if (v < m && u < m) {
                float2* w = win + (size_t)q * m * m + (size_t)v * m + u;
                float2 r = acc[p];
                if (job.accumulate) r = cadd(*w, r);
                *w = r;
            }
        }
    }
}

// ----------------------------------------------- MFMA (BF16) contraction --
// The complex product is carried by real BF16 MFMA (v_mfma_f32_16x16x32_bf16)
// through the block identity, with K running over 16 beams twice:
//   Re = [Cr | -Ci] . [Sr ; Si]        Im = [Ci | Cr] . [Sr ; Si]
// Split mode: every FP32 operand x = hi + lo with hi = bf16(x), lo = bf16(x - hi),
// and each product is hi*hi + hi*lo + lo*hi accumulated in FP32 (the lo*lo
// term, ~2^-16 relative, is dropped).  Plain mode keeps hi*hi only.
//
// Operands are staged per K step (16 beams) as records: NP parts (hi, lo) x
// (re, im) x two halves of 8 beams as bf16, one record per pixel or probe.
// Both operands are converted once per call, before the contraction, into
// records in global memory: C per (probe, K step), S per (K step, pixel) in
// pixel-major order, so that a work tile at any phase reads each of its 16
// rows of records as one contiguous 2 KB run.  A workgroup copies a K step's
// records into LDS (S chunks permuted by tile pixel, see rec_key) and feeds
// the MFMAs while the next step's loads are in flight.  (The alternative
// PRISM_CONTRACT_PRESPLIT = 0 reads S in its FP32 layout and splits it on the
// fly: no converted copy, but every phase tile converting its pixels again.)
// With W wavefronts (4 or 8), wave w owns tile rows (16/W)w .. (16/W)(w+1)-1
// (16-pixel MFMA column blocks) and all W 16-probe row blocks: 16 W probes
// per workgroup.
#ifndef PRISM_CONTRACT_PRESPLIT
#define PRISM_CONTRACT_PRESPLIT 1   // 1: S as pixel-major split records; 0: FP32 S split on the fly
#endif
#ifndef PRISM_CONTRACT_WAVES
#define PRISM_CONTRACT_WAVES 4   // wavefronts per contraction workgroup (4: 64 probes, 8: 128 probes)
#endif
namespace mfmac {
constexpr int WAVES = PRISM_CONTRACT_WAVES;
constexpr int NT = 64 * WAVES;        // threads per workgroup
constexpr int PB = 16 / WAVES;        // tile rows (16-pixel MFMA column blocks) per wave
constexpr int QB = 16 / PB;           // 16-probe row blocks
constexpr int PC = 16 * QB;           // probes per workgroup
constexpr int SH = NT / 256;          // threads per tile pixel in the S staging
constexpr int HPT = 2 / SH;           // 8-beam halves of a K step converted per thread
}

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;

// Two floats to packed bf16 (round to nearest even, v_cvt_pk_bf16_f32).
__device__ __forceinline__ unsigned int pack_bf16(float a, float b) {
    bf16x2 h = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(unsigned int, h);
}
// x = hi + lo + O(2^-16 |x|): hi = bf16(x), lo = bf16(x - hi), for a pair.
__device__ __forceinline__ void split_pair(float a, float b, unsigned int& hi, unsigned int& lo) {
    hi = pack_bf16(a, b);
    const float ra = __uint_as_float(hi << 16), rb = __uint_as_float(hi & 0xffff0000u);
    lo = pack_bf16(a - ra, b - rb);
}
__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// Record chunk c (= part * 4 + reim * 2 + half) of row r sits at chunk
// position c ^ key(r): 8 consecutive rows then touch 8 distinct 16-byte bank
// groups (records of 128 bytes: key = r & 7; of 64 bytes: two rows share a
// 128-byte line and key = (r >> 1) & 3).
template <int NP>
__device__ __forceinline__ int rec_key(int r) { return NP == 2 ? (r & 7) : ((r >> 1) & 3); }

// Records of 8 complex values v[0..7] (beams half*8 + 0..7): writes chunks
// (reim, half) of each part into ch[part * 4 + reim * 2 + half].
template <int NP>
__device__ __forceinline__ void make_chunks(const float2 (&v)[8], int half, u32x4 (&ch)[NP * 4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        unsigned int rh, rl, ih, il;
        if constexpr (NP == 2) {
            split_pair(v[2 * i].x, v[2 * i + 1].x, rh, rl);
            split_pair(v[2 * i].y, v[2 * i + 1].y, ih, il);
            ch[4 + half][i] = rl;
            ch[6 + half][i] = il;
        } else {
            rh = pack_bf16(v[2 * i].x, v[2 * i + 1].x);
            ih = pack_bf16(v[2 * i].y, v[2 * i + 1].y);
        }
        ch[half][i] = rh;
        ch[2 + half][i] = ih;
    }
}

// The record chunks of one 8-beam half of a pixel's K step, written to the
// pixel's LDS record (chunk c at position c ^ key).
template <int NP, int HALF>
__device__ __forceinline__ void stage_s_half(const float2 (&v)[8], u32x4* rec, int key) {
    u32x4 ch[NP * 4];
    make_chunks<NP>(v, HALF, ch);
#pragma unroll
    for (int part = 0; part < NP; ++part)
#pragma unroll
        for (int reim = 0; reim < 2; ++reim) {
            const int c = part * 4 + reim * 2 + HALF;
            rec[c ^ key] = ch[c];
        }
}

// Split S, pixel-major: out[(k plane + pixel) NCH + c] holds chunk c of the
// record of K step k at pixel = y ns + x (chunks in order).  Thread = (K step,
// pixel); consecutive threads read consecutive pixels of each beam plane and
// write consecutive records.
template <int NP>
__global__ __launch_bounds__(WG) void k_split_s(const float2* __restrict__ S, u32x4* __restrict__ out, int n_beams,
                                                int plane, int K) {
    constexpr int NCH = NP * 4;
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= (int64_t)K * plane) return;
    const int k = (int)(i / plane), pix = (int)(i % plane);
    const float2* src = S + pix;
    float2 v[2][8];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int b = k * KSTEP + h * 8 + j;
            v[h][j] = b < n_beams ? src[(size_t)b * plane] : make_float2(0.f, 0.f);
        }
    u32x4 ch[NCH];
    make_chunks<NP>(v[0], 0, ch);
    make_chunks<NP>(v[1], 1, ch);
    u32x4* rec = out + i * NCH;
#pragma unroll
    for (int c = 0; c < NCH; ++c) rec[c] = ch[c];
}

hipError_t launch_split_s(int precision, const float2* S, void* Ssplit, int n_beams, int ns, hipStream_t st) {
    const int K = ksteps_of(n_beams), plane = ns * ns;
    const int64_t blocks = ((int64_t)K * plane + WG - 1) / WG;
    if (precision == 1)
        hipLaunchKernelGGL(k_split_s<2>, dim3((unsigned)blocks), dim3(WG), 0, st, S, static_cast<u32x4*>(Ssplit), n_beams,
                           plane, K);
    else
        hipLaunchKernelGGL(k_split_s<1>, dim3((unsigned)blocks), dim3(WG), 0, st, S, static_cast<u32x4*>(Ssplit), n_beams,
                           plane, K);
    return hipGetLastError();
}

// Split C: thread = (probe, K step, half of 8 beams); records unpermuted.
template <int NP>
__global__ __launch_bounds__(WG) void k_coefficients_split(u32x4* __restrict__ Cs, const double2* __restrict__ xy,
                                                           const int2* __restrict__ beams,
                                                           const float2* __restrict__ aberr, int n_probes,
                                                           int n_beams, int K, double inv_L, float amp) {
    constexpr int NCH = NP * 4;
    const int64_t total = (int64_t)n_probes * K * 2;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < total; i += (int64_t)gridDim.x * WG) {
        const int p = (int)(i / (2 * K)), r = (int)(i % (2 * K)), k = r >> 1, half = r & 1;
        const double2 xyp = xy[p];
        float2 v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int b = k * KSTEP + half * 8 + j;
            v[j] = b < n_beams ? coefficient(xyp, beams[b], aberr, b, inv_L, amp) : make_float2(0.f, 0.f);
        }
        u32x4 ch[NCH];
        make_chunks<NP>(v, half, ch);
        u32x4* rec = Cs + ((size_t)p * K + k) * NCH;
#pragma unroll
        for (int part = 0; part < NP; ++part) {
            rec[part * 4 + half] = ch[part * 4 + half];
            rec[part * 4 + 2 + half] = ch[part * 4 + 2 + half];
        }
    }
}

hipError_t launch_coefficients_split(int precision, void* Csplit, const double2* xy, const int2* beams,
                                     const float2* aberr, int n_probes, int n_beams, double inv_L, float amp,
                                     hipStream_t st) {
    const int K = ksteps_of(n_beams);
    int64_t total = (int64_t)n_probes * K * 2;
    int64_t blocks = (total + WG - 1) / WG;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    u32x4* Cs = static_cast<u32x4*>(Csplit);
    if (precision == 1)
        hipLaunchKernelGGL(k_coefficients_split<2>, dim3((unsigned)blocks), dim3(WG), 0, st, Cs, xy, beams, aberr,
                           n_probes, n_beams, K, inv_L, amp);
    else
        hipLaunchKernelGGL(k_coefficients_split<1>, dim3((unsigned)blocks), dim3(WG), 0, st, Cs, xy, beams, aberr,
                           n_probes, n_beams, K, inv_L, amp);
    return hipGetLastError();
}

template <int NP>
__global__ __launch_bounds__(mfmac::NT) __attribute__((amdgpu_waves_per_eu(2))) void k_contract_mfma(ContractBatch batch) {
    using namespace mfmac;
    constexpr int NCH = NP * 4;                 // 16-byte chunks per record
    constexpr int CPT = PC * NCH / NT;          // C chunks staged per thread
    __shared__ u32x4 Ss[256 * NCH];             // one K step of the tile (pixel records, chunks permuted)
    __shared__ u32x4 Cl[PC * NCH];              // one K step of the probe chunk (records permuted)
    __shared__ int pidx[PC];

    int tile, chunk;
    ContractJob job;
    if (!locate(batch, job, tile, chunk)) return;
    float2* __restrict__ win = job.win;
    const int* __restrict__ tile_probes = job.tile_probes;
    const int2* __restrict__ corner = job.corner;
    const int ns = job.ns, m = job.m, K = job.ksteps, n_beams = job.n_beams;
    const int t0 = job.tile_start[tile], t1 = job.tile_start[tile + 1];
    const int pc0 = t0 + chunk * PC;
    if (pc0 >= t1) return;
    const int np = min(PC, t1 - pc0);
    const int2 org = job.tile_origin[tile];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid < PC) pidx[tid] = tid < np ? tile_probes[pc0 + tid] : -1;

    f32x4 accr[QB][PB], acci[QB][PB];
#pragma unroll
    for (int a = 0; a < QB; ++a)
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            accr[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
            acci[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    const size_t plane = (size_t)ns * ns;
#if PRISM_CONTRACT_PRESPLIT
    // S staging: chunks q = tid + j NT of the step's 256 x NCH chunks, i.e.
    // chunk sc of tile pixels sp0 + j PPJ, read by raw buffer loads from a
    // scalar resource at the K step's records (byte offsets per chunk kept in
    // registers; rows wrap periodically)
    constexpr int SPT = 256 * NCH / NT, PPJ = NT / NCH;
    const int sc = tid % NCH, sp0 = tid / NCH;
    const int sx = (org.x + sp0 % TILE) & (ns - 1);
    const int skey = rec_key<NP>(sp0);          // the same for every j: PPJ is a multiple of 8
    int voff[SPT];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int sy = (org.y + (sp0 + j * PPJ) / TILE) & (ns - 1);
        voff[j] = ((sy * ns + sx) * NCH + sc) * (int)sizeof(u32x4);
    }
#else
    // S staging: tile pixel sp, 8-beam halves sh0 .. sh0 + HPT - 1 of each K
    // step, read by raw buffer loads: a scalar resource at the K step's first
    // beam plane, the pixel's byte offset in a plane (one register) and the
    // beam's plane offset as a scalar, so the 16 loads of a step cost no
    // address registers
    // (sh0 is uniform over a wavefront: 0 with 4 wavefronts)
    const int sp = tid & 255, sh0 = SH == 1 ? 0 : __builtin_amdgcn_readfirstlane((tid >> 8) * HPT);
    const int sy = (org.y + sp / TILE) & (ns - 1), sx = (org.x + sp % TILE) & (ns - 1);
    const int pix_off = (sy * ns + sx) * (int)sizeof(float2);
    const int plane_bytes = (int)(plane * sizeof(float2));
    const int skey = rec_key<NP>(sp);
#endif
    __syncthreads();
    // C staging: chunk q = tid * CPT + j of the step's PC x NCH chunks
    const int crow = (tid * CPT) / NCH, cc0 = (tid * CPT) % NCH;
    const int cq = pidx[crow];
    const u32x4* __restrict__ Cg = static_cast<const u32x4*>(job.C) + (size_t)(cq < 0 ? 0 : cq) * K * NCH + cc0;
    const int ckey = rec_key<NP>(crow);
    const u32x4 zero = u32x4{0u, 0u, 0u, 0u};

    u32x4 creg[CPT];
#if PRISM_CONTRACT_PRESPLIT
    u32x4 sreg[SPT];
    auto load_s = [&](int k) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<u32x4*>(static_cast<const u32x4*>(job.S) + (size_t)k * plane * NCH), (short)0, 0x7fffffff,
            0x00020000);
#pragma unroll
        for (int j = 0; j < SPT; ++j)
            sreg[j] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff[j], 0, 0));
    };
    auto stage_s = [&]() {
#pragma unroll
        for (int j = 0; j < SPT; ++j) Ss[(sp0 + j * PPJ) * NCH + (sc ^ skey)] = sreg[j];
    };
#else
    float2 sv[HPT][8];
    auto load_s = [&](int k) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float2*>(static_cast<const float2*>(job.S) + (size_t)k * KSTEP * plane), (short)0, 0x7fffffff,
            0x00020000);
        const bool full = k * KSTEP + KSTEP <= n_beams;   // every beam of the step exists (uniform)
#pragma unroll
        for (int h = 0; h < HPT; ++h)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int jb = (SH == 1 ? h : sh0) * 8 + j;
                sv[h][j] = full || k * KSTEP + jb < n_beams
                               ? __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, pix_off, jb * plane_bytes, 0))
                               : make_float2(0.f, 0.f);
            }
    };
    // record chunks of the staged halves (the half index must be a
    // compile-time constant: it selects registers)
    auto stage_s = [&]() {
        if constexpr (SH == 1) {
            stage_s_half<NP, 0>(sv[0], Ss + sp * NCH, skey);
            stage_s_half<NP, 1>(sv[HPT - 1], Ss + sp * NCH, skey);
        } else if (sh0 == 0) {
            stage_s_half<NP, 0>(sv[0], Ss + sp * NCH, skey);
        } else {
            stage_s_half<NP, 1>(sv[0], Ss + sp * NCH, skey);
        }
    };
#endif
    load_s(0);
#pragma unroll
    for (int j = 0; j < CPT; ++j) creg[j] = cq >= 0 ? Cg[j] : zero;

    const int col = lane & 15, g = lane >> 4;   // MFMA operand lane roles
    const u32x4 sgn = u32x4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
    for (int k = 0; k < K; ++k) {
        stage_s();
#pragma unroll
        for (int j = 0; j < CPT; ++j) Cl[crow * NCH + ((cc0 + j) ^ ckey)] = creg[j];
        __syncthreads();
        if (k + 1 < K) {
            load_s(k + 1);
#pragma unroll
            for (int j = 0; j < CPT; ++j) creg[j] = cq >= 0 ? Cg[(size_t)(k + 1) * NCH + j] : zero;
        }
        // B operand of lane group g: chunk part*4 + g (re beams 0-7, 8-15, im beams 0-7, 8-15)
        u32x4 Bop[NP][PB];
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) {
            const int pix = (PB * wave + pb) * TILE + col;
            const int key = rec_key<NP>(pix);
#pragma unroll
            for (int part = 0; part < NP; ++part) Bop[part][pb] = Ss[pix * NCH + ((part * 4 + g) ^ key)];
        }
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            const int row = 16 * qb + col;
            const int key = rec_key<NP>(row);
            // A_r = [Cr | -Ci]: chunk part*4 + g, negated for g >= 2; A_i = [Ci | Cr]: chunk part*4 + (g ^ 2)
            u32x4 Ar[NP], Ai[NP];
#pragma unroll
            for (int part = 0; part < NP; ++part) {
                Ar[part] = Cl[row * NCH + ((part * 4 + g) ^ key)];
                if (g >= 2) Ar[part] ^= sgn;
                Ai[part] = Cl[row * NCH + ((part * 4 + (g ^ 2)) ^ key)];
            }
#pragma unroll
            for (int pb = 0; pb < PB; ++pb) {
                accr[qb][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(Ar[0]), as_bf16x8(Bop[0][pb]),
                                                                      accr[qb][pb], 0, 0, 0);
                acci[qb][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(Ai[0]), as_bf16x8(Bop[0][pb]),
                                                                      acci[qb][pb], 0, 0, 0);
                if constexpr (NP == 2) {
                    accr[qb][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(Ar[0]), as_bf16x8(Bop[1][pb]),
                                                                          accr[qb][pb], 0, 0, 0);
                    acci[qb][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(Ai[0]), as_bf16x8(Bop[1][pb]),
                                                                          acci[qb][pb], 0, 0, 0);
                    accr[qb][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(Ar[1]), as_bf16x8(Bop[0][pb]),
                                                                          accr[qb][pb], 0, 0, 0);
                    acci[qb][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(Ai[1]), as_bf16x8(Bop[0][pb]),
                                                                          acci[qb][pb], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    // ---- epilogue: D row = probe 16 qb + 4 g + r, column = pixel
#pragma unroll
    for (int qb = 0; qb < QB; ++qb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = pidx[16 * qb + 4 * g + r];
            if (q < 0) continue;
            const int2 c0 = corner[q];
#pragma unroll
            for (int pb = 0; pb < PB; ++pb) {
                const int py = (org.y + PB * wave + pb) & (ns - 1), px = (org.x + col) & (ns - 1);
                const int v = (py - c0.y) & (ns - 1);
                const int u = (px - c0.x) & (ns - 1);
                if (v < m && u < m) {
                    float2* w = win + (size_t)q * m * m + (size_t)v * m + u;
                    float2 res = make_float2(accr[qb][pb][r], acci[qb][pb][r]);
                    if (job.accumulate) res = cadd(*w, res);
                    *w = res;
                }
            }
        }
}

int contract_probe_chunk() { return mfmac::PC; }
bool contract_reads_split_s() { return PRISM_CONTRACT_PRESPLIT != 0; }

hipError_t launch_contract_batch(int precision, const ContractArgs* jobs, int n_jobs, hipStream_t st) {
    const int pc = precision == 0 ? fp32c::PC : mfmac::PC;
    for (int j0 = 0; j0 < n_jobs; j0 += MAX_JOBS) {
        ContractBatch b{};
        b.n_jobs = n_jobs - j0 < MAX_JOBS ? n_jobs - j0 : MAX_JOBS;
        int blocks = 0;
        for (int k = 0; k < b.n_jobs; ++k) {
            const ContractArgs& a = jobs[j0 + k];
            ContractJob& job = b.job[k];
            job.C = a.C;
            job.S = a.S;
            job.win = a.win;
            job.tile_start = a.tile_start;
            job.tile_probes = a.tile_probes;
            job.tile_origin = a.tile_origin;
            job.corner = a.corner;
            job.n_beams = a.n_beams;
            job.ns = a.ns;
            job.m = a.m;
            job.ksteps = ksteps_of(a.n_beams);
            job.accumulate = a.accumulate;
            job.chunks = (a.max_per_tile + pc - 1) / pc;
            if (job.chunks < 1) job.chunks = 1;
            job.n_tiles = a.n_tiles;
            job.block0 = blocks;
            blocks += job.chunks * job.n_tiles;
        }
        b.n_blocks = blocks;
        b.per_xcd = (blocks + 7) / 8;
        if (blocks == 0) continue;
        dim3 grid((unsigned)(8 * b.per_xcd));
        if (precision == 0)
            hipLaunchKernelGGL(k_contract_fp32, grid, dim3(WG), 0, st, b);
        else if (precision == 1)
            hipLaunchKernelGGL(k_contract_mfma<2>, grid, dim3(mfmac::NT), 0, st, b);
        else
            hipLaunchKernelGGL(k_contract_mfma<1>, grid, dim3(mfmac::NT), 0, st, b);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------ deterministic bin sums --
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ------------------------------------------------------- window detection --
// One workgroup per probe: M x M window in LDS, row then column transforms,
// |Psi|^2 / M^4, then each bin summed over its pixel list by one wavefront.
struct WindowJob {
    const float2* win;        // [n_probes][m][m]
    float* out;               // [n_probes][n_bins], or null
    float* diff;              // [n_probes][m][m] intensities (4D output), or null
    const int* perm;          // window pixels grouped by bin
    const int* bin_start;     // [n_bins + 1]
    const float2* tw_m;       // W_m twiddles
    int n_bins;
    int probe0;               // first workgroup of this job
    float scale;              // out = scale * sum (+ out when accumulating)
    int accumulate;
};
struct WindowBatch {
    int n_jobs;
    WindowJob job[MAX_JOBS];
};

// The window sits in LDS with an odd row stride RS of at least the padded
// exchange length and with that many rows (more than M), so that each row
// transform and each column transform exchanges in place, through the
// padded slots of its own row or column: no separate exchange buffers, so
// the 128-point windows take 16 wavefronts per workgroup in the LDS that
// would otherwise hold 4 wavefronts' exchange buffers.  The odd stride keeps
// the strided column accesses of 16 lanes in distinct banks.
template <int M>
struct WinCfg {
    using F = Fft<M>;
    static constexpr int NW = M >= 128 ? 16 : 4;              // wavefronts per workgroup
    static constexpr int NT = 64 * NW;
    static constexpr int RS = F::LDS | 1;                     // row stride (float2), odd
    static constexpr int ROWS = F::LDS;                       // rows (the column exchanges use all)
};

template <int M>
__global__ __launch_bounds__(WinCfg<M>::NT) void k_window_detect(WindowBatch batch) {
    using C = WinCfg<M>;
    using F = typename C::F;
    constexpr int E = F::E, LPT = F::LPT, G = 64 / LPT, NW = C::NW, NT = C::NT, RS = C::RS;
    __shared__ float2 buf[C::ROWS * RS];
    int jj = 0;
#pragma unroll
    for (int k = 1; k < MAX_JOBS; ++k)
        if (k < batch.n_jobs && batch.job[k].probe0 <= (int)blockIdx.x) jj = k;
    const WindowJob job = batch.job[jj];
    const float2* __restrict__ win = job.win;
    float* __restrict__ out = job.out;
    float* __restrict__ diff = job.diff;
    const int* __restrict__ perm = job.perm;
    const int* __restrict__ bin_start = job.bin_start;
    const float2* __restrict__ tw_m = job.tw_m;
    const int n_bins = job.n_bins;
    const int p = (int)blockIdx.x - job.probe0;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int g = lane / LPT, lt = lane % LPT;
    const float2* w = win + (size_t)p * M * M;
    {
        // batches of loads in flight before their LDS stores
        constexpr int NLD = (M * M + NT - 1) / NT, BATCH = NLD < 16 ? NLD : 16;
        static_assert(NLD % BATCH == 0, "load batches must divide the window");
#pragma unroll 1
        for (int k0 = 0; k0 < NLD; k0 += BATCH) {
            float2 ld[BATCH];
#pragma unroll
            for (int k = 0; k < BATCH; ++k) {
                const int idx = tid + (k0 + k) * NT;
                if (idx < M * M) ld[k] = w[idx];
            }
#pragma unroll
            for (int k = 0; k < BATCH; ++k) {
                const int idx = tid + (k0 + k) * NT;
                if (idx < M * M) buf[(idx / M) * RS + idx % M] = ld[k];
            }
        }
    }
    __syncthreads();
    typename F::Twiddles tw;
    tw.load(tw_m, lt);
    // rows, each exchanged in its own padded row
    for (int r0 = wave * G; r0 < M; r0 += NW * G) {
        float2* row = buf + (r0 + g) * RS;
        float2 v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = row[lt + LPT * i];
        F::template run_x<-1>(v, typename F::RowX{row}, tw, lt);
        F::sync();
#pragma unroll
        for (int i = 0; i < E; ++i) row[lt + LPT * i] = v[i];
    }
    __syncthreads();
    // columns, each exchanged in its own padded column, then intensity in place
    const float scale = 1.0f / ((float)M * (float)M * (float)M * (float)M);
    for (int c0 = wave * G; c0 < M; c0 += NW * G) {
        float2* col = buf + c0 + g;
        float2 v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = col[(lt + LPT * i) * RS];
        F::template run_x<-1>(v, typename F::template StrideX<RS>{col}, tw, lt);
        F::sync();
#pragma unroll
        for (int i = 0; i < E; ++i) col[(lt + LPT * i) * RS] = make_float2(cnorm(v[i]) * scale, 0.f);
    }
    __syncthreads();
    if (diff) {
        // the 4D output takes the same scale and accumulation as the 3D one
        float* d = diff + (size_t)p * M * M;
        for (int idx = tid; idx < M * M; idx += NT) {
            const float v = job.scale * buf[(idx / M) * RS + idx % M].x;
            d[idx] = job.accumulate ? d[idx] + v : v;
        }
    }
    if (!out) return;
    for (int b = wave; b < n_bins; b += NW) {
        float s = 0.f;
        for (int k = bin_start[b] + lane; k < bin_start[b + 1]; k += 64) {
            int pix = perm[k];
            s += buf[(pix / M) * RS + pix % M].x;
        }
        s = wave_sum(s);
        if (lane == 0) {
            float* o = out + (size_t)p * n_bins + b;
            *o = job.accumulate ? *o + job.scale * s : job.scale * s;
        }
    }
}

template <int M>
static hipError_t window_m(const WindowArgs* jobs, int n_jobs, hipStream_t st) {
    for (int j0 = 0; j0 < n_jobs; j0 += MAX_JOBS) {
        WindowBatch b{};
        b.n_jobs = n_jobs - j0 < MAX_JOBS ? n_jobs - j0 : MAX_JOBS;
        int blocks = 0;
        for (int k = 0; k < b.n_jobs; ++k) {
            const WindowArgs& a = jobs[j0 + k];
            b.job[k] = WindowJob{a.win, a.out, a.diff, a.perm, a.bin_start, a.tw_m, a.n_bins, blocks, a.scale,
                                 a.accumulate};
            blocks += a.n_probes;
        }
        if (blocks == 0) continue;
        hipLaunchKernelGGL((k_window_detect<M>), dim3((unsigned)blocks), dim3(WinCfg<M>::NT), 0, st, b);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------- large windows (M = 256, 512) --
// A window no longer fits in LDS: rows are transformed in place in HBM, then
// 16-column strips are staged through LDS for the column transforms, which
// write |Psi|^2 / M^4 to an intensity buffer binned by k_bin_reduce.
template <int M>
__global__ __launch_bounds__(WG) void k_window_rows(float2* __restrict__ win, const float2* __restrict__ tw_m,
                                                    int64_t n_rows) {
    using F = Fft<M>;
    constexpr int E = F::E, LPT = F::LPT, G = 64 / LPT;
    __shared__ float2 xch[4 * G * F::LDS];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int g = lane / LPT, lt = lane % LPT;
    const int64_t r = (int64_t)blockIdx.x * 4 * G + wave * G + g;
    if (r >= n_rows) return;
    typename F::Twiddles tw;
    tw.load(tw_m, lt);
    float2* row = win + r * M;
    float2 v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = row[lt + LPT * i];
    F::template run<-1>(v, xch + (wave * G + g) * F::LDS, tw, lt);
#pragma unroll
    for (int i = 0; i < E; ++i) row[lt + LPT * i] = v[i];
}

template <int M>
__global__ __launch_bounds__(WG) void k_window_cols(const float2* __restrict__ win, float* __restrict__ inten,
                                                    const float2* __restrict__ tw_m) {
    using F = Fft<M>;
    constexpr int E = F::E, LPT = F::LPT, G = 64 / LPT, CW = 16, ROWS = CW + 1;
    __shared__ float2 strip[M * ROWS];
    __shared__ float2 xch[4 * G * F::LDS];
    const int p = blockIdx.y, u0 = blockIdx.x * CW;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int g = lane / LPT, lt = lane % LPT;
    const float2* w = win + (size_t)p * M * M;
    {
        constexpr int NLD = M * CW / WG;
        float2 ld[NLD];
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int idx = tid + k * WG, v = idx / CW, c = idx % CW;
            ld[k] = w[(size_t)v * M + u0 + c];
        }
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int idx = tid + k * WG, v = idx / CW, c = idx % CW;
            strip[v * ROWS + c] = ld[k];
        }
    }
    __syncthreads();
    typename F::Twiddles tw;
    tw.load(tw_m, lt);
    const float scale = 1.0f / ((float)M * (float)M * (float)M * (float)M);
    float* I = inten + (size_t)p * M * M;
    for (int c0 = wave * G; c0 < CW; c0 += 4 * G) {
        const int c = c0 + g;
        float2* col = strip + c;
        float2 v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = col[(lt + LPT * i) * ROWS];
        F::template run<-1>(v, xch + (wave * G + g) * F::LDS, tw, lt);
#pragma unroll
        for (int i = 0; i < E; ++i) I[(size_t)(lt + LPT * i) * M + u0 + c] = cnorm(v[i]) * scale;
    }
}

// diff = scale * inten (+ diff when accumulating): the 4D output of a large
// window when it is scaled or accumulated (the bins read the plain intensity).
__global__ __launch_bounds__(WG) void k_scale_into(float* __restrict__ diff, const float* __restrict__ inten,
                                                   int64_t count, float scale, int accumulate) {
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < count; i += (int64_t)gridDim.x * WG) {
        const float v = scale * inten[i];
        diff[i] = accumulate ? diff[i] + v : v;
    }
}

template <int M>
static hipError_t window_large(float2* win, float* inten, float* out, const int* perm, const int* bin_start,
                               const float2* tw_m, int n_probes, int n_bins, float scale, int accumulate,
                               hipStream_t st) {
    // inten receives |Psi|^2 / M^4 (it is the 4D output when one is requested
    // unscaled and not accumulated)
    constexpr int G = 64 / Fft<M>::LPT;
    const int64_t rows = (int64_t)n_probes * M;
    hipLaunchKernelGGL((k_window_rows<M>), dim3((unsigned)((rows + 4 * G - 1) / (4 * G))), dim3(WG), 0, st, win,
                       tw_m, rows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_window_cols<M>), dim3(M / 16, (unsigned)n_probes), dim3(WG), 0, st, win, inten, tw_m);
    e = hipGetLastError();
    if (e != hipSuccess || !out) return e;
    return launch_bin_reduce(inten, (int64_t)M * M, out, perm, bin_start, n_probes, n_bins, st, scale, accumulate);
}

hipError_t launch_window_batch(int m, const WindowArgs* jobs, int n_jobs, hipStream_t st) {
    switch (m) {
        case 16: return window_m<16>(jobs, n_jobs, st);
        case 32: return window_m<32>(jobs, n_jobs, st);
        case 64: return window_m<64>(jobs, n_jobs, st);
        case 128: return window_m<128>(jobs, n_jobs, st);
        case 256:
        case 512:
            for (int k = 0; k < n_jobs; ++k) {
                const WindowArgs& a = jobs[k];
                const bool direct = a.diff && a.scale == 1.0f && !a.accumulate;
                float* I = direct ? a.diff : a.inten;
                hipError_t e = m == 256 ? window_large<256>(a.win, I, a.out, a.perm, a.bin_start, a.tw_m,
                                                            a.n_probes, a.n_bins, a.scale, a.accumulate, st)
                                        : window_large<512>(a.win, I, a.out, a.perm, a.bin_start, a.tw_m,
                                                            a.n_probes, a.n_bins, a.scale, a.accumulate, st);
                if (e != hipSuccess) return e;
                if (a.diff && !direct) {
                    const int64_t count = (int64_t)a.n_probes * m * m;
                    const int64_t blocks = std::min<int64_t>((count + WG - 1) / WG, 65536);
                    hipLaunchKernelGGL(k_scale_into, dim3((unsigned)blocks), dim3(WG), 0, st, a.diff, a.inten, count,
                                       a.scale, a.accumulate);
                    e = hipGetLastError();
                    if (e != hipSuccess) return e;
                }
            }
            return hipSuccess;
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------- bin reduce --
__global__ __launch_bounds__(WG) void k_bin_reduce(const float* __restrict__ inten, int64_t pix_per_item,
                                                   float* __restrict__ out, const int* __restrict__ perm,
                                                   const int* __restrict__ bin_start, int n_bins, float scale,
                                                   int accumulate) {
    const int item = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const float* I = inten + (size_t)item * pix_per_item;
    for (int b = wave; b < n_bins; b += 4) {
        float s = 0.f;
        for (int k = bin_start[b] + lane; k < bin_start[b + 1]; k += 64) s += I[perm[k]];
        s = wave_sum(s);
        if (lane == 0) {
            float* o = out + (size_t)item * n_bins + b;
            *o = accumulate ? *o + scale * s : scale * s;
        }
    }
}

hipError_t launch_bin_reduce(const float* inten, int64_t pix_per_item, float* out, const int* perm,
                             const int* bin_start, int n_items, int n_bins, hipStream_t st, float scale,
                             int accumulate) {
    hipLaunchKernelGGL(k_bin_reduce, dim3((unsigned)n_items), dim3(WG), 0, st, inten, pix_per_item, out, perm,
                       bin_start, n_bins, scale, accumulate);
    return hipGetLastError();
}

}  // namespace prism
