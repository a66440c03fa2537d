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
__global__ __launch_bounds__(WG) void k_coefficients(float2* __restrict__ C, const double2* __restrict__ xy,
                                                     const int2* __restrict__ beams,
                                                     const float2* __restrict__ aberr, int n_probes, int n_beams,
                                                     double inv_L, float amp) {
    int64_t total = (int64_t)n_probes * n_beams;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < total; i += (int64_t)gridDim.x * WG) {
        int p = (int)(i / n_beams), b = (int)(i % n_beams);
        double2 r = xy[p];
        int2 k = beams[b];
        double a = ((double)k.x * r.x + (double)k.y * r.y) * inv_L;
        float fr = (float)(a - rint(a));
        float s, c;
        sincosf(-6.283185307179586f * fr, &s, &c);
        float2 v = make_float2(amp * c, amp * s);
        if (aberr) v = cmul(v, aberr[b]);
        C[i] = v;
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
// The S grid is cut into 16 x 16 pixel tiles.  For each tile the plan lists
// every probe whose M x M window overlaps it.  A workgroup takes one tile and
// a chunk of PC of those probes and forms, for every tile pixel,
//     acc[p] = sum_b C[p][b] S[b][pixel]
// then stores each (probe, pixel) that lies inside the probe's window.  Each
// window element is produced by exactly one (tile, probe) pair, so no atomics.
constexpr int TILE = 16;

// Work of one (request's) probe synthesis inside a batched contraction launch.
struct ContractJob {
    const float2* C;          // [n_probes][n_beams] coefficients
    const float2* S;          // [n_beams][ns][ns]
    float2* win;              // [n_probes][m][m]
    const int* tile_start;    // [n_tiles + 1]
    const int* tile_probes;
    const int2* corner;       // window corner per probe
    int n_beams, ns, m;
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
// dealt round-robin to the 8 XCDs; logical workgroups l and l+1 are placed on
// the same XCD, so all probe chunks of a pixel tile share that XCD's L2.
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
    const float2* __restrict__ C = job.C;
    const float2* __restrict__ S = job.S;
    float2* __restrict__ win = job.win;
    const int* __restrict__ tile_probes = job.tile_probes;
    const int2* __restrict__ corner = job.corner;
    const int n_beams = job.n_beams, ns = job.ns, m = job.m;
    const int t0 = job.tile_start[tile], t1 = job.tile_start[tile + 1];
    const int pc0 = t0 + chunk * PC;
    if (pc0 >= t1) return;
    const int np = min(PC, t1 - pc0);
    const int ntx = ns / TILE;
    const int tid = threadIdx.x;
    const int px = (tile % ntx) * TILE + (tid % TILE);
    const int py = (tile / ntx) * TILE + (tid / TILE);
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
// Workgroup: one 16 x 16 pixel tile x 64 probes.  Wave w owns tile rows
// 4w..4w+3 (four 16-pixel MFMA column blocks) and all four 16-probe row blocks.
namespace mfmac {
constexpr int PC = 64;   // probes per workgroup
constexpr int KB = 16;   // beams per K step
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

template <bool SPLIT>
__global__ __launch_bounds__(WG) void k_contract_mfma(ContractBatch batch) {
    using namespace mfmac;
    constexpr int NP = SPLIT ? 2 : 1;           // hi (, lo)
    // [part][re/im][row][beam]: the 16 beams of a row are contiguous (32 B)
    __shared__ __attribute__((aligned(16))) u32x4 Ss[NP][2][256][2];
    __shared__ __attribute__((aligned(16))) uint2 Cs[NP][2][PC][4];
    __shared__ int pidx[PC];

    int tile, chunk;
    ContractJob job;
    if (!locate(batch, job, tile, chunk)) return;
    const float2* __restrict__ C = job.C;
    const float2* __restrict__ S = job.S;
    float2* __restrict__ win = job.win;
    const int* __restrict__ tile_probes = job.tile_probes;
    const int2* __restrict__ corner = job.corner;
    const int n_beams = job.n_beams, ns = job.ns, m = job.m;
    const int t0 = job.tile_start[tile], t1 = job.tile_start[tile + 1];
    const int pc0 = t0 + chunk * PC;
    if (pc0 >= t1) return;
    const int np = min(PC, t1 - pc0);
    const int ntx = ns / TILE;
    const int tx0 = (tile % ntx) * TILE, ty0 = (tile / ntx) * TILE;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid < PC) pidx[tid] = tid < np ? tile_probes[pc0 + tid] : -1;

    f32x4 accr[4][4], acci[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            accr[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
            acci[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    const size_t plane = (size_t)ns * ns;
    // S staging: thread = one tile pixel, 16 beams per K step
    const int spix = tid;
    const float2* Sp = S + (size_t)(ty0 + spix / TILE) * ns + tx0 + (spix % TILE);
    // C staging: thread = (probe, 4 beams)
    const int cp = tid >> 2, cb = (tid & 3) * 4;
    __syncthreads();
    const int cq = pidx[cp];
    const float2* Cp = C + (size_t)(cq < 0 ? 0 : cq) * n_beams + cb;

    float2 sv[KB], cv[4];
    auto load = [&](int b0) {
#pragma unroll
        for (int k = 0; k < KB; ++k)
            sv[k] = (b0 + k < n_beams) ? Sp[(size_t)(b0 + k) * plane] : make_float2(0.f, 0.f);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            cv[k] = (cq >= 0 && b0 + cb + k < n_beams) ? Cp[b0 + k] : make_float2(0.f, 0.f);
    };
    load(0);

    const int col = lane & 15, g = lane >> 4;   // MFMA operand lane roles
    for (int b0 = 0; b0 < n_beams; b0 += KB) {
        // ---- convert and stage this K step (16 B stores)
        {
            unsigned int rh[KB / 2], ih[KB / 2], rl[KB / 2], il[KB / 2];
#pragma unroll
            for (int k = 0; k < KB / 2; ++k) {
                if constexpr (SPLIT) {
                    split_pair(sv[2 * k].x, sv[2 * k + 1].x, rh[k], rl[k]);
                    split_pair(sv[2 * k].y, sv[2 * k + 1].y, ih[k], il[k]);
                } else {
                    rh[k] = pack_bf16(sv[2 * k].x, sv[2 * k + 1].x);
                    ih[k] = pack_bf16(sv[2 * k].y, sv[2 * k + 1].y);
                }
            }
            Ss[0][0][spix][0] = u32x4{rh[0], rh[1], rh[2], rh[3]};
            Ss[0][0][spix][1] = u32x4{rh[4], rh[5], rh[6], rh[7]};
            Ss[0][1][spix][0] = u32x4{ih[0], ih[1], ih[2], ih[3]};
            Ss[0][1][spix][1] = u32x4{ih[4], ih[5], ih[6], ih[7]};
            if constexpr (SPLIT) {
                Ss[NP - 1][0][spix][0] = u32x4{rl[0], rl[1], rl[2], rl[3]};
                Ss[NP - 1][0][spix][1] = u32x4{rl[4], rl[5], rl[6], rl[7]};
                Ss[NP - 1][1][spix][0] = u32x4{il[0], il[1], il[2], il[3]};
                Ss[NP - 1][1][spix][1] = u32x4{il[4], il[5], il[6], il[7]};
            }
            unsigned int crh[2], cih[2], crl[2], cil[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if constexpr (SPLIT) {
                    split_pair(cv[2 * k].x, cv[2 * k + 1].x, crh[k], crl[k]);
                    split_pair(cv[2 * k].y, cv[2 * k + 1].y, cih[k], cil[k]);
                } else {
                    crh[k] = pack_bf16(cv[2 * k].x, cv[2 * k + 1].x);
                    cih[k] = pack_bf16(cv[2 * k].y, cv[2 * k + 1].y);
                }
            }
            Cs[0][0][cp][cb / 4] = make_uint2(crh[0], crh[1]);
            Cs[0][1][cp][cb / 4] = make_uint2(cih[0], cih[1]);
            if constexpr (SPLIT) {
                Cs[NP - 1][0][cp][cb / 4] = make_uint2(crl[0], crl[1]);
                Cs[NP - 1][1][cp][cb / 4] = make_uint2(cil[0], cil[1]);
            }
        }
        __syncthreads();
        // ---- next K step's global loads fly while this step's MFMAs run
        if (b0 + KB < n_beams) load(b0 + KB);
        // ---- B operands: pixel block pb = tile row 4*wave + pb, lane column = pixel
        //      k-group g: 0,1 -> Sr beams 8g.., 2,3 -> Si beams 8(g-2)..
        u32x4 Bop[NP][4];
#pragma unroll
        for (int part = 0; part < NP; ++part)
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) {
                const int pix = (4 * wave + pb) * TILE + col;
                Bop[part][pb] = Ss[part][g >> 1][pix][g & 1];
            }
#pragma unroll
        for (int qb = 0; qb < 4; ++qb) {
            const int prow = 16 * qb + col;
            // A_r = [Cr | -Ci], A_i = [Ci | Cr]
            u32x4 Ar[NP], Ai[NP];
#pragma unroll
            for (int part = 0; part < NP; ++part) {
                const uint2* cr2 = &Cs[part][0][prow][2 * (g & 1)];
                const uint2* ci2 = &Cs[part][1][prow][2 * (g & 1)];
                u32x4 cr = u32x4{cr2[0].x, cr2[0].y, cr2[1].x, cr2[1].y};
                u32x4 ci = u32x4{ci2[0].x, ci2[0].y, ci2[1].x, ci2[1].y};
                if (g < 2) {
                    Ar[part] = cr;
                    Ai[part] = ci;
                } else {
                    Ar[part] = ci ^ u32x4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
                    Ai[part] = cr;
                }
            }
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) {
                accr[qb][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(Ar[0]), as_bf16x8(Bop[0][pb]),
                                                                      accr[qb][pb], 0, 0, 0);
                acci[qb][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(Ai[0]), as_bf16x8(Bop[0][pb]),
                                                                      acci[qb][pb], 0, 0, 0);
                if constexpr (SPLIT) {
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
    for (int qb = 0; qb < 4; ++qb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = pidx[16 * qb + 4 * g + r];
            if (q < 0) continue;
            const int2 c0 = corner[q];
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) {
                const int py = ty0 + 4 * wave + pb, px = tx0 + col;
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
            job.corner = a.corner;
            job.n_beams = a.n_beams;
            job.ns = a.ns;
            job.m = a.m;
            job.accumulate = a.accumulate;
            job.chunks = (a.max_per_tile + pc - 1) / pc;
            if (job.chunks < 1) job.chunks = 1;
            job.n_tiles = a.n_tiles;
            job.block0 = blocks;
            blocks += job.chunks * job.n_tiles;
        }
        b.n_blocks = blocks;
        b.per_xcd = (blocks + 7) / 8;
        dim3 grid((unsigned)(8 * b.per_xcd));
        if (precision == 0)
            hipLaunchKernelGGL(k_contract_fp32, grid, dim3(WG), 0, st, b);
        else if (precision == 1)
            hipLaunchKernelGGL(k_contract_mfma<true>, grid, dim3(WG), 0, st, b);
        else
            hipLaunchKernelGGL(k_contract_mfma<false>, grid, dim3(WG), 0, st, b);
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

template <int M>
__global__ __launch_bounds__(WG) void k_window_detect(WindowBatch batch) {
    using F = Fft<M>;
    constexpr int E = F::E, LPT = F::LPT, G = 64 / LPT, ROW = F::LDS + 1;
    __shared__ float2 buf[M * ROW];
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
        constexpr int NLD = (M * M + WG - 1) / WG, BATCH = NLD < 16 ? NLD : 16;
        static_assert(NLD % BATCH == 0, "load batches must divide the window");
#pragma unroll 1
        for (int k0 = 0; k0 < NLD; k0 += BATCH) {
            float2 ld[BATCH];
#pragma unroll
            for (int k = 0; k < BATCH; ++k) {
                const int idx = tid + (k0 + k) * WG;
                if (idx < M * M) ld[k] = w[idx];
            }
#pragma unroll
            for (int k = 0; k < BATCH; ++k) {
                const int idx = tid + (k0 + k) * WG;
                if (idx < M * M) buf[(idx / M) * ROW + F::pad(idx % M)] = ld[k];
            }
        }
    }
    __syncthreads();
    typename F::Twiddles tw;
    tw.load(tw_m, lt);
    // rows
    for (int r0 = wave * G; r0 < M; r0 += 4 * G) {
        float2* row = buf + (r0 + g) * ROW;
        float2 v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = row[F::pad(lt + LPT * i)];
        F::template run<-1>(v, row, tw, lt);
        wave_sync();
#pragma unroll
        for (int i = 0; i < E; ++i) row[F::pad(lt + LPT * i)] = v[i];
    }
    __syncthreads();
    // columns, then intensity in place
    const float scale = 1.0f / ((float)M * (float)M * (float)M * (float)M);
    for (int c0 = wave * G; c0 < M; c0 += 4 * G) {
        float2* col = buf + F::pad(c0 + g);
        float2 v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = col[(lt + LPT * i) * ROW];
        F::template run_col<-1>(v, col, ROW, tw, lt);
        wave_sync();
#pragma unroll
        for (int i = 0; i < E; ++i) col[(lt + LPT * i) * ROW] = make_float2(cnorm(v[i]) * scale, 0.f);
    }
    __syncthreads();
    if (diff) {
        float* d = diff + (size_t)p * M * M;
        for (int idx = tid; idx < M * M; idx += WG) d[idx] = buf[(idx / M) * ROW + F::pad(idx % M)].x;
    }
    if (!out) return;
    for (int b = wave; b < n_bins; b += 4) {
        float s = 0.f;
        for (int k = bin_start[b] + lane; k < bin_start[b + 1]; k += 64) {
            int pix = perm[k];
            s += buf[(pix / M) * ROW + F::pad(pix % M)].x;
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
        hipLaunchKernelGGL((k_window_detect<M>), dim3((unsigned)blocks), dim3(WG), 0, st, b);
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
        F::template run_col<-1>(v, col, ROWS, tw, lt);
#pragma unroll
        for (int i = 0; i < E; ++i) I[(size_t)(lt + LPT * i) * M + u0 + c] = cnorm(v[i]) * scale;
    }
}

template <int M>
static hipError_t window_large(float2* win, float* inten, float* out, const int* perm, const int* bin_start,
                               const float2* tw_m, int n_probes, int n_bins, float scale, int accumulate,
                               hipStream_t st) {
    // inten receives |Psi|^2 / M^4 (it is the 4D output when one is requested)
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
                float* I = a.diff ? a.diff : a.inten;
                hipError_t e = m == 256 ? window_large<256>(a.win, I, a.out, a.perm, a.bin_start, a.tw_m,
                                                            a.n_probes, a.n_bins, a.scale, a.accumulate, st)
                                        : window_large<512>(a.win, I, a.out, a.perm, a.bin_start, a.tw_m,
                                                            a.n_probes, a.n_bins, a.scale, a.accumulate, st);
                if (e != hipSuccess) return e;
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
