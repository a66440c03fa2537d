// api.hip -- C ABI of the PRISM / multislice library: validation, host
// planning (FP64, integer), table uploads and kernel dispatch.
//
// Floating-point decisions that pick integers (beam membership, aperture,
// detector bins, window centres) are explicit sequences of correctly rounded
// IEEE-754 float64 operations, evaluated without contraction, so that any
// conforming implementation of the same expressions reproduces them exactly.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "kernels.hpp"
#include "prism.h"

using namespace prism;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(PRISM_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------- kernel timing --
// Optional per-kernel-class timing: when enabled on the calling thread, each
// launch is bracketed by HIP events on its stream.  Totals are read after the
// caller has synchronised the stream.
struct TimedLaunch {
    int cls;
    hipEvent_t a, b;
};
thread_local bool t_timing = false;
thread_local std::vector<TimedLaunch> t_pending;
thread_local double t_total_ms[PRISM_TIMING_CLASSES];
thread_local int64_t t_count[PRISM_TIMING_CLASSES];

template <class Fn>
hipError_t timed(int cls, hipStream_t st, Fn&& fn) {
    if (!t_timing) return fn();
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, st);
    if (e != hipSuccess) return e;
    e = fn();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, st);
    if (e == hipSuccess) t_pending.push_back(TimedLaunch{cls, a, b});
    return e;
}

// ---------------------------------------------------------------- physics --
// Relativistic wavelength and interaction constant of Eqs. (1)-(2), CODATA 2018.
constexpr double kPlanck = 6.62607015e-34, kLight = 299792458.0, kCharge = 1.602176634e-19,
                 kMass0 = 9.1093837015e-31;
constexpr double kPi = 3.14159265358979323846;

double wavelength_A(double E0) {
    double eE = kCharge * E0;
    return kPlanck * kLight / std::sqrt(eE * (2.0 * kMass0 * kLight * kLight + eE)) * 1e10;
}
double sigma_per_VA(double E0) {
    double lam_m = wavelength_A(E0) * 1e-10;
    double m = kMass0 + kCharge * E0 / (kLight * kLight);
    return 2.0 * kPi * m * kCharge * lam_m / (kPlanck * kPlanck) * 1e-10;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// FFT-order integer frequency of index i on an m-point grid.
inline int freq(int i, int m) { return i < (m + 1) / 2 ? i : i - m; }
// band column j (of n/2) -> kx in [-n/4, n/4)
inline int band_k(int j, int n) { return j < n / 4 ? j : j - n / 2; }

// lambda * sqrt(kx^2 + ky^2) / Lw  (the one expression every angle test uses)
inline double angle_of(double lam, int kx, int ky, double Lw) {
    return lam * std::sqrt((double)(kx * kx + ky * ky)) / Lw;
}
inline double alpha_aa_of(double lam, int n, double L) { return lam * (double)n / (4.0 * L); }
inline int bin_of(double lam, int kx, int ky, double Lw, double a_aa, double dalpha, int n_bins) {
    double a = angle_of(lam, kx, ky, Lw);
    if (!(a < a_aa)) return -1;
    double b = std::floor(a / dalpha);
    if (b >= (double)n_bins) return -1;
    return (int)b;
}

// Beams: every f-th Fourier index inside alpha_max, ordered by (ky, kx).
// Indices beyond kmax = alpha_max L / lam (+1 for rounding) per axis are
// outside the aperture, so the scan is limited to that square.
std::vector<int2> beam_list(int n, double L, double lam, double alpha_max, int f) {
    std::vector<int2> out;
    const int kmax = (int)std::min<double>(n / 2, std::ceil(alpha_max * L / lam) + 1.0);
    for (int ky = std::max(-n / 2, -kmax); ky < std::min(n / 2, kmax + 1); ++ky)
        for (int kx = std::max(-n / 2, -kmax); kx < std::min(n / 2, kmax + 1); ++kx) {
            if (kx % f != 0 || ky % f != 0) continue;
            if (angle_of(lam, kx, ky, L) <= alpha_max) out.push_back(make_int2(kx, ky));
        }
    return out;
}

// Window centre: nearest S-grid pixel (round half up), periodic.
inline int centre_of(double x, double L, int n) {
    double c = std::floor(x / (2.0 * (L / n)) + 0.5);
    int ns = n / 2;
    long long ci = (long long)c % ns;
    if (ci < 0) ci += ns;
    return (int)ci;
}

int default_bins(double a_aa, double dalpha) { return (int)std::ceil(a_aa / dalpha); }
constexpr int MAX_BINS = 4096;   // detector bins of one output (multislice workspace bound)

// exp(-i chi(q)), chi = pi lam C1 q^2 + (pi/2) C3 lam^3 q^4, q = k/L: the phase
// is formed and reduced mod 2 pi in FP64, the factor stored in FP32.
float2 aberration_factor(int kx, int ky, double L, double lam, double C1, double C3) {
    const double q2 = ((double)kx / L) * ((double)kx / L) + ((double)ky / L) * ((double)ky / L);
    // chi / pi, reduced to (-1, 1]
    double t = lam * C1 * q2 + 0.5 * C3 * lam * lam * lam * q2 * q2;
    t -= 2.0 * std::nearbyint(t / 2.0);
    const double ph = -kPi * t;
    return make_float2((float)std::cos(ph), (float)std::sin(ph));
}

// ----------------------------------------------------- workspace carving --
struct Carve {
    char* base;
    size_t off = 0;
    explicit Carve(void* b) : base(static_cast<char*>(b)) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base + off);
        off += count * sizeof(T);
        return p;
    }
};

std::vector<float2> twiddle_table(int m) {
    std::vector<float2> t(m);
    for (int i = 0; i < m; ++i) {
        double a = 2.0 * kPi * (double)i / (double)m;
        t[i] = make_float2((float)std::cos(a), (float)-std::sin(a));
    }
    return t;
}

// Host-side tables of the propagation passes, laid out as one blob.
struct PropHost {
    std::vector<float2> tw_half, tw_full, band, prop;
};

PropHost prop_tables(int n, double L, double lam, double dz) {
    PropHost h;
    const int Lh = n / 2;
    h.tw_half = twiddle_table(Lh);
    h.tw_full = twiddle_table(n);
    h.band.resize(Lh);
    h.prop.resize(Lh);
    for (int j = 0; j < Lh; ++j) {
        int k = band_k(j, n);
        double a = 2.0 * kPi * (double)k / (double)n;
        h.band[j] = make_float2((float)std::cos(a), (float)-std::sin(a));
        // phase -pi * lam dz k^2 / L^2, reduced to (-pi, pi]
        double t = lam * dz * (double)k * (double)k / (L * L);
        t -= 2.0 * std::nearbyint(t / 2.0);
        double ph = -kPi * t;
        h.prop[j] = make_float2((float)(std::cos(ph) / n), (float)(std::sin(ph) / n));
    }
    return h;
}

struct PropDev {
    float2 *tw_half, *tw_full, *band, *prop;
    PropTables tables() const { return PropTables{tw_half, tw_full, band, prop}; }
};

PropDev carve_prop(Carve& c, int n) {
    PropDev d;
    d.tw_half = c.take<float2>(n / 2);
    d.tw_full = c.take<float2>(n);
    d.band = c.take<float2>(n / 2);
    d.prop = c.take<float2>(n / 2);
    return d;
}

// Copy a host vector into a blob at the device pointer's offset.
template <class T>
void stage(std::vector<char>& blob, const void* dev_base, const T* dev_ptr, const std::vector<T>& v) {
    size_t off = reinterpret_cast<const char*>(dev_ptr) - static_cast<const char*>(dev_base);
    if (blob.size() < off + v.size() * sizeof(T)) blob.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
}

int upload(void* dev, const std::vector<char>& blob, hipStream_t st) {
    if (blob.empty()) return PRISM_OK;
    HIP_TRY(hipMemcpyAsync(dev, blob.data(), blob.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return PRISM_OK;
}

int check_grid(const prism_grid* g) {
    if (!g) return fail(PRISM_E_INVAL, "grid is NULL");
    if (g->n <= 0 || !(g->dz > 0) || !(g->cell[0] > 0) || !(g->cell[1] > 0) || !(g->cell[2] > 0))
        return fail(PRISM_E_INVAL, "grid: n, dz and cell must be positive");
    if (g->cell[0] != g->cell[1]) return fail(PRISM_E_UNSUPPORTED, "grid: only square cells (Lx == Ly)");
    if (!is_pow2(g->n) || g->n < 64 || g->n > 2048)
        return fail(PRISM_E_UNSUPPORTED, "grid: n = %d must be a power of two in [64, 2048]", g->n);
    int s = (int)std::ceil(g->cell[2] / g->dz - 1e-12);
    if (g->n_slices != s) return fail(PRISM_E_INVAL, "grid: n_slices %d != ceil(Lz/dz) = %d", g->n_slices, s);
    return PRISM_OK;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

struct ProbeHost {
    std::vector<double2> xy;
    std::vector<int2> corner;
    std::vector<int> tile_start, tile_probes, perm, bin_start;
    std::vector<int2> tile_origin;  // first pixel of each work tile
    std::vector<float2> tw_m;
    std::vector<int2> beams;
    std::vector<float2> aberr;      // per beam, empty when there are no aberrations
};

// Detector tables: pixel indices grouped by bin (bins[i] in [-1, n_bins),
// -1 = no bin), ascending pixel index inside a bin; start[b] .. start[b+1]
// delimit bin b in perm.
void group_by_bin(const std::vector<int>& bins, int n_bins, std::vector<int>& perm, std::vector<int>& start) {
    std::vector<int> cnt(n_bins + 1, 0);
    for (int b : bins)
        if (b >= 0) cnt[b + 1]++;
    start.assign(n_bins + 1, 0);
    for (int b = 0; b < n_bins; ++b) start[b + 1] = start[b] + cnt[b + 1];
    perm.assign(start[n_bins], 0);
    std::vector<int> fill(start.begin(), start.end() - 1);
    for (size_t i = 0; i < bins.size(); ++i)
        if (bins[i] >= 0) perm[fill[bins[i]]++] = (int)i;
}

// Annular bins of an m x m FFT-order grid (pixel index ky_i * m + kx_i), or
// the caller's detector map of that grid when `dmap` is given.
void bin_tables(double lam, double Lw, double a_aa, double dalpha, int n_bins, int m, const int32_t* dmap,
                std::vector<int>& perm, std::vector<int>& start) {
    std::vector<int> bins((size_t)m * m);
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c)
            bins[(size_t)r * m + c] =
                dmap ? dmap[(size_t)r * m + c] : bin_of(lam, freq(c, m), freq(r, m), Lw, a_aa, dalpha, n_bins);
    group_by_bin(bins, n_bins, perm, start);
}

// A caller's detector map: every entry -1 (no detector) or a bin in [0, n_bins).
int check_detector_map(const int32_t* dmap, size_t count, int n_bins, const char* what) {
    if (!dmap) return fail(PRISM_E_INVAL, "%s: NULL detector map", what);
    if (n_bins < 1 || n_bins > MAX_BINS) return fail(PRISM_E_INVAL, "%s: n_bins %d outside [1, %d]", what, n_bins, MAX_BINS);
    for (size_t i = 0; i < count; ++i)
        if (dmap[i] < -1 || dmap[i] >= n_bins)
            return fail(PRISM_E_INVAL, "%s: detector map entry %zu = %d outside [-1, %d)", what, i, (int)dmap[i], n_bins);
    return PRISM_OK;
}

// Work tiles of the windowed contraction.  Each probe gets a tiling phase,
// its window corner's offset modulo 16 rounded down to a multiple of the
// quantum Q (Q = 16: one phase for all probes; Q = 1: the exact offset, so
// that the window covers whole tiles), and is listed under every 16 x 16
// tile of its phase that its window overlaps.  A work tile is a (phase,
// tile) pair with at least one probe.
struct TileCover {
    int nt, nq, Q, M, ns;
    // tiles of the phase grid covered along one axis by a window starting at c
    void span(int c, int& phase, int& first, int& count) const {
        phase = (c & 15) / Q;
        const int rel = (c - phase * Q) & (ns - 1);
        first = rel / 16;
        count = std::min((rel + M - 1) / 16 - first + 1, nt);   // a window as wide as the grid covers each tile once
    }
    int key(int ph, int tx, int ty) const { return (ph * nt + ty) * nt + tx; }
};

// One probe's tiles under a TileCover: phase index and, per axis, the first
// tile and the tile count.
struct Span {
    int ph, fx, nx, fy, ny;
};

// Spans of every probe and the probe count of every (phase, tile) key.
static void cover_counts(const TileCover& tc, const std::vector<int2>& corner, std::vector<Span>& spans,
                         std::vector<int>& count) {
    spans.resize(corner.size());
    count.assign((size_t)tc.nq * tc.nq * tc.nt * tc.nt, 0);
    const int wrap = tc.nt - 1;
    for (size_t p = 0; p < corner.size(); ++p) {
        Span& sp = spans[p];
        int phx, phy;
        tc.span(corner[p].x, phx, sp.fx, sp.nx);
        tc.span(corner[p].y, phy, sp.fy, sp.ny);
        sp.ph = phy * tc.nq + phx;
        for (int a = 0; a < sp.ny; ++a) {
            int* row = count.data() + (size_t)tc.key(sp.ph, 0, (sp.fy + a) & wrap);
            for (int b = 0; b < sp.nx; ++b) row[(sp.fx + b) & wrap]++;
        }
    }
}

// Interleaved bits of (ty, tx): work tiles near each other in the S grid get
// nearby places in the launch order.
static uint32_t morton(uint32_t ty, uint32_t tx) {
    uint32_t r = 0;
    for (int b = 0; b < 16; ++b) r |= ((tx >> b) & 1u) << (2 * b) | ((ty >> b) & 1u) << (2 * b + 1);
    return r;
}

int probe_host(const prism_smatrix_desc* d, const double* xy, int64_t n_probes, double dalpha, int n_bins,
               double C1, double C3, const int32_t* dmap, ProbeHost& h, int& max_per_tile) {
    const int n = d->grid.n, ns = d->ns, M = d->m_win;
    const double L = d->grid.cell[0];
    h.xy.resize(n_probes);
    h.corner.resize(n_probes);
    for (int64_t p = 0; p < n_probes; ++p) {
        double x = xy[2 * p], y = xy[2 * p + 1];
        if (!std::isfinite(x) || !std::isfinite(y)) return fail(PRISM_E_INVAL, "probe %lld: non-finite position", (long long)p);
        h.xy[p] = make_double2(x, y);
        int cx = centre_of(x, L, n), cy = centre_of(y, L, n);
        h.corner[p] = make_int2((cx - M / 2) & (ns - 1), (cy - M / 2) & (ns - 1));
    }
    // The quantum whose work tiles need the fewest workgroups of the MFMA
    // contraction's probe chunk.  Exact phases (Q = 1) give every window the
    // fewest tiles; when their probe chunks are also all full no tiling needs
    // fewer workgroups, and the aligned grid (Q = 16) is not evaluated.
    const int pc = contract_probe_chunk();
    auto cost_of = [&](const std::vector<int>& count, long long& entries) {
        long long cost = 0;
        entries = 0;
        for (int c : count) {
            cost += (c + pc - 1) / pc;
            entries += c;
        }
        return cost;
    };
    TileCover tc{ns / 16, 16, 1, M, ns};
    std::vector<Span> spans;
    std::vector<int> count;
    cover_counts(tc, h.corner, spans, count);
    long long entries = 0;
    const long long cost1 = cost_of(count, entries);
    if (cost1 > (entries + pc - 1) / pc) {
        TileCover t16{ns / 16, 1, 16, M, ns};
        std::vector<Span> spans16;
        std::vector<int> count16;
        cover_counts(t16, h.corner, spans16, count16);
        long long e16 = 0;
        if (cost_of(count16, e16) <= cost1) {
            tc = t16;
            spans.swap(spans16);
            count.swap(count16);
        }
    }
    std::vector<std::pair<uint64_t, int>> order;   // (position, phase) sort key, key
    const int nt2 = tc.nt * tc.nt;
    for (int k = 0; k < (int)count.size(); ++k) {
        if (!count[k]) continue;
        const int tx = k % tc.nt, ty = (k / tc.nt) % tc.nt, ph = k / nt2;
        order.emplace_back(((uint64_t)morton(ty, tx) << 16) | (uint64_t)ph, k);
    }
    std::sort(order.begin(), order.end());
    std::vector<int> slot(count.size(), -1);
    const int n_tiles = (int)order.size();
    h.tile_start.assign(n_tiles + 1, 0);
    h.tile_origin.resize(n_tiles);
    max_per_tile = 0;
    for (int t = 0; t < n_tiles; ++t) {
        const int k = order[t].second;
        const int tx = k % tc.nt, ty = (k / tc.nt) % tc.nt, ph = k / nt2;
        const int phx = ph % tc.nq, phy = ph / tc.nq;
        slot[k] = t;
        h.tile_start[t + 1] = h.tile_start[t] + count[k];
        h.tile_origin[t] = make_int2((phx * tc.Q + 16 * tx) & (ns - 1), (phy * tc.Q + 16 * ty) & (ns - 1));
        max_per_tile = std::max(max_per_tile, count[k]);
    }
    // probe lists, filled phase by phase (probes of one phase in their order)
    // so that consecutive probes land on neighbouring work tiles
    const int nph = tc.nq * tc.nq, wrap = tc.nt - 1;
    std::vector<int> by_phase(n_probes), ph_start(nph + 1, 0);
    for (const Span& sp : spans) ph_start[sp.ph + 1]++;
    for (int q = 0; q < nph; ++q) ph_start[q + 1] += ph_start[q];
    {
        std::vector<int> pos(ph_start.begin(), ph_start.end() - 1);
        for (int64_t p = 0; p < n_probes; ++p) by_phase[pos[spans[p].ph]++] = (int)p;
    }
    h.tile_probes.assign(h.tile_start[n_tiles], 0);
    // the phases' work tiles are disjoint, so phases fill in parallel, each
    // with its own write positions (a phase's keys are one contiguous block)
    auto fill_phases = [&](int q0, int q1) {
        std::vector<int> fill(nt2);
        for (int q = q0; q < q1; ++q) {
            const int* sq = slot.data() + (size_t)q * nt2;
            for (int k = 0; k < nt2; ++k) fill[k] = sq[k] >= 0 ? h.tile_start[sq[k]] : 0;
            for (int i = ph_start[q]; i < ph_start[q + 1]; ++i) {
                const int p = by_phase[i];
                const Span& sp = spans[p];
                for (int a = 0; a < sp.ny; ++a) {
                    int* frow = fill.data() + (size_t)((sp.fy + a) & wrap) * tc.nt;
                    for (int b = 0; b < sp.nx; ++b) h.tile_probes[frow[(sp.fx + b) & wrap]++] = p;
                }
            }
        }
    };
    const int nthr = std::min<int>(nph, std::max(1u, std::min(8u, std::thread::hardware_concurrency())));
    if (nthr > 1 && n_probes >= 4096) {
        std::vector<std::thread> pool;
        for (int t = 0; t < nthr; ++t) pool.emplace_back(fill_phases, nph * t / nthr, nph * (t + 1) / nthr);
        for (std::thread& th : pool) th.join();
    } else {
        fill_phases(0, nph);
    }
    bin_tables(d->lambda, L / d->f, d->alpha_aa, dalpha, n_bins, M, dmap, h.perm, h.bin_start);
    h.tw_m = twiddle_table(M);
    h.beams = beam_list(n, L, d->lambda, d->alpha_max, d->f);
    h.aberr.clear();
    if (C1 != 0.0 || C3 != 0.0) {
        h.aberr.resize(h.beams.size());
        for (size_t b = 0; b < h.beams.size(); ++b)
            h.aberr[b] = aberration_factor(h.beams[b].x, h.beams[b].y, L, d->lambda, C1, C3);
    }
    return PRISM_OK;
}

int batch_of(const prism_smatrix_desc* d) {
    return (d->beam_batch > 0 && d->beam_batch < d->n_beams) ? d->beam_batch : d->n_beams;
}

// Workspace of one probe-synthesis job: coefficients (complex64, or the
// split layout of the MFMA contraction, whichever is larger), windows and
// (for windows above 128 pixels) intensities.
struct SynthJobDev {
    void* C;
    float2* win;
    float* inten;
};
SynthJobDev synth_job_carve(const prism_smatrix_desc* d, const prism_probe_plan* plan, Carve& c) {
    const size_t P = (size_t)std::max<int64_t>(plan->n_probes, 1);
    SynthJobDev j;
    j.C = c.take<char>(split_c_bytes((int64_t)P, d->n_beams));
    j.win = c.take<float2>(P * d->m_win * d->m_win);
    j.inten = d->m_win > 128 ? c.take<float>(P * d->m_win * d->m_win) : nullptr;
    return j;
}
// The MFMA contraction reads S as split records, converted once per distinct
// S-matrix of a call (nothing is reserved when it splits S itself).
void* split_s_carve(const prism_smatrix_desc* d, Carve& c) {
    return contract_reads_split_s() ? c.take<char>(split_s_bytes(d->ns, d->n_beams)) : nullptr;
}

// Consistency of a descriptor filled by prism_smatrix_plan (without recounting
// the beams, which costs O(n^2) host work per call).
int check_desc(const prism_smatrix_desc* d) {
    if (!d) return fail(PRISM_E_INVAL, "descriptor is NULL");
    int rc = check_grid(&d->grid);
    if (rc) return rc;
    const int n = d->grid.n;
    if (d->f < 1 || d->ns != n / 2 || d->ns % d->f != 0 || d->m_win != d->ns / d->f || d->n_beams < 1 ||
        d->lambda != wavelength_A(d->E0) || d->sigma != sigma_per_VA(d->E0) ||
        d->alpha_aa != alpha_aa_of(d->lambda, n, d->grid.cell[0]) ||
        d->smatrix_bytes != (size_t)d->n_beams * d->ns * d->ns * sizeof(float2) || d->beam_batch < 0)
        return fail(PRISM_E_INVAL, "descriptor was not filled by prism_smatrix_plan");
    return PRISM_OK;
}

}  // namespace

// ------------------------------------------ fixed scratch (no allocation) --
// Workspace of prism_probe_outputs_noalloc: one array per GPU, part of the
// code object, held until the process ends.  Host code takes its device
// address from hipGetSymbolAddress (once per device, with that device
// current) and never uses the array's name, which on the host is only a
// stand-in for the symbol.
static __device__ __align__(256) char scratch[PRISM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array.
int scratch_address(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PRISM_E_DEVICE, "device index %d outside 0..%d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(PRISM_E_DEVICE, "scratch array has no device address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PRISM_OK;
}
}  // namespace

// =================================================================== ABI ==
extern "C" {

const char* prism_last_error(void) { return g_err.c_str(); }

int prism_grid_init(const double cell[3], double dz, int32_t n, prism_grid* out) {
    if (!cell || !out) return fail(PRISM_E_INVAL, "NULL argument");
    prism_grid g{};
    g.n = n;
    g.cell[0] = cell[0];
    g.cell[1] = cell[1];
    g.cell[2] = cell[2];
    g.dz = dz;
    g.n_slices = (dz > 0 && cell[2] > 0) ? (int)std::ceil(cell[2] / dz - 1e-12) : 0;
    int rc = check_grid(&g);
    if (rc) return rc;
    *out = g;
    return PRISM_OK;
}

int prism_detector_bin_map(double lambda, double Lw, double alpha_aa, double dalpha, int32_t n_bins, int32_t m,
                           int32_t* map) {
    if (!map || m <= 0 || !(lambda > 0) || !(Lw > 0) || !(dalpha > 0) || n_bins <= 0)
        return fail(PRISM_E_INVAL, "bin map: invalid argument");
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) map[(size_t)r * m + c] = bin_of(lambda, freq(c, m), freq(r, m), Lw, alpha_aa, dalpha, n_bins);
    return PRISM_OK;
}

int prism_detector_default_bins(const prism_grid* grid, double E0, double dalpha, int32_t* n_bins,
                                double* alpha_aa) {
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!n_bins || !(E0 > 0) || !(dalpha > 0)) return fail(PRISM_E_INVAL, "default bins: invalid argument");
    const double a = alpha_aa_of(wavelength_A(E0), grid->n, grid->cell[0]);
    *n_bins = default_bins(a, dalpha);
    if (alpha_aa) *alpha_aa = a;
    return PRISM_OK;
}

// ------------------------------------------------------------ potential --
int prism_project_potential_workspace(int64_t n_atoms, size_t* bytes) {
    if (!bytes || n_atoms < 0) return fail(PRISM_E_INVAL, "invalid argument");
    Carve c(nullptr);
    c.take<PotAtom>((size_t)std::max<int64_t>(n_atoms, 1));
    c.take<int>(8193);
    c.take<PotSpecies>(256);
    *bytes = c.off + 256;
    return PRISM_OK;
}

int prism_project_potential(const prism_atom* atoms, int64_t n_atoms, const prism_species* species, int32_t n_species,
                            const prism_grid* grid, float* V, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!V || (n_atoms > 0 && !atoms) || !species || n_species <= 0 || n_species > 256 || n_atoms < 0)
        return fail(PRISM_E_INVAL, "potential: invalid argument");
    if (grid->n_slices > 8192) return fail(PRISM_E_UNSUPPORTED, "potential: more than 8192 slices");
    size_t need = 0;
    prism_project_potential_workspace(n_atoms, &need);
    if (!ws || ws_bytes < need) return fail(PRISM_E_WORKSPACE, "potential: workspace %zu < %zu bytes", ws_bytes, need);
    const double L = grid->cell[0];
    const int S = grid->n_slices;
    std::vector<PotSpecies> sp(n_species);
    float rc_max = 0.f;
    for (int i = 0; i < n_species; ++i) {
        const prism_species& s = species[i];
        if (s.n_gauss < 1 || s.n_gauss > 4) return fail(PRISM_E_INVAL, "species %d: n_gauss must be 1..4", i);
        double wmax = 0;
        PotSpecies p{};
        for (int g = 0; g < s.n_gauss; ++g) {
            if (!(s.width[g] > 0)) return fail(PRISM_E_INVAL, "species %d: width must be positive", i);
            wmax = std::max(wmax, s.width[g]);
            p.amp_n[g] = (float)(s.amp[g] / (2.0 * kPi * s.width[g] * s.width[g]));
            p.inv2w2[g] = (float)(1.0 / (2.0 * s.width[g] * s.width[g]));
        }
        double rcut = 6.0 * wmax;
        if (!(2.0 * rcut < L)) return fail(PRISM_E_INVAL, "species %d: cutoff 6*max(width) must be below L/2", i);
        p.n_gauss = s.n_gauss;
        p.rc = (float)rcut;
        p.rc2 = (float)(rcut * rcut);
        rc_max = std::max(rc_max, p.rc);
        sp[i] = p;
    }
    // atoms sorted (stably) by slice
    std::vector<int> slice_of(n_atoms);
    std::vector<int> start(S + 1, 0);
    for (int64_t a = 0; a < n_atoms; ++a) {
        const prism_atom& at = atoms[a];
        if (at.species < 0 || at.species >= n_species) return fail(PRISM_E_INVAL, "atom %lld: bad species", (long long)a);
        if (!std::isfinite(at.x) || !std::isfinite(at.y) || !std::isfinite(at.z))
            return fail(PRISM_E_INVAL, "atom %lld: non-finite position", (long long)a);
        double s = std::floor(at.z / grid->dz);
        int si = s < 0 ? 0 : (s > S - 1 ? S - 1 : (int)s);
        slice_of[a] = si;
        start[si + 1]++;
    }
    for (int s = 0; s < S; ++s) start[s + 1] += start[s];
    std::vector<PotAtom> sorted(std::max<int64_t>(n_atoms, 1));
    std::vector<int> fill(start.begin(), start.end() - 1);
    for (int64_t a = 0; a < n_atoms; ++a) {
        double x = std::fmod(atoms[a].x, L), y = std::fmod(atoms[a].y, L);
        if (x < 0) x += L;
        if (y < 0) y += L;
        sorted[fill[slice_of[a]]++] = PotAtom{x, y, slice_of[a], atoms[a].species};
    }
    Carve c(ws);
    PotAtom* d_atoms = c.take<PotAtom>(sorted.size());
    int* d_start = c.take<int>(8193);
    PotSpecies* d_sp = c.take<PotSpecies>(256);
    std::vector<char> blob;
    stage(blob, ws, d_atoms, sorted);
    stage(blob, ws, d_start, start);
    stage(blob, ws, d_sp, sp);
    hipStream_t st = as_stream(stream);
    rc = upload(ws, blob, st);
    if (rc) return rc;
    HIP_TRY(timed(PRISM_K_POTENTIAL, st, [&] { return launch_potential(V, grid->n, S, L, d_atoms, d_start, d_sp, rc_max, st); }));
    return PRISM_OK;
}

// ------------------------------------------------------------- S-matrix --
int prism_smatrix_plan(prism_smatrix_desc* d) {
    if (!d) return fail(PRISM_E_INVAL, "descriptor is NULL");
    int rc = check_grid(&d->grid);
    if (rc) return rc;
    if (!(d->E0 > 0) || !(d->alpha_max > 0) || d->f < 1 || d->beam_batch < 0)
        return fail(PRISM_E_INVAL, "smatrix: E0, alpha_max must be positive, f >= 1, beam_batch >= 0");
    const int n = d->grid.n;
    const double L = d->grid.cell[0];
    d->lambda = wavelength_A(d->E0);
    d->sigma = sigma_per_VA(d->E0);
    d->alpha_aa = alpha_aa_of(d->lambda, n, L);
    if (!(d->alpha_max < d->alpha_aa))
        return fail(PRISM_E_UNSUPPORTED, "smatrix: alpha_max %.6g must be below alpha_AA %.6g", d->alpha_max,
                    d->alpha_aa);
    d->ns = n / 2;
    if (d->ns % d->f != 0) return fail(PRISM_E_UNSUPPORTED, "smatrix: f = %d must divide n/2 = %d", d->f, d->ns);
    d->m_win = d->ns / d->f;
    if (d->m_win < 16 || d->m_win > 512)
        return fail(PRISM_E_UNSUPPORTED, "smatrix: window side n/(2f) = %d outside [16, 512]", d->m_win);
    d->n_beams = (int32_t)beam_list(n, L, d->lambda, d->alpha_max, d->f).size();
    d->smatrix_bytes = (size_t)d->n_beams * d->ns * d->ns * sizeof(float2);
    Carve c(nullptr);
    carve_prop(c, n);
    c.take<int2>(d->n_beams);
    c.take<float2>((size_t)d->grid.n_slices * n * n);
    c.take<float2>((size_t)n * n);                           // row spectrum of the first slice
    c.take<float2>((size_t)batch_of(d) * (n / 2) * wave_col_stride(n));
    d->build_ws_bytes = c.off + 256;
    return PRISM_OK;
}

int prism_beam_list(const prism_smatrix_desc* d, int32_t* k_out, int32_t cap) {
    int rc = check_desc(d);
    if (rc) return rc;
    if (!k_out || cap < d->n_beams) return fail(PRISM_E_INVAL, "beam list: capacity %d < %d", cap, d->n_beams);
    auto b = beam_list(d->grid.n, d->grid.cell[0], d->lambda, d->alpha_max, d->f);
    for (size_t i = 0; i < b.size(); ++i) {
        k_out[2 * i] = b[i].x;
        k_out[2 * i + 1] = b[i].y;
    }
    return PRISM_OK;
}

// ------------------------------------------------ overlapped build streams --
// The S-matrix build splits each beam batch into parts, one per stream: the
// caller's stream and up to three partner streams (created once per caller
// stream, default priority, kept for the life of the process).  Stream k
// starts after the first slice of stream k-1 (its plane-wave gather and
// first column pass), so that row passes (bound by VALU issue) of one part
// share the GPU with column passes (bound by memory latency) of another,
// each kernel at its own occupancy.
constexpr int kMaxBuildStreams = 4;
// Part k starts after part k-1's first row pass (0), first column pass (1)
// or second row pass (2): 1245 beams at 1024^2 on two streams took 261.1,
// 256.5 and 261.5 ms per build.
#ifndef PRISM_FORK_STAGE
#define PRISM_FORK_STAGE 1
#endif
// 0: by grid size.  Four streams up to n = 1024 (1245 beams at 1024^2 on 1,
// 2, 3 and 4 streams: 262.4, 253.9, 251.0 and 249.5 ms per build), one above
// (1245 beams at 2048^2: 1.419, 1.410, 1.418 and 1.426 s, no gain beyond the
// spread between runs).
std::atomic<int> g_build_streams{0};
int build_streams_for(int n) {
    const int s = g_build_streams.load();
    return s > 0 ? s : (n <= 1024 ? 4 : 1);
}
std::mutex g_partner_mu;
std::map<hipStream_t, std::vector<hipStream_t>> g_partner;

// The first `count` partner streams of st, created on first use.  At most
// kMaxPartnered caller streams get partners (the library never destroys a
// stream that may still hold work); *out_count is 0 for any further caller
// stream, whose builds then run on that stream alone.
constexpr size_t kMaxPartnered = 32;
int partner_streams(hipStream_t st, int count, hipStream_t* out, int* out_count) {
    std::lock_guard<std::mutex> lk(g_partner_mu);
    *out_count = 0;
    if (g_partner.find(st) == g_partner.end() && g_partner.size() >= kMaxPartnered) return PRISM_OK;
    std::vector<hipStream_t>& v = g_partner[st];
    while ((int)v.size() < count) {
        hipStream_t p = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&p, hipStreamNonBlocking));
        v.push_back(p);
    }
    for (int i = 0; i < count; ++i) out[i] = v[i];
    *out_count = count;
    return PRISM_OK;
}

// Events that order the build's streams, destroyed with the call.
struct BuildEvents {
    hipEvent_t ev[2 * kMaxBuildStreams] = {};
    ~BuildEvents() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

int prism_set_build_streams(int32_t n) {
    if (n < 0 || n > kMaxBuildStreams)
        return fail(PRISM_E_INVAL, "build streams must be 1 to %d (0: by grid size)", kMaxBuildStreams);
    g_build_streams.store(n);
    return PRISM_OK;
}

// S-matrix layers [first, first + count): all slices of each beam batch,
// then the real-space store.
static int build_range(const prism_smatrix_desc* d, const float* V, void* S, int first, int count, void* ws,
                       size_t ws_bytes, void* stream) {
    int rc = check_desc(d);
    if (rc) return rc;
    if (!V || !S) return fail(PRISM_E_INVAL, "build: NULL V or S");
    if (first < 0 || count < 0 || first > d->n_beams - count)
        return fail(PRISM_E_INVAL, "build: beam range [%d, %d + %d) outside [0, %d)", first, first, count, d->n_beams);
    if (!ws || ws_bytes < d->build_ws_bytes)
        return fail(PRISM_E_WORKSPACE, "build: workspace %zu < %zu bytes", ws_bytes, d->build_ws_bytes);
    if (count == 0) return PRISM_OK;
    const int n = d->grid.n, B = d->n_beams, nsl = d->grid.n_slices, NB = std::min(batch_of(d), count);
    const int end = first + count;
    const double L = d->grid.cell[0];
    hipStream_t st = as_stream(stream);
    Carve c(ws);
    PropDev pd = carve_prop(c, n);
    int2* d_beams = c.take<int2>(B);
    float2* T = c.take<float2>((size_t)nsl * n * n);
    float2* R0 = c.take<float2>((size_t)n * n);
    float2* W = c.take<float2>((size_t)NB * (n / 2) * wave_col_stride(n));
    PropHost ph = prop_tables(n, L, d->lambda, d->grid.dz);
    std::vector<char> blob;
    stage(blob, ws, pd.tw_half, ph.tw_half);
    stage(blob, ws, pd.tw_full, ph.tw_full);
    stage(blob, ws, pd.band, ph.band);
    stage(blob, ws, pd.prop, ph.prop);
    stage(blob, ws, d_beams, beam_list(n, L, d->lambda, d->alpha_max, d->f));
    rc = upload(ws, blob, st);
    if (rc) return rc;
    const PropTables tb = pd.tables();
    HIP_TRY(timed(PRISM_K_TRANSMISSION, st, [&] { return launch_transmission(V, T, (int64_t)nsl * n * n, (float)d->sigma, st); }));
    HIP_TRY(timed(PRISM_K_TRANSMISSION, st, [&] { return launch_row_spectrum(n, T, R0, tb, st); }));
    float2* Sout = static_cast<float2*>(S);
    const size_t item_w = (size_t)(n / 2) * wave_col_stride(n), layer = (size_t)(n / 2) * (n / 2);
    // items [i0, i0 + cnt) of the batch starting at beam b0, all slices then the store, on stream q
    auto run_items = [&](int b0, int i0, int cnt, hipStream_t q, hipEvent_t after_first_a) -> int {
        float2* Wq = W + (size_t)i0 * item_w;
        const int2* bq = d_beams + b0 + i0;
        for (int s = 0; s < nsl; ++s) {
            if (s == 0)
                HIP_TRY(timed(PRISM_K_FIRST, q, [&] { return launch_first_from_spectrum(n, Wq, R0, tb, bq, cnt, q); }));
            else
                HIP_TRY(timed(PRISM_K_PASS_A, q, [&] { return launch_pass_a(n, Wq, T + (size_t)s * n * n, tb, cnt, q); }));
            if (PRISM_FORK_STAGE == 0 && s == 0 && after_first_a) HIP_TRY(hipEventRecord(after_first_a, q));
            if (PRISM_FORK_STAGE == 2 && s == std::min(1, nsl - 1) && after_first_a)
                HIP_TRY(hipEventRecord(after_first_a, q));
            HIP_TRY(timed(PRISM_K_PASS_B, q, [&] {
                return launch_pass_b(n, s == nsl - 1 ? PASSB_LAST_S : PASSB_MID, Wq, tb, nullptr, nullptr, nullptr,
                                     nullptr, 0.0, 0.f, cnt, q);
            }));
            if (PRISM_FORK_STAGE == 1 && s == 0 && after_first_a) HIP_TRY(hipEventRecord(after_first_a, q));
        }
        float2* Sq = Sout + (size_t)(b0 + i0) * layer;
        HIP_TRY(timed(PRISM_K_FINAL, q, [&] { return launch_smatrix_final(n, Wq, Sq, pd.tw_half, cnt, q); }));
        return PRISM_OK;
    };
    int P = std::min(build_streams_for(n), NB);
    hipStream_t q[kMaxBuildStreams] = {st};
    if (P > 1) {
        int got = 0;
        rc = partner_streams(st, P - 1, q + 1, &got);
        if (rc) return rc;
        if (got < P - 1) P = 1;
    }
    if (P <= 1) {
        for (int b0 = first; b0 < end; b0 += NB) {
            rc = run_items(b0, 0, std::min(NB, end - b0), st, nullptr);
            if (rc) return rc;
        }
        return PRISM_OK;
    }
    // Wave-buffer item i always holds beam b0 + i of the current batch, and
    // stream k owns items [off(k), off(k + 1)) in every batch (a short last
    // batch leaves the tail parts empty), so no two streams ever touch the
    // same item; the forks of the first batch and the final joins are the
    // only cross-stream orderings needed.
    BuildEvents be;
    for (int k = 0; k < 2 * P; ++k) HIP_TRY(hipEventCreateWithFlags(&be.ev[k], hipEventDisableTiming));
    auto off = [&](int k) { return (int)((int64_t)k * NB / P); };
    int forked = 1;                              // streams that may hold work of this call
    auto enqueue = [&]() -> int {
        for (int b0 = first; b0 < end; b0 += NB) {
            const int nb = std::min(NB, end - b0);
            for (int k = 0; k < P; ++k) {
                const int i0 = off(k), cnt = std::min(off(k + 1), nb) - i0;
                if (b0 == first && k > 0) {
                    HIP_TRY(hipStreamWaitEvent(q[k], be.ev[k - 1], 0));
                    forked = k + 1;
                }
                if (cnt > 0) {
                    int r = run_items(b0, i0, cnt, q[k], b0 == first ? be.ev[k] : nullptr);
                    if (r) return r;
                } else if (b0 == first) {
                    HIP_TRY(hipEventRecord(be.ev[k], q[k]));
                }
            }
        }
        return PRISM_OK;
    };
    rc = enqueue();
    // join every partner that may hold work, also after an error, so that
    // the caller's stream orders all of this call's work
    for (int k = 1; k < forked; ++k) {
        hipError_t e = hipEventRecord(be.ev[P + k], q[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, be.ev[P + k], 0);
        if (e != hipSuccess && rc == PRISM_OK) rc = fail(PRISM_E_DEVICE, "build: stream join: %s", hipGetErrorString(e));
    }
    return rc;
}

int prism_build_smatrix(const prism_smatrix_desc* d, const float* V, void* S, void* ws, size_t ws_bytes,
                        void* stream) {
    if (!d) return fail(PRISM_E_INVAL, "descriptor is NULL");
    return build_range(d, V, S, 0, d->n_beams, ws, ws_bytes, stream);
}

int prism_build_smatrix_range(const prism_smatrix_desc* d, const float* V, void* S, int32_t first, int32_t count,
                              void* ws, size_t ws_bytes, void* stream) {
    if (!d) return fail(PRISM_E_INVAL, "descriptor is NULL");
    return build_range(d, V, S, first, count, ws, ws_bytes, stream);
}

// -------------------------------------------------------- probe outputs --
// Plan of either detector: annular bins of width dalpha (dmap NULL) or the
// caller's map of the window grid (dalpha recorded as 0).
// The host tables of the last plan made on this thread, with every input they
// depend on, so that uploading that plan right after making it does not
// compute them again (inputs compared exactly, positions included).
struct PlanMemo {
    bool valid = false;
    int n, f, ns, m_win, n_bins;
    double L, lambda, alpha_max, alpha_aa, dalpha, C1, C3;
    std::vector<int32_t> dmap;
    ProbeHost h;
    int maxpt = 0;
};
thread_local PlanMemo t_plan_memo;

static bool memo_matches(const PlanMemo& m, const prism_smatrix_desc* d, const double* xy, int64_t n_probes,
                         double dalpha, int n_bins, double C1, double C3, const int32_t* dmap) {
    if (!m.valid || m.n != d->grid.n || m.f != d->f || m.ns != d->ns || m.m_win != d->m_win || m.n_bins != n_bins ||
        m.L != d->grid.cell[0] || m.lambda != d->lambda || m.alpha_max != d->alpha_max || m.alpha_aa != d->alpha_aa ||
        m.dalpha != dalpha || m.C1 != C1 || m.C3 != C3 || (int64_t)m.h.xy.size() != n_probes ||
        m.dmap.empty() != (dmap == nullptr))
        return false;
    if (dmap && std::memcmp(m.dmap.data(), dmap, m.dmap.size() * sizeof(int32_t)) != 0) return false;
    return n_probes == 0 || std::memcmp(m.h.xy.data(), xy, (size_t)n_probes * sizeof(double2)) == 0;
}

static void memo_store(const prism_smatrix_desc* d, double dalpha, int n_bins, double C1, double C3,
                       const int32_t* dmap, ProbeHost&& h, int maxpt) {
    PlanMemo& m = t_plan_memo;
    m.valid = true;
    m.n = d->grid.n;
    m.f = d->f;
    m.ns = d->ns;
    m.m_win = d->m_win;
    m.n_bins = n_bins;
    m.L = d->grid.cell[0];
    m.lambda = d->lambda;
    m.alpha_max = d->alpha_max;
    m.alpha_aa = d->alpha_aa;
    m.dalpha = dalpha;
    m.C1 = C1;
    m.C3 = C3;
    m.dmap.assign(dmap, dmap ? dmap + (size_t)d->m_win * d->m_win : dmap);
    m.h = std::move(h);
    m.maxpt = maxpt;
}

static int probe_plan_make(const prism_smatrix_desc* d, const double* probe_xy, int64_t n_probes, double dalpha,
                           int32_t n_bins, const int32_t* dmap, const prism_aberrations* ab, prism_probe_plan* plan) {
    int rc = check_desc(d);
    if (rc) return rc;
    if (!plan || (n_probes > 0 && !probe_xy) || n_probes < 0 || n_probes > (1 << 30) || (!dmap && !(dalpha > 0)))
        return fail(PRISM_E_INVAL, "probe plan: invalid argument");
    const double C1 = ab ? ab->C1 : 0.0, C3 = ab ? ab->C3 : 0.0;
    if (!std::isfinite(C1) || !std::isfinite(C3)) return fail(PRISM_E_INVAL, "probe plan: non-finite aberrations");
    if (dmap) {
        rc = check_detector_map(dmap, (size_t)d->m_win * d->m_win, n_bins, "probe plan");
        if (rc) return rc;
        dalpha = 0.0;
    } else if (n_bins <= 0) {
        n_bins = default_bins(d->alpha_aa, dalpha);
    }
    ProbeHost h;
    int maxpt = 0;
    rc = probe_host(d, probe_xy, n_probes, dalpha, n_bins, C1, C3, dmap, h, maxpt);
    if (rc) return rc;
    prism_probe_plan p{};
    p.n_probes = n_probes;
    p.n_bins = n_bins;
    p.n_tiles = (int32_t)(h.tile_start.size() - 1);
    p.n_entries = (int64_t)h.tile_probes.size();
    p.max_per_tile = maxpt;
    p.n_binned = (int32_t)h.perm.size();
    p.dalpha = dalpha;
    p.C1 = C1;
    p.C3 = C3;
    Carve c(nullptr);
    const size_t P = (size_t)std::max<int64_t>(n_probes, 1);
    p.off[0] = (size_t)c.take<double2>(P);
    p.off[1] = (size_t)c.take<int2>(P);
    p.off[2] = (size_t)c.take<int>(h.tile_start.size());
    p.off[3] = (size_t)c.take<int>(std::max<size_t>(h.tile_probes.size(), 1));
    p.off[4] = (size_t)c.take<int>(std::max<size_t>(h.perm.size(), 1));
    p.off[5] = (size_t)c.take<int>(h.bin_start.size());
    p.off[6] = (size_t)c.take<float2>(h.tw_m.size());
    p.off[7] = (size_t)c.take<int2>(h.beams.size());
    p.off[8] = h.aberr.empty() ? 0 : (size_t)c.take<float2>(h.aberr.size());
    p.off[9] = (size_t)c.take<int2>(std::max<size_t>(h.tile_origin.size(), 1));
    p.plan_bytes = c.off + 256;
    Carve w(nullptr);
    synth_job_carve(d, &p, w);
    split_s_carve(d, w);
    p.ws_bytes = w.off + 256;
    *plan = p;
    memo_store(d, dalpha, n_bins, C1, C3, dmap, std::move(h), maxpt);
    return PRISM_OK;
}

int prism_probe_plan_init(const prism_smatrix_desc* d, const double* probe_xy, int64_t n_probes, double dalpha,
                          int32_t n_bins, const prism_aberrations* ab, prism_probe_plan* plan) {
    return probe_plan_make(d, probe_xy, n_probes, dalpha, n_bins, nullptr, ab, plan);
}

int prism_probe_plan_init_map(const prism_smatrix_desc* d, const double* probe_xy, int64_t n_probes,
                              const int32_t* detector_map, int32_t n_bins, const prism_aberrations* ab,
                              prism_probe_plan* plan) {
    if (!detector_map) return fail(PRISM_E_INVAL, "probe plan: NULL detector map");
    return probe_plan_make(d, probe_xy, n_probes, 0.0, n_bins, detector_map, ab, plan);
}

static int probe_plan_put(const prism_smatrix_desc* d, const double* probe_xy, const int32_t* dmap,
                          const prism_probe_plan* plan, void* plan_dev, void* stream) {
    int rc = check_desc(d);
    if (rc) return rc;
    if (!plan || !plan_dev) return fail(PRISM_E_INVAL, "probe plan upload: NULL argument");
    if (dmap) {
        if (plan->dalpha != 0.0)
            return fail(PRISM_E_INVAL, "probe plan upload: the plan has annular bins; upload it without a map");
        rc = check_detector_map(dmap, (size_t)d->m_win * d->m_win, plan->n_bins, "probe plan upload");
        if (rc) return rc;
    } else if (!(plan->dalpha > 0)) {
        return fail(PRISM_E_INVAL, "probe plan upload: the plan was made for a detector map; upload it with that map");
    }
    if (plan->n_probes > 0 && !probe_xy) return fail(PRISM_E_INVAL, "probe plan upload: NULL positions");
    ProbeHost local;
    const ProbeHost* hp = &t_plan_memo.h;
    int maxpt = t_plan_memo.maxpt;
    if (!memo_matches(t_plan_memo, d, probe_xy, plan->n_probes, plan->dalpha, plan->n_bins, plan->C1, plan->C3,
                      dmap)) {
        rc = probe_host(d, probe_xy, plan->n_probes, plan->dalpha, plan->n_bins, plan->C1, plan->C3, dmap, local,
                        maxpt);
        if (rc) return rc;
        hp = &local;
    }
    const ProbeHost& h = *hp;
    // every size the kernels and the workspace depend on must be the plan's
    if ((int64_t)h.tile_probes.size() != plan->n_entries || (int)h.perm.size() != plan->n_binned ||
        maxpt != plan->max_per_tile || (int64_t)h.tile_start.size() - 1 != plan->n_tiles)
        return fail(PRISM_E_INVAL, "probe plan upload: plan does not match these probes");
    std::vector<char> blob(plan->plan_bytes, 0);
    auto put = [&](size_t off, const void* src, size_t bytes) {
        if (bytes) std::memcpy(blob.data() + off, src, bytes);
    };
    put(plan->off[0], h.xy.data(), h.xy.size() * sizeof(double2));
    put(plan->off[1], h.corner.data(), h.corner.size() * sizeof(int2));
    put(plan->off[2], h.tile_start.data(), h.tile_start.size() * sizeof(int));
    put(plan->off[3], h.tile_probes.data(), h.tile_probes.size() * sizeof(int));
    put(plan->off[4], h.perm.data(), h.perm.size() * sizeof(int));
    put(plan->off[5], h.bin_start.data(), h.bin_start.size() * sizeof(int));
    put(plan->off[6], h.tw_m.data(), h.tw_m.size() * sizeof(float2));
    put(plan->off[7], h.beams.data(), h.beams.size() * sizeof(int2));
    if (!h.aberr.empty()) put(plan->off[8], h.aberr.data(), h.aberr.size() * sizeof(float2));
    put(plan->off[9], h.tile_origin.data(), h.tile_origin.size() * sizeof(int2));
    return upload(plan_dev, blob, as_stream(stream));
}

int prism_probe_plan_upload(const prism_smatrix_desc* d, const double* probe_xy, const prism_probe_plan* plan,
                            void* plan_dev, void* stream) {
    return probe_plan_put(d, probe_xy, nullptr, plan, plan_dev, stream);
}

int prism_probe_plan_upload_map(const prism_smatrix_desc* d, const double* probe_xy, const int32_t* detector_map,
                                const prism_probe_plan* plan, void* plan_dev, void* stream) {
    if (!detector_map) return fail(PRISM_E_INVAL, "probe plan upload: NULL detector map");
    return probe_plan_put(d, probe_xy, detector_map, plan, plan_dev, stream);
}

// Index of the first job that reads the same S-matrix (same pointer and shape).
static int first_with_same_s(const prism_probe_job* jobs, int k) {
    for (int j = 0; j < k; ++j)
        if (jobs[j].S == jobs[k].S && jobs[j].desc->n_beams == jobs[k].desc->n_beams &&
            jobs[j].desc->ns == jobs[k].desc->ns)
            return j;
    return k;
}

static int synth_validate(const prism_probe_job* jobs, int n_jobs, int precision, size_t* need) {
    if (!jobs || n_jobs < 0) return fail(PRISM_E_INVAL, "probe outputs: invalid job list");
    if (precision != PRISM_FP32 && precision != PRISM_SPLIT_BF16X3 && precision != PRISM_BF16)
        return fail(PRISM_E_INVAL, "probe outputs: unknown precision %d", precision);
    Carve c(nullptr);
    for (int k = 0; k < n_jobs; ++k) {
        const prism_probe_job& jb = jobs[k];
        int rc = check_desc(jb.desc);
        if (rc) return rc;
        if (!jb.S || !jb.plan || !jb.plan_dev || (!jb.out && !jb.diffraction && jb.plan->n_probes > 0))
            return fail(PRISM_E_INVAL, "probe outputs: job %d has a NULL pointer", k);
        if (!std::isfinite(jb.out_scale) || (jb.accumulate != 0 && jb.accumulate != 1))
            return fail(PRISM_E_INVAL, "probe outputs: job %d: bad out_scale or accumulate", k);
        synth_job_carve(jb.desc, jb.plan, c);
    }
    for (int k = 0; k < n_jobs; ++k)
        if (first_with_same_s(jobs, k) == k) split_s_carve(jobs[k].desc, c);
    *need = c.off + 256;
    return PRISM_OK;
}

// Probe synthesis for several (S-matrix, probe plan) jobs on one stream:
// coefficients per job, split S per distinct S-matrix (MFMA precisions), one
// contraction launch for all jobs, one window launch per window side.
static int synth_run(const prism_probe_job* jobs, int n_jobs, int precision, void* ws, hipStream_t st) {
    std::vector<ContractArgs> ca;
    std::vector<std::vector<WindowArgs>> wa(10);   // by log2(m)
    const bool split = precision != PRISM_FP32;
    const bool split_s = split && contract_reads_split_s();
    Carve c(ws);
    std::vector<SynthJobDev> jd(n_jobs);
    for (int k = 0; k < n_jobs; ++k) jd[k] = synth_job_carve(jobs[k].desc, jobs[k].plan, c);
    std::vector<const void*> s_op(n_jobs, nullptr);
    for (int k = 0; k < n_jobs; ++k) {
        const int j = first_with_same_s(jobs, k);
        if (j < k) {
            s_op[k] = s_op[j];
            continue;
        }
        void* ss = split_s_carve(jobs[k].desc, c);
        s_op[k] = split_s ? ss : jobs[k].S;
        // the split copy serves every job on this S-matrix: convert it when
        // any of them has probes (the first may have none)
        bool used = false;
        for (int i = k; i < n_jobs && !used; ++i)
            used = jobs[i].plan->n_probes > 0 && first_with_same_s(jobs, i) == k;
        if (split_s && used) {
            const prism_smatrix_desc* d = jobs[k].desc;
            HIP_TRY(timed(PRISM_K_SPLIT, st, [&] {
                return launch_split_s(precision, static_cast<const float2*>(jobs[k].S), ss, d->n_beams, d->ns, st);
            }));
        }
    }
    for (int k = 0; k < n_jobs; ++k) {
        const prism_probe_job& jb = jobs[k];
        const prism_smatrix_desc* d = jb.desc;
        const prism_probe_plan* plan = jb.plan;
        const char* pb = static_cast<const char*>(jb.plan_dev);
        const int P = (int)plan->n_probes, B = d->n_beams, M = d->m_win;
        if (P == 0) continue;
        auto xy = reinterpret_cast<const double2*>(pb + plan->off[0]);
        auto corner = reinterpret_cast<const int2*>(pb + plan->off[1]);
        auto tstart = reinterpret_cast<const int*>(pb + plan->off[2]);
        auto tprobes = reinterpret_cast<const int*>(pb + plan->off[3]);
        auto perm = reinterpret_cast<const int*>(pb + plan->off[4]);
        auto bstart = reinterpret_cast<const int*>(pb + plan->off[5]);
        auto tw_m = reinterpret_cast<const float2*>(pb + plan->off[6]);
        auto beams = reinterpret_cast<const int2*>(pb + plan->off[7]);
        auto aberr = (plan->C1 != 0.0 || plan->C3 != 0.0) ? reinterpret_cast<const float2*>(pb + plan->off[8]) : nullptr;
        auto torigin = reinterpret_cast<const int2*>(pb + plan->off[9]);
        const double inv_L = 1.0 / d->grid.cell[0];
        const float amp = (float)(1.0 / std::sqrt((double)B));
        HIP_TRY(timed(PRISM_K_COEFFICIENTS, st, [&] {
            return split ? launch_coefficients_split(precision, jd[k].C, xy, beams, aberr, P, B, inv_L, amp, st)
                         : launch_coefficients(static_cast<float2*>(jd[k].C), xy, beams, aberr, P, B, inv_L, amp, st);
        }));
        ca.push_back(ContractArgs{jd[k].C, s_op[k], jd[k].win, tstart, tprobes, torigin, corner, plan->n_tiles,
                                  plan->max_per_tile, B, d->ns, M});
        int lg = 0;
        while ((1 << lg) < M) ++lg;
        wa[lg].push_back(WindowArgs{jd[k].win, jd[k].inten, jb.out, jb.diffraction, perm, bstart, tw_m, P,
                                    plan->n_bins, jb.out_scale, jb.accumulate});
    }
    if (!ca.empty())
        HIP_TRY(timed(PRISM_K_CONTRACT, st, [&] { return launch_contract_batch(precision, ca.data(), (int)ca.size(), st); }));
    for (int lg = 0; lg < 10; ++lg)
        if (!wa[lg].empty())
            HIP_TRY(timed(PRISM_K_WINDOW, st, [&] { return launch_window_batch(1 << lg, wa[lg].data(), (int)wa[lg].size(), st); }));
    return PRISM_OK;
}

int prism_probe_outputs(const prism_smatrix_desc* d, const void* S, const prism_probe_plan* plan,
                        const void* plan_dev, int32_t precision, float* out, void* ws, size_t ws_bytes,
                        void* stream) {
    prism_probe_job jb{d, S, plan, plan_dev, out, nullptr, 1.0f, 0};
    size_t need = 0;
    int rc = synth_validate(&jb, 1, precision, &need);
    if (rc) return rc;
    if (!ws || ws_bytes < plan->ws_bytes)
        return fail(PRISM_E_WORKSPACE, "probe outputs: workspace %zu < %zu bytes", ws_bytes, plan->ws_bytes);
    if (plan->n_probes == 0) return PRISM_OK;
    return synth_run(&jb, 1, precision, ws, as_stream(stream));
}

int prism_probe_outputs_noalloc(const prism_smatrix_desc* d, const void* S, const prism_probe_plan* plan,
                                const void* plan_dev, int32_t precision, float* out, void* stream) {
    prism_probe_job jb{d, S, plan, plan_dev, out, nullptr, 1.0f, 0};
    size_t need = 0;
    int rc = synth_validate(&jb, 1, precision, &need);
    if (rc) return rc;
    const size_t want = std::max(need, plan->ws_bytes);
    if (want > (size_t)PRISM_NOALLOC_SCRATCH_BYTES)
        return fail(PRISM_E_WORKSPACE, "probe outputs (no allocation): %zu bytes of workspace needed, the fixed scratch holds %zu",
                    want, (size_t)PRISM_NOALLOC_SCRATCH_BYTES);
    if (plan->n_probes == 0) return PRISM_OK;
    void* ws = nullptr;
    rc = scratch_address(&ws);
    if (rc) return rc;
    return synth_run(&jb, 1, precision, ws, as_stream(stream));
}

int prism_probe_diffraction(const prism_smatrix_desc* d, const void* S, const prism_probe_plan* plan,
                            const void* plan_dev, int32_t precision, float* out4d, void* ws, size_t ws_bytes,
                            void* stream) {
    prism_probe_job jb{d, S, plan, plan_dev, nullptr, out4d, 1.0f, 0};
    size_t need = 0;
    int rc = synth_validate(&jb, 1, precision, &need);
    if (rc) return rc;
    if (!out4d && plan->n_probes > 0) return fail(PRISM_E_INVAL, "probe diffraction: NULL output");
    if (!ws || ws_bytes < plan->ws_bytes)
        return fail(PRISM_E_WORKSPACE, "probe diffraction: workspace %zu < %zu bytes", ws_bytes, plan->ws_bytes);
    if (plan->n_probes == 0) return PRISM_OK;
    return synth_run(&jb, 1, precision, ws, as_stream(stream));
}

int prism_probe_batch_workspace(const prism_probe_job* jobs, int32_t n_jobs, size_t* bytes) {
    if (!bytes) return fail(PRISM_E_INVAL, "batch workspace: NULL argument");
    return synth_validate(jobs, n_jobs, PRISM_FP32, bytes);
}

int prism_probe_outputs_batched(const prism_probe_job* jobs, int32_t n_jobs, int32_t precision, void* ws,
                                size_t ws_bytes, void* stream) {
    size_t need = 0;
    int rc = synth_validate(jobs, n_jobs, precision, &need);
    if (rc) return rc;
    if (!ws || ws_bytes < need)
        return fail(PRISM_E_WORKSPACE, "batched probe outputs: workspace %zu < %zu bytes", ws_bytes, need);
    return synth_run(jobs, n_jobs, precision, ws, as_stream(stream));
}

// ------------------------------------------------------------ multislice --
// Host side of a multislice call: aperture, aberration table, bin tables.
struct MsHost {
    double lam, sig, a_aa;
    int n_bins;
    long long n_ap;
    std::vector<int> kymax, perm, bstart;
    std::vector<float2> aberr;
    std::vector<double2> xy;
};

static int multislice_host(const prism_grid* grid, double E0, double alpha_max, const prism_aberrations* ab,
                           const double* probe_xy, int64_t n_probes, double dalpha, int32_t n_bins,
                           const int32_t* dmap, MsHost& h) {
    const int n = grid->n, Lh = n / 2;
    const double L = grid->cell[0];
    h.lam = wavelength_A(E0);
    h.sig = sigma_per_VA(E0);
    h.a_aa = alpha_aa_of(h.lam, n, L);
    if (!(alpha_max < h.a_aa))
        return fail(PRISM_E_UNSUPPORTED, "multislice: alpha_max %.6g must be below alpha_AA %.6g", alpha_max, h.a_aa);
    if (dmap) {
        int rc = check_detector_map(dmap, (size_t)n * n, n_bins, "multislice");
        if (rc) return rc;
    } else if (n_bins <= 0) {
        n_bins = default_bins(h.a_aa, dalpha);
    }
    if (n_bins > MAX_BINS) return fail(PRISM_E_UNSUPPORTED, "multislice: more than %d bins", MAX_BINS);
    h.n_bins = n_bins;
    // aperture per band column and its size
    h.kymax.assign(Lh, -1);
    h.n_ap = 0;
    for (int j = 0; j < Lh; ++j) {
        int kx = band_k(j, n);
        int m = -1;
        while (m + 1 < n / 4 && angle_of(h.lam, kx, m + 1, L) <= alpha_max) ++m;
        h.kymax[j] = m;
        if (m >= 0) h.n_ap += 2 * m + 1;
    }
    if (h.n_ap == 0) return fail(PRISM_E_INVAL, "multislice: empty aperture");
    // aberration factor of every band pixel [j][j'] (kx from j, ky from j')
    const double C1 = ab ? ab->C1 : 0.0, C3 = ab ? ab->C3 : 0.0;
    if (!std::isfinite(C1) || !std::isfinite(C3)) return fail(PRISM_E_INVAL, "multislice: non-finite aberrations");
    if (C1 != 0.0 || C3 != 0.0) {
        h.aberr.resize((size_t)Lh * Lh);
        for (int j = 0; j < Lh; ++j)
            for (int jp = 0; jp < Lh; ++jp)
                h.aberr[(size_t)j * Lh + jp] = aberration_factor(band_k(j, n), band_k(jp, n), L, h.lam, C1, C3);
    }
    // bins over band pixels, index j * (n/2) + j' (kx from j, ky from j');
    // the band holds every pixel of nonzero intensity (the propagator's
    // mask), so a map's entries outside it add nothing
    std::vector<int> bins((size_t)Lh * Lh);
    for (int j = 0; j < Lh; ++j)
        for (int jp = 0; jp < Lh; ++jp) {
            const int kx = band_k(j, n), ky = band_k(jp, n);
            bins[(size_t)j * Lh + jp] = dmap ? dmap[(size_t)((ky + n) % n) * n + (kx + n) % n]
                                             : bin_of(h.lam, kx, ky, L, h.a_aa, dalpha, n_bins);
        }
    group_by_bin(bins, n_bins, h.perm, h.bstart);
    h.xy.resize(std::max<int64_t>(n_probes, 1));
    for (int64_t p = 0; p < n_probes; ++p) {
        if (!std::isfinite(probe_xy[2 * p]) || !std::isfinite(probe_xy[2 * p + 1]))
            return fail(PRISM_E_INVAL, "probe %lld: non-finite position", (long long)p);
        h.xy[p] = make_double2(probe_xy[2 * p], probe_xy[2 * p + 1]);
    }
    return PRISM_OK;
}

// Device layout of a multislice call.  Resident: transmission of every slice.
// Streaming: one transmission slice and two potential-slice buffers.
struct MsDev {
    PropDev pd;
    int *kymax, *perm, *bstart;
    double2* xy;
    float2 *T, *W, *aberr;
    float* I;
    float* vslot[2];
};

static void multislice_carve(Carve& c, int n, int nsl, int64_t n_probes, int batch, int n_bins, size_t n_binned,
                             bool streaming, MsDev& m) {
    m.pd = carve_prop(c, n);
    m.aberr = c.take<float2>((size_t)(n / 2) * (n / 2));
    m.kymax = c.take<int>(n / 2);
    m.perm = c.take<int>(std::max<size_t>(n_binned, 1));
    m.bstart = c.take<int>(n_bins + 1);
    m.xy = c.take<double2>((size_t)std::max<int64_t>(n_probes, 1));
    m.T = c.take<float2>((size_t)(streaming ? 1 : nsl) * n * n);
    m.W = c.take<float2>((size_t)batch * (n / 2) * wave_col_stride(n));
    m.I = c.take<float>((size_t)batch * (n / 2) * (n / 2));
    m.vslot[0] = streaming ? c.take<float>((size_t)n * n) : nullptr;
    m.vslot[1] = streaming ? c.take<float>((size_t)n * n) : nullptr;
}

static int multislice_ws(const prism_grid* grid, int32_t batch, int64_t n_probes, bool streaming, size_t* bytes) {
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!bytes || batch < 1 || n_probes < 0) return fail(PRISM_E_INVAL, "multislice workspace: invalid argument");
    Carve c(nullptr);
    MsDev m;
    // bins can cover at most the (n/2)^2 band pixels
    multislice_carve(c, grid->n, grid->n_slices, n_probes, batch, MAX_BINS, (size_t)(grid->n / 2) * (grid->n / 2),
                     streaming, m);
    *bytes = c.off + 256;
    return PRISM_OK;
}

// Two-slot staging ring: slot k is filled on one stream after `freed[k]`
// and consumed on another after `ready[k]`.
struct Ring2 {
    hipEvent_t ready[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
    bool used[2] = {false, false};
    hipError_t init() {
        for (int k = 0; k < 2; ++k) {
            hipError_t e = hipEventCreateWithFlags(&ready[k], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&freed[k], hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    ~Ring2() {
        for (int k = 0; k < 2; ++k) {
            if (ready[k]) (void)hipEventDestroy(ready[k]);
            if (freed[k]) (void)hipEventDestroy(freed[k]);
        }
    }
};

// Streamed slice: copy slice s of V_host into slot (g & 1) on h2d once that
// slot's previous transmission has run, then compute its transmission into T
// on st.  The caller's next kernels on st read T.
static int feed_slice(Ring2& r, long long g, const float* V_host, int s, int n, float* const vslot[2], float2* T,
                      float sigma, hipStream_t st, hipStream_t h2d) {
    const int k = (int)(g & 1);
    const size_t n2 = (size_t)n * n;
    if (r.used[k]) HIP_TRY(hipStreamWaitEvent(h2d, r.freed[k], 0));
    HIP_TRY(hipMemcpyAsync(vslot[k], V_host + (size_t)s * n2, n2 * sizeof(float), hipMemcpyHostToDevice, h2d));
    HIP_TRY(hipEventRecord(r.ready[k], h2d));
    HIP_TRY(hipStreamWaitEvent(st, r.ready[k], 0));
    HIP_TRY(timed(PRISM_K_TRANSMISSION, st, [&] { return launch_transmission(vslot[k], T, (int64_t)n2, sigma, st); }));
    HIP_TRY(hipEventRecord(r.freed[k], st));
    r.used[k] = true;
    return PRISM_OK;
}

// Make `side` wait for all work enqueued so far on st, so that side-stream
// copies see the results of the caller's earlier work on st.
static int order_after(hipStream_t side, hipStream_t st) {
    if (side == st) return PRISM_OK;
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipError_t r = hipEventRecord(e, st);
    if (r == hipSuccess) r = hipStreamWaitEvent(side, e, 0);
    (void)hipEventDestroy(e);
    if (r != hipSuccess) return fail(PRISM_E_DEVICE, "ordering copy stream: %s", hipGetErrorString(r));
    return PRISM_OK;
}

// Make st wait for the last use of every slot on the other stream.
static int join_ring(const Ring2& r, bool on_freed, hipStream_t st) {
    for (int k = 0; k < 2; ++k)
        if (r.used[k]) HIP_TRY(hipStreamWaitEvent(st, on_freed ? r.freed[k] : r.ready[k], 0));
    return PRISM_OK;
}

static int multislice_run(const prism_grid* grid, double E0, double alpha_max, const prism_aberrations* ab,
                          const float* V, const float* V_host, const double* probe_xy, int64_t n_probes,
                          double dalpha, int32_t n_bins, const int32_t* dmap, int32_t batch, float* out, void* ws,
                          size_t ws_bytes, hipStream_t st, hipStream_t h2d) {
    int rc = check_grid(grid);
    if (rc) return rc;
    const bool streaming = V_host != nullptr;
    if ((!V && !V_host) || (!out && n_probes > 0) || (n_probes > 0 && !probe_xy) || n_probes < 0 || batch < 1 ||
        !(E0 > 0) ||
        !(alpha_max > 0) || (!dmap && !(dalpha > 0)))
        return fail(PRISM_E_INVAL, "multislice: invalid argument");
    const int n = grid->n, Lh = n / 2, nsl = grid->n_slices;
    const double L = grid->cell[0];
    MsHost h;
    rc = multislice_host(grid, E0, alpha_max, ab, probe_xy, n_probes, dalpha, n_bins, dmap, h);
    if (rc) return rc;
    n_bins = h.n_bins;
    size_t need = 0;
    rc = multislice_ws(grid, batch, n_probes, streaming, &need);
    if (rc) return rc;
    if (!ws || ws_bytes < need) return fail(PRISM_E_WORKSPACE, "multislice: workspace %zu < %zu bytes", ws_bytes, need);
    Carve c(ws);
    MsDev m;
    multislice_carve(c, n, nsl, n_probes, batch, n_bins, h.perm.size(), streaming, m);
    PropHost ph = prop_tables(n, L, h.lam, grid->dz);
    std::vector<char> blob;
    stage(blob, ws, m.pd.tw_half, ph.tw_half);
    stage(blob, ws, m.pd.tw_full, ph.tw_full);
    stage(blob, ws, m.pd.band, ph.band);
    stage(blob, ws, m.pd.prop, ph.prop);
    stage(blob, ws, m.kymax, h.kymax);
    stage(blob, ws, m.perm, h.perm);
    stage(blob, ws, m.bstart, h.bstart);
    stage(blob, ws, m.xy, h.xy);
    if (!h.aberr.empty()) stage(blob, ws, m.aberr, h.aberr);
    rc = upload(ws, blob, st);
    if (rc) return rc;
    const PropTables tb = m.pd.tables();
    Ring2 ring;
    if (streaming) {
        HIP_TRY(ring.init());
        rc = order_after(h2d, st);
        if (rc) return rc;
    } else {
        HIP_TRY(timed(PRISM_K_TRANSMISSION, st, [&] { return launch_transmission(V, m.T, (int64_t)nsl * n * n, (float)h.sig, st); }));
    }
    const float amp = (float)(1.0 / std::sqrt((double)h.n_ap));
    long long g = 0;
    for (int64_t p0 = 0; p0 < n_probes; p0 += batch) {
        const int nb = (int)std::min<int64_t>(batch, n_probes - p0);
        HIP_TRY(timed(PRISM_K_PASS_B, st, [&] {
            return launch_pass_b(n, PASSB_INIT, m.W, tb, h.aberr.empty() ? nullptr : m.aberr, nullptr, m.kymax,
                                 m.xy + p0, 1.0 / L, amp, nb, st);
        }));
        for (int s = 0; s < nsl; ++s) {
            const float2* Ts = m.T + (size_t)s * n * n;
            if (streaming) {
                rc = feed_slice(ring, g++, V_host, s, n, m.vslot, m.T, (float)h.sig, st, h2d);
                if (rc) return rc;
                Ts = m.T;
            }
            HIP_TRY(timed(PRISM_K_PASS_A, st, [&] { return launch_pass_a(n, m.W, Ts, tb, nb, st); }));
            HIP_TRY(timed(PRISM_K_PASS_B, st, [&] {
                return launch_pass_b(n, s == nsl - 1 ? PASSB_LAST_I : PASSB_MID, m.W, tb, nullptr, m.I, nullptr,
                                     nullptr, 0.0, 0.f, nb, st);
            }));
        }
        HIP_TRY(timed(PRISM_K_BIN_REDUCE, st, [&] {
            return launch_bin_reduce(m.I, (int64_t)Lh * Lh, out + p0 * n_bins, m.perm, m.bstart, nb, n_bins, st);
        }));
    }
    return PRISM_OK;
}

int multislice_workspace(const prism_grid* grid, int32_t batch, int64_t n_probes, size_t* bytes) {
    return multislice_ws(grid, batch, n_probes, false, bytes);
}

int multislice_outputs(const prism_grid* grid, double E0, double alpha_max, const prism_aberrations* ab,
                       const float* V, const double* probe_xy, int64_t n_probes, double dalpha, int32_t n_bins,
                       int32_t batch, float* out, void* ws, size_t ws_bytes, void* stream) {
    if (!V) return fail(PRISM_E_INVAL, "multislice: NULL V");
    return multislice_run(grid, E0, alpha_max, ab, V, nullptr, probe_xy, n_probes, dalpha, n_bins, nullptr, batch,
                          out, ws, ws_bytes, as_stream(stream), nullptr);
}

int multislice_outputs_map(const prism_grid* grid, double E0, double alpha_max, const prism_aberrations* ab,
                           const float* V, const double* probe_xy, int64_t n_probes, const int32_t* detector_map,
                           int32_t n_bins, int32_t batch, float* out, void* ws, size_t ws_bytes, void* stream) {
    if (!V) return fail(PRISM_E_INVAL, "multislice: NULL V");
    if (!detector_map) return fail(PRISM_E_INVAL, "multislice: NULL detector map");
    return multislice_run(grid, E0, alpha_max, ab, V, nullptr, probe_xy, n_probes, 0.0, n_bins, detector_map, batch,
                          out, ws, ws_bytes, as_stream(stream), nullptr);
}

int multislice_streaming_workspace(const prism_grid* grid, int32_t batch, int64_t n_probes, size_t* bytes) {
    return multislice_ws(grid, batch, n_probes, true, bytes);
}

int multislice_outputs_streaming(const prism_grid* grid, double E0, double alpha_max, const prism_aberrations* ab,
                                 const float* V_host, const double* probe_xy, int64_t n_probes, double dalpha,
                                 int32_t n_bins, int32_t batch, float* out, void* ws, size_t ws_bytes, void* stream,
                                 void* h2d_stream) {
    if (!V_host) return fail(PRISM_E_INVAL, "multislice streaming: NULL V_host");
    return multislice_run(grid, E0, alpha_max, ab, nullptr, V_host, probe_xy, n_probes, dalpha, n_bins, nullptr,
                          batch, out, ws, ws_bytes, as_stream(stream), as_stream(h2d_stream));
}

// ----------------------------------------------------- streaming S-matrix --
struct StreamBuildDev {
    PropDev pd;
    int2* beams;
    float* vslot[2];
    float2 *T, *R0, *W;
    float2* Sst[2];
};

static void stream_build_carve(Carve& c, const prism_smatrix_desc* d, StreamBuildDev& m) {
    const int n = d->grid.n, NB = batch_of(d);
    m.pd = carve_prop(c, n);
    m.beams = c.take<int2>(d->n_beams);
    m.vslot[0] = c.take<float>((size_t)n * n);
    m.vslot[1] = c.take<float>((size_t)n * n);
    m.T = c.take<float2>((size_t)n * n);
    m.R0 = c.take<float2>((size_t)n * n);
    m.W = c.take<float2>((size_t)NB * (n / 2) * wave_col_stride(n));
    m.Sst[0] = c.take<float2>((size_t)NB * d->ns * d->ns);
    m.Sst[1] = c.take<float2>((size_t)NB * d->ns * d->ns);
}

int prism_streaming_build_workspace(const prism_smatrix_desc* d, size_t* bytes) {
    int rc = check_desc(d);
    if (rc) return rc;
    if (!bytes) return fail(PRISM_E_INVAL, "streaming build workspace: NULL argument");
    Carve c(nullptr);
    StreamBuildDev m;
    stream_build_carve(c, d, m);
    *bytes = c.off + 256;
    return PRISM_OK;
}

int prism_build_smatrix_streaming(const prism_smatrix_desc* d, const float* V_host, void* S_host, void* ws,
                                  size_t ws_bytes, void* stream, void* h2d_stream, void* d2h_stream) {
    size_t need = 0;
    int rc = prism_streaming_build_workspace(d, &need);
    if (rc) return rc;
    if (!V_host || !S_host) return fail(PRISM_E_INVAL, "streaming build: NULL V_host or S_host");
    if (!ws || ws_bytes < need) return fail(PRISM_E_WORKSPACE, "streaming build: workspace %zu < %zu bytes", ws_bytes, need);
    const int n = d->grid.n, B = d->n_beams, nsl = d->grid.n_slices, NB = batch_of(d);
    const double L = d->grid.cell[0];
    const size_t layer = (size_t)d->ns * d->ns;
    hipStream_t st = as_stream(stream), h2d = as_stream(h2d_stream), d2h = as_stream(d2h_stream);
    Carve c(ws);
    StreamBuildDev m;
    stream_build_carve(c, d, m);
    PropHost ph = prop_tables(n, L, d->lambda, d->grid.dz);
    std::vector<char> blob;
    stage(blob, ws, m.pd.tw_half, ph.tw_half);
    stage(blob, ws, m.pd.tw_full, ph.tw_full);
    stage(blob, ws, m.pd.band, ph.band);
    stage(blob, ws, m.pd.prop, ph.prop);
    stage(blob, ws, m.beams, beam_list(n, L, d->lambda, d->alpha_max, d->f));
    rc = upload(ws, blob, st);
    if (rc) return rc;
    const PropTables tb = m.pd.tables();
    Ring2 vr, sr;
    HIP_TRY(vr.init());
    HIP_TRY(sr.init());
    rc = order_after(h2d, st);
    if (rc) return rc;
    rc = order_after(d2h, st);
    if (rc) return rc;
    float2* Sout = static_cast<float2*>(S_host);
    long long g = 0;
    int bi = 0;
    for (int b0 = 0; b0 < B; b0 += NB, ++bi) {
        const int nb = std::min(NB, B - b0);
        const int2* bb = m.beams + b0;
        for (int s = 0; s < nsl; ++s) {
            rc = feed_slice(vr, g++, V_host, s, n, m.vslot, m.T, (float)d->sigma, st, h2d);
            if (rc) return rc;
            if (s == 0) {
                // the first slice's row spectrum, rebuilt per batch (the slice buffer is reused)
                HIP_TRY(timed(PRISM_K_TRANSMISSION, st, [&] { return launch_row_spectrum(n, m.T, m.R0, tb, st); }));
                HIP_TRY(timed(PRISM_K_FIRST, st, [&] { return launch_first_from_spectrum(n, m.W, m.R0, tb, bb, nb, st); }));
            } else {
                HIP_TRY(timed(PRISM_K_PASS_A, st, [&] { return launch_pass_a(n, m.W, m.T, tb, nb, st); }));
            }
            HIP_TRY(timed(PRISM_K_PASS_B, st, [&] {
                return launch_pass_b(n, s == nsl - 1 ? PASSB_LAST_S : PASSB_MID, m.W, tb, nullptr, nullptr, nullptr,
                                     nullptr, 0.0, 0.f, nb, st);
            }));
        }
        // S staging slot k is rewritten once its previous copy-out has run
        const int k = bi & 1;
        if (sr.used[k]) HIP_TRY(hipStreamWaitEvent(st, sr.freed[k], 0));
        HIP_TRY(timed(PRISM_K_FINAL, st, [&] { return launch_smatrix_final(n, m.W, m.Sst[k], m.pd.tw_half, nb, st); }));
        HIP_TRY(hipEventRecord(sr.ready[k], st));
        HIP_TRY(hipStreamWaitEvent(d2h, sr.ready[k], 0));
        HIP_TRY(hipMemcpyAsync(Sout + (size_t)b0 * layer, m.Sst[k], (size_t)nb * layer * sizeof(float2),
                               hipMemcpyDeviceToHost, d2h));
        HIP_TRY(hipEventRecord(sr.freed[k], d2h));
        sr.used[k] = true;
    }
    return join_ring(sr, true, st);
}

// --------------------------------------------------- streaming synthesis --
struct StreamSynthDev {
    float2* Sst[2];
    void *C, *Ssplit;
    float2* win;
    float* inten;
};

// Beam-chunked synthesis layout: two chunk slots when S is streamed from
// host memory (none when S is device-resident), the coefficients and split S
// of one chunk, the windows of all probes.
static void stream_synth_carve(Carve& c, const prism_smatrix_desc* d, const prism_probe_plan* plan, int chunk,
                               bool slots, StreamSynthDev& m) {
    const size_t P = (size_t)std::max<int64_t>(plan->n_probes, 1), M = d->m_win;
    m.Sst[0] = slots ? c.take<float2>((size_t)chunk * d->ns * d->ns) : nullptr;
    m.Sst[1] = slots ? c.take<float2>((size_t)chunk * d->ns * d->ns) : nullptr;
    m.C = c.take<char>(split_c_bytes((int64_t)P, chunk));
    m.Ssplit = contract_reads_split_s() ? c.take<char>(split_s_bytes(d->ns, chunk)) : nullptr;
    m.win = c.take<float2>(P * M * M);
    m.inten = M > 128 ? c.take<float>(P * M * M) : nullptr;
}

static int chunked_ws(const prism_smatrix_desc* d, const prism_probe_plan* plan, int32_t beam_chunk, bool slots,
                      size_t* bytes) {
    int rc = check_desc(d);
    if (rc) return rc;
    if (!plan || !bytes || beam_chunk < 1 || beam_chunk > d->n_beams)
        return fail(PRISM_E_INVAL, "chunked synthesis workspace: invalid argument (beam_chunk in [1, %d])",
                    d->n_beams);
    Carve c(nullptr);
    StreamSynthDev m;
    stream_synth_carve(c, d, plan, beam_chunk, slots, m);
    *bytes = c.off + 256;
    return PRISM_OK;
}

// Probe synthesis over beam chunks accumulated in the FP32 windows.  With
// h2d set, S is host memory and each chunk is first copied into one of two
// device slots (one chunk ahead); otherwise S is device memory read in place.
static int synth_chunked(const prism_smatrix_desc* d, const void* S, const prism_probe_plan* plan,
                         const void* plan_dev, int32_t precision, int32_t beam_chunk, float* out, float* out4d,
                         void* ws, size_t ws_bytes, hipStream_t st, hipStream_t h2d, bool streamed) {
    size_t need = 0;
    int rc = chunked_ws(d, plan, beam_chunk, streamed, &need);
    if (rc) return rc;
    if (precision != PRISM_FP32 && precision != PRISM_SPLIT_BF16X3 && precision != PRISM_BF16)
        return fail(PRISM_E_INVAL, "chunked synthesis: unknown precision %d", precision);
    if (!S || !plan_dev || (!out && !out4d && plan->n_probes > 0))
        return fail(PRISM_E_INVAL, "chunked synthesis: NULL argument");
    if (!ws || ws_bytes < need)
        return fail(PRISM_E_WORKSPACE, "chunked synthesis: workspace %zu < %zu bytes", ws_bytes, need);
    if (plan->n_probes == 0) return PRISM_OK;
    Carve c(ws);
    StreamSynthDev m;
    stream_synth_carve(c, d, plan, beam_chunk, streamed, m);
    const char* pb = static_cast<const char*>(plan_dev);
    const int P = (int)plan->n_probes, B = d->n_beams, M = d->m_win;
    const size_t layer = (size_t)d->ns * d->ns;
    auto xy = reinterpret_cast<const double2*>(pb + plan->off[0]);
    auto corner = reinterpret_cast<const int2*>(pb + plan->off[1]);
    auto tstart = reinterpret_cast<const int*>(pb + plan->off[2]);
    auto tprobes = reinterpret_cast<const int*>(pb + plan->off[3]);
    auto perm = reinterpret_cast<const int*>(pb + plan->off[4]);
    auto bstart = reinterpret_cast<const int*>(pb + plan->off[5]);
    auto tw_m = reinterpret_cast<const float2*>(pb + plan->off[6]);
    auto beams = reinterpret_cast<const int2*>(pb + plan->off[7]);
    auto aberr = (plan->C1 != 0.0 || plan->C3 != 0.0) ? reinterpret_cast<const float2*>(pb + plan->off[8]) : nullptr;
    auto torigin = reinterpret_cast<const int2*>(pb + plan->off[9]);
    const float amp = (float)(1.0 / std::sqrt((double)B));
    const bool split = precision != PRISM_FP32;
    const double inv_L = 1.0 / d->grid.cell[0];
    const float2* Sb = static_cast<const float2*>(S);
    Ring2 r;
    if (streamed) {
        HIP_TRY(r.init());
        rc = order_after(h2d, st);
        if (rc) return rc;
    }
    int ci = 0;
    for (int c0 = 0; c0 < B; c0 += beam_chunk, ++ci) {
        const int nb = std::min(beam_chunk, B - c0);
        const int k = ci & 1;
        const float2* chunk = Sb + (size_t)c0 * layer;
        if (streamed) {
            if (r.used[k]) HIP_TRY(hipStreamWaitEvent(h2d, r.freed[k], 0));
            HIP_TRY(hipMemcpyAsync(m.Sst[k], chunk, (size_t)nb * layer * sizeof(float2), hipMemcpyHostToDevice, h2d));
            HIP_TRY(hipEventRecord(r.ready[k], h2d));
            HIP_TRY(hipStreamWaitEvent(st, r.ready[k], 0));
            chunk = m.Sst[k];
        }
        const float2* ab = aberr ? aberr + c0 : nullptr;
        const void* s_op = chunk;
        if (split && contract_reads_split_s()) {
            HIP_TRY(timed(PRISM_K_SPLIT, st, [&] { return launch_split_s(precision, chunk, m.Ssplit, nb, d->ns, st); }));
            s_op = m.Ssplit;
        }
        HIP_TRY(timed(PRISM_K_COEFFICIENTS, st, [&] {
            return split ? launch_coefficients_split(precision, m.C, xy, beams + c0, ab, P, nb, inv_L, amp, st)
                         : launch_coefficients(static_cast<float2*>(m.C), xy, beams + c0, ab, P, nb, inv_L, amp, st);
        }));
        ContractArgs ca{m.C, s_op, m.win, tstart, tprobes, torigin, corner, plan->n_tiles, plan->max_per_tile, nb,
                        d->ns, M, ci > 0 ? 1 : 0};
        HIP_TRY(timed(PRISM_K_CONTRACT, st, [&] { return launch_contract_batch(precision, &ca, 1, st); }));
        // a streamed slot is free again once its chunk has been read
        if (streamed) HIP_TRY(hipEventRecord(r.freed[k], st));
        if (streamed) r.used[k] = true;
    }
    WindowArgs wa{m.win, m.inten, out, out4d, perm, bstart, tw_m, P, plan->n_bins, 1.0f, 0};
    HIP_TRY(timed(PRISM_K_WINDOW, st, [&] { return launch_window_batch(M, &wa, 1, st); }));
    return PRISM_OK;
}

int prism_probe_streaming_workspace(const prism_smatrix_desc* d, const prism_probe_plan* plan, int32_t beam_chunk,
                                    size_t* bytes) {
    return chunked_ws(d, plan, beam_chunk, true, bytes);
}

int prism_probe_outputs_streaming(const prism_smatrix_desc* d, const void* S_host, const prism_probe_plan* plan,
                                  const void* plan_dev, int32_t precision, int32_t beam_chunk, float* out,
                                  float* out4d, void* ws, size_t ws_bytes, void* stream, void* h2d_stream) {
    return synth_chunked(d, S_host, plan, plan_dev, precision, beam_chunk, out, out4d, ws, ws_bytes,
                         as_stream(stream), as_stream(h2d_stream), true);
}

int prism_probe_chunked_workspace(const prism_smatrix_desc* d, const prism_probe_plan* plan, int32_t beam_chunk,
                                  size_t* bytes) {
    return chunked_ws(d, plan, beam_chunk, false, bytes);
}

int prism_probe_outputs_chunked(const prism_smatrix_desc* d, const void* S, const prism_probe_plan* plan,
                                const void* plan_dev, int32_t precision, int32_t beam_chunk, float* out, float* out4d,
                                void* ws, size_t ws_bytes, void* stream) {
    return synth_chunked(d, S, plan, plan_dev, precision, beam_chunk, out, out4d, ws, ws_bytes, as_stream(stream),
                         nullptr, false);
}

// ------------------------------------------------------------ diagnostics --
__global__ __launch_bounds__(256) void k_copy16(const float4* __restrict__ src, float4* __restrict__ dst,
                                                size_t n) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

int prism_device_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst || bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16)
        return fail(PRISM_E_INVAL, "copy: NULL, misaligned or not a multiple of 16 bytes");
    const uintptr_t s0 = (uintptr_t)src, d0 = (uintptr_t)dst;
    if (s0 < d0 + bytes && d0 < s0 + bytes) return fail(PRISM_E_INVAL, "copy: overlapping buffers");
    const size_t n = bytes / 16;
    if (n == 0) return PRISM_OK;
    if ((n + 255) / 256 > 0x7fffffffu) return fail(PRISM_E_INVAL, "copy: too large");
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, as_stream(stream),
                       static_cast<const float4*>(src), static_cast<float4*>(dst), n);
    HIP_TRY(hipGetLastError());
    return PRISM_OK;
}

int prism_timing_enable(int32_t enable) {
    t_timing = enable != 0;
    return PRISM_OK;
}

int prism_timing_reset(void) {
    for (auto& r : t_pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    t_pending.clear();
    for (int i = 0; i < PRISM_TIMING_CLASSES; ++i) {
        t_total_ms[i] = 0.0;
        t_count[i] = 0;
    }
    return PRISM_OK;
}

int prism_timing_read(int32_t cls, double* total_ms, int64_t* launches) {
    if (cls < 0 || cls >= PRISM_TIMING_CLASSES || !total_ms || !launches)
        return fail(PRISM_E_INVAL, "timing: invalid argument");
    for (auto& r : t_pending) {
        float ms = 0.f;
        HIP_TRY(hipEventSynchronize(r.b));
        HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        t_total_ms[r.cls] += ms;
        t_count[r.cls] += 1;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    t_pending.clear();
    *total_ms = t_total_ms[cls];
    *launches = t_count[cls];
    return PRISM_OK;
}

}  // extern "C"
