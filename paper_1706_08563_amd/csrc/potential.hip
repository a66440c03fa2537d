// potential.hip -- projected potential slices ("Calculation of the Projected
// Potentials", Fig. 1a-b).  Each atom adds its species' Gaussian terms
// A/(2 pi w^2) exp(-d^2/(2 w^2)) at minimum-image distance d < rc to the slab
// that holds it.
//
// One workgroup per (16 x 16 pixel tile, slice): the slice's atoms are
// filtered against the tile's bounding box (wave-ballot compaction, so the
// list keeps atom order and the sums are deterministic), then every pixel
// accumulates the listed atoms.
#include "kernels.hpp"

namespace prism {

constexpr int WG = 256;
constexpr int PT = 16;            // tile side (pixels)
constexpr int CAP = 1024;         // listed atoms per flush

struct ListAtom { float dx, dy; int species; int pad; };

__global__ __launch_bounds__(WG) void k_potential(float* __restrict__ V, int n, int n_slices, double L,
                                                  const PotAtom* __restrict__ atoms,
                                                  const int* __restrict__ slice_start,
                                                  const PotSpecies* __restrict__ species, float rc_max) {
    __shared__ ListAtom list[CAP];
    __shared__ int wave_cnt[4];
    __shared__ int n_list;
    const int ntx = n / PT;
    const int tile = blockIdx.x;
    const int s = blockIdx.y;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const double dx = L / n;
    const double half = 0.5 * (PT - 1) * dx;
    const double cx = ((tile % ntx) * PT) * dx + half;      // tile centre
    const double cy = ((tile / ntx) * PT) * dx + half;
    const int ix = tid % PT, iy = tid / PT;
    // pixel offset from the tile centre
    const float ox = (float)(ix * dx - half), oy = (float)(iy * dx - half);
    const float Lf = (float)L, hL = 0.5f * (float)L;
    const double lim = (double)rc_max + half * 1.0000001 + 1e-9;
    float acc = 0.f;
    if (tid == 0) n_list = 0;
    __syncthreads();
    const int a0 = slice_start[s], a1 = slice_start[s + 1];
    for (int base = a0; base < a1; base += WG) {
        const int a = base + tid;
        bool near = false;
        ListAtom la{0.f, 0.f, 0, 0};
        if (a < a1) {
            PotAtom at = atoms[a];
            double ddx = at.x - cx, ddy = at.y - cy;
            ddx -= L * rint(ddx / L);
            ddy -= L * rint(ddy / L);
            double ex = fmax(fabs(ddx) - half, 0.0), ey = fmax(fabs(ddy) - half, 0.0);
            near = fabs(ddx) < lim && fabs(ddy) < lim && ex * ex + ey * ey < (double)rc_max * rc_max;
            la = ListAtom{(float)ddx, (float)ddy, at.species, 0};
        }
        unsigned long long mask = __ballot(near);
        if (lane == 0) wave_cnt[wave] = __popcll(mask);
        __syncthreads();
        int off = n_list;
        for (int w = 0; w < wave; ++w) off += wave_cnt[w];
        const int total = wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
        if (near) {
            unsigned long long lower = lane ? (mask & ((1ull << lane) - 1ull)) : 0ull;
            list[off + __popcll(lower)] = la;
        }
        __syncthreads();
        int cnt = n_list + total;
        if (cnt > CAP - WG || base + WG >= a1) {
            for (int k = 0; k < cnt; ++k) {
                ListAtom e = list[k];
                float ddx = ox - e.dx, ddy = oy - e.dy;
                ddx = ddx > hL ? ddx - Lf : (ddx < -hL ? ddx + Lf : ddx);
                ddy = ddy > hL ? ddy - Lf : (ddy < -hL ? ddy + Lf : ddy);
                float d2 = ddx * ddx + ddy * ddy;
                const PotSpecies& sp = species[e.species];
                if (d2 < sp.rc2) {
                    for (int gi = 0; gi < sp.n_gauss; ++gi) acc += sp.amp_n[gi] * expf(-d2 * sp.inv2w2[gi]);
                }
            }
            cnt = 0;
        }
        __syncthreads();
        if (tid == 0) n_list = cnt;
        __syncthreads();
    }
    const int px = (tile % ntx) * PT + ix, py = (tile / ntx) * PT + iy;
    V[((size_t)s * n + py) * n + px] = acc;
}

hipError_t launch_potential(float* V, int n, int n_slices, double L, const PotAtom* atoms, const int* slice_start,
                            const PotSpecies* species, float rc_max, hipStream_t st) {
    dim3 grid((unsigned)((n / PT) * (n / PT)), (unsigned)n_slices);
    hipLaunchKernelGGL(k_potential, grid, dim3(WG), 0, st, V, n, n_slices, L, atoms, slice_start, species, rc_max);
    return hipGetLastError();
}

}  // namespace prism
