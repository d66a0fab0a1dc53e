// Smooth particle-mesh Ewald: the reciprocal-space part that completes the real-space Ewald
// forces when the paper's runs use PME (section II-C; the PME spread / solve / gather kernels
// of Fig. 2).  The paper gives no algorithm; this follows the standard smooth-PME construction
// (cardinal B-spline interpolation of the charges, FFT convolution with the Ewald kernel):
//
//   u_i = K_a x_i,a / L_a (scaled coordinates), charges spread onto the K1 x K2 x K3 grid with
//   weights M_n(u_i,a - k_a) per axis (cardinal B-splines of order n, periodic in k);
//   phi = unnormalised inverse FFT of G(m) FFT(Q)(m), with
//   G(m) = fC / (pi V) exp(-pi^2 |m|^2 / beta^2) / |m|^2 |b1|^2 |b2|^2 |b3|^2 (G(0) = 0),
//   |b_a(m)|^-2 = |sum_{k=0}^{n-2} M_n(k + 1) exp(2 pi i m k / K_a)|^2;
//   E_rec = 1/2 sum_m G(m) |FFT(Q)(m)|^2, F_i = -q_i sum over the atom's grid points of
//   grad(weights) phi.
//
// MI355X layout.  The grid is cut into tiles of about 8^3 points; the atoms are binned by the
// tile of their own grid cell (counts, one-block scan) and placed in tile order with their
// coordinates and charge.  The spread runs one workgroup per tile: it lists the atoms of its own
// and the next tile along each axis that reach its points, computes their FP64 spline weights into
// LDS, accumulates their contributions with FP64 LDS atomics and stores the finished tile with
// plain coalesced writes, so the grid needs no clearing and sees no global atomics (every point
// has one owner).  The gather runs one workgroup per tile as well: it stages the tile's potential
// plus a halo of n - 1 points below it and the spline weights and derivatives of its atoms in LDS,
// and gives each atom n^2 lanes, one per grid row, reduced in a fixed order (deterministic forces,
// FP64 sums, FP32 output).  The grid and both FFTs are FP64 (hipFFT, D2Z / Z2D); the solve runs
// over the half-complex grid and keeps per-block FP64 energy partials that one block adds in a
// fixed order.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>
#include <string>
#include <vector>

#include "nb.h"

#define NB_PME_BLOCK 256
#define NB_PME_MAX_ORDER 8
#define NB_PME_TILE 8
#define NB_PME_SCAN 1024

struct nb_pme {
    hipStream_t stream = nullptr;
    int device = 0;
    int natoms = 0, order = 0;
    int K[3] = {0, 0, 0};
    double L[3] = {0, 0, 0};
    double beta = 0, fc = 0;
    size_t nreal = 0, ncplx = 0;
    double *grid = nullptr;        // [K1][K2][K3] charges, then the potential phi
    double2 *cgrid = nullptr;      // [K1][K2][K3/2 + 1] transform
    double *infl = nullptr;        // [K1][K2][K3/2 + 1] G(m)
    double *part = nullptr;        // energy partials of the solve blocks
    int nsolve_blocks = 0;
    // tiles: nt[a] per axis, tile t covers points t K / nt .. (t + 1) K / nt - 1 (at least
    // order - 1 and at most max(NB_PME_TILE, 2 order - 3) points)
    int nt[3] = {1, 1, 1};
    int ntiles = 0, tmax[3] = {0, 0, 0};
    size_t lds_spread = 0, lds_gather = 0;   // dynamic LDS bytes of the spread and gather
    int *tcount = nullptr;         // [ntiles] atoms per tile (zero between calls)
    int *toff = nullptr;           // [ntiles + 1] first atom of each tile in tatoms
    int4 *abase = nullptr;         // [natoms] own grid cell (k1, k2, k3) and tile of each atom
    int *arank = nullptr;          // [natoms] rank of the atom within its tile
    // atoms in tile order: index, cell, coordinates and charge
    int *sidx = nullptr;
    int4 *sbase = nullptr;
    float4 *sxq = nullptr;
    hipfftHandle fwd = 0, bwd = 0;
    bool have_fwd = false, have_bwd = false;
    std::string err;
};

namespace {

thread_local std::string g_pme_error;

int pfail(nb_pme *p, int code, const std::string &msg) {
    if (p) p->err = msg;
    else g_pme_error = msg;
    return code;
}

// Cardinal B-spline weights M_n(w + j), j = 0 .. n-1, for w in [0, 1), and their derivatives
// dM_n(w + j) / dx = M_{n-1}(w + j) - M_{n-1}(w + j - 1), by the recursion
// M_k(x) = x / (k-1) M_{k-1}(x) + (k - x) / (k-1) M_{k-1}(x - 1), evaluated on the n points at
// once and unrolled for the order N.
template <int N>
__device__ __forceinline__ void pme_bspline(double w, double (&val)[N], double (&der)[N]) {
    double m[N];
    m[0] = w;          // M_2(w)
    m[1] = 1.0 - w;    // M_2(w + 1)
#pragma unroll
    for (int j = 2; j < N; ++j) m[j] = 0.0;
    // m[j] holds M_k(w + j) for j = 0 .. k-1 (zero beyond)
#pragma unroll
    for (int k = 3; k <= N; ++k) {
        if (k == N) {
#pragma unroll
            for (int j = 0; j < N; ++j) der[j] = m[j] - (j > 0 ? m[j - 1] : 0.0);
        }
        constexpr double one = 1.0;
        const double inv = one / (k - 1);
#pragma unroll
        for (int j = k - 1; j >= 0; --j) {
            const double x = w + j;
            const double lo = j > 0 ? (k - x) * m[j - 1] : 0.0;
            m[j] = (x * m[j] + lo) * inv;
        }
    }
#pragma unroll
    for (int j = 0; j < N; ++j) val[j] = m[j];
}

// Own grid cell of a coordinate along one axis: k = floor(K x / L) wrapped into 0 .. K-1, and the
// fractional part w of K x / L (the spline argument).
__device__ __forceinline__ int pme_cell(float xa, double La, int Ka, double &w) {
    const double u = (double)xa / La * Ka;
    const double fl = floor(u);
    w = u - fl;
    int c = (int)fl % Ka;
    return c + (c < 0 ? Ka : 0);
}

// Binning: each atom's own grid cell, the tile holding it and the atom's rank within the tile.
// A block first ranks its atoms per tile in an LDS hash table (tile -> count), then adds each
// table entry to the global tile count with one atomic, whose old value is the entry's base;
// the tile counts start at zero.
#define NB_PME_HASH (2 * NB_PME_BLOCK)
__global__ void __launch_bounds__(NB_PME_BLOCK) k_pme_bin(int natoms, int K1, int K2, int K3, int nt1, int nt2,
                                                           int nt3, double L1, double L2, double L3,
                                                           const float *__restrict__ x,
                                                           int4 *__restrict__ abase, int *__restrict__ arank,
                                                           int *__restrict__ tcount) {
    __shared__ int hkey[NB_PME_HASH], hcnt[NB_PME_HASH];
    for (int h = threadIdx.x; h < NB_PME_HASH; h += NB_PME_BLOCK) {
        hkey[h] = -1;
        hcnt[h] = 0;
    }
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < natoms;
    int slot = 0, lr = 0;
    if (live) {
        double w;
        const int c1 = pme_cell(x[3 * i], L1, K1, w);
        const int c2 = pme_cell(x[3 * i + 1], L2, K2, w);
        const int c3 = pme_cell(x[3 * i + 2], L3, K3, w);
        const int u1 = ((c1 + 1) * nt1 - 1) / K1, u2 = ((c2 + 1) * nt2 - 1) / K2, u3 = ((c3 + 1) * nt3 - 1) / K3;
        const int tile = (u1 * nt2 + u2) * nt3 + u3;
        abase[i] = make_int4(c1, c2, c3, tile);
        // open addressing; the table has twice as many entries as the block has atoms
        slot = (int)(((unsigned)tile * 2654435761u) >> 23) & (NB_PME_HASH - 1);
        for (;;) {
            const int old = atomicCAS(&hkey[slot], -1, tile);
            if (old == -1 || old == tile) break;
            slot = (slot + 1) & (NB_PME_HASH - 1);
        }
        lr = atomicAdd(&hcnt[slot], 1);
    }
    __syncthreads();
    for (int h = threadIdx.x; h < NB_PME_HASH; h += NB_PME_BLOCK) {
        const int k = hkey[h];
        if (k >= 0) hcnt[h] = atomicAdd(tcount + k, hcnt[h]);
    }
    __syncthreads();
    if (live) arank[i] = hcnt[slot] + lr;
}

// Exclusive scan of the tile counts into toff (toff[n] = natoms); the counts are reset to zero
// for the next call.  One block; each thread scans a contiguous run.
__global__ void __launch_bounds__(NB_PME_SCAN) k_pme_scan(int n, int *__restrict__ cnt, int *__restrict__ off) {
    __shared__ int ws[NB_PME_SCAN / 64];
    const int per = (n + NB_PME_SCAN - 1) / NB_PME_SCAN;
    const int b = min(n, (int)threadIdx.x * per), e = min(n, b + per);
    int sum = 0;
    for (int i = b; i < e; ++i) sum += cnt[i];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    if (w == 0) {
        int v = lane < NB_PME_SCAN / 64 ? ws[lane] : 0;
#pragma unroll
        for (int o = 1; o < NB_PME_SCAN / 64; o <<= 1) {
            const int y = __shfl_up(v, o, 64);
            if (lane >= o) v += y;
        }
        if (lane < NB_PME_SCAN / 64) ws[lane] = v;
    }
    __syncthreads();
    int run = inc - sum + (w > 0 ? ws[w - 1] : 0);
    for (int i = b; i < e; ++i) {
        const int c = cnt[i];
        off[i] = run;
        run += c;
        cnt[i] = 0;
    }
    if (threadIdx.x == NB_PME_SCAN - 1) off[n] = run;
}

// Placement in tile order: slot c = toff[tile] + rank receives the atom index, its cell and its
// coordinates with its charge (x, y, z, q); the spread and the gather compute the spline data of
// the atoms they stage from these.
__global__ void __launch_bounds__(NB_PME_BLOCK) k_pme_place(int natoms, const float *__restrict__ x,
                                                             const float *__restrict__ q,
                                                             const int4 *__restrict__ abase,
                                                             const int *__restrict__ arank,
                                                             const int *__restrict__ toff,
                                                             int *__restrict__ sidx, int4 *__restrict__ sbase,
                                                             float4 *__restrict__ sxq) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= natoms) return;
    const int4 kb = abase[i];
    const int c = toff[kb.w] + arank[i];
    sidx[c] = i;
    sbase[c] = kb;
    sxq[c] = make_float4(x[3 * i], x[3 * i + 1], x[3 * i + 2], q[i]);
}

// Lanes of a wave: N^2 per atom, lane (j2, j3) with j3 fastest, so that the N^2 lanes of an atom
// cover N rows of N consecutive grid points along the third axis and loop over the first; a
// wave holds 64 / N^2 atoms (4 for order 4, one for orders 6 and 8).
template <int N>
struct pme_lanes {
    static constexpr int R = N * N;
    static constexpr int APW = 64 / R;
    int slot, j2, j3;
    __device__ pme_lanes(int lane) : slot(lane / R), j2((lane % R) / N), j3(lane % N) {}
};

// First point and extent of tile t of nt along an axis of K points.
struct pme_span {
    int s, z;
    __device__ pme_span(int t, int nt, int K) : s(t * K / nt), z((t + 1) * K / nt - t * K / nt) {}
};

// Candidates tested per filter pass and hits staged per spread pass (and atoms per pass of the
// gather).
template <int N>
struct pme_chunk {
    static constexpr int FILTER = 4 * NB_PME_BLOCK;
    static constexpr int SPREAD = N == 4 ? 256 : 128;
    static constexpr int GATHER = N == 8 ? 32 : 64;
};

// Decomposition of a running index p = (l1 h2 + l2) h3 + l3 that advances by a fixed step without
// divisions (one division pair at the start).
struct pme_walk {
    int l1, l2, l3, d1, d2, d3, h2, h3;
    __device__ pme_walk(int p, int step, int h2_, int h3_) : h2(h2_), h3(h3_) {
        const int hh = h2 * h3;
        l1 = p / hh;
        l2 = (p - l1 * hh) / h3;
        l3 = p - l1 * hh - l2 * h3;
        d1 = step / hh;
        d2 = (step - d1 * hh) / h3;
        d3 = step - d1 * hh - d2 * h3;
    }
    __device__ void next() {
        l3 += d3;
        const int c3 = l3 >= h3;
        l3 -= c3 ? h3 : 0;
        l2 += d2 + c3;
        const int c2 = l2 >= h2;
        l2 -= c2 ? h2 : 0;
        l1 += d1 + c2;
    }
};

// One workgroup per tile.  Atom a touches the points k_a - j, j = 0 .. N-1 (wrapped) along each
// axis; with tiles of at least N - 1 points those lie in the atom's own tile and the one below,
// so a tile collects the atoms of itself and of the next tile along each axis (2^3 source tiles,
// fewer where an axis has one or two tiles).  A filter pass tests up to FILTER candidates (loads
// issued together) and lists those that reach the tile; the listed atoms' charge-scaled weights
// are then staged in LDS, SPREAD at a time, and the waves add their contributions to the tile
// with LDS atomics.
template <int N>
__global__ void __launch_bounds__(NB_PME_BLOCK) k_pme_spread(int K1, int K2, int K3, int nt1, int nt2, int nt3,
                                                              double L1, double L2, double L3,
                                                              const int4 *__restrict__ sbase,
                                                              const float4 *__restrict__ sxq,
                                                              const int *__restrict__ toff,
                                                              double *__restrict__ grid) {
    constexpr int CF = pme_chunk<N>::FILTER, CH = pme_chunk<N>::SPREAD;
    constexpr int UF = CF / NB_PME_BLOCK, APW = pme_lanes<N>::APW, WAVES = NB_PME_BLOCK / 64;
    constexpr int WS = 3 * N + 1;                  // staged doubles per atom (odd: fewer bank conflicts)
    extern __shared__ double lg[];                 // tile points, then CH x WS weights
    __shared__ int2 hit[CF];                       // listed atoms: slot, packed local cell
    __shared__ int nhit, csrc[9], tsrc[8];
    const int t = blockIdx.x;
    const int t3 = t % nt3, t2 = (t / nt3) % nt2, t1 = t / (nt3 * nt2);
    const pme_span a1(t1, nt1, K1), a2(t2, nt2, K2), a3(t3, nt3, K3);
    const int np = a1.z * a2.z * a3.z;
    double *wt = lg + np;
    for (int p = threadIdx.x; p < np; p += NB_PME_BLOCK) lg[p] = 0.0;
    // candidate ranges of the source tiles, as a running count over them
    const int n1 = nt1 > 1 ? 2 : 1, n2 = nt2 > 1 ? 2 : 1, n3 = nt3 > 1 ? 2 : 1, ns = n1 * n2 * n3;
    if (threadIdx.x < 64) {   // lanes 0 .. ns-1 read one source tile each; a scan gives the starts
        const int d = threadIdx.x;
        int cnt = 0;
        if (d < ns) {
            int u1 = t1 + d / (n2 * n3), u2 = t2 + (d / n3) % n2, u3 = t3 + d % n3;
            u1 -= u1 >= nt1 ? nt1 : 0;
            u2 -= u2 >= nt2 ? nt2 : 0;
            u3 -= u3 >= nt3 ? nt3 : 0;
            const int ts = (u1 * nt2 + u2) * nt3 + u3;
            const int b = toff[ts];
            cnt = toff[ts + 1] - b;
            tsrc[d] = b;
        }
        int inc = cnt;
#pragma unroll
        for (int o = 1; o < 8; o <<= 1) {
            const int y = __shfl_up(inc, o, 64);
            if (d >= o) inc += y;
        }
        if (d < ns) csrc[d + 1] = inc;
        if (d == 0) {
            csrc[0] = 0;
            nhit = 0;
        }
    }
    __syncthreads();
    const int total = csrc[ns];
    const pme_lanes<N> ln(threadIdx.x & 63);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int f0 = 0; f0 < total; f0 += CF) {
        // filter: UF candidates per thread, loads first
        int4 kb[UF];
        int cs[UF];
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            const int r = f0 + u * NB_PME_BLOCK + (int)threadIdx.x;
            cs[u] = -1;
            if (r < total) {
                int d = 0;
#pragma unroll
                for (int k = 1; k < 8; ++k) d += (k < ns && r >= csrc[k]) ? 1 : 0;
                cs[u] = tsrc[d] + (r - csrc[d]);
                kb[u] = sbase[cs[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            // local index of the atom's cell relative to the tile start; the atom reaches the tile
            // along an axis if some k - j, j < N, falls in it
            bool h = false;
            int pk = 0;
            if (cs[u] >= 0) {
                int l1 = kb[u].x - a1.s, l2 = kb[u].y - a2.s, l3 = kb[u].z - a3.s;
                l1 += l1 < 0 ? K1 : 0;
                l2 += l2 < 0 ? K2 : 0;
                l3 += l3 < 0 ? K3 : 0;
                h = (l1 < a1.z + N - 1) && (l2 < a2.z + N - 1) && (l3 < a3.z + N - 1);
                pk = h ? (l1 << 20) | (l2 << 10) | l3 : 0;   // l < tile extent + N - 1 < 1024
            }
            const uint64_t m = __ballot(h);
            int base = 0;
            if (lane == 0 && m) base = atomicAdd(&nhit, __popcll(m));
            base = __shfl(base, 0, 64);
            if (h) hit[base + __popcll(m & ((1ull << lane) - 1ull))] = make_int2(cs[u], pk);
        }
        __syncthreads();
        const int nh = nhit;
        for (int h0 = 0; h0 < nh; h0 += CH) {
            const int nc = min(CH, nh - h0);
            if ((int)threadIdx.x < nc) {   // weights of the listed atom, the first axis scaled by q
                const float4 p = sxq[hit[h0 + threadIdx.x].x];
                double *w = wt + threadIdx.x * WS;
                const float xa[3] = {p.x, p.y, p.z};
                const double La[3] = {L1, L2, L3};
                const int Ka[3] = {K1, K2, K3};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    double u, v[N], d[N];
                    pme_cell(xa[a], La[a], Ka[a], u);
                    pme_bspline<N>(u, v, d);
#pragma unroll
                    for (int j = 0; j < N; ++j) w[a * N + j] = a == 0 ? (double)p.w * v[j] : v[j];
                }
            }
            __syncthreads();
            for (int g = wave * APW; g < nc; g += WAVES * APW) {
                const int s = g + ln.slot;
                if (ln.slot >= APW || s >= nc) continue;
                const int pk = hit[h0 + s].y;
                // local point (l - j) wrapped: below the tile start it lands at K - ..., outside
                // the tile unless the tile spans the whole axis
                int l2 = ((pk >> 10) & 1023) - ln.j2, l3 = (pk & 1023) - ln.j3;
                l2 += l2 < 0 ? K2 : 0;
                l3 += l3 < 0 ? K3 : 0;
                if ((unsigned)l2 >= (unsigned)a2.z || (unsigned)l3 >= (unsigned)a3.z) continue;
                const double *w = wt + s * WS;
                const double w23 = w[N + ln.j2] * w[2 * N + ln.j3];
                double *row = lg + l2 * a3.z + l3;
                const int lb1 = pk >> 20;
#pragma unroll
                for (int j1 = 0; j1 < N; ++j1) {
                    int l1 = lb1 - j1;
                    l1 += l1 < 0 ? K1 : 0;
                    if ((unsigned)l1 < (unsigned)a1.z) atomicAdd(row + l1 * (a2.z * a3.z), w23 * w[j1]);
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) nhit = 0;
        __syncthreads();
    }
    pme_walk wk((int)threadIdx.x, NB_PME_BLOCK, a2.z, a3.z);
    for (int p = threadIdx.x; p < np; p += NB_PME_BLOCK, wk.next())
        grid[(unsigned)(((a1.s + wk.l1) * K2 + (a2.s + wk.l2)) * K3 + (a3.s + wk.l3))] = lg[p];   // < 2^30
}

// c(m) <- G(m) c(m) over the half-complex grid [K1][K2][K3h]; per-block partial sums of the
// energy 1/2 sum_m G |c|^2 over the full spectrum: a stored k3 other than 0 and K3/2 (even K3)
// stands for m and -m, so its weight is 1, else 1/2.
__global__ void __launch_bounds__(NB_PME_BLOCK) k_pme_solve(unsigned ncplx, unsigned K3h, unsigned k3nyq,
                                                             const double *__restrict__ infl,
                                                             double2 *__restrict__ c,
                                                             double *__restrict__ part) {
    __shared__ double s[NB_PME_BLOCK / 64];
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < ncplx) {
        const unsigned k3 = i % K3h;
        const double g = infl[i];
        const double2 z = c[i];
        e = ((k3 == 0u || k3 == k3nyq) ? 0.5 : 1.0) * g * (z.x * z.x + z.y * z.y);
        c[i] = make_double2(g * z.x, g * z.y);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x / 64] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < NB_PME_BLOCK / 64; ++k) t += s[k];
        part[blockIdx.x] = t;
    }
}

// Sum of the solve's energy partials in a fixed order, by one block (the gather's first block).
__device__ void pme_energy_sum(int nblk, const double *__restrict__ part, double *__restrict__ e) {
    __shared__ double s[NB_PME_BLOCK / 64];
    double t = 0.0;
    for (int k = threadIdx.x; k < nblk; k += NB_PME_BLOCK) t += part[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x / 64] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int k = 0; k < NB_PME_BLOCK / 64; ++k) r += s[k];
        e[0] = r;
    }
}

// One workgroup per tile: the potential on the tile and N - 1 points below it along each axis
// (wrapped) is staged in LDS, and so are the spline data of the tile's atoms, GATHER atoms per
// pass; each atom gets N^2 lanes (same layout as the spread), each summing its N points along the
// first axis, and the lanes of an atom are reduced in a fixed order (deterministic forces).
template <int N>
__global__ void __launch_bounds__(NB_PME_BLOCK) k_pme_gather(int K1, int K2, int K3, int nt1, int nt2, int nt3,
                                                              double L1, double L2, double L3,
                                                              const int *__restrict__ sidx,
                                                              const int4 *__restrict__ sbase,
                                                              const float4 *__restrict__ sxq,
                                                              const int *__restrict__ toff,
                                                              const double *__restrict__ phi,
                                                              float *__restrict__ f, int nblk,
                                                              const double *__restrict__ part,
                                                              double *__restrict__ e) {
    constexpr int CH = pme_chunk<N>::GATHER, R = pme_lanes<N>::R, APW = pme_lanes<N>::APW;
    constexpr int WAVES = NB_PME_BLOCK / 64;
    constexpr int RED = APW > 1 ? R : 64;   // reduction width, a power of two
    constexpr int SD = 6 * N + 1;           // staged doubles per atom (odd: fewer bank conflicts)
    extern __shared__ double lp[];          // staged potential, then CH x SD spline data
    __shared__ int4 ab[CH];                 // cells, charges and indices of the staged atoms
    __shared__ float aq[CH];
    __shared__ int ai[CH];
    const int t = blockIdx.x;
    const int t3 = t % nt3, t2 = (t / nt3) % nt2, t1 = t / (nt3 * nt2);
    const pme_span a1(t1, nt1, K1), a2(t2, nt2, K2), a3(t3, nt3, K3);
    // staged box: points s_a - (N - 1) .. s_a + z_a - 1 along each axis
    if (t == 0) pme_energy_sum(nblk, part, e);
    const int c0 = toff[t], c1 = toff[t + 1];
    if (c0 == c1) return;   // no atoms in this tile
    const int h1 = a1.z + N - 1, h2 = a2.z + N - 1, h3 = a3.z + N - 1, hh = h2 * h3;
    double *sd = lp + h1 * hh;
    {
        // GU loads per thread issued together, then stored
        constexpr int GU = 8;
        const int nbox = h1 * hh;
        pme_walk wk((int)threadIdx.x, NB_PME_BLOCK, h2, h3);
        for (int p0 = 0; p0 < nbox; p0 += GU * NB_PME_BLOCK) {
            double v[GU];
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int p = p0 + u * NB_PME_BLOCK + (int)threadIdx.x;
                if (p < nbox) {
                    int k1 = a1.s - (N - 1) + wk.l1, k2 = a2.s - (N - 1) + wk.l2, k3 = a3.s - (N - 1) + wk.l3;
                    k1 += k1 < 0 ? K1 : 0;
                    k2 += k2 < 0 ? K2 : 0;
                    k3 += k3 < 0 ? K3 : 0;
                    v[u] = phi[(unsigned)((k1 * K2 + k2) * K3 + k3)];   // K1 K2 K3 <= 2^30
                }
                wk.next();
            }
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int p = p0 + u * NB_PME_BLOCK + (int)threadIdx.x;
                if (p < nbox) lp[p] = v[u];
            }
        }
    }
    const pme_lanes<N> ln(threadIdx.x & 63);
    const int wave = threadIdx.x >> 6;
    for (int cb = c0; cb < c1; cb += CH) {
        const int nc = min(CH, c1 - cb);
        if (cb != c0) __syncthreads();   // previous pass done with the staged atoms
        // spline weights and derivatives of the staged atoms, one (atom, axis) per thread
        for (int e = threadIdx.x; e < 3 * CH; e += NB_PME_BLOCK) {
            const int a = e % CH, ax = e / CH;
            if (a < nc) {
                const float4 p = sxq[cb + a];
                const float xa = ax == 0 ? p.x : (ax == 1 ? p.y : p.z);
                const double La = ax == 0 ? L1 : (ax == 1 ? L2 : L3);
                const int Ka = ax == 0 ? K1 : (ax == 1 ? K2 : K3);
                double u, v[N], d[N];
                pme_cell(xa, La, Ka, u);
                pme_bspline<N>(u, v, d);
                double *th = sd + a * SD;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    th[ax * N + j] = v[j];
                    th[3 * N + ax * N + j] = d[j];
                }
            }
        }
        if ((int)threadIdx.x < nc) {
            ab[threadIdx.x] = sbase[cb + threadIdx.x];
            aq[threadIdx.x] = sxq[cb + threadIdx.x].w;
            ai[threadIdx.x] = sidx[cb + threadIdx.x];
        }
        __syncthreads();   // staged potential and atoms ready
        for (int g = wave * APW; g < nc; g += WAVES * APW) {   // wave-uniform trip count
            const int s = g + ln.slot;
            const bool live = ln.slot < APW && s < nc;
            double gx = 0.0, gy = 0.0, gz = 0.0;
            if (live) {
                const int4 kb = ab[s];
                const double *th = sd + s * SD;
                const double *dh = th + 3 * N;
                // local coordinates in the staged box: k_a - j - (s_a - (N - 1)), in 0 .. h_a - 1
                // (the atom's own cell k_a lies in this tile)
                const int l2 = kb.y - a2.s + (N - 1) - ln.j2;
                const int l3 = kb.z - a3.s + (N - 1) - ln.j3;
                const int l1 = kb.x - a1.s + (N - 1);
                const double *col = lp + l2 * h3 + l3;
                double sa = 0.0, sb = 0.0;
#pragma unroll
                for (int j1 = 0; j1 < N; ++j1) {
                    const double p = col[(l1 - j1) * hh];
                    sa += dh[j1] * p;
                    sb += th[j1] * p;
                }
                const double v2 = th[N + ln.j2], d2 = dh[N + ln.j2];
                const double v3 = th[2 * N + ln.j3], d3 = dh[2 * N + ln.j3];
                gx = sa * v2 * v3;
                gy = sb * d2 * v3;
                gz = sb * v2 * d3;
            }
#pragma unroll
            for (int o = RED / 2; o > 0; o >>= 1) {
                gx += __shfl_xor(gx, o, 64);
                gy += __shfl_xor(gy, o, 64);
                gz += __shfl_xor(gz, o, 64);
            }
            if (live && (threadIdx.x & (RED - 1)) == 0) {
                const double qi = aq[s];
                const int i = ai[s];
                f[3 * i] = (float)(-qi * gx * K1 / L1);
                f[3 * i + 1] = (float)(-qi * gy * K2 / L2);
                f[3 * i + 2] = (float)(-qi * gz * K3 / L3);
            }
        }
    }
}

// Host side: cardinal B-spline values M_n(k), k = 1 .. n-1, and the moduli |b(m)|^2.
std::vector<double> bspline_int(int n) {
    // M_n at the integers 0 .. n by the same recursion, from M_2(1) = 1
    std::vector<double> m(n + 1, 0.0);
    m[1] = 1.0;
    for (int k = 3; k <= n; ++k) {
        std::vector<double> nm(n + 1, 0.0);
        for (int x = 1; x < k; ++x) nm[x] = (x * m[x] + (k - x) * m[x - 1]) / (k - 1);
        m = nm;
    }
    return m;
}

std::vector<double> bmod2(int K, int n) {
    const std::vector<double> M = bspline_int(n);
    std::vector<double> out(K);
    for (int m = 0; m < K; ++m) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k <= n - 2; ++k) {
            const double ph = 2.0 * M_PI * m * k / K;
            re += M[k + 1] * cos(ph);
            im += M[k + 1] * sin(ph);
        }
        out[m] = 1.0 / (re * re + im * im);
    }
    return out;
}

template <typename T>
int palloc(nb_pme *p, T **ptr, size_t count, const char *what) {
    if (hipMalloc((void **)ptr, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) {
        *ptr = nullptr;
        return pfail(p, NB_ERR_OOM, std::string("hipMalloc ") + what);
    }
    return NB_OK;
}

void pme_free(nb_pme *p) {
    if (p->have_fwd) hipfftDestroy(p->fwd);
    if (p->have_bwd) hipfftDestroy(p->bwd);
    void *bufs[] = {p->grid, p->cgrid, p->infl, p->part, p->tcount, p->toff, p->abase, p->arank,
                    p->sidx, p->sbase, p->sxq};
    for (void *b : bufs)
        if (b) hipFree(b);
}

}  // namespace

extern "C" {

int nb_pme_setup(nb_pme **out, const nb_pme_params *prm, void *stream) {
    if (!out || !prm) return pfail(nullptr, NB_ERR_ARG, "NULL argument");
    *out = nullptr;
    for (int a = 0; a < 3; ++a) {
        if (!(std::isfinite(prm->box[a]) && prm->box[a] > 0.0)) return pfail(nullptr, NB_ERR_ARG, "box edges must be finite and > 0");
        if (prm->grid[a] < 2 * prm->order || prm->grid[a] > 1024) return pfail(nullptr, NB_ERR_ARG, "grid sizes must be in 2*order .. 1024");
    }
    if (prm->order < 4 || prm->order > NB_PME_MAX_ORDER || (prm->order & 1))
        return pfail(nullptr, NB_ERR_ARG, "order must be 4, 6 or 8");
    if (!(std::isfinite(prm->ewald_beta) && prm->ewald_beta > 0.0)) return pfail(nullptr, NB_ERR_ARG, "ewald_beta must be > 0");
    if (!(std::isfinite(prm->coulomb_const) && prm->coulomb_const > 0.0)) return pfail(nullptr, NB_ERR_ARG, "coulomb_const must be > 0");
    if (prm->natoms < 1 || prm->natoms > (1 << 27)) return pfail(nullptr, NB_ERR_ARG, "natoms must be in 1..2^27");
    nb_pme *p = new nb_pme();
    p->stream = (hipStream_t)stream;
    hipGetDevice(&p->device);
    p->natoms = prm->natoms;
    p->order = prm->order;
    for (int a = 0; a < 3; ++a) {
        p->K[a] = prm->grid[a];
        p->L[a] = prm->box[a];
    }
    p->beta = prm->ewald_beta;
    p->fc = prm->coulomb_const;
    const int K1 = p->K[0], K2 = p->K[1], K3 = p->K[2], K3h = K3 / 2 + 1;
    p->nreal = (size_t)K1 * K2 * K3;
    p->ncplx = (size_t)K1 * K2 * K3h;
    p->nsolve_blocks = (int)((p->ncplx + NB_PME_BLOCK - 1) / NB_PME_BLOCK);
    // tiles of about NB_PME_TILE points, never fewer than order - 1 (so that an atom's points lie
    // in its own tile and the one below)
    for (int a = 0; a < 3; ++a) {
        const int K = p->K[a];
        p->nt[a] = std::max(1, std::min((K + NB_PME_TILE - 1) / NB_PME_TILE, K / (p->order - 1)));
        p->tmax[a] = (K + p->nt[a] - 1) / p->nt[a];
    }
    p->ntiles = p->nt[0] * p->nt[1] * p->nt[2];
    {
        const int n = p->order, chs = n == 4 ? 256 : 128, chg = n == 8 ? 32 : 64;   // atoms per pass
        p->lds_spread = sizeof(double) * ((size_t)p->tmax[0] * p->tmax[1] * p->tmax[2] + (size_t)chs * (3 * n + 1));
        p->lds_gather = sizeof(double) * ((size_t)(p->tmax[0] + n - 1) * (p->tmax[1] + n - 1) * (p->tmax[2] + n - 1) +
                                          (size_t)chg * (6 * n + 1));
        // 64 KiB per workgroup, less the static arrays (spread: candidate list of 8 KiB)
        if (p->lds_spread > 65536 - 8448 || p->lds_gather > 65536 - 2048) {
            delete p;
            return pfail(nullptr, NB_ERR_ARG, "grid tiles exceed the LDS of a workgroup");
        }
    }
    int r;
    if ((r = palloc(p, &p->tcount, (size_t)p->ntiles, "tile counts")) != NB_OK ||
        (r = palloc(p, &p->toff, (size_t)p->ntiles + 1, "tile offsets")) != NB_OK ||
        (r = palloc(p, &p->abase, (size_t)p->natoms, "atom cells")) != NB_OK ||
        (r = palloc(p, &p->arank, (size_t)p->natoms, "atom ranks")) != NB_OK ||
        (r = palloc(p, &p->sidx, (size_t)p->natoms, "sorted atoms")) != NB_OK ||
        (r = palloc(p, &p->sbase, (size_t)p->natoms, "sorted cells")) != NB_OK ||
        (r = palloc(p, &p->sxq, (size_t)p->natoms, "sorted coordinates")) != NB_OK ||
        (r = palloc(p, &p->grid, p->nreal, "grid")) != NB_OK ||
        (r = palloc(p, &p->cgrid, p->ncplx, "transform")) != NB_OK ||
        (r = palloc(p, &p->infl, p->ncplx, "influence function")) != NB_OK ||
        (r = palloc(p, &p->part, (size_t)p->nsolve_blocks, "energy partials")) != NB_OK) {
        g_pme_error = p->err;
        pme_free(p);
        delete p;
        return r;
    }
    // influence function G(m)
    const std::vector<double> b1 = bmod2(K1, p->order), b2 = bmod2(K2, p->order), b3 = bmod2(K3, p->order);
    const double V = p->L[0] * p->L[1] * p->L[2];
    std::vector<double> g(p->ncplx);
    for (int k1 = 0; k1 < K1; ++k1) {
        const double m1 = (k1 <= K1 / 2 ? k1 : k1 - K1) / p->L[0];
        for (int k2 = 0; k2 < K2; ++k2) {
            const double m2 = (k2 <= K2 / 2 ? k2 : k2 - K2) / p->L[1];
            for (int k3 = 0; k3 < K3h; ++k3) {
                const double m3 = k3 / p->L[2];
                const double msq = m1 * m1 + m2 * m2 + m3 * m3;
                const size_t i = ((size_t)k1 * K2 + k2) * K3h + k3;
                g[i] = msq > 0.0 ? p->fc / (M_PI * V) * exp(-M_PI * M_PI * msq / (p->beta * p->beta)) / msq *
                                       b1[k1] * b2[k2] * b3[k3]
                                 : 0.0;
            }
        }
    }
    hipError_t e = hipMemcpy(p->infl, g.data(), sizeof(double) * g.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(p->tcount, 0, sizeof(int) * p->ntiles);
    if (e != hipSuccess) {
        pme_free(p);
        delete p;
        return pfail(nullptr, NB_ERR_HIP, std::string("upload influence function: ") + hipGetErrorString(e));
    }
    if (hipfftPlan3d(&p->fwd, K1, K2, K3, HIPFFT_D2Z) != HIPFFT_SUCCESS ||
        !(p->have_fwd = true) || hipfftPlan3d(&p->bwd, K1, K2, K3, HIPFFT_Z2D) != HIPFFT_SUCCESS) {
        pme_free(p);
        delete p;
        return pfail(nullptr, NB_ERR_HIP, "hipfftPlan3d");
    }
    p->have_bwd = true;
    if (hipfftSetStream(p->fwd, p->stream) != HIPFFT_SUCCESS || hipfftSetStream(p->bwd, p->stream) != HIPFFT_SUCCESS) {
        pme_free(p);
        delete p;
        return pfail(nullptr, NB_ERR_HIP, "hipfftSetStream");
    }
    *out = p;
    return NB_OK;
}

int nb_pme_forces(nb_pme *p, const float *x, const float *q, float *f, double *e) {
    if (!p || !x || !q || !f || !e) return pfail(p, NB_ERR_ARG, "NULL argument");
    hipSetDevice(p->device);
    const int K1 = p->K[0], K2 = p->K[1], K3 = p->K[2];
    const unsigned ab = (unsigned)((p->natoms + NB_PME_BLOCK - 1) / NB_PME_BLOCK);
    const int n = p->order;
    const size_t lds_spread = p->lds_spread, lds_gather = p->lds_gather;
    hipLaunchKernelGGL(k_pme_bin, dim3(ab), dim3(NB_PME_BLOCK), 0, p->stream, p->natoms, K1, K2, K3, p->nt[0],
                       p->nt[1], p->nt[2], p->L[0], p->L[1], p->L[2], x, p->abase, p->arank, p->tcount);
    hipLaunchKernelGGL(k_pme_scan, dim3(1), dim3(NB_PME_SCAN), 0, p->stream, p->ntiles, p->tcount, p->toff);
#define NB_PME_SPREAD(N)                                                                                      \
    hipLaunchKernelGGL(k_pme_spread<N>, dim3(p->ntiles), dim3(NB_PME_BLOCK), lds_spread, p->stream, K1, K2, K3, \
                       p->nt[0], p->nt[1], p->nt[2], p->L[0], p->L[1], p->L[2], p->sbase, p->sxq, p->toff, p->grid)
    hipLaunchKernelGGL(k_pme_place, dim3(ab), dim3(NB_PME_BLOCK), 0, p->stream, p->natoms, x, q, p->abase,
                       p->arank, p->toff, p->sidx, p->sbase, p->sxq);
    if (n == 4) NB_PME_SPREAD(4);
    else if (n == 6) NB_PME_SPREAD(6);
    else NB_PME_SPREAD(8);
#undef NB_PME_SPREAD
    if (hipGetLastError() != hipSuccess) return pfail(p, NB_ERR_HIP, "spread launch");
    if (hipfftExecD2Z(p->fwd, (hipfftDoubleReal *)p->grid, (hipfftDoubleComplex *)p->cgrid) != HIPFFT_SUCCESS)
        return pfail(p, NB_ERR_HIP, "forward FFT");
    hipLaunchKernelGGL(k_pme_solve, dim3(p->nsolve_blocks), dim3(NB_PME_BLOCK), 0, p->stream, (unsigned)p->ncplx,
                       (unsigned)(K3 / 2 + 1), (unsigned)(K3 % 2 == 0 ? K3 / 2 : 0), p->infl, p->cgrid, p->part);
    if (hipGetLastError() != hipSuccess) return pfail(p, NB_ERR_HIP, "solve launch");
    if (hipfftExecZ2D(p->bwd, (hipfftDoubleComplex *)p->cgrid, (hipfftDoubleReal *)p->grid) != HIPFFT_SUCCESS)
        return pfail(p, NB_ERR_HIP, "inverse FFT");
#define NB_PME_GATHER(N)                                                                                      \
    hipLaunchKernelGGL(k_pme_gather<N>, dim3(p->ntiles), dim3(NB_PME_BLOCK), lds_gather, p->stream, K1, K2, K3, \
                       p->nt[0], p->nt[1], p->nt[2], p->L[0], p->L[1], p->L[2], p->sidx, p->sbase, p->sxq,    \
                       p->toff, p->grid, f, p->nsolve_blocks, p->part, e)
    if (n == 4) NB_PME_GATHER(4);
    else if (n == 6) NB_PME_GATHER(6);
    else NB_PME_GATHER(8);
#undef NB_PME_GATHER
    if (hipGetLastError() != hipSuccess) return pfail(p, NB_ERR_HIP, "gather launch");
    return NB_OK;
}

const char *nb_pme_last_error(nb_pme *p) { return p ? p->err.c_str() : g_pme_error.c_str(); }

int nb_pme_destroy(nb_pme *p) {
    if (!p) return NB_OK;
    hipSetDevice(p->device);
    hipStreamSynchronize(p->stream);
    pme_free(p);
    delete p;
    return NB_OK;
}

}  // extern "C"
