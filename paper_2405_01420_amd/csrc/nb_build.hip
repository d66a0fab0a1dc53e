// Pair-list construction on the GPU: wrap + column binning, counting sort over columns, z-sort
// inside each column, clusters of C atoms, cluster bounding boxes, cluster-pair search under
// periodic shifts with the half-list rule, topology masks and atom-level prune.
//
// The paper names these pieces (a buffered pair list with a "list range", a prune step and
// list sorting; section III-A, the list of differences between the GROMACS versions) but
// gives no algorithm; this is a from-scratch GPU design: every stage is one kernel on the
// context's stream and nothing is read back except the overflow flag.
#include "nb_device.h"

namespace {

#define NB_BIN_LDS_MAX 12288  // columns the per-block LDS histogram of k_bin holds

// Wrap into the box, column index, rank inside the column.  With lds != 0 each block first
// counts its atoms per column in LDS and then takes one global atomic per column it touched,
// which keeps the global atomics few (atoms in input order are spatially coherent); the rank is
// the block's base in the column plus the LDS rank.  The order inside a column is arbitrary
// here: the column sort orders atoms by (z, index).
__global__ void __launch_bounds__(256) k_bin(int n, const float *__restrict__ x, nb_geom g,
                                             float4 *__restrict__ off, float *__restrict__ xbuild,
                                             int *__restrict__ col, int *__restrict__ rank,
                                             int *__restrict__ colcount, nb_meta *meta, int lds) {
    extern __shared__ int hist[];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (lds) {
        for (int k = threadIdx.x; k < g.ncol; k += blockDim.x) hist[k] = 0;
        __syncthreads();
    }
    int c = -1, lrank = 0;
    if (i < n) {
        float xv[3], o[3], w[3];
        bool fin = true;
        for (int d = 0; d < 3; ++d) {
            xv[d] = x[3 * i + d];
            xbuild[3 * i + d] = xv[d];
            if (!isfinite(xv[d])) {
                fin = false;
                xv[d] = 0.0f;
            }
        }
        if (!fin) atomicOr(&meta->flags, NB_F_BUILD_NONFINITE);
        for (int d = 0; d < 3; ++d) {
            const float L = g.L[d];
            o[d] = -floorf(xv[d] / L) * L;
            w[d] = xv[d] + o[d];
            if (w[d] < 0.0f) {
                o[d] += L;
                w[d] = xv[d] + o[d];
            }
            if (w[d] >= L) {
                o[d] -= L;
                w[d] = xv[d] + o[d];
            }
        }
        off[i] = make_float4(o[0], o[1], o[2], 0.0f);
        const int cx = min(max((int)(w[0] * g.invw[0]), 0), g.ncx - 1);
        const int cy = min(max((int)(w[1] * g.invw[1]), 0), g.ncy - 1);
        c = cy * g.ncx + cx;
        col[i] = c;
        if (lds) lrank = atomicAdd(&hist[c], 1);
        else rank[i] = atomicAdd(&colcount[c], 1);
    }
    if (lds) {
        __syncthreads();
        for (int k = threadIdx.x; k < g.ncol; k += blockDim.x) {
            const int h = hist[k];
            if (h) hist[k] = atomicAdd(&colcount[k], h);
        }
        __syncthreads();
        if (i < n) rank[i] = hist[c] + lrank;
    }
}

// Exclusive scans of column populations and of cluster counts ceil(n / C); one block of 1024
// threads, each over a contiguous run of columns: wave scans, then one thread over the waves.
__global__ void __launch_bounds__(1024) k_colscan(int ncol, int C, const int *__restrict__ colcount,
                                                   int *__restrict__ colstart, int *__restrict__ colcl,
                                                   nb_meta *meta) {
    __shared__ int wa[1024 / NB_WAVE], wb[1024 / NB_WAVE];
    const int t = threadIdx.x, lane = t & (NB_WAVE - 1), wv = t / NB_WAVE;
    const int per = (ncol + 1023) / 1024;
    const int c0 = min(ncol, t * per), c1 = min(ncol, c0 + per);
    int a = 0, b = 0, mx = 0;
    for (int c = c0; c < c1; ++c) {
        const int v = colcount[c];
        a += v;
        b += (v + C - 1) / C;
        mx = max(mx, v);
    }
    int ia = a, ib = b;
#pragma unroll
    for (int o = 1; o < NB_WAVE; o <<= 1) {
        const int va = __shfl_up(ia, o, NB_WAVE), vb = __shfl_up(ib, o, NB_WAVE);
        if (lane >= o) {
            ia += va;
            ib += vb;
        }
        mx = max(mx, __shfl_xor(mx, o, NB_WAVE));
    }
    if (lane == NB_WAVE - 1) {
        wa[wv] = ia;
        wb[wv] = ib;
    }
    __syncthreads();
    if (t == 0) {
        int ra = 0, rb = 0;
        for (int k = 0; k < 1024 / NB_WAVE; ++k) {
            const int xa = wa[k], xb = wb[k];
            wa[k] = ra;
            wb[k] = rb;
            ra += xa;
            rb += xb;
        }
        colstart[ncol] = ra;
        colcl[ncol] = rb;
        meta->nclusters = rb;
        meta->npad = rb * C;
    }
    __syncthreads();
    int pa = wa[wv] + ia - a, pb = wb[wv] + ib - b;
    for (int c = c0; c < c1; ++c) {
        const int v = colcount[c];
        colstart[c] = pa;
        colcl[c] = pb;
        pa += v;
        pb += (v + C - 1) / C;
    }
    if (lane == 0) atomicMax(&meta->maxcolumn, mx);
}

// Clears the column histogram and the build's part of the status block before a build (one
// launch instead of a memset per buffer).  Conditions raised by earlier force calls (stale list,
// non-finite coordinates, force range) stay set until nb_check has reported them.
__global__ void k_begin(int ncol, int *__restrict__ colcount, nb_meta *meta) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ncol) colcount[i] = 0;
    if (i == 0) {
        const uint32_t keep = meta->flags & NB_F_CALL_MASK;
        *meta = nb_meta{};
        meta->flags = keep;
    }
}

// Atom indices in column order; also marks every slot of perm empty (-1) for the column sort,
// which fills the slots of real atoms.
__global__ void k_scatter(int n, int npad_max, const int *__restrict__ col,
                          const int *__restrict__ rank, const int *__restrict__ colstart,
                          int *__restrict__ tmp, int *__restrict__ perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (int p = i; p < npad_max; p += gridDim.x * blockDim.x) perm[p] = -1;
    if (i >= n) return;
    tmp[colstart[col[i]] + rank[i]] = i;
}

#define NB_COLSORT_THREADS 256
#define NB_COLSORT_POS 512  // columns of at most this many atoms keep the slot positions in LDS
static_assert(NB_COLSORT_POS == 2 * NB_COLSORT_THREADS, "the rank sort takes up to two atoms per thread");

// One block per column: sort the column's atoms by (z, index) in LDS (by rank for columns of
// at most two atoms per thread, bitonic otherwise), then lay them out as clusters of C slots;
// the tail of the last cluster is padding (perm = -1).  The block then writes the bounding
// boxes of its clusters over their real atoms (from the slots it has just written), and the
// column's z table: for every bin edge z_k = k / zinv, k = 0 .. nz, the number of its clusters
// whose upper z bound is below z_k and the number whose lower z bound is at most z_k (both
// bounds grow with the index, so these are the first cluster that can reach above z_k and the
// first that lies wholly above it); the end edges count as -inf and +inf.
template <int C>
__global__ void __launch_bounds__(NB_COLSORT_THREADS) k_colsort(nb_geom g, const float *__restrict__ x,
                                                 const float4 *__restrict__ off,
                                                 const int *__restrict__ colcount,
                                                 const int *__restrict__ colstart,
                                                 const int *__restrict__ colcl,
                                                 const int *__restrict__ tmp, int *__restrict__ perm,
                                                 int *__restrict__ slot_of, float4 *__restrict__ xs,
                                                 float4 *__restrict__ xq, int *__restrict__ tsort,
                                                 float4 *__restrict__ bblo, float4 *__restrict__ bbhi,
                                                 int2 *__restrict__ colz, nb_meta *meta) {
    __shared__ unsigned long long key[NB_SORT_MAX];
    __shared__ float zlo[NB_SORT_MAX / C], zhi[NB_SORT_MAX / C];  // the clusters' z bounds
    // the slots' positions (w = 1 for an atom, 0 for padding), from which the bounding boxes are
    // formed, for columns of at most NB_COLSORT_POS + C slots
    __shared__ float4 spos[NB_COLSORT_POS + C];
    const int c = blockIdx.x, tid = threadIdx.x;
    const int n = colcount[c], start = colstart[c];
    const int cl0 = colcl[c], nslot = (colcl[c + 1] - cl0) * C;
    // a padding slot: far coordinates (distinct per slot) and type 0 in the build's and the force
    // path's copies; the per-call pack writes only the slots of atoms, so these last until the
    // next build
    auto pad = [&](int slot) {
        perm[slot] = -1;
        xs[slot] = nb_pad_coord(slot);
        xq[slot] = nb_pad_coord(slot);
        tsort[slot] = 0;
    };
    if (n > NB_SORT_MAX) {   // reported; the column's clusters are left empty
        if (tid == 0) atomicOr(&meta->flags, NB_F_COLUMN);
        for (int r = tid; r < nslot; r += blockDim.x) pad(cl0 * C + r);
    } else if (n <= 2 * (int)blockDim.x) {
        // one or two atoms per thread: an atom's place in the sorted column is the number of
        // smaller (z, index) keys (distinct: the atom index is their low word), read from LDS
        // as broadcasts
        const bool two = n > (int)blockDim.x;
        unsigned long long v[2] = {~0ull, ~0ull};
        int a[2] = {-1, -1};
        float4 pa[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int idx = tid + j * (int)blockDim.x;
            pa[j] = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
            if (idx < n) {
                a[j] = tmp[start + idx];
                const float4 o = off[a[j]];
                pa[j].x = x[3 * a[j]] + o.x;
                pa[j].y = x[3 * a[j] + 1] + o.y;
                pa[j].z = x[3 * a[j] + 2] + o.z;
                float z = pa[j].z;
                if (!(z > 0.0f)) z = 0.0f;
                v[j] = ((unsigned long long)__float_as_uint(z) << 32) | (unsigned)a[j];
                key[idx] = v[j];
            }
        }
        __syncthreads();
        int rank[2] = {0, 0};
        if (two) {
            for (int k = 0; k < n; ++k) {
                const unsigned long long kk = key[k];
                rank[0] += kk < v[0] ? 1 : 0;
                rank[1] += kk < v[1] ? 1 : 0;
            }
        } else {
            for (int k = 0; k < n; ++k) rank[0] += key[k] < v[0] ? 1 : 0;
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (a[j] < 0) continue;
            const int slot = cl0 * C + rank[j];
            perm[slot] = a[j];
            slot_of[a[j]] = slot;
            xs[slot] = pa[j];
            spos[rank[j]] = pa[j];
        }
        for (int r = n + tid; r < nslot; r += blockDim.x) {
            pad(cl0 * C + r);
            spos[r] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
    } else {
    int npow = 1;
    while (npow < n) npow <<= 1;
    for (int k = tid; k < npow; k += blockDim.x) {
        unsigned long long v = ~0ull;
        if (k < n) {
            int a = tmp[start + k];
            float z = x[3 * a + 2] + off[a].z;
            if (!(z > 0.0f)) z = 0.0f;
            v = ((unsigned long long)__float_as_uint(z) << 32) | (unsigned)a;
        }
        key[k] = v;
    }
    for (int size = 2; size <= npow; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int k = tid; k < npow; k += blockDim.x) {
                int j = k ^ stride;
                if (j > k) {
                    unsigned long long a = key[k], b = key[j];
                    bool up = (k & size) == 0;
                    if ((a > b) == up) {
                        key[k] = b;
                        key[j] = a;
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int r = tid; r < nslot; r += blockDim.x) {
        int slot = cl0 * C + r;
        float4 pa = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (r < n) {
            int a = (int)(key[r] & 0xffffffffu);
            perm[slot] = a;
            slot_of[a] = slot;
            float4 o = off[a];
            pa = make_float4(x[3 * a] + o.x, x[3 * a + 1] + o.y, x[3 * a + 2] + o.z, 1.0f);
            xs[slot] = pa;
        } else {
            pad(slot);
        }
        if (r < NB_COLSORT_POS + C) spos[r] = pa;
    }
    }
    // the block's writes of perm, xs and spos are visible to the whole block after the barrier
    __syncthreads();
    // (larger columns read the slots back from memory, all C of a cluster at once)
    const bool lds_pos = n <= NB_SORT_MAX && nslot <= NB_COLSORT_POS + C;
    for (int k = tid; k < nslot / C; k += blockDim.x) {
        const int cl = cl0 + k;
        float3 a = make_float3(3e38f, 3e38f, 3e38f), b = make_float3(-3e38f, -3e38f, -3e38f);
        float4 ps[C];
        if (lds_pos) {
#pragma unroll
            for (int r = 0; r < C; ++r) ps[r] = spos[k * C + r];
        } else {
            int pr[C];
#pragma unroll
            for (int r = 0; r < C; ++r) {
                pr[r] = perm[cl * C + r];
                ps[r] = xs[cl * C + r];
            }
#pragma unroll
            for (int r = 0; r < C; ++r) ps[r].w = pr[r] < 0 ? 0.0f : 1.0f;
        }
#pragma unroll
        for (int r = 0; r < C; ++r) {
            const float4 p = ps[r];
            if (p.w == 0.0f) continue;
            a.x = fminf(a.x, p.x);
            a.y = fminf(a.y, p.y);
            a.z = fminf(a.z, p.z);
            b.x = fmaxf(b.x, p.x);
            b.y = fmaxf(b.y, p.y);
            b.z = fmaxf(b.z, p.z);
        }
        bblo[cl] = make_float4(a.x, a.y, a.z, 0.0f);
        bbhi[cl] = make_float4(b.x, b.y, b.z, 0.0f);
        if (k < NB_SORT_MAX / C) {
            zlo[k] = a.z;
            zhi[k] = b.z;
        }
    }
    __syncthreads();
    const int ncl = min(nslot / C, NB_SORT_MAX / C);
    for (int k = tid; k <= g.nz; k += blockDim.x) {
        const float zk = (float)k / g.zinv;
        int below = 0, upto = 0;
        for (int i = 0; i < ncl; ++i) {
            below += zhi[i] < zk ? 1 : 0;
            upto += zlo[i] <= zk ? 1 : 0;
        }
        // the end edges stand for -inf and +inf: no coordinate, however rounded, lies outside
        if (k == 0) below = 0;
        if (k == g.nz) upto = ncl;
        colz[(size_t)c * (g.nz + 1) + k] = make_int2(below, upto);
    }
}

__device__ __forceinline__ float gap(float alo, float ahi, float blo, float bhi) {
    return fmaxf(0.0f, fmaxf(blo - ahi, alo - bhi));
}


#define NB_QCAP 128       // candidate queue slots per wavefront
#ifndef NB_SEARCH_WAVES
#define NB_SEARCH_WAVES 6
#endif
#define NB_PART_MAX 256   // exclusion partners of one i-cluster held in LDS

// Wave-local ordering of LDS writes before reads by other lanes of the same wavefront.
__device__ __forceinline__ void nb_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Mask bits (b * C + a) with b > a: the upper triangle kept for the self pair at t = 0.
template <int C>
__device__ __forceinline__ unsigned long long nb_triangle() {
    unsigned long long m = 0ull;
#pragma unroll
    for (int b = 0; b < C; ++b)
#pragma unroll
        for (int a = 0; a < C; ++a)
            if (b > a) m |= 1ull << (b * C + a);
    return m;
}

// One wave per i-cluster.  For every periodic shift t whose image can reach the i-cluster's
// bounding box within rlist, the clusters of the columns overlapping the dilated box are tested
// one per lane (bounding-box distance below rlist and the half-list rule: cj > ci for any t;
// cj == ci only for t = 0, with the upper triangle, or t lexicographically positive, which covers
// both images +t and -t).  Passing candidates are appended, in order, to a per-wave queue in
// LDS; every 64 queued candidates are evaluated one per lane: the topology mask (real atoms,
// self triangle, exclusions looked up as slot numbers) and whether any unmasked atom pair is
// within rlist at the build positions (atom-level prune), separately for each 4-atom j-group of
// the candidate.  Kept group entries are written in queue order, so the entries of one
// i-cluster are contiguous at jl[ci * cap] and grouped by shift.
template <int C>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NB_SEARCH_WAVES))) k_search(nb_geom g, int cap, const int *__restrict__ colcl,
                                                const int2 *__restrict__ colz,
                                                const float4 *__restrict__ bblo,
                                                const float4 *__restrict__ bbhi,
                                                const int *__restrict__ perm,
                                                const float4 *__restrict__ xs,
                                                const int *__restrict__ eoff,
                                                const int *__restrict__ eidx,
                                                const int *__restrict__ slot_of,
                                                int *__restrict__ icount,
                                                nb_entry *__restrict__ jl, nb_meta *meta) {
    __shared__ int q_cj[4][NB_QCAP], q_s[4][NB_QCAP];
    __shared__ int part[4][NB_PART_MAX];  // (a << 24) | partner slot
    const int lane = threadIdx.x & (NB_WAVE - 1);
    const int wv = threadIdx.x / NB_WAVE;
    const int ci = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / NB_WAVE) + wv);
    if (ci >= meta->nclusters) return;
    const float4 lo = bblo[ci], hi = bbhi[ci];
    const float rl = g.rl;
    // i-cluster atoms (wave-uniform)
    float xi[C], yi[C], zi[C];
    unsigned ireal = 0u;
#pragma unroll
    for (int a = 0; a < C; ++a) {
        const float4 p = xs[ci * C + a];
        xi[a] = p.x;
        yi[a] = p.y;
        zi[a] = p.z;
        if (p.w > 0.0f) ireal |= 1u << a;
    }
    // exclusion partners of the i-cluster atoms, as slots, into LDS
    int npart = 0;
    if (eoff) {
        int ne = 0, eb = 0;
        if (lane < C && ((ireal >> lane) & 1u)) {
            const int ia = perm[ci * C + lane];
            eb = eoff[ia];
            ne = eoff[ia + 1] - eb;
        }
        // exclusive prefix of ne over lanes 0 .. C-1
        int pre = 0;
        for (int a = 0; a < C; ++a) {
            const int na = __shfl(ne, a, NB_WAVE);
            if (a < lane) pre += na;
            npart += na;
        }
        npart = __builtin_amdgcn_readfirstlane(npart);
        if (npart > NB_PART_MAX) {
            if (lane == 0) atomicOr(&meta->flags, NB_F_OVERFLOW | NB_F_COLUMN);
            npart = 0;
        } else if (lane < C) {
            for (int k = 0; k < ne; ++k) part[wv][pre + k] = (lane << 24) | slot_of[eidx[eb + k]];
        }
        nb_wave_sync();
    }
    const unsigned long long tri = nb_triangle<C>();
    int count = 0, nq = 0;

    // evaluate queue slots 0 .. n-1 (n <= 64), one candidate per lane, and append kept entries
    auto flush = [&](int n) {
        bool keep0 = false, keep1 = false;
        unsigned long long m = 0ull;
        int cj = 0, s = 0;
        if (lane < n) {
            cj = q_cj[wv][lane];
            s = q_s[wv][lane];
            const float sx = nb_tx(s) * g.L[0], sy = nb_ty(s) * g.L[1], sz = nb_tz(s) * g.L[2];
            float jx[C], jy[C], jz[C];
#pragma unroll
            for (int b = 0; b < C; ++b) {
                const float4 p = xs[cj * C + b];
                jx[b] = p.x + sx;
                jy[b] = p.y + sy;
                jz[b] = p.z + sz;
            }
            // every pair of the C x C candidate, padding included (its distance excludes it)
            m = C == 8 ? ~0ull : 0xFFFFull;
            if (cj == ci && s == NB_SHIFT_ZERO) m &= tri;
            for (int k = 0; k < npart; ++k) {
                const int pe = part[wv][k];
                const int ps = pe & 0xffffff;
                if (ps / C == cj) m &= ~(1ull << ((ps % C) * C + (pe >> 24)));
            }
            // atom-level prune per j-group (the whole cluster for C = 4, each half for C = 8): a
            // group is kept if it has an unmasked pair and some pair within rlist.  Testing the
            // distances without the mask keeps a superset of the groups with an unmasked pair in
            // range (padding sits far away, so only excluded or self pairs can differ; the force
            // kernel applies the mask), at two VALU instructions less per pair.
#pragma unroll
            for (int b = 0; b < C; ++b) {
#pragma unroll
                for (int a = 0; a < C; ++a) {
                    const float dx = xi[a] - jx[b], dy = yi[a] - jy[b], dz = zi[a] - jz[b];
                    const bool in = dx * dx + dy * dy + dz * dz < g.rl2;
                    if (b < NB_JG) keep0 |= in;
                    else keep1 |= in;
                }
            }
            keep0 = keep0 && (uint32_t)m != 0u;
            keep1 = keep1 && (uint32_t)(m >> 32) != 0u;
        }
        // kept groups in (lane, half) order: the list stays in queue order, grouped by shift
        const unsigned long long k0 = __ballot(keep0), k1 = __ballot(keep1);
        const unsigned below0 = __builtin_amdgcn_mbcnt_hi((unsigned)(k0 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)k0, 0u));
        const unsigned below1 = __builtin_amdgcn_mbcnt_hi((unsigned)(k1 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)k1, 0u));
        const int pos0 = count + (int)(below0 + below1);
        nb_entry *out = jl + (size_t)ci * cap;
        if (keep0 && pos0 < cap) out[pos0] = nb_make_entry(cj * (C / NB_JG), s, (uint32_t)m);
        if (C == 8 && keep1) {
            const int pos1 = pos0 + (keep0 ? 1 : 0);
            if (pos1 < cap) out[pos1] = nb_make_entry(cj * 2 + 1, s, (uint32_t)(m >> 32));
        }
        count += __popcll(k0) + __popcll(k1);
    };

    for (int s = 0; s < 27; ++s) {
        const int tx = nb_tx(s), ty = nb_ty(s), tz = nb_tz(s);
        const float sx = tx * g.L[0], sy = ty * g.L[1], sz = tz * g.L[2];
        // j coordinates (unshifted frame) whose image x + t L can lie within rl of the bbox
        const float x0 = lo.x - rl - sx, x1 = hi.x + rl - sx;
        const float y0 = lo.y - rl - sy, y1 = hi.y + rl - sy;
        const float z0 = lo.z - rl - sz, z1 = hi.z + rl - sz;
        if (x1 < 0.0f || x0 >= g.L[0] || y1 < 0.0f || y0 >= g.L[1] || z1 < 0.0f || z0 >= g.L[2])
            continue;
        const int cx0 = max(0, (int)floorf(x0 * g.invw[0])), cx1 = min(g.ncx - 1, (int)floorf(x1 * g.invw[0]));
        const int cy0 = max(0, (int)floorf(y0 * g.invw[1])), cy1 = min(g.ncy - 1, (int)floorf(y1 * g.invw[1]));
        // The candidate columns of this shift, up to 64 at a time: lane c holds the z-window of
        // column c's clusters, and the wave walks the concatenated windows 64 clusters per pass,
        // so the loads of one pass are independent of each other.
        if (cx1 < cx0 || cy1 < cy0) continue;
        const int ncx_r = cx1 - cx0 + 1;
        const int ncols = ncx_r * (cy1 - cy0 + 1);
        for (int c0 = 0; c0 < ncols; c0 += NB_WAVE) {
            const int c = c0 + lane;
            int cstart = 0, cnt = 0;
            if (c < ncols) {
                const int col = (cy0 + c / ncx_r) * g.ncx + cx0 + c % ncx_r;
                cstart = colcl[col];
                // clusters are z-ordered within a column, so both bounding-box z ends increase
                // with the index: keep only a run that holds every cluster whose z extent meets
                // [z0, z1] widened by 2^-10 nm (all the bounding-box test below can pass), from
                // the column's z table at the bin edges below and above that range (one bin
                // further out on each side, so that the rounding of the bin index cannot narrow
                // the run); the extra clusters fail the bounding-box test
                const float zw0 = z0 - 0x1p-10f, zw1 = z1 + 0x1p-10f;
                const int k0 = min(max((int)floorf(zw0 * g.zinv) - 1, 0), g.nz);
                const int k1 = min(max((int)ceilf(zw1 * g.zinv) + 1, 0), g.nz);
                const int a = colz[(size_t)col * (g.nz + 1) + k0].x;  // no cluster before a reaches z0
                const int e = colz[(size_t)col * (g.nz + 1) + k1].y;  // none from e on starts below z1
                cstart += a;
                cnt = max(e - a, 0);
            }
            int incl = cnt;  // inclusive prefix sum of the counts over the lanes
#pragma unroll
            for (int o = 1; o < NB_WAVE; o <<= 1) {
                const int v = __shfl_up(incl, o, NB_WAVE);
                if (lane >= o) incl += v;
            }
            const int total = __builtin_amdgcn_readlane(incl, NB_WAVE - 1);
            for (int f0 = 0; f0 < total; f0 += NB_WAVE) {
                const int f = f0 + lane;
                // column lane q: the first lane whose inclusive prefix exceeds f
                int q = 0;
#pragma unroll
                for (int step = NB_WAVE / 2; step >= 1; step >>= 1) {
                    const int v = __shfl(incl, q + step - 1, NB_WAVE);
                    if (v <= f) q += step;
                }
                q = min(q, NB_WAVE - 1);
                const int qstart = __shfl(cstart, q, NB_WAVE);
                const int qexcl = __shfl(incl, q, NB_WAVE) - __shfl(cnt, q, NB_WAVE);
                const int cjl = qstart + (f - qexcl);
                bool cand = f < total;
                if (cand) {
                    const bool half = cjl > ci || (cjl == ci && s >= NB_SHIFT_ZERO);
                    const float4 jlo = bblo[cjl], jhi = bbhi[cjl];
                    const float gx = gap(lo.x, hi.x, jlo.x + sx, jhi.x + sx);
                    const float gy = gap(lo.y, hi.y, jlo.y + sy, jhi.y + sy);
                    const float gz = gap(lo.z, hi.z, jlo.z + sz, jhi.z + sz);
                    cand = half && (gx * gx + gy * gy + gz * gz < g.rl2);
                }
                const unsigned long long cbal = __ballot(cand);
                if (cbal == 0ull) continue;
                if (cand) {
                    const int pos = nq + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(cbal >> 32),
                                                                       __builtin_amdgcn_mbcnt_lo((unsigned)cbal, 0u));
                    q_cj[wv][pos] = cjl;
                    q_s[wv][pos] = s;
                }
                nq += __popcll(cbal);
                nb_wave_sync();
                if (nq >= NB_WAVE) {
                    flush(NB_WAVE);
                    // move the overflow (slots 64 .. nq-1) to the front
                    const int rest = nq - NB_WAVE;
                    int mc = 0, ms = 0;
                    if (lane < rest) {
                        mc = q_cj[wv][NB_WAVE + lane];
                        ms = q_s[wv][NB_WAVE + lane];
                    }
                    nb_wave_sync();
                    if (lane < rest) {
                        q_cj[wv][lane] = mc;
                        q_s[wv][lane] = ms;
                    }
                    nq = rest;
                    nb_wave_sync();
                }
            }
        }
    }
    if (nq > 0) flush(nq);
    // No per-wave atomics on shared counters (they serialise across the whole grid): only an
    // overflowing i-cluster touches meta; list totals are summed from icount on request.
    if (lane == 0) {
        icount[ci] = min(count, cap);
        if (count > cap) {
            atomicOr(&meta->flags, NB_F_OVERFLOW);
            atomicMax(&meta->maxcount, count);
        }
    }
}

#define NB_UNIT_MIN 4  // batches per work unit at least (a unit's fixed cost is about one)
#define NB_UNITS_BLOCKS 16   // workgroups of k_units
#define NB_UNITS_THREADS 1024
#define NB_UNITS_LOADS 16    // batch counts a k_units thread loads at a time

// Cost class of a work unit (or list) of nb >= 1 batches: floor(log2 nb), at most NB_HIST_BINS - 1.
__device__ __forceinline__ int nb_cost_class(int nb) {
    return min(31 - __clz(max(nb, 1)), NB_HIST_BINS - 1);
}

// Exclusive prefix of v over the 1024 threads of the block (thread order) and the block total;
// wa is LDS scratch of 16 ints.  Every thread of the block must call it.
__device__ __forceinline__ int nb_block_scan(int v, int *wa, int *total) {
    const int tid = threadIdx.x, lane = tid & (NB_WAVE - 1), wv = tid / NB_WAVE;
    int incl = v;
#pragma unroll
    for (int o = 1; o < NB_WAVE; o <<= 1) {
        const int u = __shfl_up(incl, o, NB_WAVE);
        if (lane >= o) incl += u;
    }
    __syncthreads();  // wa may still be read from the previous call
    if (lane == NB_WAVE - 1) wa[wv] = incl;
    __syncthreads();
    int base = 0, tot = 0;
    for (int k = 0; k < (int)(blockDim.x / NB_WAVE); ++k) {
        const int t = wa[k];
        base += k < wv ? t : 0;
        tot += t;
    }
    *total = tot;
    return base + incl - v;
}

// Work units of the force kernel: every i-cluster with a non-empty list becomes ceil(nb / P)
// units of at most P 64-lane batches, nb being its list length in batches and
// P = max(4, ceil(total batches / (2 * SIMDs))).  The SIMDs share their time among resident
// waves, so a kernel lasts about max(total batches / SIMDs, longest list) batch times; lists are
// split only when the longest list would set that (small boxes), never at 96k atoms.  The lists
// of the last `tail` clusters are also split in halves (units of ceil(nb / 2) batches): those
// units run while the device drains, and shorter ones let the SIMDs finish together (96k atoms:
// 82 -> 78 us).  The unit index is also its energy slot.  Order: with sorted = 0 units stay in
// cluster order, so that neighbouring waves work on neighbouring clusters, whose j-atoms they
// share in the caches (ordering them longest first was measured slower at 96k atoms); with
// sorted != 0 they are emitted longest first by cost class (floor(log2 batches), stable in
// cluster order within a class), the post-prune list sorting of the paper (section III-A) that
// starts the long lists before the short ones to shorten the tail.  The histogram of list
// lengths over the same classes goes to meta->hist.
//
// NB_UNITS_BLOCKS workgroups, each emitting the units of one chunk of consecutive clusters, with
// no synchronisation between them: every workgroup sums the batch counts of all clusters itself
// (for P) and counts the units of the clusters before its chunk (for its first unit index, or per
// cost class in the sorted order), reading the counts in coalesced passes.
__device__ __forceinline__ int nb_block_sum(int v, int *wa) {
    int t;
    nb_block_scan(v, wa, &t);
    return t;
}

__global__ void __launch_bounds__(NB_UNITS_THREADS) k_units(int slots, int unit_cap, int sorted, int tail,
                                                            const int *__restrict__ icount,
                                                            int4 *__restrict__ units, nb_meta *meta) {
    __shared__ int wa[NB_UNITS_THREADS / NB_WAVE];
    __shared__ int s_cnt[2][NB_HIST_BINS];  // per cost class: units before the chunk, all units
    __shared__ int s_hist[NB_HIST_BINS];
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & (NB_WAVE - 1);
    const bool lead = blockIdx.x == 0, last = blockIdx.x == gridDim.x - 1;
    const int ncl = meta->nclusters;
    const int chunk = (ncl + gridDim.x - 1) / gridDim.x;
    const int lo = min(ncl, (int)blockIdx.x * chunk), hi = min(ncl, lo + chunk);
    if (tid < NB_HIST_BINS) {
        s_hist[tid] = 0;
        s_cnt[0][tid] = 0;
        s_cnt[1][tid] = 0;
    }
    __syncthreads();
    auto batches = [&](int c) { return (icount[c] + NB_JPB - 1) / NB_JPB; };
    // the batch counts of clusters c0 + j nthr + tid (j < NB_UNITS_LOADS) below `end`, loaded
    // together from clamped indices (zero past the end), passed to f(c, nb)
    auto pass = [&](int end, auto &&f) {
        for (int c0 = 0; c0 < end; c0 += NB_UNITS_LOADS * nthr) {
            int nb[NB_UNITS_LOADS];
#pragma unroll
            for (int j = 0; j < NB_UNITS_LOADS; ++j) nb[j] = icount[min(c0 + j * nthr + tid, end - 1)];
#pragma unroll
            for (int j = 0; j < NB_UNITS_LOADS; ++j) {
                const int c = c0 + j * nthr + tid;
                f(c, c < end ? (nb[j] + NB_JPB - 1) / NB_JPB : 0);
            }
        }
    };
    // pass over all clusters: total batches, longest list; the list-length histogram (first
    // workgroup; per-wave counts from ballots)
    int nb_sum = 0, nb_max = 0;
    int hw[NB_HIST_BINS];
#pragma unroll
    for (int b = 0; b < NB_HIST_BINS; ++b) hw[b] = 0;
    pass(ncl, [&](int c, int nb) {
        nb_sum += nb;
        nb_max = max(nb_max, nb);
        if (lead) {
            const int k = nb > 0 ? nb_cost_class(nb) : -1;
#pragma unroll
            for (int b = 0; b < NB_HIST_BINS; ++b) hw[b] += __popcll(__builtin_amdgcn_ballot_w64(k == b));
        }
    });
    if (lead && lane == 0) {
#pragma unroll
        for (int b = 0; b < NB_HIST_BINS; ++b)
            if (hw[b]) atomicAdd(&s_hist[b], hw[b]);
    }
    nb_sum = nb_block_sum(nb_sum, wa);
    int m = nb_max;
#pragma unroll
    for (int o = NB_WAVE / 2; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, NB_WAVE));
    __syncthreads();
    if (lane == 0) wa[tid / NB_WAVE] = m;
    __syncthreads();
    for (int k = 0; k < nthr / NB_WAVE; ++k) m = max(m, wa[k]);
    const int P = max(NB_UNIT_MIN, (nb_sum + 2 * slots - 1) / (2 * slots));
    // the lists of the last `tail` clusters are split into halves (units of ceil(nb / 2) batches;
    // longer than P, they are split by P anyway): batches per unit and units of cluster c
    const int c_split = ncl - tail;
    auto halve = [&](int c, int nb) { return c >= c_split && nb <= P; };
    auto pmax = [&](int c, int nb) { return halve(c, nb) ? (nb + 1) >> 1 : P; };
    auto nunits_of = [&](int c, int nb) {
        return halve(c, nb) ? min(nb, 2) : (nb <= P ? (nb > 0 ? 1 : 0) : (nb + P - 1) / P);
    };
    // this thread's clusters of the chunk: a contiguous run, so that unit order is cluster order
    const int sub = (hi - lo + nthr - 1) / nthr;
    const int t_lo = min(hi, lo + tid * sub), t_hi = min(hi, t_lo + sub);
    if (!sorted) {
        // units before the chunk, then the exclusive prefix over the chunk's threads
        int before = 0;
        pass(lo, [&](int c, int nb) { before += nunits_of(c, nb); });
        before = nb_block_sum(before, wa);
        int mine = 0;
        for (int c = t_lo; c < t_hi; ++c) mine += nunits_of(c, batches(c));
        int tot = 0;
        int u = before + nb_block_scan(mine, wa, &tot);
        if (last && tid == 0) {
            const int run = before + tot;
            meta->nunits = min(run, unit_cap);
            if (run > unit_cap) atomicOr(&meta->flags, NB_F_COLUMN);  // not reachable: <= ncl + tail + 2 slots
        }
        for (int c = t_lo; c < t_hi; ++c) {
            const int nb = batches(c), pc = pmax(c, nb);
            for (int b = 0; b < nb; b += pc) {
                if (u < unit_cap) units[u] = make_int4(c, b, min(pc, nb - b), u);
                ++u;
            }
        }
    } else {
        // per cost class: the units before the chunk and all units (a cluster's units are all
        // of length pc but the last)
        int hb[NB_HIST_BINS], ha[NB_HIST_BINS];  // before the chunk, all (selects on the values,
#pragma unroll                                // so that both stay in registers)
        for (int b = 0; b < NB_HIST_BINS; ++b) hb[b] = ha[b] = 0;
        pass(ncl, [&](int c, int nb) {
            if (nb <= 0) return;
            const int nu = nunits_of(c, nb), pc = pmax(c, nb);
            const int kf = nb_cost_class(pc), kl = nb_cost_class(nb - (nu - 1) * pc);
            const bool before = c < lo;
#pragma unroll
            for (int b = 0; b < NB_HIST_BINS; ++b) {
                const int add = (b == kf ? nu - 1 : 0) + (b == kl ? 1 : 0);
                ha[b] += add;
                hb[b] += before ? add : 0;
            }
        });
#pragma unroll
        for (int b = 0; b < NB_HIST_BINS; ++b) {
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                int v = w == 0 ? hb[b] : ha[b];
#pragma unroll
                for (int o = NB_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, NB_WAVE);
                if (lane == 0 && v) atomicAdd(&s_cnt[w][b], v);
            }
        }
        __syncthreads();
        if (last && tid == 0) {
            int run = 0;
            for (int b = 0; b < NB_HIST_BINS; ++b) run += s_cnt[1][b];
            meta->nunits = min(run, unit_cap);
            if (run > unit_cap) atomicOr(&meta->flags, NB_F_COLUMN);
        }
        // one pass per cost class, from the highest: the class's units of the chunk follow those
        // of all higher classes and the class's units before the chunk
        int base = 0;
        for (int k = NB_HIST_BINS - 1; k >= 0; --k) {
            int mine = 0;
            for (int c = t_lo; c < t_hi; ++c) {
                const int nb = batches(c), pc = pmax(c, nb);
                for (int b = 0; b < nb; b += pc) mine += nb_cost_class(min(pc, nb - b)) == k ? 1 : 0;
            }
            int tot = 0;
            int u = base + s_cnt[0][k] + nb_block_scan(mine, wa, &tot);
            for (int c = t_lo; c < t_hi; ++c) {
                const int nb = batches(c), pc = pmax(c, nb);
                for (int b = 0; b < nb; b += pc) {
                    const int len = min(pc, nb - b);
                    if (nb_cost_class(len) != k) continue;
                    if (u < unit_cap) units[u] = make_int4(c, b, len, u);
                    ++u;
                }
            }
            base += s_cnt[1][k];
        }
    }
    if (lead) {
        __syncthreads();
        if (tid < NB_HIST_BINS) meta->hist[tid] = s_hist[tid];
        if (tid == 0) {
            meta->maxbatches = m;
            meta->split = P;
        }
    }
}

// Export of interacting pairs with the force kernel's arithmetic: the same lane layout (one
// j atom per lane, the i atoms of the cluster in turn) and the same displacement formula.
template <int C>
__global__ void __launch_bounds__(256) k_pairs(nb_geom g, float rc2, int cap,
                                               const float4 *__restrict__ xq,
                                               const int *__restrict__ perm,
                                               const int *__restrict__ icount,
                                               const nb_entry *__restrict__ jl,
                                               const nb_meta *meta,
                                               unsigned long long *counter, int64_t outcap,
                                               int64_t *__restrict__ out) {
    const int lane = threadIdx.x & (NB_WAVE - 1);
    const int ci = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / NB_WAVE) +
                                                  threadIdx.x / NB_WAVE);
    if (ci >= meta->nclusters) return;
    const int nj = icount[ci];
    const int b = lane % NB_JG;
    for (int base = 0; base < nj; base += NB_JPB) {
        const int e = base + lane / NB_JG;
        if (e >= nj) continue;
        const nb_entry en = jl[(size_t)ci * cap + e];
        const int s = nb_entry_shift(en);
        const int tx = nb_tx(s), ty = nb_ty(s), tz = nb_tz(s);
        const int jslot = nb_entry_group(en) * NB_JG + b;
        const float4 xj = xq[jslot];
        const float xjs = xj.x + nb_dj(tx, g.L[0]), yjs = xj.y + nb_dj(ty, g.L[1]),
                    zjs = xj.z + nb_dj(tz, g.L[2]);
        const float dix = nb_di(tx, g.L[0]), diy = nb_di(ty, g.L[1]), diz = nb_di(tz, g.L[2]);
        const unsigned mcol = nb_mask_column<C>(en.mask, b);
        const int jb = perm[jslot];
        for (int k = 0; k < C; ++k) {
            if (!((mcol >> k) & 1u)) continue;
            const float4 xi = xq[ci * C + k];
            float dx = (xi.x + dix) - xjs, dy = (xi.y + diy) - yjs, dz = (xi.z + diz) - zjs;
            float r2 = nb_r2(dx, dy, dz);
            if (r2 < rc2) {
                int ia = perm[ci * C + k];
                unsigned long long w = atomicAdd(counter, 1ull);
                if ((int64_t)w < outcap) {
                    out[2 * w] = min(ia, jb);
                    out[2 * w + 1] = max(ia, jb);
                }
            }
        }
    }
}

// Rolling prune: the pruned list keeps the entries of the full list that have an unmasked atom
// pair within r_inner at the current positions (the masks are kept as they are; the force
// kernel still tests r < rc).  One wave per i-cluster with the lanes of the pair export (entry =
// lane / 4, j-atom = lane % 4, the C i-atoms in a loop), on the positions the per-call pack has
// just written (so the distances are the ones the force kernel sees).  Kept entries are
// compacted in order with a ballot per batch.
template <int C>
__global__ void __launch_bounds__(256) k_prune(nb_geom g, float rin2, int cap, int ncl_max,
                                               const float4 *__restrict__ xq,
                                               const int *__restrict__ icount,
                                               const nb_entry *__restrict__ jl,
                                               int *__restrict__ icount_p,
                                               nb_entry *__restrict__ jl_p, const nb_meta *meta) {
    const int lane = threadIdx.x & (NB_WAVE - 1);
    const int ci = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / NB_WAVE) +
                                                  threadIdx.x / NB_WAVE);
    if (ci >= ncl_max) return;
    if (ci >= meta->nclusters) {
        if (lane == 0) icount_p[ci] = 0;
        return;
    }
    float4 xi[C];
#pragma unroll
    for (int k = 0; k < C; ++k) xi[k] = xq[ci * C + k];
    const int nj = icount[ci];
    const int b = lane % NB_JG, eo = lane / NB_JG;
    int kept = 0;
    for (int base = 0; base < nj; base += NB_JPB) {   // wave-uniform
        const int e = base + eo;
        const nb_entry en = e < nj ? jl[(size_t)ci * cap + e] : nb_make_entry(0, NB_SHIFT_ZERO, 0u);
        const int s = nb_entry_shift(en);
        const int tx = nb_tx(s), ty = nb_ty(s), tz = nb_tz(s);
        const float4 xj = xq[nb_entry_group(en) * NB_JG + b];
        const float xjs = xj.x + nb_dj(tx, g.L[0]), yjs = xj.y + nb_dj(ty, g.L[1]), zjs = xj.z + nb_dj(tz, g.L[2]);
        const float dix = nb_di(tx, g.L[0]), diy = nb_di(ty, g.L[1]), diz = nb_di(tz, g.L[2]);
        const unsigned mcol = nb_mask_column<C>(en.mask, b);   // empty past the end of the list
        bool hit = false;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const float dx = (xi[k].x + dix) - xjs, dy = (xi[k].y + diy) - yjs, dz = (xi[k].z + diz) - zjs;
            hit |= ((mcol >> k) & 1u) && nb_r2(dx, dy, dz) < rin2;
        }
        const uint64_t m = __ballot(hit);
        uint32_t em = 0;   // entries of this batch with a pair in range
#pragma unroll
        for (int q = 0; q < NB_JPB; ++q) em |= ((m >> (NB_JG * q)) & 0xFull) ? (1u << q) : 0u;
        if (b == 0 && ((em >> eo) & 1u))
            jl_p[(size_t)ci * cap + kept + __popc(em & ((1u << eo) - 1u))] = en;
        kept += __popc(em);
    }
    if (lane == 0) icount_p[ci] = kept;
}

// Displacement check against the positions of the last prune ((r_inner - rc) / 2).
__global__ void k_prune_check(int n, const float *__restrict__ x, const float *__restrict__ xp,
                              float stale2, nb_meta *meta) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float d0 = x[3 * i] - xp[3 * i], d1 = x[3 * i + 1] - xp[3 * i + 1], d2 = x[3 * i + 2] - xp[3 * i + 2];
    if (!(d0 * d0 + d1 * d1 + d2 * d2 < stale2)) atomicOr(&meta->flags, NB_F_STALE);
}

template <int C>
hipError_t build_impl(nb_ctx *c, const float *x) {
    const int n = c->natoms;
    const int tb = 256;
    hipLaunchKernelGGL(k_begin, dim3((c->geom.ncol + tb - 1) / tb), dim3(tb), 0, c->stream,
                       c->geom.ncol, c->colcount, c->meta);
    const int lds = c->geom.ncol <= NB_BIN_LDS_MAX;
    hipLaunchKernelGGL(k_bin, dim3((n + tb - 1) / tb), dim3(tb), lds ? sizeof(int) * c->geom.ncol : 0,
                       c->stream, n, x, c->geom, c->off, c->xbuild, c->col, c->rank, c->colcount,
                       c->meta, lds);
    hipLaunchKernelGGL(k_colscan, dim3(1), dim3(1024), 0, c->stream, c->geom.ncol, C, c->colcount,
                       c->colstart, c->colcl, c->meta);
    // every slot is marked empty here; the column sort fills the slots of its clusters (atoms and
    // padding), which are the only ones the force path reads
    hipLaunchKernelGGL(k_scatter, dim3((n + tb - 1) / tb), dim3(tb), 0, c->stream, n, c->npad_max,
                       c->col, c->rank, c->colstart, c->tmp, c->perm);
    hipLaunchKernelGGL((k_colsort<C>), dim3(c->geom.ncol), dim3(NB_COLSORT_THREADS), 0, c->stream, c->geom, x, c->off,
                       c->colcount, c->colstart, c->colcl, c->tmp, c->perm, c->slot_of, c->xs,
                       c->xq, c->tsort, c->bblo, c->bbhi, c->colz, c->meta);
    hipLaunchKernelGGL((k_search<C>), dim3((c->ncl_max + 3) / 4), dim3(256), 0, c->stream,
                       c->geom, c->cap, c->colcl, c->colz, c->bblo, c->bbhi, c->perm, c->xs,
                       c->nnz_excl > 0 ? c->excl_off : nullptr, c->excl_idx, c->slot_of, c->icount, c->jl,
                       c->meta);
    hipLaunchKernelGGL(k_units, dim3(NB_UNITS_BLOCKS), dim3(NB_UNITS_THREADS), 0, c->stream, c->slots,
                       c->unit_cap, (c->flags & NB_SORT_UNITS) ? 1 : 0, c->tail_n, c->icount, c->units,
                       c->meta);
    return hipGetLastError();
}

template <int C>
hipError_t pairs_impl(nb_ctx *c, int64_t cap) {
    unsigned long long *counter = (unsigned long long *)&c->meta->npairs_out;
    const hipError_t e = hipMemsetAsync(counter, 0, sizeof(unsigned long long), c->stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_pairs<C>), dim3((c->ncl_max + 3) / 4), dim3(256), 0, c->stream, c->geom,
                       c->fp.rc2, c->cap, c->xq, c->perm, c->icount, c->jl, c->meta, counter, cap,
                       c->dbg_pairs);
    return hipGetLastError();
}

}  // namespace

hipError_t nb_launch_build(nb_ctx *c, const float *x) {
    return c->C == 4 ? build_impl<4>(c, x) : build_impl<8>(c, x);
}

hipError_t nb_launch_debug_pairs(nb_ctx *c, int64_t cap) {
    return c->C == 4 ? pairs_impl<4>(c, cap) : pairs_impl<8>(c, cap);
}

namespace {
template <int C>
hipError_t prune_impl(nb_ctx *c, float rin2, const int *icount, const nb_entry *jl, int *icount_p,
                      nb_entry *jl_p) {
    hipLaunchKernelGGL((k_prune<C>), dim3((c->ncl_max + 3) / 4), dim3(256), 0, c->stream, c->geom, rin2,
                       c->cap, c->ncl_max, c->xq, icount, jl, icount_p, jl_p, c->meta);
    // work units of the pruned lists (the shorter lists are split by the same rule)
    hipLaunchKernelGGL(k_units, dim3(NB_UNITS_BLOCKS), dim3(NB_UNITS_THREADS), 0, c->stream, c->slots,
                       c->unit_cap, (c->flags & NB_SORT_UNITS) ? 1 : 0, c->tail_n, icount_p, c->units,
                       c->meta);
    return hipGetLastError();
}
}  // namespace

hipError_t nb_launch_prune(nb_ctx *c, float rin2, const int *icount, const nb_entry *jl, int *icount_p,
                           nb_entry *jl_p) {
    return c->C == 4 ? prune_impl<4>(c, rin2, icount, jl, icount_p, jl_p) : prune_impl<8>(c, rin2, icount, jl, icount_p, jl_p);
}

hipError_t nb_launch_prune_check(nb_ctx *c, const float *x) {
    const int tb = 256;
    hipLaunchKernelGGL(k_prune_check, dim3((c->natoms + tb - 1) / tb), dim3(tb), 0, c->stream, c->natoms, x,
                       c->xprune, c->stale2_prune, c->meta);
    return hipGetLastError();
}
