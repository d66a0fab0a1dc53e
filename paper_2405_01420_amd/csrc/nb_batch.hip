// Batched form: independent boxes (an ensemble) evaluated together.  Every box keeps its own
// context (grid, list, buffers); the force phase is one persistent launch per cluster shape in
// which each wavefront pulls chunks of (box, i-cluster) work items from an atomic counter.  The
// items are in descending order of j-list length so that the longest start first, and the chunks
// are cut by guided self-scheduling (each holds about 1/(2W) of the work still left, W waves), so
// the queue head is touched a few times per wave instead of once per i-cluster.  Pack,
// finalize and energy reduction each run as one launch over all boxes (2-D grids), so the
// whole force call is four launches that a HIP graph replays with one host call.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "nb_force_body.h"

struct nb_box_desc {
    const int *perm;
    const int *slot_of;
    const float4 *off;
    float4 *xq;
    int *tsort;
    const int *icount;
    const nb_entry *jl;
    float *fj;
    double *epart;
    const nb_meta *meta;
    int cap, npad_max, natoms, atom_off;
    float L[3];
    int pad;
};

struct nb_batch {
    hipStream_t stream = nullptr;
    int device = 0;
    int nbox = 0;
    int64_t natoms = 0;
    std::vector<nb_ctx *> box;
    std::vector<int> atom_off, cluster;
    nb_fparams fp{};        // shared constants (L is set per box on the device)
    double shift_coul = 0;
    float4 *ljtab = nullptr;  // the LJ table of box 0 (identical for all boxes)
    bool eprec = false;       // FP64 Coulomb energies (tables of box 0)
    int flav = 0;             // NB_FLAV(elec, vdw) of all boxes
    double2 *etab = nullptr;
    int etab_n = 0;
    float etab_invh = 0.0f;
    double fc = 0;
    int ntypes = 0;
    nb_box_desc *d_desc = nullptr;
    int2 *d_items[2] = {nullptr, nullptr};  // work items for C = 4 and C = 8
    int *d_chunks[2] = {nullptr, nullptr};  // chunk boundaries into the work items
    int nitems[2] = {0, 0};
    int nchunks[2] = {0, 0};
    int item_cap[2] = {0, 0};
    unsigned *d_counter = nullptr;           // two queue heads
    int max_npad = 0, max_natoms = 0;
    int sorted = 1, blocks_per_cu = 0;
    int grid[2] = {0, 0};
    bool have_list = false;
    bool graph_ready = false;
    hipGraphExec_t gexec = nullptr;
    const void *gptr[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int64_t nentries = 0, evaluated = 0;
    double build_ms = 0;
    std::string err;
};

namespace {

__global__ void k_batch_pack(const nb_box_desc *__restrict__ desc, const float *__restrict__ x,
                             const float *__restrict__ q, const int32_t *__restrict__ type,
                             int ntypes, unsigned *counter) {
    const int bidx = blockIdx.y;
    const nb_box_desc d = desc[bidx];
    if (bidx == 0 && blockIdx.x == 0 && threadIdx.x < 2) counter[threadIdx.x] = 0u;
    // slots past a box's current padded count hold perm = -1 (set at every build)
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d.npad_max) return;
    const int a = d.perm[p];
    if (a >= 0) {
        const int g = d.atom_off + a;
        const float4 o = d.off[a];
        int t = type[g];
        t = min(max(t, 0), ntypes - 1);
        d.xq[p] = make_float4(x[3 * g] + o.x, x[3 * g + 1] + o.y, x[3 * g + 2] + o.z, q[g]);
        d.tsort[p] = t;
    } else {
        d.xq[p] = nb_pad_coord(p);
        d.tsort[p] = 0;
    }
    d.fj[p] = 0.0f;
    d.fj[d.npad_max + p] = 0.0f;
    d.fj[2 * d.npad_max + p] = 0.0f;
}

// Persistent force kernel: every wavefront loops, taking the next chunk of work items from the
// queue, until the queue is empty; every wave reaches that exit.
template <int C, bool EPREC, int FLAV>
__global__ void __launch_bounds__(256) NB_FORCE_OCCUPANCY k_batch_force(nb_fparams fp, const nb_box_desc *__restrict__ desc,
                                                     const int2 *__restrict__ items,
                                                     const int *__restrict__ chunks, int nchunks,
                                                     const float4 *__restrict__ ljtab,
                                                     const double2 *__restrict__ etab, int etab_n,
                                                     float etab_invh, unsigned *counter,
                                                     unsigned *flags) {
    extern __shared__ float4 tab[];
    __shared__ __attribute__((aligned(C * NB_WAVE * 4))) nb_wg_lds<C, EPREC, FLAV, 256 / NB_WAVE> wl;
    const int ntt = fp.ntypes * fp.ntypes;
    nb_load_ljtab(tab, ljtab, ntt);
    nb_etab et;
    et.seg = reinterpret_cast<const double2 *>(tab + 2 * ntt);
    et.invh = etab_invh;
    et.n = etab_n;
    et.fseg = nullptr;  // the tabulated flavour is not built for batches
    if (EPREC) {
        double2 *dst = reinterpret_cast<double2 *>(tab + 2 * ntt);
        for (int k = threadIdx.x; k < NB_ETAB_W * etab_n; k += blockDim.x) dst[k] = etab[k];
    }
    __syncthreads();
    const int lane = threadIdx.x & (NB_WAVE - 1);
    const nb_wv wvw = nb_wave_view(wl, __builtin_amdgcn_readfirstlane(threadIdx.x / NB_WAVE));
    // Every lane executes the queue atomic (lane 0 adds 1, the others 0; the compiler issues
    // one atomic per wave), so no divergent region precedes the uniform exit test; the value
    // lane 0 saw is the chunk of this wave.  The trip count is bounded by nchunks even if the
    // queue misbehaved.
    for (int iter = 0; iter < nchunks; ++iter) {
        const unsigned c = (unsigned)__builtin_amdgcn_readfirstlane(
            (int)atomicAdd(counter, lane == 0 ? 1u : 0u));
        if (c >= (unsigned)nchunks) break;
        const int i0 = __builtin_amdgcn_readfirstlane(chunks[c]);
        const int i1 = __builtin_amdgcn_readfirstlane(chunks[c + 1]);
        for (int it = i0; it < i1; ++it) {
            const int2 w = items[it];
            const int b = __builtin_amdgcn_readfirstlane(w.x);
            const int ci = __builtin_amdgcn_readfirstlane(w.y);
            const nb_box_desc &d = desc[b];
            nb_fparams f = fp;
            f.L[0] = d.L[0];
            f.L[1] = d.L[1];
            f.L[2] = d.L[2];
            f.nL[0] = -d.L[0];
            f.nL[1] = -d.L[1];
            f.nL[2] = -d.L[2];
            // the descriptor's pointers are global memory; typed so, their accesses are global
            const nb_esum es = nb_force_cluster<C, EPREC, FLAV, false>(
                f, tab, et, wvw, ci, 0, 1 << 20, d.cap, d.npad_max, nb_g(d.xq), nb_g(d.tsort),
                nb_g(d.icount), nb_g(d.jl), nb_g(d.fj), nb_g(flags));
            if (lane == 0) {
                NB_G double *ep = nb_g(d.epart) + 4 * ci;
                nb_st(ep, es.elj);
                nb_st(ep + 1, es.ec);
                nb_st(ep + 2, es.qq);
            }
        }
    }
}

__global__ void k_batch_finalize(const nb_box_desc *__restrict__ desc, float *__restrict__ f) {
    const nb_box_desc d = desc[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.natoms) return;
    const int p = d.slot_of[i];
    const int g = d.atom_off + i;
    // fixed-point sums (the force body's layout): x in the low 32 bits of the xy word, y above
    const unsigned long long w = reinterpret_cast<const unsigned long long *>(d.fj)[p];
    const int ix = (int)(unsigned)w;
    const int iy = (int)((w - (unsigned long long)(long long)ix) >> 32);
    const int iz = reinterpret_cast<const int *>(d.fj + 2 * d.npad_max)[p];
    f[3 * g] = (float)ix * (1.0f / NB_FSCALE);
    f[3 * g + 1] = (float)iy * (1.0f / NB_FSCALE);
    f[3 * g + 2] = (float)iz * (1.0f / NB_FSCALE);
}

__global__ void __launch_bounds__(256) k_batch_energy(const nb_box_desc *__restrict__ desc,
                                                      double shift_coul, double coul_scale,
                                                      double *__restrict__ e) {
    __shared__ double s[3][256 / NB_WAVE];
    const nb_box_desc d = desc[blockIdx.x];
    const int ncl = d.meta->nclusters;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int k = threadIdx.x; k < ncl; k += blockDim.x) {
        a += d.epart[4 * k];
        b += d.epart[4 * k + 1];
        c += d.epart[4 * k + 2];
    }
    a = nb_wave_sum_d(a);
    b = nb_wave_sum_d(b);
    c = nb_wave_sum_d(c);
    const int w = threadIdx.x / NB_WAVE;
    if ((threadIdx.x & (NB_WAVE - 1)) == 0) {
        s[0][w] = a;
        s[1][w] = b;
        s[2][w] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0, tc = 0.0;
        for (int k = 0; k < (int)(blockDim.x / NB_WAVE); ++k) {
            ta += s[0][k];
            tb += s[1][k];
            tc += s[2][k];
        }
        e[2 * blockIdx.x] = ta;
        e[2 * blockIdx.x + 1] = coul_scale * (tb - shift_coul * tc);
    }
}

thread_local std::string g_batch_error;

int bfail(nb_batch *bt, int code, const std::string &msg) {
    if (bt) bt->err = msg;
    else g_batch_error = msg;
    return code;
}

void free_batch(nb_batch *bt) {
    for (nb_ctx *c : bt->box)
        if (c) nb_destroy(c);
    if (bt->gexec) hipGraphExecDestroy(bt->gexec);
    void *bufs[] = {bt->d_desc, bt->d_items[0], bt->d_items[1], bt->d_chunks[0], bt->d_chunks[1],
                    bt->d_counter};
    for (void *p : bufs)
        if (p) hipFree(p);
}

int upload_desc(nb_batch *bt) {
    std::vector<nb_box_desc> h(bt->nbox);
    for (int b = 0; b < bt->nbox; ++b) {
        nb_ctx *c = bt->box[b];
        nb_box_desc &d = h[b];
        d.perm = c->perm;
        d.slot_of = c->slot_of;
        d.off = c->off;
        d.xq = c->xq;
        d.tsort = c->tsort;
        d.icount = c->icount;
        d.jl = c->jl;
        d.fj = c->fj;
        d.epart = c->epart;
        d.meta = c->meta;
        d.cap = c->cap;
        d.npad_max = c->npad_max;
        d.natoms = c->natoms;
        d.atom_off = bt->atom_off[b];
        for (int k = 0; k < 3; ++k) d.L[k] = (float)c->box[k];
        d.pad = 0;
    }
    hipError_t e = hipMemcpy(bt->d_desc, h.data(), sizeof(nb_box_desc) * h.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bfail(bt, NB_ERR_HIP, std::string("upload box descriptors: ") + hipGetErrorString(e));
    return NB_OK;
}

size_t batch_shm(const nb_batch *bt) {
    return sizeof(float4) * 2 * bt->ntypes * bt->ntypes + (bt->eprec ? sizeof(double2) * NB_ETAB_W * bt->etab_n : 0);
}

template <int C>
int grid_for(nb_batch *bt) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, bt->device) != hipSuccess) return 0;
    int per_cu = bt->blocks_per_cu;
    if (per_cu <= 0) {
        hipError_t e = bt->eprec
                           ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_force<C, true, 0>, 256, batch_shm(bt))
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_force<C, false, 0>, 256, batch_shm(bt));
        if (e != hipSuccess || per_cu <= 0) per_cu = 1;
    }
    return per_cu * prop.multiProcessorCount;
}

template <int C, bool EPREC, int FLAV>
void launch_batch_t(nb_batch *bt, int s) {
    hipLaunchKernelGGL((k_batch_force<C, EPREC, FLAV>), dim3(bt->grid[s]), dim3(256), batch_shm(bt),
                       bt->stream, bt->fp, bt->d_desc, bt->d_items[s], bt->d_chunks[s], bt->nchunks[s],
                       bt->ljtab, bt->etab, bt->etab_n, bt->etab_invh, bt->d_counter + s,
                       bt->d_counter + 2);
}

template <int C>
void launch_batch_c(nb_batch *bt, int s) {
    switch (bt->flav) {
    case NB_FLAV(NB_ELEC_EWALD, NB_VDW_SHIFT):
        if (bt->eprec) launch_batch_t<C, true, NB_FLAV(NB_ELEC_EWALD, NB_VDW_SHIFT)>(bt, s);
        else launch_batch_t<C, false, NB_FLAV(NB_ELEC_EWALD, NB_VDW_SHIFT)>(bt, s);
        break;
    case NB_FLAV(NB_ELEC_EWALD, NB_VDW_FSWITCH):
        if (bt->eprec) launch_batch_t<C, true, NB_FLAV(NB_ELEC_EWALD, NB_VDW_FSWITCH)>(bt, s);
        else launch_batch_t<C, false, NB_FLAV(NB_ELEC_EWALD, NB_VDW_FSWITCH)>(bt, s);
        break;
    case NB_FLAV(NB_ELEC_RF, NB_VDW_SHIFT):
        if (bt->eprec) launch_batch_t<C, true, NB_FLAV(NB_ELEC_RF, NB_VDW_SHIFT)>(bt, s);
        else launch_batch_t<C, false, NB_FLAV(NB_ELEC_RF, NB_VDW_SHIFT)>(bt, s);
        break;
    default:
        if (bt->eprec) launch_batch_t<C, true, NB_FLAV(NB_ELEC_RF, NB_VDW_FSWITCH)>(bt, s);
        else launch_batch_t<C, false, NB_FLAV(NB_ELEC_RF, NB_VDW_FSWITCH)>(bt, s);
        break;
    }
}

hipError_t launch_forces(nb_batch *bt, const float *x, const float *q, const int32_t *type, float *f,
                         double *e) {
    const int tb = 256;
    hipLaunchKernelGGL(k_batch_pack, dim3((bt->max_npad + tb - 1) / tb, bt->nbox), dim3(tb), 0,
                       bt->stream, bt->d_desc, x, q, type, bt->ntypes, bt->d_counter);
    if (bt->nitems[0] > 0) launch_batch_c<4>(bt, 0);
    if (bt->nitems[1] > 0) launch_batch_c<8>(bt, 1);
    hipLaunchKernelGGL(k_batch_finalize, dim3((bt->max_natoms + tb - 1) / tb, bt->nbox), dim3(tb), 0,
                       bt->stream, bt->d_desc, f);
    hipLaunchKernelGGL(k_batch_energy, dim3(bt->nbox), dim3(256), 0, bt->stream, bt->d_desc,
                       bt->shift_coul, bt->eprec ? bt->fc : 1.0, e);
    return hipGetLastError();
}

}  // namespace

extern "C" {

int nb_batch_setup(nb_batch **out, int32_t nbox, const int32_t *atom_off, const double *boxes,
                   const int32_t *clusters, const nb_params *common, void *stream) {
    if (!out || !atom_off || !boxes || !common || nbox < 1) return bfail(nullptr, NB_ERR_ARG, "bad argument");
    if (common->flags & NB_EWALD_CORR)
        return bfail(nullptr, NB_ERR_ARG, "NB_EWALD_CORR is not available in the batched form");
    if (common->elec == NB_ELEC_EWALD_TAB)
        return bfail(nullptr, NB_ERR_ARG, "the tabulated Ewald flavour is not available in the batched form");
    *out = nullptr;
    if (atom_off[0] != 0 || atom_off[nbox] != common->natoms)
        return bfail(nullptr, NB_ERR_ARG, "atom_off must start at 0 and end at common->natoms");
    for (int b = 0; b < nbox; ++b)
        if (atom_off[b + 1] <= atom_off[b]) return bfail(nullptr, NB_ERR_ARG, "every box needs at least one atom");
    nb_batch *bt = new nb_batch();
    bt->stream = (hipStream_t)stream;
    hipGetDevice(&bt->device);
    bt->nbox = nbox;
    bt->natoms = common->natoms;
    bt->atom_off.assign(atom_off, atom_off + nbox + 1);
    bt->ntypes = common->ntypes;
    int64_t items_max[2] = {0, 0};
    for (int b = 0; b < nbox; ++b) {
        const int n = atom_off[b + 1] - atom_off[b];
        nb_params pb = *common;
        pb.natoms = n;
        for (int k = 0; k < 3; ++k) pb.box[k] = boxes[3 * b + k];
        pb.cluster = clusters ? clusters[b] : common->cluster;
        pb.flags = common->flags & ~NB_ASYNC_BUILD;
        std::vector<int32_t> eo, ei;
        if (common->excl_off) {
            const int a0 = atom_off[b], base = common->excl_off[a0];
            eo.resize(n + 1);
            for (int i = 0; i <= n; ++i) eo[i] = common->excl_off[a0 + i] - base;
            ei.resize(std::max(eo[n], 1));
            for (int k = 0; k < eo[n]; ++k) {
                int g = common->excl_idx[base + k] - a0;
                if (g < 0 || g >= n) {
                    free_batch(bt);
                    delete bt;
                    return bfail(nullptr, NB_ERR_ARG, "an exclusion crosses two boxes");
                }
                ei[k] = g;
            }
            pb.excl_off = eo.data();
            pb.excl_idx = ei.data();
        }
        nb_ctx *c = nullptr;
        int r = nb_setup(&c, &pb, stream);
        if (r != NB_OK) {
            std::string msg = std::string("box ") + std::to_string(b) + ": " + nb_last_error(nullptr);
            free_batch(bt);
            delete bt;
            return bfail(nullptr, r, msg);
        }
        bt->box.push_back(c);
        bt->cluster.push_back(c->C);
        items_max[c->C == 8] += c->ncl_max;
        bt->max_npad = std::max(bt->max_npad, c->npad_max);
        bt->max_natoms = std::max(bt->max_natoms, n);
    }
    bt->fp = bt->box[0]->fp;
    bt->shift_coul = bt->box[0]->shift_coul;
    bt->ljtab = bt->box[0]->ljtab;
    bt->eprec = (common->flags & NB_ENERGY_FP64) != 0;
    bt->flav = NB_FLAV(common->elec, common->vdw);
    bt->etab = bt->box[0]->etab;
    bt->etab_n = bt->box[0]->etab_n;
    bt->etab_invh = bt->box[0]->etab_invh;
    bt->fc = bt->box[0]->fc;
    hipError_t e = hipMalloc((void **)&bt->d_desc, sizeof(nb_box_desc) * nbox);
    // two queue heads (reset by the pack kernel of every call) and the force range flag
    if (e == hipSuccess) e = hipMalloc((void **)&bt->d_counter, sizeof(unsigned) * 3);
    if (e == hipSuccess) e = hipMemset(bt->d_counter, 0, sizeof(unsigned) * 3);
    for (int s = 0; s < 2 && e == hipSuccess; ++s) {
        bt->item_cap[s] = (int)std::max<int64_t>(items_max[s], 1);
        e = hipMalloc((void **)&bt->d_items[s], sizeof(int2) * bt->item_cap[s]);
        if (e == hipSuccess) e = hipMalloc((void **)&bt->d_chunks[s], sizeof(int) * (bt->item_cap[s] + 1));
    }
    if (e != hipSuccess) {
        free_batch(bt);
        delete bt;
        return bfail(nullptr, NB_ERR_OOM, "batch buffers");
    }
    int r = upload_desc(bt);
    if (r != NB_OK) {
        std::string msg = bt->err;
        free_batch(bt);
        delete bt;
        return bfail(nullptr, r, msg);
    }
    bt->grid[0] = items_max[0] > 0 ? grid_for<4>(bt) : 0;
    bt->grid[1] = items_max[1] > 0 ? grid_for<8>(bt) : 0;
    *out = bt;
    return NB_OK;
}

int nb_batch_set_schedule(nb_batch *bt, int32_t sorted, int32_t blocks_per_cu) {
    if (!bt || blocks_per_cu < 0) return bfail(bt, NB_ERR_ARG, "bad argument");
    bt->sorted = sorted != 0;
    bt->blocks_per_cu = blocks_per_cu;
    hipSetDevice(bt->device);
    bool any4 = false, any8 = false;
    for (int c : bt->cluster) (c == 8 ? any8 : any4) = true;
    bt->grid[0] = any4 ? grid_for<4>(bt) : 0;
    bt->grid[1] = any8 ? grid_for<8>(bt) : 0;
    bt->graph_ready = false;
    if (bt->have_list) {
        // re-order the existing work list
        return nb_batch_pairlist(bt, nullptr);
    }
    return NB_OK;
}

int nb_batch_pairlist(nb_batch *bt, const float *x) {
    if (!bt) return bfail(bt, NB_ERR_ARG, "NULL batch");
    hipSetDevice(bt->device);
    auto t0 = std::chrono::steady_clock::now();
    if (x) {
        bt->have_list = false;
        std::vector<bool> todo(bt->nbox, true);
        for (int attempt = 0; attempt < 4; ++attempt) {
            for (int b = 0; b < bt->nbox; ++b)
                if (todo[b]) {
                    nb_ctx *c = bt->box[b];
                    hipError_t e = nb_launch_build(c, x + 3 * (size_t)bt->atom_off[b]);
                    if (e != hipSuccess) return bfail(bt, NB_ERR_HIP, std::string("build: ") + hipGetErrorString(e));
                }
            hipError_t e = hipStreamSynchronize(bt->stream);
            if (e != hipSuccess) return bfail(bt, NB_ERR_HIP, std::string("build: ") + hipGetErrorString(e));
            bool again = false;
            for (int b = 0; b < bt->nbox; ++b) {
                if (!todo[b]) continue;
                nb_ctx *c = bt->box[b];
                nb_meta m;
                if (nb_read_meta(c, &m) != NB_OK) return bfail(bt, NB_ERR_HIP, c->err);
                todo[b] = false;
                if (m.flags & NB_F_COLUMN) return bfail(bt, NB_ERR_OVERFLOW, "a grid column overflowed");
                if (m.flags & NB_F_BUILD_NONFINITE) return bfail(bt, NB_ERR_NONFINITE, "non-finite coordinates");
                if (m.flags & NB_F_OVERFLOW) {
                    if (nb_regrow_list(c, m.maxcount) != NB_OK) return bfail(bt, NB_ERR_OOM, c->err);
                    todo[b] = true;
                    again = true;
                }
                c->have_list = !todo[b];
            }
            if (!again) break;
            if (attempt == 3) return bfail(bt, NB_ERR_OVERFLOW, "pair list still overflowing");
        }
    } else if (!bt->have_list) {
        return bfail(bt, NB_ERR_STATE, "no pair lists");
    }
    // work list: (box, i-cluster) with the j-list length as cost
    std::vector<std::pair<int, int2>> items[2];
    bt->nentries = 0;
    bt->evaluated = 0;
    for (int b = 0; b < bt->nbox; ++b) {
        nb_ctx *c = bt->box[b];
        nb_meta m;
        if (nb_read_meta(c, &m) != NB_OK) return bfail(bt, NB_ERR_HIP, c->err);
        std::vector<int> cnt(std::max(m.nclusters, 1));
        if (m.nclusters > 0 &&
            hipMemcpy(cnt.data(), c->icount, sizeof(int) * m.nclusters, hipMemcpyDeviceToHost) != hipSuccess)
            return bfail(bt, NB_ERR_HIP, "read list lengths");
        const int s = c->C == 8;
        int64_t ne = 0;
        for (int ci = 0; ci < m.nclusters; ++ci) {
            items[s].push_back({cnt[ci], make_int2(b, ci)});
            ne += cnt[ci];
        }
        bt->nentries += ne;
        bt->evaluated += ne * (int64_t)c->C * NB_JG;
    }
    for (int s = 0; s < 2; ++s) {
        if (bt->sorted)
            std::stable_sort(items[s].begin(), items[s].end(),
                             [](const std::pair<int, int2> &a, const std::pair<int, int2> &b) { return a.first > b.first; });
        std::vector<int2> flat(items[s].size());
        for (size_t k = 0; k < flat.size(); ++k) flat[k] = items[s][k].second;
        bt->nitems[s] = (int)flat.size();
        if (bt->nitems[s] > bt->item_cap[s]) return bfail(bt, NB_ERR_OVERFLOW, "work list capacity");
        // guided chunks: each takes about 1/(2W) of the remaining cost (j-entries plus one batch
        // of per-cluster overhead per item), at least one item
        std::vector<int> chunks(1, 0);
        double remaining = 0.0;
        for (const auto &it : items[s]) remaining += it.first + NB_JPB;
        const double waves = 4.0 * std::max(bt->grid[s], 1);
        double acc = 0.0, target = remaining / (2.0 * waves);
        for (size_t k = 0; k < items[s].size(); ++k) {
            acc += items[s][k].first + NB_JPB;
            if (acc >= target || k + 1 == items[s].size()) {
                chunks.push_back((int)k + 1);
                remaining -= acc;
                acc = 0.0;
                target = remaining / (2.0 * waves);
            }
        }
        bt->nchunks[s] = (int)chunks.size() - 1;
        if (!flat.empty() &&
            (hipMemcpy(bt->d_items[s], flat.data(), sizeof(int2) * flat.size(), hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(bt->d_chunks[s], chunks.data(), sizeof(int) * chunks.size(), hipMemcpyHostToDevice) != hipSuccess))
            return bfail(bt, NB_ERR_HIP, "upload work list");
    }
    int r = upload_desc(bt);
    if (r != NB_OK) return r;
    bt->have_list = true;
    bt->graph_ready = false;
    bt->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return NB_OK;
}

int nb_batch_forces(nb_batch *bt, const float *x, const float *q, const int32_t *type, float *f,
                    double *e) {
    if (!bt || !x || !q || !type || !f || !e) return bfail(bt, NB_ERR_ARG, "NULL argument");
    if (!bt->have_list) return bfail(bt, NB_ERR_STATE, "nb_batch_forces before nb_batch_pairlist");
    hipError_t err = launch_forces(bt, x, q, type, f, e);
    if (err != hipSuccess) return bfail(bt, NB_ERR_HIP, std::string("batch force launch: ") + hipGetErrorString(err));
    return NB_OK;
}

int nb_batch_tune_schedule(nb_batch *bt, const float *x, const float *q, const int32_t *type, float *f,
                           double *e, int32_t reps, double *us_out, int32_t *best) {
    if (!bt || !x || !q || !type || !f || !e || reps < 1) return bfail(bt, NB_ERR_ARG, "bad argument");
    if (!bt->have_list) return bfail(bt, NB_ERR_STATE, "nb_batch_tune_schedule before nb_batch_pairlist");
    hipSetDevice(bt->device);
    // candidates: cost-sorted items with a persistent grid of as many blocks as fit, or 1, 2, 4
    // blocks per compute unit; items in box order with as many blocks as fit
    static const int32_t cand[NB_BATCH_NSCHED][2] = {{1, 0}, {1, 1}, {1, 2}, {1, 4}, {0, 0}};
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) {
        if (ev[0]) hipEventDestroy(ev[0]);
        return bfail(bt, NB_ERR_HIP, "hipEventCreate");
    }
    int r = NB_OK, pick = 0;
    double us[NB_BATCH_NSCHED], best_us = 0.0;
    for (int k = 0; k < NB_BATCH_NSCHED && r == NB_OK; ++k) {
        if ((r = nb_batch_set_schedule(bt, cand[k][0], cand[k][1])) != NB_OK) break;
        for (int w = 0; w < 2 && r == NB_OK; ++w) r = nb_batch_forces(bt, x, q, type, f, e);
        if (r != NB_OK) break;
        hipError_t err = hipEventRecord(ev[0], bt->stream);
        for (int i = 0; i < reps && r == NB_OK; ++i) r = nb_batch_forces(bt, x, q, type, f, e);
        if (err == hipSuccess) err = hipEventRecord(ev[1], bt->stream);
        float ms = 0.0f;
        if (err == hipSuccess) err = hipEventSynchronize(ev[1]);
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (r == NB_OK && err != hipSuccess) r = bfail(bt, NB_ERR_HIP, std::string("schedule timing: ") + hipGetErrorString(err));
        us[k] = 1e3 * ms / reps;
        if (r == NB_OK && (k == 0 || us[k] < best_us)) {
            best_us = us[k];
            pick = k;
        }
    }
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    if (r != NB_OK) return r;
    if ((r = nb_batch_set_schedule(bt, cand[pick][0], cand[pick][1])) != NB_OK) return r;
    if (us_out)
        for (int k = 0; k < NB_BATCH_NSCHED; ++k) us_out[k] = us[k];
    if (best) {
        best[0] = cand[pick][0];
        best[1] = cand[pick][1];
    }
    return NB_OK;
}

int nb_batch_graph_forces(nb_batch *bt, const float *x, const float *q, const int32_t *type,
                          float *f, double *e) {
    if (!bt || !x || !q || !type || !f || !e) return bfail(bt, NB_ERR_ARG, "NULL argument");
    if (!bt->have_list) return bfail(bt, NB_ERR_STATE, "nb_batch_graph_forces before nb_batch_pairlist");
    const void *ptrs[5] = {x, q, type, f, e};
    bool same = bt->graph_ready;
    for (int k = 0; k < 5 && same; ++k) same = ptrs[k] == bt->gptr[k];
    if (!same) {
        if (bt->gexec) {
            hipGraphExecDestroy(bt->gexec);
            bt->gexec = nullptr;
        }
        hipGraph_t g = nullptr;
        hipError_t err = hipStreamBeginCapture(bt->stream, hipStreamCaptureModeThreadLocal);
        if (err != hipSuccess) return bfail(bt, NB_ERR_HIP, std::string("begin capture: ") + hipGetErrorString(err));
        hipError_t lerr = launch_forces(bt, x, q, type, f, e);
        err = hipStreamEndCapture(bt->stream, &g);
        if (lerr != hipSuccess || err != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return bfail(bt, NB_ERR_HIP, std::string("capture: ") + hipGetErrorString(lerr != hipSuccess ? lerr : err));
        }
        err = hipGraphInstantiate(&bt->gexec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (err != hipSuccess) return bfail(bt, NB_ERR_HIP, std::string("instantiate: ") + hipGetErrorString(err));
        for (int k = 0; k < 5; ++k) bt->gptr[k] = ptrs[k];
        bt->graph_ready = true;
    }
    hipError_t err = hipGraphLaunch(bt->gexec, bt->stream);
    if (err != hipSuccess) return bfail(bt, NB_ERR_HIP, std::string("graph launch: ") + hipGetErrorString(err));
    return NB_OK;
}

int nb_batch_get_info(nb_batch *bt, nb_batch_info *info) {
    if (!bt || !info) return bfail(bt, NB_ERR_ARG, "NULL argument");
    memset(info, 0, sizeof(*info));
    info->nbox = bt->nbox;
    info->sorted = bt->sorted;
    info->natoms = bt->natoms;
    info->nitems = (int64_t)bt->nitems[0] + bt->nitems[1];
    info->nentries = bt->nentries;
    info->evaluated_pairs = bt->evaluated;
    info->grid_blocks[0] = bt->grid[0];
    info->grid_blocks[1] = bt->grid[1];
    info->graph_ready = bt->graph_ready;
    info->build_ms_last = bt->build_ms;
    return NB_OK;
}

int nb_batch_check(nb_batch *bt) {
    if (!bt) return bfail(bt, NB_ERR_ARG, "NULL argument");
    hipSetDevice(bt->device);
    unsigned flag = 0u;
    hipError_t e = hipMemcpyAsync(&flag, bt->d_counter + 2, sizeof(unsigned), hipMemcpyDeviceToHost, bt->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(bt->stream);
    if (e != hipSuccess) return bfail(bt, NB_ERR_HIP, std::string("read batch status: ") + hipGetErrorString(e));
    if (flag & NB_F_RANGE) {
        const unsigned zero = 0u;
        e = hipMemcpy(bt->d_counter + 2, &zero, sizeof(unsigned), hipMemcpyHostToDevice);
        if (e != hipSuccess) return bfail(bt, NB_ERR_HIP, std::string("clear batch status: ") + hipGetErrorString(e));
        return bfail(bt, NB_ERR_RANGE, "a pair force component exceeded 131072 kJ/mol/nm (or was not finite): "
                                       "net force components beyond 524288 would not be represented");
    }
    return NB_OK;
}

const char *nb_batch_last_error(nb_batch *bt) { return bt ? bt->err.c_str() : g_batch_error.c_str(); }

int nb_batch_destroy(nb_batch *bt) {
    if (!bt) return NB_OK;
    hipSetDevice(bt->device);
    hipStreamSynchronize(bt->stream);
    free_batch(bt);
    delete bt;
    return NB_OK;
}

}  // extern "C"
