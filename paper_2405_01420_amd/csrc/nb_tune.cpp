// Autotuner of the batched form (nb_autotune): cluster shape per box-size bucket and the work
// schedule of the persistent force kernel, timed on the caller's own boxes, with decisions kept
// in a JSON cache file.
//
// The order of the work and the shape of the clusters decide how much of a small box's kernel
// is tail and how many pairs are evaluated per useful one: the effects the paper's post-prune
// list sorting addresses (section III-A, the list of differences between the GROMACS versions)
// and the small-system efficiency it measures (section IV-C).  Every candidate is timed with HIP
// events on the caller's stream around repeated nb_batch_forces calls; the tuner itself does no
// force arithmetic.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "nb_internal.h"

namespace {

// ---- the cache file: {"key": {"field": number, ...}, ...} ---------------------------------
using tune_record = std::map<std::string, double>;
using tune_cache = std::map<std::string, tune_record>;

struct json_in {
    const std::string &s;
    size_t p = 0;
    explicit json_in(const std::string &t) : s(t) {}
    void ws() {
        while (p < s.size() && (s[p] == ' ' || s[p] == '\n' || s[p] == '\t' || s[p] == '\r')) ++p;
    }
    bool lit(char c) {
        ws();
        if (p < s.size() && s[p] == c) {
            ++p;
            return true;
        }
        return false;
    }
    bool str(std::string &out) {
        ws();
        if (p >= s.size() || s[p] != '"') return false;
        ++p;
        out.clear();
        while (p < s.size() && s[p] != '"') {
            if (s[p] == '\\') {
                if (++p >= s.size()) return false;
            }
            out.push_back(s[p++]);
        }
        if (p >= s.size()) return false;
        ++p;
        return true;
    }
    bool num(double &v) {
        ws();
        const char *b = s.c_str() + p;
        char *e = nullptr;
        v = strtod(b, &e);
        if (e == b) return false;
        p += (size_t)(e - b);
        return true;
    }
};

// Parses the cache text; false if it is not an object of objects of numbers.
bool parse_cache(const std::string &text, tune_cache &out) {
    json_in in(text);
    if (!in.lit('{')) return false;
    if (in.lit('}')) return true;
    do {
        std::string key;
        if (!in.str(key) || !in.lit(':') || !in.lit('{')) return false;
        tune_record rec;
        if (!in.lit('}')) {
            do {
                std::string f;
                double v;
                if (!in.str(f) || !in.lit(':') || !in.num(v)) return false;
                rec[f] = v;
            } while (in.lit(','));
            if (!in.lit('}')) return false;
        }
        out[key] = rec;
    } while (in.lit(','));
    if (!in.lit('}')) return false;
    in.ws();
    return in.p == text.size();
}

std::string format_cache(const tune_cache &c) {
    std::string o = "{\n";
    bool first = true;
    for (const auto &kv : c) {
        if (!first) o += ",\n";
        first = false;
        o += " \"" + kv.first + "\": {";
        bool f2 = true;
        for (const auto &fv : kv.second) {
            char buf[64];
            snprintf(buf, sizeof(buf), "%.17g", fv.second);
            if (!f2) o += ", ";
            f2 = false;
            o += "\"" + fv.first + "\": " + buf;
        }
        o += "}";
    }
    o += "\n}\n";
    return o;
}

int read_file(const char *path, std::string &text, bool &exists) {
    exists = false;
    FILE *f = fopen(path, "rb");
    if (!f) return NB_OK;  // no cache yet
    exists = true;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
    const bool bad = ferror(f) != 0;
    fclose(f);
    return bad ? NB_ERR_IO : NB_OK;
}

int write_file(const char *path, const std::string &text) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return NB_ERR_IO;
    const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
    if (fclose(f) != 0 || !ok) {
        remove(tmp.c_str());
        return NB_ERR_IO;
    }
    if (rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        return NB_ERR_IO;
    }
    return NB_OK;
}

thread_local std::string g_tune_error;

int tfail(int code, const std::string &msg) {
    g_tune_error = msg;
    return code;
}

// Logarithmic size buckets over [NB_TUNE_NMIN, NB_TUNE_NMAX); sizes outside fall into the first
// and last bucket.
int bucket_of(int natoms) {
    const double r = std::log((double)NB_TUNE_NMAX / NB_TUNE_NMIN) / NB_TUNE_BUCKETS;
    const int b = (int)std::floor(std::log((double)natoms / NB_TUNE_NMIN) / r);
    return std::min(std::max(b, 0), NB_TUNE_BUCKETS - 1);
}

int bucket_edge(int k) {
    return (int)std::lround(NB_TUNE_NMIN * std::pow((double)NB_TUNE_NMAX / NB_TUNE_NMIN, (double)k / NB_TUNE_BUCKETS));
}

// Device arrays of a subset of boxes, gathered from the caller's concatenated arrays.
struct sample_set {
    std::vector<int32_t> atom_off;
    std::vector<double> boxes;
    std::vector<int32_t> eoff, eidx;
    float *x = nullptr, *q = nullptr, *f = nullptr;
    int32_t *t = nullptr;
    double *e = nullptr;
    ~sample_set() {
        void *bufs[] = {x, q, f, t, e};
        for (void *b : bufs)
            if (b) hipFree(b);
    }
};

int gather(const std::vector<int> &members, const int32_t *atom_off, const double *boxes,
           const nb_params *common, const float *x, const float *q, const int32_t *type,
           hipStream_t stream, sample_set &s) {
    s.atom_off.assign(1, 0);
    for (int b : members) {
        s.atom_off.push_back(s.atom_off.back() + (atom_off[b + 1] - atom_off[b]));
        for (int k = 0; k < 3; ++k) s.boxes.push_back(boxes[3 * b + k]);
    }
    const size_t n = (size_t)s.atom_off.back();
    if (hipMalloc((void **)&s.x, 3 * n * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&s.q, n * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&s.f, 3 * n * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&s.t, n * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&s.e, 2 * members.size() * sizeof(double)) != hipSuccess)
        return tfail(NB_ERR_OOM, "autotune sample buffers");
    for (size_t k = 0; k < members.size(); ++k) {
        const int b = members[k];
        const size_t a0 = (size_t)atom_off[b], na = (size_t)(atom_off[b + 1] - atom_off[b]);
        const size_t d0 = (size_t)s.atom_off[k];
        hipError_t e = hipMemcpyAsync(s.x + 3 * d0, x + 3 * a0, 3 * na * sizeof(float), hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(s.q + d0, q + a0, na * sizeof(float), hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(s.t + d0, type + a0, na * sizeof(int32_t), hipMemcpyDeviceToDevice, stream);
        if (e != hipSuccess) return tfail(NB_ERR_HIP, std::string("autotune gather: ") + hipGetErrorString(e));
        if (common->excl_off) {
            if (k == 0) s.eoff.assign(1, 0);
            for (size_t i = 0; i < na; ++i) {
                const int g = (int)(a0 + i);
                for (int m = common->excl_off[g]; m < common->excl_off[g + 1]; ++m)
                    s.eidx.push_back(common->excl_idx[m] - (int)a0 + (int)d0);
                s.eoff.push_back((int32_t)s.eidx.size());
            }
        }
    }
    if (s.eidx.empty()) s.eidx.push_back(0);
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return tfail(NB_ERR_HIP, std::string("autotune gather: ") + hipGetErrorString(e));
    return NB_OK;
}

// Microseconds per nb_batch_forces of the sample with all boxes at cluster size C.
int time_sample(const sample_set &s, const nb_params *common, int C, hipStream_t stream, double *us) {
    const int nbox = (int)s.atom_off.size() - 1;
    nb_params p = *common;
    p.natoms = s.atom_off.back();
    p.excl_off = common->excl_off ? s.eoff.data() : nullptr;
    p.excl_idx = common->excl_off ? s.eidx.data() : nullptr;
    std::vector<int32_t> cl(nbox, C);
    nb_batch *bt = nullptr;
    int r = nb_batch_setup(&bt, nbox, s.atom_off.data(), s.boxes.data(), cl.data(), &p, stream);
    if (r != NB_OK) return tfail(r, std::string("autotune sample: ") + nb_batch_last_error(nullptr));
    hipEvent_t ev[2] = {nullptr, nullptr};
    if ((r = nb_batch_pairlist(bt, s.x)) == NB_OK)
        for (int w = 0; w < 3 && r == NB_OK; ++w) r = nb_batch_forces(bt, s.x, s.q, s.t, s.f, s.e);
    if (r != NB_OK) g_tune_error = nb_batch_last_error(bt);
    const int reps = 10;
    if (r == NB_OK) {
        hipError_t e = hipEventCreate(&ev[0]);
        if (e == hipSuccess) e = hipEventCreate(&ev[1]);
        if (e == hipSuccess) e = hipEventRecord(ev[0], stream);
        for (int i = 0; i < reps && e == hipSuccess && r == NB_OK; ++i) r = nb_batch_forces(bt, s.x, s.q, s.t, s.f, s.e);
        if (e == hipSuccess) e = hipEventRecord(ev[1], stream);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (r == NB_OK && e != hipSuccess) r = tfail(NB_ERR_HIP, std::string("autotune timing: ") + hipGetErrorString(e));
        *us = 1e3 * ms / reps;
    }
    for (hipEvent_t v : ev)
        if (v) hipEventDestroy(v);
    nb_batch_destroy(bt);
    return r;
}

}  // namespace

extern "C" {

const char *nb_autotune_last_error(void) { return g_tune_error.c_str(); }

int nb_autotune(int32_t nbox, const int32_t *atom_off, const double *boxes, const nb_params *common,
                const float *x, const float *q, const int32_t *type, const char *cache_path,
                void *stream, int32_t *clusters_out, nb_tune_result *res) {
    g_tune_error.clear();
    if (nbox < 1 || !atom_off || !boxes || !common || !x || !q || !type || !clusters_out || !res)
        return tfail(NB_ERR_ARG, "NULL argument or no boxes");
    for (int b = 0; b < nbox; ++b)
        if (atom_off[b + 1] <= atom_off[b]) return tfail(NB_ERR_ARG, "every box needs at least one atom");
    const auto t0 = std::chrono::steady_clock::now();
    memset(res, 0, sizeof(*res));
    // the cache is read (and checked) before the device is touched
    tune_cache cache;
    if (cache_path) {
        std::string text;
        bool exists = false;
        if (read_file(cache_path, text, exists) != NB_OK) return tfail(NB_ERR_IO, std::string("cannot read ") + cache_path);
        if (exists && !parse_cache(text, cache)) return tfail(NB_ERR_IO, std::string("not a tuning cache: ") + cache_path);
    }
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return tfail(NB_ERR_HIP, "hipGetDeviceProperties");
    int rtv = 0;
    hipRuntimeGetVersion(&rtv);
    char pre[256];
    snprintf(pre, sizeof(pre), "%s|hip%d|rc%.4f|%s%s%s", prop.gcnArchName, rtv, common->cutoff,
             common->elec == NB_ELEC_RF ? "rf" : "ewald", common->vdw == NB_VDW_FSWITCH ? "-fsw" : "",
             (common->flags & NB_ENERGY_FP64) ? "|e64" : "");
    // ---- cluster shape per bucket
    std::vector<std::vector<int>> members(NB_TUNE_BUCKETS);
    for (int b = 0; b < nbox; ++b) members[bucket_of(atom_off[b + 1] - atom_off[b])].push_back(b);
    res->nbuckets = NB_TUNE_BUCKETS;
    int choice[NB_TUNE_BUCKETS] = {0};
    for (int k = 0; k < NB_TUNE_BUCKETS; ++k) {
        res->bucket_lo[k] = bucket_edge(k);
        res->bucket_hi[k] = bucket_edge(k + 1);
        res->bucket_boxes[k] = (int32_t)members[k].size();
        if (members[k].empty()) continue;
        char key[320];
        snprintf(key, sizeof(key), "%s|bucket%d-%d", pre, res->bucket_lo[k], res->bucket_hi[k]);
        auto it = cache.find(key);
        if (it != cache.end() && it->second.count("cluster")) {
            choice[k] = (int)it->second["cluster"];
            res->bucket_cached[k] = 1;
            if (choice[k] != 4 && choice[k] != 8) return tfail(NB_ERR_IO, std::string("bad cluster size in cache entry ") + key);
            continue;
        }
        std::vector<int> sample(members[k].begin(), members[k].begin() + std::min<size_t>(members[k].size(), NB_TUNE_SAMPLE));
        sample_set ss;
        int r = gather(sample, atom_off, boxes, common, x, q, type, s, ss);
        if (r != NB_OK) return r;
        const int shapes[2] = {4, 8};
        for (int c = 0; c < 2; ++c)
            if ((r = time_sample(ss, common, shapes[c], s, &res->bucket_us[k][c])) != NB_OK) return r;
        choice[k] = res->bucket_us[k][1] < res->bucket_us[k][0] ? 8 : 4;
        tune_record rec;
        rec["cluster"] = choice[k];
        rec["us4"] = res->bucket_us[k][0];
        rec["us8"] = res->bucket_us[k][1];
        rec["boxes"] = (double)sample.size();
        cache[key] = rec;
    }
    for (int k = 0; k < NB_TUNE_BUCKETS; ++k) res->bucket_cluster[k] = choice[k];
    for (int b = 0; b < nbox; ++b) clusters_out[b] = choice[bucket_of(atom_off[b + 1] - atom_off[b])];
    // ---- schedule of the whole batch with those shapes
    char skey[320];
    snprintf(skey, sizeof(skey), "%s|schedule|n%d|atoms%d", pre, nbox, atom_off[nbox]);
    auto it = cache.find(skey);
    if (it != cache.end() && it->second.count("sorted") && it->second.count("blocks_per_cu")) {
        res->sorted = (int32_t)it->second["sorted"];
        res->blocks_per_cu = (int32_t)it->second["blocks_per_cu"];
        res->schedule_cached = 1;
    } else {
        nb_batch *bt = nullptr;
        int r = nb_batch_setup(&bt, nbox, atom_off, boxes, clusters_out, common, stream);
        if (r != NB_OK) return tfail(r, std::string("autotune batch: ") + nb_batch_last_error(nullptr));
        float *f = nullptr;
        double *e = nullptr;
        if (hipMalloc((void **)&f, 3 * (size_t)atom_off[nbox] * sizeof(float)) != hipSuccess ||
            hipMalloc((void **)&e, 2 * (size_t)nbox * sizeof(double)) != hipSuccess)
            r = tfail(NB_ERR_OOM, "autotune output buffers");
        if (r == NB_OK && (r = nb_batch_pairlist(bt, x)) != NB_OK) g_tune_error = nb_batch_last_error(bt);
        int32_t best[2] = {1, 0};
        if (r == NB_OK && (r = nb_batch_tune_schedule(bt, x, q, type, f, e, 5, res->schedule_us, best)) != NB_OK)
            g_tune_error = nb_batch_last_error(bt);
        if (f) hipFree(f);
        if (e) hipFree(e);
        nb_batch_destroy(bt);
        if (r != NB_OK) return r;
        res->sorted = best[0];
        res->blocks_per_cu = best[1];
        tune_record rec;
        rec["sorted"] = best[0];
        rec["blocks_per_cu"] = best[1];
        for (int k = 0; k < NB_BATCH_NSCHED; ++k) rec["us" + std::to_string(k)] = res->schedule_us[k];
        cache[skey] = rec;
    }
    if (cache_path && write_file(cache_path, format_cache(cache)) != NB_OK)
        return tfail(NB_ERR_IO, std::string("cannot write ") + cache_path);
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return NB_OK;
}

}  // extern "C"
