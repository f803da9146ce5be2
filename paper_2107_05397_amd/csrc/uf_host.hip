// Host side of the striped UniFrac library: input validation, tree and table
// preparation, device upload, workspace planning and the C ABI of uf.h.
//
// No exception or abort crosses the ABI: every entry point catches, records a
// thread-local message and returns a uf_status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "uf_internal.h"
#include "uf_split.h"

namespace {

thread_local std::string g_last_error;
std::atomic<int64_t> g_chunk_nodes{0};
// Dense-set thresholds of the sparse-aware split, [0] unweighted, [1] weighted;
// negative = automatic (cost model in ensure_split).
std::atomic<double> g_split_threshold[2] = {{-1.0}, {-1.0}};

// Measured MI355X rates of the split's two halves (pair updates per second,
// chunk embedding included, C2-sized inputs): the weighted dense stripe pass
// (32-bit fixed point; FP32 is within 10%), the BF16x2 MFMA Gram, and the
// marginal rates of the slot kernel over the pairs that share a non-dense branch
// (fitted to the optimum of a threshold sweep: near the threshold the lists are
// long and the walk keeps its lanes full).
constexpr double kRateBandDense = 3.05e13;
constexpr double kRateGramMfma = 3.78e14;
constexpr double kRatePairsWeighted = 7.3e11;
constexpr double kRatePairsUnweighted = 1.0e12;

uf_status fail(uf_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

uf_status hip_fail(hipError_t e, const char* what) {
    return fail(UF_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define UF_HIP(call)                                            \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return hip_fail(e_, #call);       \
    } while (0)

template <class F>
uf_status guarded(F&& f) {
    try {
        return f();
    } catch (const std::bad_alloc&) {
        return fail(UF_ERR_NOMEM, "host allocation failed");
    } catch (const std::exception& ex) {
        return fail(UF_ERR_ARG, std::string("unexpected error: ") + ex.what());
    } catch (...) {
        return fail(UF_ERR_ARG, "unexpected error");
    }
}

// Round an FP64 value to the nearest bfloat16 (ties to even) and return its
// bits.  Works on the FP64 bit pattern: keep sign, exponent and the top 7
// fraction bits, rounding on the 45 dropped bits.  Values below the bfloat16
// normal range are placed on its subnormal grid (spacing 2^-133).
uint16_t bf16_bits(double x) {
    if (x == 0.0 || !std::isfinite(x)) {
        float f = static_cast<float>(x);
        uint32_t b;
        std::memcpy(&b, &f, 4);
        return static_cast<uint16_t>(b >> 16);
    }
    const double ax = std::fabs(x);
    double r;
    if (ax < 0x1p-126) {
        r = std::nearbyint(ax * 0x1p133) * 0x1p-133;   // exact scaling, RNE on the grid
    } else {
        uint64_t b;
        std::memcpy(&b, &ax, 8);
        const uint64_t drop = 45;
        const uint64_t half = (uint64_t(1) << (drop - 1)) - 1;
        const uint64_t odd = (b >> drop) & 1;
        b = (b + half + odd) & ~((uint64_t(1) << drop) - 1);
        std::memcpy(&r, &b, 8);
    }
    float f = static_cast<float>(x < 0 ? -r : r);      // exact: r has <= 8 significant bits
    uint32_t fb;
    std::memcpy(&fb, &f, 4);
    return static_cast<uint16_t>(fb >> 16);
}

double bf16_value(uint16_t h) {
    uint32_t b = uint32_t(h) << 16;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

uf_status check_device(int* dev_out) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) return fail(UF_ERR_DEVICE, "no HIP device available");
    int dev = 0;
    UF_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    UF_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(UF_ERR_DEVICE, std::string("library is built for gfx950; device is ") +
                                       prop.gcnArchName);
    *dev_out = dev;
    return UF_OK;
}

// ------------------------------------------------------------------ timing
// Events around kernel launches, recorded only while profiling is enabled.
struct ProfRec {
    std::string name;
    hipEvent_t a = nullptr, b = nullptr;
};
std::mutex g_prof_mu;
std::atomic<int> g_prof_on{0};
std::vector<ProfRec> g_prof_pending;
std::map<std::string, std::pair<double, int64_t>> g_prof_done;

// set while a batch enqueues its per-table runs (possibly under graph capture)
thread_local bool t_prof_suppress = false;

class ProfScope {
  public:
    ProfScope(const char* name, hipStream_t s) : s_(s) {
        if (!g_prof_on.load() || t_prof_suppress) return;
        rec_.name = name;
        if (hipEventCreate(&rec_.a) != hipSuccess || hipEventCreate(&rec_.b) != hipSuccess ||
            hipEventRecord(rec_.a, s) != hipSuccess) {
            release();
            return;
        }
        live_ = true;
    }
    ~ProfScope() {
        if (!live_) return;
        if (hipEventRecord(rec_.b, s_) != hipSuccess) {
            release();
            return;
        }
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_pending.push_back(rec_);
    }

  private:
    void release() {
        if (rec_.a) (void)hipEventDestroy(rec_.a);
        if (rec_.b) (void)hipEventDestroy(rec_.b);
        rec_.a = rec_.b = nullptr;
    }
    hipStream_t s_;
    ProfRec rec_;
    bool live_ = false;
};

// Carve sub-buffers out of one allocation, 256-byte aligned.
struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t at = (off + 255) & ~size_t(255);
        off = at + bytes;
        return at;
    }
};

// ------------------------------------------------------------------ sparse split
ufp::Emb emb_view(const uf_embedding& e) {
    ufp::Emb v;
    v.n = e.n;
    v.row_ptr = e.row_ptr;
    v.rank = e.rank;
    v.cum = e.cum;
    v.total = e.total;
    v.lo = e.lo;
    v.hi = e.hi;
    v.len = e.len;
    v.parent_pos = e.parent_pos;
    v.tip_pos = e.tip_pos;
    v.root_pos = int32_t(e.nb);
    return v;
}

// Device temporaries of a split build: the embedding's grow-only scratch.
char* split_scratch(uf_embedding* e, size_t bytes, uf_status* st) {
    if (e->split_tmp.bytes < bytes) {
        if (e->split_tmp.buf) (void)hipFree(e->split_tmp.buf);
        e->split_tmp.buf = nullptr;
        e->split_tmp.bytes = 0;
        if (hipMalloc(&e->split_tmp.buf, bytes) != hipSuccess) {
            *st = fail(UF_ERR_NOMEM, "split temporaries");
            return nullptr;
        }
        e->split_tmp.bytes = bytes;
    }
    *st = UF_OK;
    return static_cast<char*>(e->split_tmp.buf);
}

// Samples touching each branch.  Both variants' splits classify branches by
// these counts.  The device puts +1 / -1 points on positions (ufs::branch_points);
// positions are in postorder, so the subtree of position v is the range
// [sub_first[v], v], and the count of branch v is the sum of the points there:
// a difference of two prefix sums (host, exact integers).
uf_status branch_counts(uf_embedding* e, hipStream_t s, std::vector<int32_t>* out) {
    const int64_t nb = e->nb;
    uf_status st = UF_OK;
    char* tmp = split_scratch(e, size_t(std::max<int64_t>(nb, 1)) * 4 + 256, &st);
    if (!tmp) return st;
    int32_t* dpt = reinterpret_cast<int32_t*>(tmp);
    std::vector<int32_t> pt(size_t(std::max<int64_t>(nb, 1)), 0);
    {
        ProfScope ps("branch_count", s);
        UF_HIP(ufk::zero_u32(reinterpret_cast<unsigned*>(dpt), std::max<int64_t>(nb, 1), s));
        UF_HIP(ufs::branch_points(emb_view(*e), dpt, s));
    }
    UF_HIP(hipStreamSynchronize(s));
    if (nb) UF_HIP(hipMemcpy(pt.data(), dpt, size_t(nb) * 4, hipMemcpyDeviceToHost));
    std::vector<int64_t> pre(size_t(nb) + 1, 0);   // pre[k] = sum of pt[0, k)
    for (int64_t v = 0; v < nb; ++v) pre[size_t(v) + 1] = pre[size_t(v)] + pt[size_t(v)];
    out->assign(size_t(std::max<int64_t>(nb, 1)), 0);
    for (int64_t v = 0; v < nb; ++v)
        (*out)[size_t(v)] = int32_t(pre[size_t(v) + 1] - pre[size_t(e->sub_first[size_t(v)])]);
    return UF_OK;
}

std::atomic<uint64_t> g_split_builds{0};

// Scale Q of the 32-bit fixed-point dense pass of the weighted split (0: use FP32).
// x_int = rint(x Q) is off by at most 1/(2Q) per value, so a pair's numerator is off
// by at most (nnz_i + nnz_j) / (2Q) (nnz: dense branches of nonzero length touched),
// and d by at most that over s_i + s_j <= max_s(nnz_s / s_s) / (2Q).  Q keeps every
// pair sum, Q (m_i + m_j) plus rounding, below 2^32 (m: dense mass of a sample);
// the fixed-point pass is taken when the bound on d is at most 1e-5.
double fixed_point_scale(const std::vector<double>& sw, const std::vector<unsigned long long>& sigma,
                         double unit, const std::vector<int32_t>& nnz, int64_t n_dense) {
    constexpr double kMaxDistErr = 1e-5;
    if (n_dense >= (int64_t(1) << 22)) return 0.0;
    double m_max = 0.0, ratio = 0.0;
    for (size_t s = 0; s < nnz.size(); ++s) {
        const double m = std::max(sw[s] - double(sigma[s]) * unit, 0.0);
        m_max = std::max(m_max, m);
        if (nnz[s] > 0) {
            if (!(sw[s] > 0.0)) return 0.0;
            ratio = std::max(ratio, double(nnz[s]) / sw[s]);
        }
    }
    if (m_max <= 0.0) return 1.0;   // every dense value is 0
    const double q = (0x1p32 - 0x1p23) / (2.0 * m_max);
    return ratio / (2.0 * q) <= kMaxDistErr ? q : 0.0;
}

// Build the dense set and the shared non-dense branch lists of one variant of an
// embedding at threshold thr.  Synchronous on `s`.  Caller holds e->split_mu.
//
// A branch touched by c samples costs c(c-1)/2 pair visits when left out of the
// dense set, and one pass over all N*floor(N/2) stripe slots of the dense kernel
// when put in it.  With a fixed threshold f it is dense when c > f*N; with the
// automatic one when c(c-1)/2 / (slot rate) > N*floor(N/2) / rate of the
// variant's dense kernel, i.e. when it is cheaper in the dense kernel.
uf_status build_split(uf_embedding* e, int weighted, double thr, const std::vector<int32_t>& cnt,
                      hipStream_t s, std::shared_ptr<SplitCache>* out) {
    const int64_t n = e->n, nb = e->nb;
    const ufp::Emb ev = emb_view(*e);
    auto sc = std::make_shared<SplitCache>();
    sc->build_id = ++g_split_builds;
    sc->threshold = thr;
    std::vector<int32_t> cls(size_t(std::max<int64_t>(nb, 1)), ufs::kClassAlone), dense;
    std::vector<int32_t> small_ids, large_ids;
    std::vector<int64_t> roff(1, 0);
    const double lim = thr * double(n);
    const double pair_lim = 2.0 * double(n) * double(n / 2) *
                            (weighted ? kRatePairsWeighted / kRateBandDense
                                      : kRatePairsUnweighted / kRateGramMfma);
    for (int64_t v = 0; v < nb; ++v) {
        const int64_t c = cnt[size_t(v)];
        const bool is_dense = thr >= 0.0 ? double(c) > lim : double(c) * double(c - 1) > pair_lim;
        if (is_dense) {
            cls[size_t(v)] = ufs::kClassDense;
            dense.push_back(int32_t(v));
        } else if (c >= 2) {
            const int32_t id = int32_t(roff.size()) - 1;
            cls[size_t(v)] = id;
            (c <= ufs::kSortSmall ? small_ids : large_ids).push_back(id);
            roff.push_back(roff.back() + c);
            sc->n_pairs += c * (c - 1) / 2;
        }
    }
    sc->n_dense = int64_t(dense.size());
    sc->n_lists = int64_t(roff.size()) - 1;
    sc->n_entries = roff.back();
    sc->n_dense_pad = (sc->n_dense + ufk::kGramKPad - 1) / ufk::kGramKPad * ufk::kGramKPad;
    // list entries carry a kBaseBits-bit start and a window length of up to N/2 in
    // the other 24 bits, and list lengths and positions in 24 bits; weighted
    // members hold the sample in kSampleBits bits
    if (n >= (int64_t(1) << ufs::kSampleBits))
        return fail(UF_ERR_UNSUPPORTED, "the sparse split takes fewer than 2^24 samples");
    if (sc->n_entries >= (int64_t(1) << ufs::kBaseBits))
        return fail(UF_ERR_UNSUPPORTED, "the sparse split takes fewer than 2^40 list entries");
    if (weighted) {
        // weighted members hold the value in the 40 bits above the sample: choose
        // the fixed-point step so that l * u <= max l stays below 2^40
        std::vector<double> len(size_t(std::max<int64_t>(nb, 1)), 0.0);
        if (nb) UF_HIP(hipMemcpy(len.data(), e->len, size_t(nb) * 8, hipMemcpyDeviceToHost));
        double lmax = 0.0;
        for (int64_t v = 0; v < nb; ++v)
            if (cls[size_t(v)] != ufs::kClassDense) lmax = std::max(lmax, len[size_t(v)]);
        int ex = 0;
        while (lmax >= std::ldexp(1.0 - 0x1p-20, ex)) ++ex;
        sc->unit = std::ldexp(1.0, ex - 40);
    }
    const size_t ne = size_t(std::max<int64_t>(sc->n_entries, 1));
    const size_t nl = size_t(std::max<int64_t>(sc->n_lists, 1));
    const size_t nn = size_t(std::max<int64_t>(n, 1));
    Carver c;
    const size_t o_dense = c.take(size_t(std::max<int64_t>(sc->n_dense, 1)) * 4);
    const size_t o_cls = c.take(size_t(std::max<int64_t>(nb, 1)) * 4);
    const size_t o_roff = c.take(roff.size() * 8);
    const size_t o_rs = weighted ? 0 : c.take(ne * 4);
    const size_t o_rw = weighted ? c.take(ne * 8) : 0;
    const size_t o_sig = c.take(nn * 8);
    const size_t o_dhi = c.take(size_t(std::max<int64_t>(sc->n_dense_pad, 1)) * 2);
    const size_t o_dlo = c.take(size_t(std::max<int64_t>(sc->n_dense_pad, 1)) * 2);
    const size_t o_rl = c.take(nl * 8);
    const size_t o_soff = c.take(size_t(n + 1) * 8);
    const size_t o_ent = c.take(ne * sizeof(ufs::SlotEntry));
    const size_t o_lord = weighted ? c.take(size_t(std::max<int64_t>(sc->n_dense, 1)) * 4) : 0;
    if (hipMalloc(&sc->arena, c.off + 256) != hipSuccess) {
        sc->arena = nullptr;
        return fail(UF_ERR_NOMEM, "split lists");
    }
    char* b = static_cast<char*>(sc->arena);
    sc->dense = reinterpret_cast<int32_t*>(b + o_dense);
    sc->cls = reinterpret_cast<int32_t*>(b + o_cls);
    sc->roff = reinterpret_cast<int64_t*>(b + o_roff);
    sc->rs = weighted ? nullptr : reinterpret_cast<int32_t*>(b + o_rs);
    sc->rw = weighted ? reinterpret_cast<unsigned long long*>(b + o_rw) : nullptr;
    sc->sigma = reinterpret_cast<unsigned long long*>(b + o_sig);
    sc->dlen_hi = reinterpret_cast<uint16_t*>(b + o_dhi);
    sc->dlen_lo = reinterpret_cast<uint16_t*>(b + o_dlo);
    sc->rl = reinterpret_cast<int64_t*>(b + o_rl);
    sc->soff = reinterpret_cast<int64_t*>(b + o_soff);
    sc->entries = reinterpret_cast<ufs::SlotEntry*>(b + o_ent);
    sc->lo_ord = weighted ? reinterpret_cast<int32_t*>(b + o_lord) : nullptr;
    // temporaries in the embedding's scratch: unsorted list members, list fill
    // cursors, per-sample counts and cursors, and the list ids by sort class
    Carver t;
    const size_t t_rs = t.take(ne * 4);
    const size_t t_rq = t.take(ne * 8);
    const size_t t_fill = t.take(nl * 4);
    const size_t t_scnt = t.take(nn * 4);
    const size_t t_scur = t.take(nn * 4);
    const size_t t_dnnz = t.take(nn * 4);
    const size_t t_small = t.take(std::max<size_t>(small_ids.size(), 1) * 4);
    const size_t t_large = t.take(std::max<size_t>(large_ids.size(), 1) * 4);
    const size_t t_nodes = t.take(size_t(std::max<int64_t>(nb, 1)) * 16);
    uf_status sst = UF_OK;
    char* tb = split_scratch(e, t.off + 256, &sst);
    if (!tb) return sst;
    int32_t* rs_tmp = reinterpret_cast<int32_t*>(tb + t_rs);
    int64_t* rq_tmp = reinterpret_cast<int64_t*>(tb + t_rq);
    int32_t* fill = reinterpret_cast<int32_t*>(tb + t_fill);
    int32_t* scnt = reinterpret_cast<int32_t*>(tb + t_scnt);
    int32_t* scur = reinterpret_cast<int32_t*>(tb + t_scur);
    int32_t* dnnz = reinterpret_cast<int32_t*>(tb + t_dnnz);
    int32_t* d_small = reinterpret_cast<int32_t*>(tb + t_small);
    int32_t* d_large = reinterpret_cast<int32_t*>(tb + t_large);
    int4* nodes = reinterpret_cast<int4*>(tb + t_nodes);
    if (sc->n_dense) UF_HIP(hipMemcpy(sc->dense, dense.data(), size_t(sc->n_dense) * 4, hipMemcpyHostToDevice));
    if (weighted && sc->n_dense) {
        // the dense list in ascending lo, for the merge embedding of the dense chunks
        std::vector<int32_t> lo(size_t(nb + 1));
        UF_HIP(hipMemcpy(lo.data(), e->lo, size_t(nb + 1) * 4, hipMemcpyDeviceToHost));
        std::vector<int32_t> ord(size_t(sc->n_dense));
        for (int64_t k = 0; k < sc->n_dense; ++k) ord[size_t(k)] = int32_t(k);
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
            return lo[size_t(dense[size_t(x)])] < lo[size_t(dense[size_t(y)])];
        });
        UF_HIP(hipMemcpy(sc->lo_ord, ord.data(), ord.size() * 4, hipMemcpyHostToDevice));
    }
    if (nb) UF_HIP(hipMemcpy(sc->cls, cls.data(), size_t(nb) * 4, hipMemcpyHostToDevice));
    UF_HIP(hipMemcpy(sc->roff, roff.data(), roff.size() * 8, hipMemcpyHostToDevice));
    if (!small_ids.empty())
        UF_HIP(hipMemcpy(d_small, small_ids.data(), small_ids.size() * 4, hipMemcpyHostToDevice));
    if (!large_ids.empty())
        UF_HIP(hipMemcpy(d_large, large_ids.data(), large_ids.size() * 4, hipMemcpyHostToDevice));
    {
        ProfScope ps("split_fill", s);
        UF_HIP(ufk::zero_u32(reinterpret_cast<unsigned*>(fill), int64_t(nl), s));
        UF_HIP(ufk::zero_u32(reinterpret_cast<unsigned*>(scnt), int64_t(nn), s));
        UF_HIP(ufk::zero_u32(reinterpret_cast<unsigned*>(scur), int64_t(nn), s));
        UF_HIP(ufk::zero_u32(reinterpret_cast<unsigned*>(dnnz), int64_t(nn), s));
        UF_HIP(ufk::zero_u32(reinterpret_cast<unsigned*>(sc->sigma), int64_t(nn) * 2, s));
        UF_HIP(ufs::split_fill(ev, weighted != 0, sc->cls, nodes, sc->roff, fill, rs_tmp, rq_tmp,
                               sc->sigma, scnt, dnnz, 1.0 / sc->unit, s));
    }
    std::vector<int32_t> hcnt(nn, 0), hdnnz(nn, 0);
    std::vector<double> hsw(nn, 0.0);
    std::vector<unsigned long long> hsig(nn, 0);
    UF_HIP(hipStreamSynchronize(s));
    if (n) {
        UF_HIP(hipMemcpy(hcnt.data(), scnt, size_t(n) * 4, hipMemcpyDeviceToHost));
        UF_HIP(hipMemcpy(hdnnz.data(), dnnz, size_t(n) * 4, hipMemcpyDeviceToHost));
        UF_HIP(hipMemcpy(hsw.data(), e->sw, size_t(n) * 8, hipMemcpyDeviceToHost));
        UF_HIP(hipMemcpy(hsig.data(), sc->sigma, size_t(n) * 8, hipMemcpyDeviceToHost));
    }
    if (weighted) sc->q_scale = fixed_point_scale(hsw, hsig, sc->unit, hdnnz, sc->n_dense);
    std::vector<int64_t> soff(size_t(n + 1), 0);
    for (int64_t i = 0; i < n; ++i) soff[size_t(i + 1)] = soff[size_t(i)] + hcnt[size_t(i)];
    if (soff[size_t(n)] != sc->n_entries)
        return fail(UF_ERR_DEVICE, "sparse split: list entry counts disagree");
    UF_HIP(hipMemcpy(sc->soff, soff.data(), soff.size() * 8, hipMemcpyHostToDevice));
    {
        ProfScope ps("sort_lists", s);
        UF_HIP(ufs::sort_lists(sc->roff, d_small, int64_t(small_ids.size()), d_large,
                               int64_t(large_ids.size()), n, ufs::slot_segment_len(0, n / 2),
                               rs_tmp, rq_tmp, sc->rs, sc->rw, sc->soff, scur, sc->entries, s));
    }
    {
        ProfScope ps("split_lengths", s);
        UF_HIP(ufs::split_lengths(sc->cls, nb, sc->dense, sc->n_dense, sc->n_dense_pad, e->len_hi,
                                  e->len_lo, sc->dlen_hi, sc->dlen_lo, sc->rl, s));
        if (!weighted) UF_HIP(ufs::entry_lengths(sc->entries, sc->n_entries, sc->rl, s));
    }
    UF_HIP(hipStreamSynchronize(s));
    *out = std::move(sc);
    return UF_OK;
}

// The split of one variant at the current threshold: the cached one, or a new
// build (also when force is set).  The returned reference keeps it alive for the
// caller even if another thread replaces it meanwhile.
uf_status ensure_split(const uf_embedding* ce, int weighted, void* stream,
                       std::shared_ptr<SplitCache>* out, bool force = false,
                       const std::vector<int32_t>* counts = nullptr) {
    if (!ce) return fail(UF_ERR_ARG, "embedding is NULL");
    uf_embedding* e = const_cast<uf_embedding*>(ce);   // the cache is internal state
    const int w = weighted ? 1 : 0;
    std::lock_guard<std::mutex> lk(e->split_mu);
    const double thr = g_split_threshold[w].load();
    if (!force && e->split[w] && e->split[w]->threshold == thr) {
        *out = e->split[w];
        return UF_OK;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int32_t> own;
    if (!counts) {
        uf_status st = branch_counts(e, s, &own);
        if (st != UF_OK) return st;
        counts = &own;
    }
    std::shared_ptr<SplitCache> sc;
    uf_status st = build_split(e, w, thr, *counts, s, &sc);
    if (st != UF_OK) return st;
    e->split[w] = sc;   // a previous split is freed when its last user lets go
    *out = std::move(sc);
    return UF_OK;
}

// ------------------------------------------------------------------ planning
struct Plan {
    int64_t n = 0, S = 0, sb = 0, se = 0, sr = 0;
    int weighted = 0;
    uf_precision prec = UF_FP64;
    bool rowstats = false;
    int64_t kc = 0, nchunks = 0, kpad = 0;
    int64_t n_parts = 0;
    size_t off_acc = 0, off_q = 0, off_chunk = 0, off_part = 0, off_rm = 0, off_m = 0, total = 0;
};

// sp: the variant's split for the split precisions (ignored otherwise).
// fit > 0: the node chunk is sized so that the whole workspace fits in fit bytes
// (at least 32 branches per chunk, or all of them when fewer), else UF_ERR_RANGE.
uf_status make_plan(const uf_embedding* e, int weighted, uf_precision prec, int64_t sb,
                    int64_t se, bool rowstats, Plan* p, const SplitCache* sp = nullptr,
                    size_t fit = 0) {
    if (!e) return fail(UF_ERR_ARG, "embedding is NULL");
    if (prec != UF_FP64 && prec != UF_FP32 && prec != UF_MFMA_BF16X2 && prec != UF_FP32_SPLIT &&
        prec != UF_MFMA_SPLIT)
        return fail(UF_ERR_ARG, "unknown precision");
    if (weighted && (prec == UF_MFMA_BF16X2 || prec == UF_MFMA_SPLIT))
        return fail(UF_ERR_UNSUPPORTED,
                    "the MFMA Gram path exists for the unweighted variant only");
    if (!weighted && prec == UF_FP32_SPLIT)
        return fail(UF_ERR_UNSUPPORTED,
                    "UF_FP32_SPLIT is the weighted-normalized split; use UF_MFMA_SPLIT");
    const int64_t n = e->n;
    const int64_t S = n / 2;
    if (sb < 0 || se < sb || se > S)
        return fail(UF_ERR_RANGE, "stripe range must satisfy 0 <= begin <= end <= floor(N/2)");
    p->n = n;
    p->S = S;
    p->sb = sb;
    p->se = se;
    p->sr = se - sb;
    p->weighted = weighted;
    p->prec = prec;
    p->rowstats = rowstats;
    const bool split = prec == UF_FP32_SPLIT || prec == UF_MFMA_SPLIT;
    const bool mfma = prec == UF_MFMA_BF16X2 || prec == UF_MFMA_SPLIT;
    if (split && !sp) return fail(UF_ERR_ARG, "split precision without a split");
    const int64_t nb = split ? sp->n_dense : e->nb;
    const size_t elem = prec == UF_FP64 ? 8 : (mfma ? 1 : 4);
    p->n_parts = std::max<int64_t>(1, (p->sr + 255) / 256);
    const size_t acc_elem = (prec == UF_FP64) ? 8 : 4;
    // workspace layout for a chunk of kc branches
    auto layout = [&](int64_t kc) {
        p->kc = kc;
        p->nchunks = nb > 0 && kc > 0 ? (nb + kc - 1) / kc : 0;
        p->kpad = (kc + ufk::kGramKPad - 1) / ufk::kGramKPad * ufk::kGramKPad;
        Carver c;
        p->off_acc = c.take(size_t(p->sr) * size_t(n) * acc_elem);
        p->off_q = rowstats ? c.take(size_t(p->sr) * size_t(n) * 8) : 0;
        if (mfma)
            p->off_chunk = c.take(size_t(n) * size_t(p->kpad));   // FP8 presence
        else
            p->off_chunk = c.take(size_t(kc) * size_t(n) * elem);
        p->off_part = rowstats ? c.take(size_t(p->n_parts) * size_t(n) * 8) : 0;
        p->off_rm = rowstats ? c.take(size_t(n) * 8) : 0;
        p->off_m = split ? c.take(size_t(p->sr) * size_t(n) * 8) : 0;
        p->total = c.off + 256;
    };
    auto shape = [&](int64_t kc) {
        kc = std::max<int64_t>(kc, 32);
        if (mfma) kc = (kc + ufk::kGramKPad - 1) / ufk::kGramKPad * ufk::kGramKPad;
        return std::min<int64_t>(kc, std::max<int64_t>(nb, 1));
    };
    if (fit > 0) {
        // the chunk takes what the rest leaves (each carved piece may lose up to
        // 255 bytes to alignment)
        layout(0);
        const size_t rest = p->total + 6 * 256;
        const size_t per = mfma ? size_t(n) : size_t(n) * elem;
        const int64_t room = rest < fit ? int64_t((fit - rest) / std::max<size_t>(per, 1)) : 0;
        const int64_t kc = std::min<int64_t>(room, std::max<int64_t>(nb, 1));
        if (mfma || kc < std::min<int64_t>(32, std::max<int64_t>(nb, 1)))
            return fail(UF_ERR_RANGE, "problem too large for the fixed scratch (" +
                                          std::to_string(fit) + " bytes)");
        layout(kc);
        if (p->total > fit)
            return fail(UF_ERR_RANGE, "problem too large for the fixed scratch (" +
                                          std::to_string(fit) + " bytes)");
        return UF_OK;
    }
    int64_t kc = g_chunk_nodes.load();
    if (kc <= 0) {
        const double budget = 8.0 * 1024 * 1024 * 1024;
        kc = static_cast<int64_t>(budget / (double(std::max<int64_t>(n, 1)) * double(elem)));
    }
    layout(shape(kc));
    return UF_OK;
}

uf_status run_dm(const uf_embedding* e, int weighted, uf_precision prec, int64_t sb, int64_t se,
                 int layout, uf_out_dtype odt, void* out, double* row_out, double* grand_mean,
                 bool full_means, void* ws, size_t ws_bytes, void* stream, bool fit_ws = false) {
    if (!e) return fail(UF_ERR_ARG, "embedding is NULL");
    if (!out) return fail(UF_ERR_ARG, "output pointer is NULL");
    if (layout != UF_CONDENSED && layout != UF_STRIPES) return fail(UF_ERR_ARG, "bad layout");
    if (odt != UF_OUT_F64 && odt != UF_OUT_F32) return fail(UF_ERR_ARG, "bad output dtype");
    const bool rowstats = row_out != nullptr || grand_mean != nullptr;
    int dev = 0;
    uf_status st = check_device(&dev);
    if (st != UF_OK) return st;
    if (dev != e->device) return fail(UF_ERR_DEVICE, "embedding lives on another device");
    Plan p;
    std::shared_ptr<SplitCache> hold;   // keeps the split alive while this call enqueues
    if ((prec == UF_FP32_SPLIT && weighted) || (prec == UF_MFMA_SPLIT && !weighted)) {
        st = ensure_split(e, weighted, stream, &hold);
        if (st != UF_OK) return st;
    }
    st = make_plan(e, weighted, prec, sb, se, rowstats, &p, hold.get(), fit_ws ? ws_bytes : 0);
    if (st != UF_OK) return st;
    if (!ws || ws_bytes < p.total)
        return fail(UF_ERR_WORKSPACE, "workspace missing or smaller than uf_workspace_size()");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p.sr == 0 || p.n < 2) {
        // zeroed by a kernel, so that the call can be captured into a graph
        if (row_out && p.n > 0) UF_HIP(ufk::zero_u32(reinterpret_cast<unsigned*>(row_out), 2 * p.n, s));
        if (grand_mean) UF_HIP(ufk::zero_u32(reinterpret_cast<unsigned*>(grand_mean), 2, s));
        return UF_OK;
    }
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
    void* acc = base + p.off_acc;
    double* q = rowstats ? reinterpret_cast<double*>(base + p.off_q) : nullptr;
    void* chunk = base + p.off_chunk;
    const int64_t nb = e->nb;
    const bool split = prec == UF_FP32_SPLIT || prec == UF_MFMA_SPLIT;
    const SplitCache* sp = split ? hold.get() : nullptr;
    // Dense part: node chunks (all branches, or the split's dense list) into acc.
    for (int64_t c = 0; c < p.nchunks; ++c) {
        const int64_t k0 = c * p.kc;
        const int64_t kc = std::min<int64_t>(p.kc, (sp ? sp->n_dense : nb) - k0);
        const int first = c == 0;
        if (prec == UF_FP64) {
            double* E = static_cast<double*>(chunk);
            {
                ProfScope ps("embed_nm", s);
                UF_HIP(ufk::embed_node_major_f64(*e, k0, kc, weighted, E, s));
            }
            ProfScope ps(weighted ? "band_wn_f64" : "band_uw_f64", s);
            UF_HIP(ufk::band_f64(E, e->len + k0, kc, p.n, p.sb, p.se, weighted, first,
                                 static_cast<double*>(acc), s));
        } else if (prec == UF_FP32) {
            float* E = static_cast<float*>(chunk);
            {
                ProfScope ps("embed_nm", s);
                UF_HIP(ufk::embed_node_major_f32(*e, k0, kc, weighted, E, s));
            }
            ProfScope ps(weighted ? "band_wn_f32" : "band_uw_f32", s);
            UF_HIP(ufk::band_f32(E, e->len32 + k0, kc, p.n, p.sb, p.se, weighted, first,
                                 static_cast<float*>(acc), s));
        } else if (prec == UF_FP32_SPLIT && sp->q_scale > 0.0) {
            uint32_t* E = static_cast<uint32_t*>(chunk);
            {
                ProfScope ps("embed_nm", s);
                UF_HIP(ufs::embed_list_u32(emb_view(*e), sp->dense, sp->lo_ord, sp->n_dense,
                                           e->max_total < (int64_t(1) << 32), k0, kc,
                                           sp->q_scale, E, s));
            }
            ProfScope ps("band_wn_u32", s);
            UF_HIP(ufk::band_u32(E, kc, p.n, p.sb, p.se, first, static_cast<uint32_t*>(acc), s));
        } else if (prec == UF_FP32_SPLIT) {
            float* E = static_cast<float*>(chunk);
            {
                ProfScope ps("embed_nm", s);
                UF_HIP(ufs::embed_list_f32(emb_view(*e), sp->dense, sp->lo_ord, sp->n_dense,
                                           e->max_total < (int64_t(1) << 32), k0, kc, E, s));
            }
            ProfScope ps("band_wn_f32", s);
            UF_HIP(ufk::band_f32(E, nullptr, kc, p.n, p.sb, p.se, 1, first,
                                 static_cast<float*>(acc), s));
        } else {
            const bool ms = prec == UF_MFMA_SPLIT;
            uint8_t* P = static_cast<uint8_t*>(chunk);
            const int64_t kpad = (kc + ufk::kGramKPad - 1) / ufk::kGramKPad * ufk::kGramKPad;
            {
                ProfScope ps("embed_pres", s);
                UF_HIP(ufk::embed_presence_fp8(*e, k0, kc, kpad, P, s,
                                                ms ? sp->dense : nullptr));
            }
            ProfScope ps("gram_mfma", s);
            UF_HIP(ufk::gram_mfma(P, (ms ? sp->dlen_hi : e->len_hi) + k0,
                                  (ms ? sp->dlen_lo : e->len_lo) + k0, kpad, p.n, p.sb,
                                  p.se, first, static_cast<float*>(acc), s));
        }
    }
    if (p.nchunks == 0) {  // no (dense) branch: the dense part is 0
        const int64_t words = p.sr * p.n * (prec == UF_FP64 ? 2 : 1);
        UF_HIP(ufk::zero_u32(static_cast<unsigned*>(acc), words, s));
    }
    // Non-dense part of a split: exact fixed-point pair sums into M (every
    // element of the range written).
    unsigned long long* M = nullptr;
    if (sp) {
        M = reinterpret_cast<unsigned long long*>(base + p.off_m);
        ProfScope ps(weighted ? "rare_slots_wn" : "rare_slots_uw", s);
        UF_HIP(ufs::rare_slots(sp->rs, sp->rw, sp->soff, sp->entries, p.n, p.sb, p.se, M, s));
    }
    const double* scal = weighted ? e->sw
                                  : (prec == UF_FP64 ? e->wu : (prec == UF_FP32 ? e->wu32 : e->wub));
    {
        ProfScope ps("finalize", s);
        const bool fixed = sp && weighted && sp->q_scale > 0.0;
        const int acc_type = prec == UF_FP64 ? ufk::kAccF64 : (fixed ? ufk::kAccU32 : ufk::kAccF32);
        UF_HIP(ufk::finalize(weighted ? 0 : 1, acc, acc_type, fixed ? 1.0 / sp->q_scale : 1.0, scal,
                             p.n, p.sb, p.se, layout, odt == UF_OUT_F32 ? 1 : 0, out, q, s, M,
                             sp && weighted ? sp->sigma : nullptr,
                             sp && weighted ? sp->unit : 0x1p-40));
    }
    if (rowstats) {
        ProfScope ps("row_sums", s);
        double* part = reinterpret_cast<double*>(base + p.off_part);
        double* rm = row_out ? row_out : reinterpret_cast<double*>(base + p.off_rm);
        const double scale = full_means ? 1.0 / double(p.n) : 1.0;
        UF_HIP(ufk::row_sums(q, p.n, p.sb, p.se, part, p.n_parts, scale, rm, s));
        if (grand_mean) UF_HIP(ufk::grand_mean(rm, p.n, grand_mean, s));
    }
    return UF_OK;
}

}  // namespace

namespace ufh {
uf_status fail(uf_status st, const std::string& msg) { return ::fail(st, msg); }
uf_status hip_fail(hipError_t e, const char* what) { return ::hip_fail(e, what); }
uf_status check_device(int* dev_out) { return ::check_device(dev_out); }
struct ProfHandle {
    ProfScope scope;
    ProfHandle(const char* name, hipStream_t s) : scope(name, s) {}
};
ProfHandle* prof_begin(const char* name, hipStream_t s) {
    if (!g_prof_on.load() || t_prof_suppress) return nullptr;
    return new (std::nothrow) ProfHandle(name, s);
}
void prof_end(ProfHandle* h) { delete h; }
}  // namespace ufh

// =========================================================================
// C ABI
// =========================================================================
extern "C" {

const char* uf_status_string(uf_status s) {
    switch (s) {
        case UF_OK: return "ok";
        case UF_ERR_ARG: return "invalid argument";
        case UF_ERR_TREE: return "invalid tree";
        case UF_ERR_TABLE: return "invalid table";
        case UF_ERR_EMPTY_SAMPLE: return "sample with zero total count";
        case UF_ERR_RANGE: return "stripe range out of bounds";
        case UF_ERR_NOMEM: return "out of memory";
        case UF_ERR_DEVICE: return "device error";
        case UF_ERR_UNSUPPORTED: return "unsupported precision for this variant";
        case UF_ERR_WORKSPACE: return "workspace too small";
    }
    return "unknown status";
}

const char* uf_last_error_message(void) { return g_last_error.c_str(); }

int64_t uf_n_stripes(int64_t n) { return n < 0 ? 0 : n / 2; }

int64_t uf_condensed_index(int64_t n, int64_t i, int64_t j) {
    if (i < 0 || j < 0 || i >= n || j >= n || i == j) return -1;
    if (i > j) std::swap(i, j);
    return n * i - i * (i + 1) / 2 + (j - i - 1);
}

void uf_set_chunk_nodes(int64_t nodes) { g_chunk_nodes.store(nodes < 0 ? 0 : nodes); }

uf_status uf_set_split_threshold(int weighted, double fraction) {
    if (!(fraction <= 1.0)) return fail(UF_ERR_ARG, "split threshold must be <= 1 (or < 0: automatic)");
    g_split_threshold[weighted ? 1 : 0].store(fraction < 0.0 ? -1.0 : fraction);
    return UF_OK;
}

uf_status uf_split_stats(const uf_embedding* e, int weighted, int64_t* n_dense, int64_t* n_lists,
                         int64_t* n_pairs) {
    return guarded([&]() -> uf_status {
        if (!e) return fail(UF_ERR_ARG, "embedding is NULL");
        std::shared_ptr<SplitCache> sc;
        uf_status st = ensure_split(e, weighted, nullptr, &sc);
        if (st != UF_OK) return st;
        if (n_dense) *n_dense = sc->n_dense;
        if (n_lists) *n_lists = sc->n_lists;
        if (n_pairs) *n_pairs = sc->n_pairs;
        return UF_OK;
    });
}

void uf_profile_enable(int on) { g_prof_on.store(on ? 1 : 0); }

void uf_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& r : g_prof_pending) {
        (void)hipEventSynchronize(r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof_pending.clear();
    g_prof_done.clear();
}

uf_status uf_profile_read(const char* kernel, double* total_ms, int64_t* launches) {
    return guarded([&]() -> uf_status {
        if (!kernel || !total_ms || !launches) return fail(UF_ERR_ARG, "NULL argument");
        std::lock_guard<std::mutex> lk(g_prof_mu);
        uf_status st = UF_OK;
        for (auto& r : g_prof_pending) {
            float ms = 0.0f;
            hipError_t e = hipEventSynchronize(r.b);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
            if (e != hipSuccess) st = hip_fail(e, "profile event");
            auto& d = g_prof_done[r.name];
            d.first += ms;
            d.second += 1;
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        g_prof_pending.clear();
        auto it = g_prof_done.find(kernel);
        *total_ms = it == g_prof_done.end() ? 0.0 : it->second.first;
        *launches = it == g_prof_done.end() ? 0 : it->second.second;
        return st;
    });
}

// ------------------------------------------------------------------ tree
uf_status uf_tree_load(int64_t m, const int64_t* parent, const double* length, uf_tree** out) {
    return guarded([&]() -> uf_status {
        if (!out) return fail(UF_ERR_ARG, "out is NULL");
        *out = nullptr;
        if (m < 1 || !parent || !length) return fail(UF_ERR_ARG, "need n_nodes >= 1 and arrays");
        if (m > (int64_t(1) << 30)) return fail(UF_ERR_ARG, "more than 2^30 nodes");
        int64_t root = -1;
        for (int64_t v = 0; v < m; ++v) {
            const int64_t p = parent[v];
            if (p == -1) {
                if (root >= 0) return fail(UF_ERR_TREE, "more than one root");
                root = v;
            } else if (p < 0 || p >= m || p == v) {
                return fail(UF_ERR_TREE, "parent id out of range at node " + std::to_string(v));
            } else if (!std::isfinite(length[v]) || length[v] < 0.0) {
                return fail(UF_ERR_TREE, "branch length must be finite and >= 0 at node " +
                                             std::to_string(v));
            }
        }
        if (root < 0) return fail(UF_ERR_TREE, "no root (parent -1)");
        // children in CSR, ascending child id
        std::vector<int64_t> first(m + 1, 0), kids(m > 1 ? m - 1 : 1);
        for (int64_t v = 0; v < m; ++v)
            if (parent[v] >= 0) first[parent[v] + 1]++;
        for (int64_t v = 0; v < m; ++v) first[v + 1] += first[v];
        {
            std::vector<int64_t> fill(first.begin(), first.end() - 1);
            for (int64_t v = 0; v < m; ++v)
                if (parent[v] >= 0) kids[fill[parent[v]]++] = v;
        }
        auto t = new uf_tree();
        std::unique_ptr<uf_tree> guard(t);
        t->n_nodes = m;
        t->node_at.reserve(m);
        // iterative postorder from the root
        std::vector<std::pair<int64_t, int64_t>> stack;
        stack.reserve(64);
        stack.emplace_back(root, first[root]);
        while (!stack.empty()) {
            auto& top = stack.back();
            if (top.second < first[top.first + 1]) {
                const int64_t c = kids[top.second++];
                if (int64_t(stack.size()) > m) return fail(UF_ERR_TREE, "cycle");
                stack.emplace_back(c, first[c]);
            } else {
                t->node_at.push_back(top.first);
                stack.pop_back();
            }
        }
        if (int64_t(t->node_at.size()) != m)
            return fail(UF_ERR_TREE, "not every node is reachable from the root (cycle?)");
        t->pos_of.assign(m, -1);
        for (int64_t k = 0; k < m; ++k) t->pos_of[t->node_at[k]] = k;
        t->parent_pos.resize(m);
        t->len.resize(m);
        t->tip_rank.assign(m, -1);
        std::vector<int64_t> size(m, 1);
        std::vector<int64_t> tips_before(m + 1, 0);
        for (int64_t k = 0; k < m; ++k) {
            const int64_t v = t->node_at[k];
            t->parent_pos[k] = parent[v] >= 0 ? int32_t(t->pos_of[parent[v]]) : -1;
            t->len[k] = parent[v] >= 0 ? length[v] : 0.0;
            const bool is_tip = first[v + 1] == first[v];
            tips_before[k + 1] = tips_before[k] + (is_tip ? 1 : 0);
            if (is_tip) {
                t->tip_rank[v] = int32_t(tips_before[k]);
                t->tip_pos.push_back(int32_t(k));
            }
        }
        for (int64_t k = 0; k < m - 1; ++k) size[t->parent_pos[k]] += size[k];
        t->lo.resize(m);
        t->hi.resize(m);
        for (int64_t k = 0; k < m; ++k) {
            t->lo[k] = int32_t(tips_before[k - size[k] + 1]);
            t->hi[k] = int32_t(tips_before[k + 1]);
        }
        t->n_tips = tips_before[m];
        *out = guard.release();
        return UF_OK;
    });
}

int64_t uf_tree_n_nodes(const uf_tree* t) { return t ? t->n_nodes : -1; }
int64_t uf_tree_n_tips(const uf_tree* t) { return t ? t->n_tips : -1; }
void uf_free_tree(uf_tree* t) { delete t; }

// ------------------------------------------------------------------ table
uf_status uf_table_load(const uf_tree* t, int64_t n, const int64_t* indptr, const int64_t* tip,
                        const int64_t* counts, uf_table** out) {
    return guarded([&]() -> uf_status {
        if (!out) return fail(UF_ERR_ARG, "out is NULL");
        *out = nullptr;
        if (!t || n < 0 || !indptr) return fail(UF_ERR_ARG, "need a tree and indptr");
        if (indptr[0] != 0) return fail(UF_ERR_TABLE, "indptr[0] must be 0");
        for (int64_t s = 0; s < n; ++s)
            if (indptr[s + 1] < indptr[s]) return fail(UF_ERR_TABLE, "indptr must not decrease");
        const int64_t nnz = indptr[n];
        if (nnz > 0 && (!tip || !counts)) return fail(UF_ERR_ARG, "tip/count arrays are NULL");
        if (n > (int64_t(1) << 31) - 1) return fail(UF_ERR_ARG, "too many samples");
        auto tb = new uf_table();
        std::unique_ptr<uf_table> guard(tb);
        tb->n_samples = n;
        tb->n_tips = t->n_tips;
        tb->row_ptr.assign(n + 1, 0);
        tb->total.assign(n, 0);
        tb->rank.reserve(nnz);
        tb->count.reserve(nnz);
        std::vector<std::pair<int32_t, int64_t>> row;
        for (int64_t s = 0; s < n; ++s) {
            row.clear();
            for (int64_t e = indptr[s]; e < indptr[s + 1]; ++e) {
                const int64_t v = tip[e];
                if (v < 0 || v >= t->n_nodes)
                    return fail(UF_ERR_TABLE, "feature id out of range in sample " + std::to_string(s));
                if (t->tip_rank[v] < 0)
                    return fail(UF_ERR_TABLE, "feature maps to an internal node in sample " +
                                                  std::to_string(s));
                if (counts[e] < 0) return fail(UF_ERR_TABLE, "negative count in sample " + std::to_string(s));
                row.emplace_back(t->tip_rank[v], counts[e]);
            }
            std::sort(row.begin(), row.end());
            int64_t total = 0;
            for (size_t k = 0; k < row.size(); ++k) {
                if (k > 0 && row[k].first == row[k - 1].first)
                    return fail(UF_ERR_TABLE, "duplicate feature in sample " + std::to_string(s));
                if (row[k].second == 0) continue;
                if (total > (int64_t(1) << 52) - row[k].second)
                    return fail(UF_ERR_TABLE, "sample total exceeds 2^52");
                total += row[k].second;
                tb->rank.push_back(row[k].first);
                tb->count.push_back(row[k].second);
            }
            if (total <= 0)
                return fail(UF_ERR_EMPTY_SAMPLE, "sample " + std::to_string(s) + " has zero total count");
            tb->total[s] = total;
            tb->row_ptr[s + 1] = int64_t(tb->rank.size());
        }
        *out = guard.release();
        return UF_OK;
    });
}

int64_t uf_table_n_samples(const uf_table* t) { return t ? t->n_samples : -1; }
void uf_free_table(uf_table* t) { delete t; }

// ------------------------------------------------------------------ embedding
}  // extern "C"

namespace {
uf_status embed_impl(const uf_tree* t, const uf_table* tb, void* stream, uf_embedding** out) {
    {
        if (!out) return fail(UF_ERR_ARG, "out is NULL");
        *out = nullptr;
        if (!t || !tb) return fail(UF_ERR_ARG, "tree or table is NULL");
        if (tb->n_tips != t->n_tips) return fail(UF_ERR_ARG, "table was loaded against another tree");
        int dev = 0;
        uf_status st = check_device(&dev);
        if (st != UF_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int64_t n = tb->n_samples;
        const int64_t m = t->n_nodes;
        const int64_t nb = m - 1;
        const int64_t nnz = int64_t(tb->rank.size());
        const int64_t nb_pad = (nb + ufk::kGramKPad + 63) / 64 * 64;  // room for the last K step
        // host-side arrays
        std::vector<int64_t> cum(size_t(nnz + n), 0);
        for (int64_t r = 0; r < n; ++r) {
            int64_t acc = 0;
            const int64_t a = tb->row_ptr[r], b = tb->row_ptr[r + 1];
            for (int64_t e = a; e < b; ++e) {
                cum[a + r + (e - a)] = acc;
                acc += tb->count[e];
            }
            cum[b + r] = acc;
        }
        std::vector<double> total(n);
        for (int64_t r = 0; r < n; ++r) total[r] = double(tb->total[r]);
        std::vector<float> len32(nb_pad, 0.0f);
        std::vector<uint16_t> lhi(nb_pad, 0), llo(nb_pad, 0);
        for (int64_t k = 0; k < nb; ++k) {
            len32[k] = static_cast<float>(t->len[k]);
            lhi[k] = bf16_bits(t->len[k]);
            llo[k] = bf16_bits(t->len[k] - bf16_value(lhi[k]));
        }
        // root distances by position for the three length roundings (FP64 sums)
        std::vector<double> d64(m, 0.0), d32(m, 0.0), dbf(m, 0.0);
        for (int64_t k = m - 2; k >= 0; --k) {
            const int32_t p = t->parent_pos[k];
            d64[k] = d64[p] + t->len[k];
            d32[k] = d32[p] + double(len32[k]);
            dbf[k] = dbf[p] + (bf16_value(lhi[k]) + bf16_value(llo[k]));
        }
        // one device allocation for everything
        Carver c;
        const size_t o_rowptr = c.take(size_t(n + 1) * 8);
        const size_t o_rank = c.take(size_t(std::max<int64_t>(nnz, 1)) * 4);
        const size_t o_cum = c.take(size_t(nnz + n) * 8 + 8);
        const size_t o_total = c.take(size_t(std::max<int64_t>(n, 1)) * 8);
        const size_t o_lo = c.take(size_t(m) * 4);   // includes the root's interval
        const size_t o_hi = c.take(size_t(m) * 4);
        const size_t o_len = c.take(size_t(std::max<int64_t>(nb, 1)) * 8);
        const size_t o_len32 = c.take(size_t(nb_pad) * 4);
        const size_t o_lhi = c.take(size_t(nb_pad) * 2);
        const size_t o_llo = c.take(size_t(nb_pad) * 2);
        const size_t o_sw = c.take(size_t(std::max<int64_t>(n, 1)) * 8);
        const size_t o_wu = c.take(size_t(std::max<int64_t>(n, 1)) * 8);
        const size_t o_wu32 = c.take(size_t(std::max<int64_t>(n, 1)) * 8);
        const size_t o_wub = c.take(size_t(std::max<int64_t>(n, 1)) * 8);
        const size_t o_ppos = c.take(size_t(m) * 4);
        const size_t o_tpos = c.take(size_t(std::max<int64_t>(t->n_tips, 1)) * 4);
        const size_t o_d64 = c.take(size_t(m) * 8);
        const size_t o_d32 = c.take(size_t(m) * 8);
        const size_t o_dbf = c.take(size_t(m) * 8);
        void* arena = nullptr;
        hipError_t he = hipMalloc(&arena, c.off + 256);
        if (he != hipSuccess) return fail(UF_ERR_NOMEM, "device allocation of the embedding failed");
        auto e = new uf_embedding();
        std::unique_ptr<uf_embedding> guard(e);
        e->arena = arena;
        e->device = dev;
        e->n = n;
        e->nb = nb;
        e->nnz = nnz;
        for (int64_t r = 0; r < n; ++r) e->max_total = std::max<int64_t>(e->max_total, tb->total[r]);
        char* b = static_cast<char*>(arena);
        e->row_ptr = reinterpret_cast<int64_t*>(b + o_rowptr);
        e->rank = reinterpret_cast<int32_t*>(b + o_rank);
        e->cum = reinterpret_cast<int64_t*>(b + o_cum);
        e->total = reinterpret_cast<double*>(b + o_total);
        e->lo = reinterpret_cast<int32_t*>(b + o_lo);
        e->hi = reinterpret_cast<int32_t*>(b + o_hi);
        e->len = reinterpret_cast<double*>(b + o_len);
        e->len32 = reinterpret_cast<float*>(b + o_len32);
        e->len_hi = reinterpret_cast<uint16_t*>(b + o_lhi);
        e->len_lo = reinterpret_cast<uint16_t*>(b + o_llo);
        e->sw = reinterpret_cast<double*>(b + o_sw);
        e->wu = reinterpret_cast<double*>(b + o_wu);
        e->wu32 = reinterpret_cast<double*>(b + o_wu32);
        e->wub = reinterpret_cast<double*>(b + o_wub);
        int32_t* ppos = reinterpret_cast<int32_t*>(b + o_ppos);
        int32_t* tpos = reinterpret_cast<int32_t*>(b + o_tpos);
        e->parent_pos = ppos;
        e->tip_pos = tpos;
        // first position of each position's subtree: its leftmost tip's
        e->sub_first.resize(size_t(nb));
        for (int64_t k = 0; k < nb; ++k) e->sub_first[size_t(k)] = t->tip_pos[size_t(t->lo[size_t(k)])];
        double* dd64 = reinterpret_cast<double*>(b + o_d64);
        double* dd32 = reinterpret_cast<double*>(b + o_d32);
        double* ddbf = reinterpret_cast<double*>(b + o_dbf);
        e->d64 = dd64;
        e->d32 = dd32;
        e->dbf = ddbf;
        auto cleanup = [&](uf_status code) {
            (void)hipFree(arena);
            e->arena = nullptr;
            return code;
        };
        // synchronous copies (pageable host memory), then the scalar kernel
        auto H2D = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
            if (bytes == 0) return hipSuccess;
            return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
        };
        hipError_t rc = hipSuccess;
        if (rc == hipSuccess) rc = H2D(e->row_ptr, tb->row_ptr.data(), size_t(n + 1) * 8);
        if (rc == hipSuccess) rc = H2D(e->rank, tb->rank.data(), size_t(nnz) * 4);
        if (rc == hipSuccess) rc = H2D(e->cum, cum.data(), size_t(nnz + n) * 8);
        if (rc == hipSuccess) rc = H2D(e->total, total.data(), size_t(n) * 8);
        if (rc == hipSuccess) rc = H2D(e->lo, t->lo.data(), size_t(m) * 4);
        if (rc == hipSuccess) rc = H2D(e->hi, t->hi.data(), size_t(m) * 4);
        if (rc == hipSuccess) rc = H2D(e->len, t->len.data(), size_t(nb) * 8);
        if (rc == hipSuccess) rc = H2D(e->len32, len32.data(), size_t(nb_pad) * 4);
        if (rc == hipSuccess) rc = H2D(e->len_hi, lhi.data(), size_t(nb_pad) * 2);
        if (rc == hipSuccess) rc = H2D(e->len_lo, llo.data(), size_t(nb_pad) * 2);
        if (rc == hipSuccess) rc = H2D(ppos, t->parent_pos.data(), size_t(m) * 4);
        if (rc == hipSuccess) rc = H2D(tpos, t->tip_pos.data(), size_t(t->n_tips) * 4);
        if (rc == hipSuccess) rc = H2D(dd64, d64.data(), size_t(m) * 8);
        if (rc == hipSuccess) rc = H2D(dd32, d32.data(), size_t(m) * 8);
        if (rc == hipSuccess) rc = H2D(ddbf, dbf.data(), size_t(m) * 8);
        if (rc != hipSuccess) return cleanup(hip_fail(rc, "upload of the embedding inputs"));
        if (n > 0) {
            rc = ufk::sample_scalars(*e, ppos, tpos, dd64, dd32, ddbf, s);
            if (rc != hipSuccess) return cleanup(hip_fail(rc, "sample scalar kernel launch"));
        }
        rc = hipStreamSynchronize(s);
        if (rc != hipSuccess) return cleanup(hip_fail(rc, "sample scalar kernel"));
        *out = guard.release();
        return UF_OK;
    }
}
}  // namespace

extern "C" {

uf_status uf_embed(const uf_tree* t, const uf_table* tb, void* stream, uf_embedding** out) {
    return guarded([&]() -> uf_status { return embed_impl(t, tb, stream, out); });
}

int64_t uf_embedding_n_samples(const uf_embedding* e) { return e ? e->n : -1; }

uf_status uf_embedding_scalars(const uf_embedding* e, double* sw, double* wu) {
    return guarded([&]() -> uf_status {
        if (!e) return fail(UF_ERR_ARG, "embedding is NULL");
        if (sw && e->n) UF_HIP(hipMemcpy(sw, e->sw, size_t(e->n) * 8, hipMemcpyDeviceToHost));
        if (wu && e->n) UF_HIP(hipMemcpy(wu, e->wu, size_t(e->n) * 8, hipMemcpyDeviceToHost));
        return UF_OK;
    });
}

uf_status uf_embedding_prepare(const uf_embedding* ce, int what, void* stream) {
    return guarded([&]() -> uf_status {
        if (!ce) return fail(UF_ERR_ARG, "embedding is NULL");
        if (what & ~(UF_PREP_SCALARS | UF_PREP_SPLIT_UNWEIGHTED | UF_PREP_SPLIT_WEIGHTED))
            return fail(UF_ERR_ARG, "unknown preparation flag");
        int dev = 0;
        uf_status st = check_device(&dev);
        if (st != UF_OK) return st;
        if (dev != ce->device) return fail(UF_ERR_DEVICE, "embedding lives on another device");
        uf_embedding* e = const_cast<uf_embedding*>(ce);
        hipStream_t s = static_cast<hipStream_t>(stream);
        if ((what & UF_PREP_SCALARS) && e->n > 0) {
            ProfScope ps("sample_scalars", s);
            UF_HIP(ufk::sample_scalars(*e, e->parent_pos, e->tip_pos, e->d64, e->d32, e->dbf, s));
        }
        const bool sw = (what & UF_PREP_SPLIT_WEIGHTED) != 0, su = (what & UF_PREP_SPLIT_UNWEIGHTED) != 0;
        if (sw || su) {
            // the branch sample counts serve both variants' dense sets
            std::vector<int32_t> counts;
            {
                std::lock_guard<std::mutex> lk(e->split_mu);
                st = branch_counts(e, s, &counts);
            }
            if (st != UF_OK) return st;
            std::shared_ptr<SplitCache> sc;
            if (sw && (st = ensure_split(e, 1, stream, &sc, true, &counts)) != UF_OK) return st;
            if (su && (st = ensure_split(e, 0, stream, &sc, true, &counts)) != UF_OK) return st;
        }
        return UF_OK;
    });
}

void uf_free_embedding(uf_embedding* e) {
    if (!e) return;
    e->split[0].reset();
    e->split[1].reset();
    if (e->arena) (void)hipFree(e->arena);
    delete e;
}

// ------------------------------------------------------------------ workspace
uf_status uf_workspace_size(const uf_embedding* e, int weighted, uf_precision prec, int64_t sb,
                            int64_t se, int want_row_stats, size_t* bytes) {
    return guarded([&]() -> uf_status {
        if (!bytes) return fail(UF_ERR_ARG, "bytes is NULL");
        std::shared_ptr<SplitCache> sc;
        if (e && ((weighted && prec == UF_FP32_SPLIT) || (!weighted && prec == UF_MFMA_SPLIT))) {
            uf_status sst = ensure_split(e, weighted, nullptr, &sc);
            if (sst != UF_OK) return sst;
        }
        Plan p;
        uf_status st = make_plan(e, weighted ? 1 : 0, prec, sb, se, want_row_stats != 0, &p, sc.get());
        if (st != UF_OK) return st;
        *bytes = p.total;
        return UF_OK;
    });
}

// ------------------------------------------------------------------ distances
uf_status uf_dm_unweighted(const uf_embedding* e, uf_precision prec, uf_out_dtype odt, void* out,
                           double* row_means, double* grand_mean, void* ws, size_t ws_bytes,
                           void* stream) {
    return guarded([&]() -> uf_status {
        if (!e) return fail(UF_ERR_ARG, "embedding is NULL");
        return run_dm(e, 0, prec, 0, e->n / 2, UF_CONDENSED, odt, out, row_means, grand_mean,
                      true, ws, ws_bytes, stream);
    });
}

uf_status uf_dm_weighted_normalized(const uf_embedding* e, uf_precision prec, uf_out_dtype odt,
                                    void* out, double* row_means, double* grand_mean, void* ws,
                                    size_t ws_bytes, void* stream) {
    return guarded([&]() -> uf_status {
        if (!e) return fail(UF_ERR_ARG, "embedding is NULL");
        return run_dm(e, 1, prec, 0, e->n / 2, UF_CONDENSED, odt, out, row_means, grand_mean,
                      true, ws, ws_bytes, stream);
    });
}

uf_status uf_dm_unweighted_stripes(const uf_embedding* e, uf_precision prec, int64_t sb,
                                   int64_t se, uf_layout layout, uf_out_dtype odt, void* out,
                                   double* row_sums, void* ws, size_t ws_bytes, void* stream) {
    return guarded([&]() -> uf_status {
        return run_dm(e, 0, prec, sb, se, layout, odt, out, row_sums, nullptr, false, ws,
                      ws_bytes, stream);
    });
}

uf_status uf_dm_weighted_normalized_stripes(const uf_embedding* e, uf_precision prec, int64_t sb,
                                            int64_t se, uf_layout layout, uf_out_dtype odt,
                                            void* out, double* row_sums, void* ws,
                                            size_t ws_bytes, void* stream) {
    return guarded([&]() -> uf_status {
        return run_dm(e, 1, prec, sb, se, layout, odt, out, row_sums, nullptr, false, ws,
                      ws_bytes, stream);
    });
}

}  // extern "C"

// ------------------------------------------------------------------ no allocation
// Workspace of uf_dm_weighted_normalized_noalloc: a fixed device array.  Every
// device the library runs on holds its own copy, at its own address, for the
// life of the process.  In host code `scratch` names a host-side stand-in, so
// kernels only ever receive the per-device address looked up below.
static __device__ __align__(256) unsigned char scratch[UF_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (which must be current): looked up
// once per device.
uf_status scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(UF_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t he = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (he != hipSuccess || !ptr) return hip_fail(he, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return UF_OK;
}
}  // namespace

extern "C" {

uf_status uf_dm_weighted_normalized_noalloc(const uf_embedding* e, uf_precision prec,
                                            uf_out_dtype odt, void* out, double* row_means,
                                            double* grand_mean, void* stream) {
    return guarded([&]() -> uf_status {
        if (!e) return fail(UF_ERR_ARG, "embedding is NULL");
        if (prec != UF_FP64 && prec != UF_FP32)
            return fail(UF_ERR_UNSUPPORTED,
                        "the no-allocation call takes UF_FP64 or UF_FP32 (the split precisions "
                        "build their split with device allocations)");
        int dev = 0;
        uf_status st = check_device(&dev);
        if (st != UF_OK) return st;
        if (dev != e->device) return fail(UF_ERR_DEVICE, "embedding lives on another device");
        void* ws = nullptr;
        st = scratch_address(dev, &ws);
        if (st != UF_OK) return st;
        return run_dm(e, 1, prec, 0, e->n / 2, UF_CONDENSED, odt, out, row_means, grand_mean,
                      true, ws, size_t(UF_NOALLOC_SCRATCH_BYTES), stream, true);
    });
}

}  // extern "C"

// =========================================================================
// Batches: many tables on one tree (weighted normalized, FP32), one graph
// =========================================================================
struct uf_batch {
    const uf_tree* tree = nullptr;            // caller's tree (must outlive the batch)
    uf_embedding* emb = nullptr;              // concatenated tables, device
    int64_t n_tables = 0;
    std::vector<BatchTable> tabs;        // host copy
    std::vector<int64_t> acc_elems;           // per table
    int64_t n_items = 0, max_items = 0;
    int64_t kc = 0, n_chunks = 0;
    int stage_branches = 16, wgs_per_cu = 2, tile_stripes = 128, n_cu = 256;
    int64_t n_bucket = 0;
    void* arena = nullptr;                    // descs, tab_of, items, queue bounds
    BatchTable* d_tabs = nullptr;
    int32_t* d_tab_of = nullptr;
    int2* d_items = nullptr;
    int64_t* d_qbeg = nullptr;
    int64_t* d_qend = nullptr;
    int32_t* d_lo_chunks = nullptr;           // positions of each chunk ordered by lo
    size_t off_E = 0, off_acc = 0, off_cnt = 0, ws_total = 0;
    hipStream_t cap = nullptr;                // capture stream (default priority)
    hipEvent_t last_run = nullptr;            // recorded after every run's work
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uintptr_t> graph_key;         // workspace + outputs the graph was built for
    // sparse-split mode: per-table embeddings, runs forked over `n_streams` streams
    bool split = false;
    std::vector<uf_embedding*> tembs;         // [n_tables], nullptr below 2 samples
    std::vector<int64_t> order;               // tables by decreasing size
    size_t slot_bytes = 0;                    // workspace per stream
    int n_streams = 4;
    std::vector<hipStream_t> streams;         // kMaxBatchStreams, default priority
    std::vector<hipEvent_t> events;           // fork + one join event per stream

    ~uf_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        if (last_run) (void)hipEventDestroy(last_run);
        for (hipStream_t q : streams) (void)hipStreamDestroy(q);
        for (hipEvent_t ev : events) (void)hipEventDestroy(ev);
        for (uf_embedding* t : tembs) uf_free_embedding(t);
        if (arena) (void)hipFree(arena);
        uf_free_embedding(emb);
    }
};

namespace {

const int kBatchStages[] = {8, 16, 32};
const int kBatchTiles[] = {64, 128, 256};

// (stage branches, resident blocks per CU, stripes per tile) is valid when the
// kernel exists and that many of its blocks fit on a CU (LDS, registers)
bool config_valid(int ks, int w, int ts) {
    return w >= 1 && w <= ufk::band_persistent_max_blocks(ks, ts);
}

std::string cache_key_arch() { return "gfx950"; }

// Cache file: {"gfx950": {"weighted_normalized_fp32": {"n_bucket_B": {"stage_branches": K,
// "wgs_per_cu": W, "tile_stripes": S, "ms": T}, ...}}}.  Entries are parsed
// leniently by pattern; an entry without tile_stripes means 128.
struct TuneEntry {
    int ks, w, ts;
    double ms;
};
std::map<int64_t, TuneEntry> read_tune_cache(const char* path) {
    std::map<int64_t, TuneEntry> m;
    if (!path) return m;
    FILE* f = std::fopen(path, "rb");
    if (!f) return m;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    std::fclose(f);
    size_t pos = 0;
    while ((pos = text.find("\"n_bucket_", pos)) != std::string::npos) {
        long long b = 0;
        int ks = 0, w = 0, ts = 128;
        double ms = 0;
        const char* at = text.c_str() + pos;
        const bool ok =
            std::sscanf(at, "\"n_bucket_%lld\": {\"stage_branches\": %d, \"wgs_per_cu\": %d, "
                            "\"tile_stripes\": %d, \"ms\": %lf",
                        &b, &ks, &w, &ts, &ms) == 5 ||
            (ts = 128, std::sscanf(at, "\"n_bucket_%lld\": {\"stage_branches\": %d, \"wgs_per_cu\": %d, "
                                       "\"ms\": %lf",
                                   &b, &ks, &w, &ms) == 4);
        if (ok && config_valid(ks, w, ts)) m[b] = TuneEntry{ks, w, ts, ms};
        pos += 10;
    }
    return m;
}

bool write_tune_cache(const char* path, const std::map<int64_t, TuneEntry>& m) {
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    std::fprintf(f, "{\"%s\": {\"weighted_normalized_fp32\": {", cache_key_arch().c_str());
    bool firstc = true;
    for (const auto& kv : m) {
        std::fprintf(f,
                     "%s\n  \"n_bucket_%lld\": {\"stage_branches\": %d, \"wgs_per_cu\": %d, "
                     "\"tile_stripes\": %d, \"ms\": %.6f}",
                     firstc ? "" : ",", (long long)kv.first, kv.second.ks, kv.second.w, kv.second.ts,
                     kv.second.ms);
        firstc = false;
    }
    std::fprintf(f, "\n}}}\n");
    std::fclose(f);
    return std::rename(tmp.c_str(), path) == 0;
}

const char* tune_path(const char* p) { return p ? p : std::getenv("UF_TUNE_CACHE"); }

// Work items of the persistent kernel for tiles of ts stripes: (table, tile) with
// the tile's i-block fastest, tables in order.
std::vector<int2> batch_items(const std::vector<BatchTable>& tabs, int ts) {
    std::vector<int2> items;
    for (size_t r = 0; r < tabs.size(); ++r) {
        const BatchTable& t = tabs[r];
        if (t.n < 2) continue;
        const int64_t n_sblk = (t.n / 2 + ts - 1) / ts;
        for (int64_t tt = 0; tt < t.n_iblk * n_sblk; ++tt) items.push_back(make_int2(int(r), int(tt)));
    }
    return items;
}

// Upload the items for tiles of ts stripes and the 8 queue bounds (synchronous).
uf_status batch_set_tiles(uf_batch* b, int ts) {
    const std::vector<int2> items = batch_items(b->tabs, ts);
    // a run still in flight reads the current items
    if (b->last_run) UF_HIP(hipEventSynchronize(b->last_run));
    if (int64_t(items.size()) > b->max_items) return fail(UF_ERR_ARG, "tile size below the smallest");
    b->n_items = int64_t(items.size());
    std::vector<int64_t> qb(8), qe(8);
    for (int q = 0; q < 8; ++q) {
        qb[size_t(q)] = b->n_items * q / 8;
        qe[size_t(q)] = b->n_items * (q + 1) / 8;
    }
    if (b->n_items)
        UF_HIP(hipMemcpy(b->d_items, items.data(), sizeof(int2) * size_t(b->n_items), hipMemcpyHostToDevice));
    UF_HIP(hipMemcpy(b->d_qbeg, qb.data(), 64, hipMemcpyHostToDevice));
    UF_HIP(hipMemcpy(b->d_qend, qe.data(), 64, hipMemcpyHostToDevice));
    b->tile_stripes = ts;
    return UF_OK;
}

// node-major FP32 embedding of chunk [k0, k0+kc) of every table: forward merge
// when every sample total is below 2^32, else binary searches (same values)
hipError_t batch_embed(const uf_batch* b, int64_t k0, int64_t kc, float* E, hipStream_t s) {
    const uf_embedding& e = *b->emb;
    if (b->d_lo_chunks && e.max_total < (int64_t(1) << 32))
        return ufs::embed_batch_merge_f32(emb_view(e), b->d_tabs, b->d_tab_of, b->d_lo_chunks + k0,
                                          k0, kc, E, s);
    return ufk::embed_batch_f32(e, b->d_tabs, b->d_tab_of, k0, kc, E, s);
}

// enqueue the whole batch on stream s (also used under graph capture)
uf_status batch_enqueue(uf_batch* b, float* const* outs, char* base, hipStream_t s) {
    float* E = reinterpret_cast<float*>(base + b->off_E);
    float* acc = reinterpret_cast<float*>(base + b->off_acc);
    unsigned* cnt = reinterpret_cast<unsigned*>(base + b->off_cnt);
    const uf_embedding& e = *b->emb;
    const int nblk = b->n_cu * b->wgs_per_cu;
    UF_HIP(ufk::zero_u32(cnt, std::max<int64_t>(b->n_chunks, 1) * 8, s));
    for (int64_t c = 0; c < b->n_chunks; ++c) {
        const int64_t k0 = c * b->kc;
        const int64_t kc = std::min<int64_t>(b->kc, e.nb - k0);
        UF_HIP(batch_embed(b, k0, kc, E, s));
        if (b->n_items > 0)
            UF_HIP(ufk::band_persistent_f32(E, b->d_tabs, b->d_items, b->d_qbeg, b->d_qend,
                                            cnt + c * 8, kc, c == 0, acc, b->stage_branches,
                                            b->tile_stripes, nblk, s));
    }
    for (int64_t r = 0; r < b->n_tables; ++r) {
        const BatchTable& t = b->tabs[r];
        if (t.n < 2) continue;
        if (b->n_chunks == 0) {
            UF_HIP(ufk::zero_u32(reinterpret_cast<unsigned*>(acc + t.acc_off), (t.n / 2) * t.n, s));
        }
        UF_HIP(ufk::finalize(0, acc + t.acc_off, ufk::kAccF32, 1.0, e.sw + t.off, t.n, 0, t.n / 2,
                             UF_CONDENSED, 1, outs[r], nullptr, s));
    }
    return UF_OK;
}

constexpr int kMaxBatchStreams = 8;

// Sparse-split mode: table r runs on stream (rank of r by size) mod n_streams, in
// decreasing size, each stream with its own workspace slot; the streams fork from
// and join back into s (also under graph capture).
uf_status batch_split_enqueue(uf_batch* b, float* const* outs, char* base, hipStream_t s) {
    t_prof_suppress = true;
    struct Reset {
        ~Reset() { t_prof_suppress = false; }
    } reset;
    const int k = b->n_streams;
    UF_HIP(hipEventRecord(b->events[0], s));
    for (int q = 0; q < k; ++q) UF_HIP(hipStreamWaitEvent(b->streams[size_t(q)], b->events[0], 0));
    for (size_t rank = 0; rank < b->order.size(); ++rank) {
        const int64_t r = b->order[rank];
        const uf_embedding* e = b->tembs[size_t(r)];
        const int q = int(rank % size_t(k));
        char* slot = base + size_t(q) * b->slot_bytes;
        uf_status st = run_dm(e, 1, UF_FP32_SPLIT, 0, e->n / 2, UF_CONDENSED, UF_OUT_F32, outs[r],
                              nullptr, nullptr, false, slot, b->slot_bytes, b->streams[size_t(q)]);
        if (st != UF_OK) return st;
    }
    for (int q = 0; q < k; ++q) {
        UF_HIP(hipEventRecord(b->events[size_t(q) + 1], b->streams[size_t(q)]));
        UF_HIP(hipStreamWaitEvent(s, b->events[size_t(q) + 1], 0));
    }
    return UF_OK;
}

uf_status batch_enqueue_any(uf_batch* b, float* const* outs, char* base, hipStream_t s) {
    return b->split ? batch_split_enqueue(b, outs, base, s) : batch_enqueue(b, outs, base, s);
}

void drop_graph(uf_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_key.clear();
}

}  // namespace

extern "C" {

uf_status uf_batch_set_precision(uf_batch* b, uf_precision prec, const uf_table* const* tables,
                                 void* stream) {
    return guarded([&]() -> uf_status {
        if (!b) return fail(UF_ERR_ARG, "batch is NULL");
        if (prec == UF_FP32) {
            b->split = false;
            drop_graph(b);
            return UF_OK;
        }
        if (prec != UF_FP32_SPLIT) return fail(UF_ERR_UNSUPPORTED, "batches run UF_FP32 or UF_FP32_SPLIT");
        if (!tables) return fail(UF_ERR_ARG, "tables are NULL");
        if (b->tembs.empty()) {
            for (int64_t r = 0; r < b->n_tables; ++r)
                if (!tables[r] || tables[r]->n_samples != b->tabs[size_t(r)].n)
                    return fail(UF_ERR_ARG, "tables differ from the ones the batch was created with");
            b->tembs.assign(size_t(b->n_tables), nullptr);
            for (int64_t r = 0; r < b->n_tables; ++r) {
                if (b->tabs[size_t(r)].n < 2) continue;
                uf_status st = embed_impl(b->tree, tables[r], stream, &b->tembs[size_t(r)]);
                if (st != UF_OK) return st;
            }
        }
        size_t slot = 0;
        b->order.clear();
        for (int64_t r = 0; r < b->n_tables; ++r) {
            const uf_embedding* e = b->tembs[size_t(r)];
            if (!e) continue;
            std::shared_ptr<SplitCache> sc;
            uf_status st = ensure_split(e, 1, stream, &sc);
            if (st != UF_OK) return st;
            Plan p;
            st = make_plan(e, 1, UF_FP32_SPLIT, 0, e->n / 2, false, &p, sc.get());
            if (st != UF_OK) return st;
            slot = std::max(slot, (p.total + 255) & ~size_t(255));
            b->order.push_back(r);
        }
        std::stable_sort(b->order.begin(), b->order.end(), [&](int64_t x, int64_t y) {
            return b->tabs[size_t(x)].n > b->tabs[size_t(y)].n;
        });
        b->slot_bytes = slot;
        if (b->streams.empty()) {
            b->streams.assign(kMaxBatchStreams, nullptr);
            for (auto& q : b->streams) UF_HIP(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
            b->events.assign(kMaxBatchStreams + 1, nullptr);
            for (auto& ev : b->events) UF_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        }
        b->split = true;
        drop_graph(b);
        return UF_OK;
    });
}

uf_status uf_batch_create(const uf_tree* tree, const uf_table* const* tables, int64_t n_tables,
                          const char* tune_cache, void* stream, uf_batch** out) {
    return guarded([&]() -> uf_status {
        if (!out) return fail(UF_ERR_ARG, "out is NULL");
        *out = nullptr;
        if (!tree || !tables || n_tables < 1) return fail(UF_ERR_ARG, "need a tree and >= 1 table");
        // concatenate the tables on the host
        uf_table cat;
        cat.n_tips = tree->n_tips;
        cat.row_ptr.push_back(0);
        for (int64_t r = 0; r < n_tables; ++r) {
            const uf_table* t = tables[r];
            if (!t) return fail(UF_ERR_ARG, "table pointer is NULL");
            if (t->n_tips != tree->n_tips) return fail(UF_ERR_ARG, "table loaded against another tree");
            const int64_t base = int64_t(cat.rank.size());
            cat.rank.insert(cat.rank.end(), t->rank.begin(), t->rank.end());
            cat.count.insert(cat.count.end(), t->count.begin(), t->count.end());
            cat.total.insert(cat.total.end(), t->total.begin(), t->total.end());
            for (int64_t sidx = 1; sidx <= t->n_samples; ++sidx) cat.row_ptr.push_back(base + t->row_ptr[sidx]);
        }
        cat.n_samples = int64_t(cat.total.size());
        auto b = new uf_batch();
        std::unique_ptr<uf_batch> guard(b);
        b->tree = tree;
        uf_status st = embed_impl(tree, &cat, stream, &b->emb);
        if (st != UF_OK) return st;
        b->n_tables = n_tables;
        int dev = 0;
        UF_HIP(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        UF_HIP(hipGetDeviceProperties(&prop, dev));
        b->n_cu = prop.multiProcessorCount;
        // chunk length: 16 GiB of embedding for all tables, or the process-wide setting
        const int64_t n_all = std::max<int64_t>(cat.n_samples, 1);
        int64_t kc = g_chunk_nodes.load();
        if (kc <= 0) kc = int64_t(16.0 * 1024 * 1024 * 1024 / (double(n_all) * 4.0));
        kc = std::min<int64_t>(std::max<int64_t>(kc, 32), std::max<int64_t>(b->emb->nb, 1));
        b->kc = kc;
        b->n_chunks = b->emb->nb > 0 ? (b->emb->nb + kc - 1) / kc : 0;
        // per-table layout
        int64_t off = 0, eoff = 0, aoff = 0;
        std::vector<int32_t> tab_of(size_t(n_all), 0);
        double mean_n = 0;
        for (int64_t r = 0; r < n_tables; ++r) {
            BatchTable t;
            t.n = tables[r]->n_samples;
            t.off = off;
            t.e_off = eoff;
            t.acc_off = aoff;
            t.n_iblk = (t.n + ufk::kBandI - 1) / ufk::kBandI;
            b->tabs.push_back(t);
            for (int64_t i = 0; i < t.n; ++i) tab_of[size_t(off + i)] = int32_t(r);
            const int64_t S = t.n / 2;
            off += t.n;
            eoff += kc * t.n;
            aoff += ((S * t.n + 63) / 64) * 64;
            mean_n += double(t.n) / double(n_tables);
        }
        // work items: the arena holds those of the smallest tile (the most)
        b->max_items = int64_t(batch_items(b->tabs, kBatchTiles[0]).size());
        b->n_bucket = mean_n > 1 ? int64_t(std::ceil(std::log2(mean_n))) : 0;
        Carver c;
        const size_t o_tabs = c.take(sizeof(BatchTable) * size_t(n_tables));
        const size_t o_tabof = c.take(size_t(n_all) * 4);
        const size_t o_items = c.take(sizeof(int2) * size_t(std::max<int64_t>(b->max_items, 1)));
        const size_t o_qb = c.take(8 * 8);
        const size_t o_qe = c.take(8 * 8);
        const int64_t nb = b->emb->nb;
        const size_t o_lord = c.take(size_t(std::max<int64_t>(nb, 1)) * 4);
        if (hipMalloc(&b->arena, c.off + 256) != hipSuccess) return fail(UF_ERR_NOMEM, "batch descriptors");
        char* base = static_cast<char*>(b->arena);
        b->d_tabs = reinterpret_cast<BatchTable*>(base + o_tabs);
        b->d_tab_of = reinterpret_cast<int32_t*>(base + o_tabof);
        b->d_items = reinterpret_cast<int2*>(base + o_items);
        b->d_qbeg = reinterpret_cast<int64_t*>(base + o_qb);
        b->d_qend = reinterpret_cast<int64_t*>(base + o_qe);
        b->d_lo_chunks = reinterpret_cast<int32_t*>(base + o_lord);
        {
            // positions of each chunk [c kc, (c+1) kc) in ascending lo (stable)
            std::vector<int32_t> ord(size_t(std::max<int64_t>(nb, 1)));
            for (int64_t k = 0; k < nb; ++k) ord[size_t(k)] = int32_t(k);
            for (int64_t k0 = 0; k0 < nb; k0 += kc) {
                const auto first = ord.begin() + k0, last = ord.begin() + std::min<int64_t>(nb, k0 + kc);
                std::stable_sort(first, last, [&](int32_t x, int32_t y) {
                    return tree->lo[size_t(x)] < tree->lo[size_t(y)];
                });
            }
            if (nb) UF_HIP(hipMemcpy(b->d_lo_chunks, ord.data(), size_t(nb) * 4, hipMemcpyHostToDevice));
        }
        UF_HIP(hipMemcpy(b->d_tabs, b->tabs.data(), sizeof(BatchTable) * size_t(n_tables), hipMemcpyHostToDevice));
        UF_HIP(hipMemcpy(b->d_tab_of, tab_of.data(), size_t(n_all) * 4, hipMemcpyHostToDevice));
        Carver w;
        b->off_E = w.take(size_t(eoff) * 4);
        b->off_acc = w.take(size_t(aoff) * 4);
        b->off_cnt = w.take(size_t(std::max<int64_t>(b->n_chunks, 1)) * 8 * 4);
        b->ws_total = w.off + 256;
        // launch configuration from the tuning cache, if it has this size bucket
        auto cache = read_tune_cache(tune_path(tune_cache));
        auto it = cache.find(b->n_bucket);
        int ts = 128;
        if (it != cache.end()) {
            b->stage_branches = it->second.ks;
            b->wgs_per_cu = it->second.w;
            ts = it->second.ts;
        }
        st = batch_set_tiles(b, ts);
        if (st != UF_OK) return st;
        UF_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        UF_HIP(hipEventCreateWithFlags(&b->last_run, hipEventDisableTiming));
        *out = guard.release();
        return UF_OK;
    });
}

uf_status uf_batch_plan_create(const uf_tree* tree, const uf_table* const* tables, int64_t n_tables,
                               uf_precision prec, const char* tune_cache, void* stream,
                               uf_batch** out) {
    if (prec != UF_FP32 && prec != UF_FP32_SPLIT) {
        if (out) *out = nullptr;
        return fail(UF_ERR_UNSUPPORTED, "batches run UF_FP32 or UF_FP32_SPLIT");
    }
    uf_status st = uf_batch_create(tree, tables, n_tables, tune_cache, stream, out);
    if (st != UF_OK || prec == UF_FP32) return st;
    st = uf_batch_set_precision(*out, prec, tables, stream);
    if (st != UF_OK) {
        uf_free_batch(*out);
        *out = nullptr;
    }
    return st;
}

int64_t uf_batch_n_tables(const uf_batch* b) { return b ? b->n_tables : -1; }

size_t batch_ws_bytes(const uf_batch* b) {
    return b->split ? b->slot_bytes * size_t(kMaxBatchStreams) + 256 : b->ws_total;
}

uf_status uf_batch_workspace_size(const uf_batch* b, size_t* bytes) {
    if (!b || !bytes) return fail(UF_ERR_ARG, "NULL argument");
    *bytes = batch_ws_bytes(b);
    return UF_OK;
}

uf_status uf_batch_config(const uf_batch* b, int* stage_branches, int* wgs_per_cu,
                          int* tile_stripes, int64_t* chunk_nodes) {
    if (!b) return fail(UF_ERR_ARG, "batch is NULL");
    if (stage_branches) *stage_branches = b->stage_branches;
    if (wgs_per_cu) *wgs_per_cu = b->wgs_per_cu;
    if (tile_stripes) *tile_stripes = b->tile_stripes;
    if (chunk_nodes) *chunk_nodes = b->kc;
    return UF_OK;
}

uf_status uf_batch_set_config(uf_batch* b, int stage_branches, int wgs_per_cu, int tile_stripes) {
    return guarded([&]() -> uf_status {
        if (!b) return fail(UF_ERR_ARG, "batch is NULL");
        if (!config_valid(stage_branches, wgs_per_cu, tile_stripes))
            return fail(UF_ERR_ARG, "unsupported (stage_branches, wgs_per_cu, tile_stripes)");
        if (tile_stripes != b->tile_stripes) {
            const uf_status st = batch_set_tiles(b, tile_stripes);
            if (st != UF_OK) return st;
        }
        b->stage_branches = stage_branches;
        b->wgs_per_cu = wgs_per_cu;
        if (b->exec) {
            (void)hipGraphExecDestroy(b->exec);
            (void)hipGraphDestroy(b->graph);
            b->exec = nullptr;
            b->graph = nullptr;
            b->graph_key.clear();
        }
        return UF_OK;
    });
}

uf_status uf_batch_run(uf_batch* b, float* const* outs, int use_graph, void* ws, size_t ws_bytes,
                       void* stream) {
    return guarded([&]() -> uf_status {
        if (!b || !outs) return fail(UF_ERR_ARG, "NULL argument");
        if (!ws || ws_bytes < batch_ws_bytes(b)) return fail(UF_ERR_WORKSPACE, "batch workspace too small");
        for (int64_t r = 0; r < b->n_tables; ++r)
            if (!outs[r] && b->tabs[r].n >= 2) return fail(UF_ERR_ARG, "output pointer is NULL");
        int dev = 0;
        uf_status st = check_device(&dev);
        if (st != UF_OK) return st;
        char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
        hipStream_t s = static_cast<hipStream_t>(stream);
        std::vector<uintptr_t> key;
        if (b->split) {
            // splits are built outside any capture (a changed threshold rebuilds them)
            for (int64_t r : b->order) {
                std::shared_ptr<SplitCache> sc;
                st = ensure_split(b->tembs[size_t(r)], 1, stream, &sc);
                if (st != UF_OK) return st;
                key.push_back(uintptr_t(sc->build_id));
            }
            key.push_back(uintptr_t(b->n_streams));
        }
        if (!use_graph) {
            st = batch_enqueue_any(b, outs, base, s);
            if (st != UF_OK) return st;
            UF_HIP(hipEventRecord(b->last_run, s));
            return UF_OK;
        }
        key.push_back(reinterpret_cast<uintptr_t>(base));
        for (int64_t r = 0; r < b->n_tables; ++r) key.push_back(reinterpret_cast<uintptr_t>(outs[r]));
        if (!b->exec || key != b->graph_key) {
            if (b->exec) {
                (void)hipGraphExecDestroy(b->exec);
                (void)hipGraphDestroy(b->graph);
                b->exec = nullptr;
                b->graph = nullptr;
            }
            UF_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
            uf_status est = batch_enqueue_any(b, outs, base, b->cap);
            hipGraph_t g = nullptr;
            hipError_t ce = hipStreamEndCapture(b->cap, &g);
            if (est != UF_OK) {
                if (g) (void)hipGraphDestroy(g);
                return est;
            }
            if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
            hipGraphExec_t ex = nullptr;
            hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            if (ie != hipSuccess) {
                (void)hipGraphDestroy(g);
                return hip_fail(ie, "hipGraphInstantiate");
            }
            b->graph = g;
            b->exec = ex;
            b->graph_key = key;
        }
        UF_HIP(hipGraphLaunch(b->exec, s));
        UF_HIP(hipEventRecord(b->last_run, s));
        return UF_OK;
    });
}

uf_status uf_autotune(uf_batch* b, void* ws, size_t ws_bytes, const char* tune_cache,
                      void* stream, double* best_ms) {
    return guarded([&]() -> uf_status {
        if (!b) return fail(UF_ERR_ARG, "batch is NULL");
        if (!ws || ws_bytes < batch_ws_bytes(b)) return fail(UF_ERR_WORKSPACE, "batch workspace too small");
        int dev = 0;
        uf_status st = check_device(&dev);
        if (st != UF_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
        if (b->split) {
            // sparse-split mode: time whole eager runs over 1, 2, 4 and 8 streams into
            // scratch outputs in the workspace's slots (output sizes are the tables')
            std::vector<void*> scratch(size_t(b->n_tables), nullptr);
            struct Free {
                std::vector<void*>& v;
                ~Free() {
                    for (void* q : v)
                        if (q) (void)hipFree(q);
                }
            } fr{scratch};
            for (int64_t r : b->order) {
                const int64_t n = b->tabs[size_t(r)].n;
                if (hipMalloc(&scratch[size_t(r)], size_t(n * (n - 1) / 2) * 4 + 256) != hipSuccess)
                    return fail(UF_ERR_NOMEM, "autotune outputs");
            }
            std::vector<float*> outs(size_t(b->n_tables), nullptr);
            for (int64_t r = 0; r < b->n_tables; ++r) outs[size_t(r)] = static_cast<float*>(scratch[size_t(r)]);
            hipEvent_t e0, e1;
            UF_HIP(hipEventCreate(&e0));
            UF_HIP(hipEventCreate(&e1));
            int best_k = b->n_streams;
            double best_t = 1e300;
            for (int k : {1, 2, 4, 8}) {
                b->n_streams = k;
                double tmin = 1e300;
                for (int rep = 0; rep < 2; ++rep) {
                    UF_HIP(hipEventRecord(e0, s));
                    st = batch_split_enqueue(b, outs.data(), base, s);
                    if (st != UF_OK) return st;
                    UF_HIP(hipEventRecord(e1, s));
                    UF_HIP(hipEventSynchronize(e1));
                    float ms = 0;
                    UF_HIP(hipEventElapsedTime(&ms, e0, e1));
                    tmin = std::min(tmin, double(ms));
                }
                if (tmin < best_t) {
                    best_t = tmin;
                    best_k = k;
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            b->n_streams = best_k;
            drop_graph(b);
            if (best_ms) *best_ms = best_t;
            return UF_OK;
        }
        float* E = reinterpret_cast<float*>(base + b->off_E);
        float* acc = reinterpret_cast<float*>(base + b->off_acc);
        unsigned* cnt = reinterpret_cast<unsigned*>(base + b->off_cnt);
        const uf_embedding& e = *b->emb;
        if (b->n_chunks == 0 || b->n_items == 0) return UF_OK;
        // timed on the first 2,048 branches of the first chunk: every configuration
        // pays the same per-branch work, so a part of the chunk ranks them
        const int64_t kc = std::min<int64_t>(std::min<int64_t>(b->kc, e.nb), 2048);
        UF_HIP(batch_embed(b, 0, kc, E, s));
        hipEvent_t e0, e1;
        UF_HIP(hipEventCreate(&e0));
        UF_HIP(hipEventCreate(&e1));
        struct Ev {
            hipEvent_t a, b;
            ~Ev() {
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
            }
        } ev{e0, e1};
        TuneEntry best{b->stage_branches, b->wgs_per_cu, b->tile_stripes, 1e300};
        for (int ts : kBatchTiles) {
            st = batch_set_tiles(b, ts);
            if (st != UF_OK) return st;
            for (int ks : kBatchStages) {
                // the two highest occupancies the configuration allows
                const int wmax = ufk::band_persistent_max_blocks(ks, ts);
                for (int w = std::max(1, wmax - 1); w <= wmax; ++w) {
                    double tmin = 1e300;
                    for (int rep = 0; rep < 2; ++rep) {
                        UF_HIP(ufk::zero_u32(cnt, 8, s));
                        UF_HIP(hipEventRecord(e0, s));
                        UF_HIP(ufk::band_persistent_f32(E, b->d_tabs, b->d_items, b->d_qbeg, b->d_qend,
                                                        cnt, kc, 1, acc, ks, ts, b->n_cu * w, s));
                        UF_HIP(hipEventRecord(e1, s));
                        UF_HIP(hipEventSynchronize(e1));
                        float ms = 0;
                        UF_HIP(hipEventElapsedTime(&ms, e0, e1));
                        tmin = std::min(tmin, double(ms));
                    }
                    if (tmin < best.ms) best = TuneEntry{ks, w, ts, tmin};
                }
            }
        }
        if (best_ms) *best_ms = best.ms;
        st = batch_set_tiles(b, best.ts);
        if (st != UF_OK) return st;
        st = uf_batch_set_config(b, best.ks, best.w, best.ts);
        if (st != UF_OK) return st;
        const char* path = tune_path(tune_cache);
        if (path) {
            auto cache = read_tune_cache(path);
            cache[b->n_bucket] = best;
            if (!write_tune_cache(path, cache)) return fail(UF_ERR_ARG, "cannot write the tuning cache");
        }
        return UF_OK;
    });
}

void uf_free_batch(uf_batch* b) { delete b; }

}  // extern "C"
