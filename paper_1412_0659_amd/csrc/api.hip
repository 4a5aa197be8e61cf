// C ABI of the tree-code library: context, argument checks, the order of the
// launches for a build / force evaluation / leapfrog step, statistics and
// array export.  Declarations and contracts are in include/bh.h.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "bh_internal.h"

using namespace bh;

namespace {

int fail(bh_ctx *c, int code, const std::string &msg) {
    if (c) c->last_error = msg;
    return code;
}

#define BH_HIP(ctx, call)                                                                 \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail((ctx), BH_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
bool dalloc(T **p, size_t count, std::string &err) {
    hipError_t e = hipMalloc((void **)p, sizeof(T) * std::max<size_t>(count, 1));
    if (e != hipSuccess) {
        *p = nullptr;
        err = std::string("hipMalloc: ") + hipGetErrorString(e);
        (void)hipGetLastError();
        return false;
    }
    return true;
}

void free_all(bh_ctx *c) {
    auto f = [](void *p) {
        if (p) (void)hipFree(p);
    };
    for (int k = 0; k < 2; ++k) {
        State &s = c->st[k];
        f(s.x); f(s.y); f(s.z); f(s.m); f(s.vx); f(s.vy); f(s.vz); f(s.cid);
        f(s.x64); f(s.y64); f(s.z64);
        f(c->sort.key[k]); f(c->sort.idx[k]);
    }
    f(c->acc); f(c->xyzm); f(c->spill); f(c->box); f(c->box_part); f(c->status); f(c->work); f(c->totals);
    f(c->sort.counts); f(c->sort.scan_part);
    Cells &q = c->cells;
    f(q.prefix); f(q.level); f(q.begin); f(q.count); f(q.child0); f(q.nchild); f(q.parent);
    f(q.ls); f(q.part); f(q.lbt); f(q.cbnd); f(q.M); f(q.S); f(q.com); f(q.Q); f(q.wA); f(q.wN); f(q.P0); f(q.P1);
    f(q.P2); f(q.size);
    Groups &g = c->groups;
    f(g.flag); f(g.scan); f(g.begin); f(g.count_dev); f(g.box); f(g.npp); f(g.npc);
    f(c->lcell); f(c->gsrc); f(c->lhot); f(c->usort); f(c->leafof); f(c->cic); f(c->inv); f(c->diag);
    Boundary &b = c->bnd;
    f(b.flag); f(b.scan); f(b.ids); f(b.box); f(b.cmin); f(b.cmax); f(b.lvl); f(b.part);
    Let &t = c->let;
    f(t.wA); f(t.P0); f(t.P1); f(t.P2); f(t.xyzm); f(t.wN); f(t.origin);
    f(t.cmark); f(t.omark); f(t.cscan); f(t.pmark); f(t.pscan); f(t.spart); f(t.word);
    f(c->cut.S); f(c->cut.cuts); f(c->seg);
    if (c->hint_host) (void)hipHostFree(c->hint_host);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
}

bool valid_theta(float t) { return std::isfinite(t) && t > 0.f && t <= 1.f; }
bool valid_eps(float e) { return std::isfinite(e) && e >= 0.f; }

int check_status(bh_ctx *c) {
    uint32_t st = 0;
    BH_HIP(c, hipMemcpy(&st, c->status, sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (st == 0) return BH_OK;
    BH_HIP(c, hipMemset(c->status, 0, sizeof(uint32_t)));
    if (st & kStNonFinite) return fail(c, BH_ENONFINITE, "non-finite position or velocity");
    if (st & kStMass) return fail(c, BH_EMASS, "mass <= 0 or not finite");
    if (st & kStIndex) return fail(c, BH_EINVAL, "target index outside [0, n)");
    if (st & kStOutside) return fail(c, BH_EINVAL, "particle outside the box set by bh_set_box");
    return fail(c, BH_ECAPACITY, "cell or stack capacity exceeded");
}

// Levels the grid kernels split: one past the deepest level of a recent tree
// of the same particle set when one has been published (a tail kernel splits
// any deeper level), else all of them.  The published copy is read without
// waiting: its two build numbers agree only if it was read whole.
int grid_levels(bh_ctx *c, bool fresh) {
    if (c->forced_grid_levels >= 0) return std::min(c->forced_grid_levels, kLevels - 1);
    if (fresh || !c->hint_host) return kLevels - 1;
    const volatile uint32_t *h = c->hint_host;
    const uint32_t last = h[1];
    std::atomic_thread_fence(std::memory_order_acquire);
    uint32_t ls[kLevels + 1];
    for (int k = 0; k < kLevels + 1; ++k) ls[k] = h[2 + k];
    std::atomic_thread_fence(std::memory_order_acquire);
    const uint32_t first = h[0];
    if (first != last || last < c->hint_gen_min || last > c->build_gen) return kLevels - 1;
    int deepest = -1;
    for (int l = 0; l < kLevels; ++l)
        if (ls[l + 1] > ls[l]) deepest = l;
    return deepest < 0 ? kLevels - 1 : std::min(kLevels - 1, deepest + 1);
}

// fresh: a new particle set (no earlier tree describes it)
void rebuild(bh_ctx *c, uint32_t n, hipStream_t s, bool fresh) {
    if (fresh) c->hint_gen_min = c->build_gen + 1;
    const int L = grid_levels(c, fresh);
    ++c->build_gen;
    record_event(c, 0, s);
    launch_bbox(c, c->st[c->cur], n, s);
    launch_keys(c, c->st[c->cur], n, s);
    launch_radix_sort(c, n, s);
    launch_gather(c, n, s);
    record_event(c, 1, s);
    launch_build(c, n, s, L);
    launch_groups(c, n, s);
    record_event(c, 2, s);
    launch_moments(c, s, L);
    record_event(c, 3, s);
    c->built = true;
    c->have_acc = false;
    c->counts_valid = false;
    c->bnd.valid = false;
    c->let.valid = false;
}

void force(bh_ctx *c, float theta, float eps, hipStream_t s) {
    launch_walk_prep(c, theta, s);
    launch_walk(c, eps, s);
    launch_totals(c, (uint32_t)c->n, s);
    c->have_acc = true;
    c->counts_valid = true;
    c->acc_theta = theta;
    c->acc_eps = eps;
}

// lazily sized device buffers of the multi-domain calls
template <class T>
bool grow(T **p, int64_t &cap, int64_t need, std::string &err) {
    if (*p && cap >= need) return true;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    cap = 0;
    if (!dalloc(p, (size_t)need, err)) return false;
    cap = need;
    return true;
}

bool same_box(const bh_ctx *a, const bh_ctx *b) {
    return a->fixed_box && b->fixed_box && a->box_lo[0] == b->box_lo[0] &&
           a->box_lo[1] == b->box_lo[1] && a->box_lo[2] == b->box_lo[2] &&
           a->box_side == b->box_side;
}

int check_n(bh_ctx *c, int64_t n) {
    if (n <= 0) return fail(c, BH_EINVAL, "n must be positive");
    if (n > c->nmax) return fail(c, BH_ECAPACITY, "n exceeds the context capacity");
    return BH_OK;
}

// C = floor(cap n / p), at most n (a larger C clamps nothing more)
int64_t cap_count(float cap, int64_t n, int32_t p) {
    const double v = std::floor((double)cap * (double)n / (double)p);
    return v >= (double)n ? n : (int64_t)v;
}

// Per sorted particle: 23 npp + 65 npc of its group's last walk (host).
int particle_costs(bh_ctx *c, std::vector<int64_t> &cost) {
    uint32_t ng = 0;
    BH_HIP(c, hipMemcpy(&ng, c->groups.count_dev, sizeof(ng), hipMemcpyDeviceToHost));
    std::vector<uint32_t> b((size_t)ng + 1), pp(ng), pc(ng);
    BH_HIP(c, hipMemcpy(b.data(), c->groups.begin, 4 * ((size_t)ng + 1), hipMemcpyDeviceToHost));
    BH_HIP(c, hipMemcpy(pp.data(), c->groups.npp, 4 * (size_t)ng, hipMemcpyDeviceToHost));
    BH_HIP(c, hipMemcpy(pc.data(), c->groups.npc, 4 * (size_t)ng, hipMemcpyDeviceToHost));
    cost.assign((size_t)c->n, 0);
    for (uint32_t g = 0; g < ng; ++g)
        for (uint32_t i = b[g]; i < b[g + 1]; ++i)
            cost[i] = 23 * (int64_t)pp[g] + 65 * (int64_t)pc[g];
    return BH_OK;
}

// clamp cuts[1..p-1] so that no domain holds more than C particles
void clamp_cuts(int64_t *cuts, int32_t p, int64_t n, int64_t C) {
    for (int32_t k = 1; k < p; ++k) {
        const int64_t lo = std::max(cuts[k - 1], n - (int64_t)(p - k) * C);
        const int64_t hi = std::min(cuts[k - 1] + C, n);
        cuts[k] = std::min(std::max(cuts[k], lo), hi);
    }
    cuts[p] = n;
}

// m cost-weighted samples of one process's particles (key order): sample j
// is the first particle whose inclusive running cost S has
// 2 m S >= (2 j + 1) W, W the process total
void draw_samples(const std::vector<uint64_t> &keys, const std::vector<int64_t> &cost,
                  int32_t m, std::vector<uint64_t> &out, int64_t &W) {
    W = 0;
    for (int64_t v : cost) W += v;
    out.clear();
    __int128 S = 0;
    int32_t j = 0;
    for (size_t i = 0; i < keys.size() && j < m; ++i) {
        S += cost[i];
        while (j < m && (__int128)2 * m * S >= (__int128)(2 * j + 1) * W) {
            out.push_back(keys[i]);
            ++j;
        }
    }
}

// (key, weight) samples -> pieces - 1 boundary keys of equal weight; a
// boundary past the last sample is reported missing (have = 0)
void weight_cuts(std::vector<std::pair<uint64_t, int64_t>> smp, int32_t pieces,
                 std::vector<uint64_t> &key, std::vector<char> &have) {
    std::stable_sort(smp.begin(), smp.end(),
                     [](const std::pair<uint64_t, int64_t> &a,
                        const std::pair<uint64_t, int64_t> &b) { return a.first < b.first; });
    __int128 T = 0, S = 0;
    for (auto &e : smp) T += e.second;
    key.assign((size_t)std::max(pieces - 1, 0), 0);
    have.assign(key.size(), 0);
    int32_t t = 1;
    for (auto &e : smp) {
        while (t < pieces && S * pieces >= T * t) {
            key[(size_t)t - 1] = e.first;
            have[(size_t)t - 1] = 1;
            ++t;
        }
        S += e.second;
    }
}

}  // namespace

// ---- the entry point that allocates nothing ----------------------------------
//
// tree_force_static runs the whole path (build + walk + unsort) for up to
// BH_STATIC_MAX_N particles with every intermediate buffer carved out of one
// file-scope device array, for callers that cannot allocate device memory.
// Each device the library runs on holds its own copy of the array for the
// life of the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device.

namespace {

constexpr int64_t kStaticMaxN = BH_STATIC_MAX_N;
constexpr int kStaticWalkGrid = 1024;          // persistent walk waves (stack spill per wave)
constexpr size_t kStaticBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {

struct StaticDevice {
    unsigned char *ptr = nullptr;  // device address of `scratch` on this device
    int cus = 0, walk_grid = 0;
};
StaticDevice g_static[kMaxDevices];
std::mutex g_static_mu;

// Point every buffer of the path at consecutive 256-byte-aligned pieces of
// base (nothing is written when base is null); returns the bytes used.
size_t static_layout(bh_ctx *c, unsigned char *base) {
    size_t off = 0;
    auto take = [&](auto **p, size_t count) {
        using T = std::remove_pointer_t<std::remove_reference_t<decltype(*p)>>;
        off = (off + 255) & ~size_t(255);
        *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += sizeof(T) * std::max<size_t>(count, 1);
    };
    const size_t n = (size_t)c->nmax, nc = (size_t)c->cap_cells;
    for (int k = 0; k < 2; ++k) {
        State &st = c->st[k];
        take(&st.x, n); take(&st.y, n); take(&st.z, n); take(&st.m, n);
        take(&st.vx, n); take(&st.vy, n); take(&st.vz, n); take(&st.cid, n);
        st.x64 = st.y64 = st.z64 = nullptr;
        take(&c->sort.key[k], n);
        take(&c->sort.idx[k], n);
    }
    c->sort.counts_len = sort_counts_len(c->nmax);
    c->sort.scan_part_len = std::max(scan_part_len(c->sort.counts_len), scan_part_len(c->nmax));
    take(&c->sort.counts, (size_t)c->sort.counts_len);
    take(&c->sort.scan_part, (size_t)c->sort.scan_part_len);
    take(&c->acc, n); take(&c->xyzm, n);
    take(&c->spill, (size_t)c->walk_grid * kStackMax);
    take(&c->box, 8); take(&c->box_part, 6 * 1024); take(&c->status, 4); take(&c->work, 8);
    take(&c->totals, 4);
    Cells &q = c->cells;
    take(&q.prefix, nc); take(&q.level, nc); take(&q.begin, nc); take(&q.count, nc);
    take(&q.child0, nc); take(&q.nchild, nc); take(&q.parent, nc); take(&q.ls, kLsSize);
    take(&q.part, kBuildGrid + 1); take(&q.lbt, ((size_t)1 << (3 * kTableLevel)) + 1);
    take(&q.cbnd, 8 * n);
    take(&q.M, nc); take(&q.S, 3 * nc); take(&q.com, 3 * nc); take(&q.Q, 6 * nc);
    take(&q.wA, nc); take(&q.wN, nc); take(&q.P0, nc); take(&q.P1, nc); take(&q.P2, nc);
    take(&q.size, nc);
    Groups &g = c->groups;
    take(&g.flag, n); take(&g.scan, n); take(&g.begin, n + 1); take(&g.count_dev, 1);
    take(&g.box, 2 * n); take(&g.npp, n); take(&g.npc, n);
    return off;
}

// Once per device, with that device current: the address of `scratch` there.
int static_device(int dev, StaticDevice &out) {
    if (dev < 0 || dev >= kMaxDevices) return BH_EINVAL;
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticDevice &d = g_static[dev];
    if (!d.ptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return BH_EHIP;
        }
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            return BH_EHIP;
        }
        d.cus = std::max(cus, 1);
        d.walk_grid = std::min(d.cus * walk_blocks_per_cu(), kStaticWalkGrid);
        d.ptr = static_cast<unsigned char *>(p);
    }
    out = d;
    return BH_OK;
}

}  // namespace

extern "C" {

const char *bh_strerror(int status) {
    switch (status) {
        case BH_OK: return "ok";
        case BH_EINVAL: return "invalid argument";
        case BH_ECAPACITY: return "capacity exceeded";
        case BH_ENOMEM: return "device allocation failed";
        case BH_EHIP: return "HIP runtime error";
        case BH_ENONFINITE: return "non-finite particle data";
        case BH_ESTATE: return "call out of order";
        case BH_EMASS: return "non-positive mass";
        default: return "unknown status";
    }
}

const char *bh_last_error(const bh_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int bh_create(bh_ctx **out, int64_t n_max, const bh_params *p) {
    if (!out) return BH_EINVAL;
    *out = nullptr;
    bh_params prm{};
    prm.nleaf = 16;
    prm.ncrit = 64;
    if (p) prm = *p;
    if (n_max <= 0 || prm.nleaf < 1 || prm.nleaf > 64 || prm.ncrit < 1 || prm.ncrit > 64 ||
        prm.far_fp16 < 0 || prm.far_fp16 > 1 || prm.pos_fp64 < 0 || prm.pos_fp64 > 1 ||
        prm.adjoint < 0 || prm.adjoint > 1 || prm.curve < 0 || prm.curve > 1 ||
        prm.pair_groups < 0 || prm.pair_groups == 1 || prm.pair_groups > 64)
        return BH_EINVAL;
    // cells: <= n leaves + 21 levels x n / (nleaf + 1) internal cells; the walk
    // packs a cell index into 29 bits
    int64_t cap = n_max + 21 * (n_max / (prm.nleaf + 1)) + 1;
    if (cap >= (int64_t(1) << 29)) return BH_EINVAL;

    bh_ctx *c = new (std::nothrow) bh_ctx();
    if (!c) return BH_ENOMEM;
    c->nmax = n_max;
    c->cap_cells = cap;
    c->p = prm;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return BH_EHIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) {
        delete c;
        return BH_EHIP;
    }
    c->cus = prop.multiProcessorCount;

    std::string err;
    bool ok = true;
    size_t n = (size_t)n_max, nc = (size_t)cap;
    for (int k = 0; k < 2 && ok; ++k) {
        State &s = c->st[k];
        ok = dalloc(&s.x, n, err) && dalloc(&s.y, n, err) && dalloc(&s.z, n, err) &&
             dalloc(&s.m, n, err) && dalloc(&s.vx, n, err) && dalloc(&s.vy, n, err) &&
             dalloc(&s.vz, n, err) && dalloc(&s.cid, n, err) && dalloc(&c->sort.key[k], n, err) &&
             dalloc(&c->sort.idx[k], n, err);
        if (ok && prm.pos_fp64)
            ok = dalloc(&s.x64, n, err) && dalloc(&s.y64, n, err) && dalloc(&s.z64, n, err);
    }
    c->sort.counts_len = sort_counts_len(n_max);
    c->sort.scan_part_len = std::max(scan_part_len(c->sort.counts_len), scan_part_len(n_max));
    Cells &q = c->cells;
    Groups &g = c->groups;
    c->walk_grid = std::max(1, c->cus) * walk_blocks_per_cu();
    {
        // test hook: a smaller LDS window of the walk stack, so that tests
        // reach the spill / refill path with moderate trees
        const char *v = std::getenv("BH_WALK_SMALL_STACK");
        c->walk_small_stack = v && v[0] == '1';
        // test hook: the number of levels the grid kernels split in every
        // build (the single-workgroup tail splits the rest)
        const char *g = std::getenv("BH_BUILD_GRID_LEVELS");
        c->forced_grid_levels = g && g[0] ? std::atoi(g) : -1;
    }
    c->pair_groups = (uint32_t)prm.pair_groups;
    ok = ok && dalloc(&c->acc, n, err) && dalloc(&c->xyzm, n, err) &&
         dalloc(&c->spill, (size_t)c->walk_grid * kStackMax, err) && dalloc(&c->box, 8, err) &&
         dalloc(&c->box_part, 6 * 1024, err) && dalloc(&c->status, 4, err) &&
         dalloc(&c->work, 8, err) && dalloc(&c->totals, 4, err) &&
         dalloc(&c->sort.counts, (size_t)c->sort.counts_len, err) &&
         dalloc(&c->sort.scan_part, (size_t)c->sort.scan_part_len, err) &&
         dalloc(&q.prefix, nc, err) && dalloc(&q.level, nc, err) && dalloc(&q.begin, nc, err) &&
         dalloc(&q.count, nc, err) && dalloc(&q.child0, nc, err) && dalloc(&q.nchild, nc, err) &&
         dalloc(&q.parent, nc, err) && dalloc(&q.ls, kLsSize, err) && dalloc(&q.cbnd, 8 * n, err) &&
         dalloc(&q.part, kBuildGrid + 1, err) &&
         dalloc(&q.lbt, ((size_t)1 << (3 * kTableLevel)) + 1, err) && dalloc(&q.M, nc, err) && dalloc(&q.S, 3 * nc, err) &&
         dalloc(&q.com, 3 * nc, err) && dalloc(&q.Q, 6 * nc, err) && dalloc(&q.wA, nc, err) &&
         dalloc(&q.wN, nc, err) && dalloc(&q.P0, nc, err) && dalloc(&q.P1, nc, err) &&
         dalloc(&q.P2, nc, err) && dalloc(&q.size, nc, err) && dalloc(&g.flag, n, err) &&
         dalloc(&g.scan, n, err) && dalloc(&g.begin, n + 1, err) &&
         dalloc(&g.count_dev, 1, err) && dalloc(&g.box, 2 * n, err) && dalloc(&g.npp, n, err) &&
         dalloc(&g.npc, n, err) && dalloc(&c->cic, 65536, err) && dalloc(&c->inv, n, err) &&
         dalloc(&c->diag, (size_t)(kDiagBlocks + 1) * kDiagN, err);
    if (ok && prm.adjoint)
        ok = dalloc(&c->lcell, 8 * 10 * nc, err) && dalloc(&c->gsrc, 8 * 4 * n, err) &&
             dalloc(&c->lhot, (size_t)kHotCopies * kHotCopy, err) &&
             dalloc(&c->usort, n, err) && dalloc(&c->leafof, n, err);
    for (auto &e : c->ev)
        if (ok && hipEventCreate(&e) != hipSuccess) ok = false;
    // pinned, device-visible copy of a recent build's level starts (zeroed: none yet)
    // (coherent, so the device's stores reach host memory in the order fenced)
    if (ok && hipHostMalloc((void **)&c->hint_host, (kLevels + 3) * sizeof(uint32_t),
                            hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        c->hint_host = nullptr;
        (void)hipGetLastError();
        ok = false;
    }
    if (ok) std::memset(c->hint_host, 0, (kLevels + 3) * sizeof(uint32_t));
    if (ok && hipHostGetDevicePointer((void **)&c->hint_dev, c->hint_host, 0) != hipSuccess) {
        (void)hipGetLastError();
        ok = false;
    }
    if (ok && hipMemset(c->status, 0, 4 * sizeof(uint32_t)) != hipSuccess) ok = false;
    if (!ok) {
        free_all(c);
        delete c;
        return BH_ENOMEM;
    }
    *out = c;
    return BH_OK;
}

int bh_destroy(bh_ctx *c) {
    if (!c) return BH_EINVAL;
    (void)hipDeviceSynchronize();
    free_all(c);
    delete c;
    return BH_OK;
}

int tree_build(bh_ctx *c, const float *pos, const float *mass, int64_t n, hipStream_t s) {
    return bh_set_state(c, pos, nullptr, mass, n, s);
}

int bh_set_state(bh_ctx *c, const float *pos, const float *vel, const float *mass, int64_t n,
                 hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!pos || !mass) return fail(c, BH_EINVAL, "null pointer");
    int rc = check_n(c, n);
    if (rc) return rc;
    c->n = n;
    c->cur = 0;
    launch_ingest(c, pos, vel, mass, (uint32_t)n, s);
    rebuild(c, (uint32_t)n, s, true);
    c->ev_rec[6] = c->ev_rec[7] = false;
    BH_HIP(c, hipGetLastError());
    return BH_OK;
}

int tree_force(bh_ctx *c, float theta, float eps, float *acc, float *pot, hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!valid_theta(theta)) return fail(c, BH_EINVAL, "theta must be in (0, 1]");
    if (!valid_eps(eps)) return fail(c, BH_EINVAL, "eps must be finite and >= 0");
    if (!c->built) return fail(c, BH_ESTATE, "tree_force before tree_build");
    force(c, theta, eps, s);
    if (acc || pot) launch_unsort(c, acc, pot, (uint32_t)c->n, s);
    BH_HIP(c, hipGetLastError());
    return BH_OK;
}

int leapfrog_step(bh_ctx *c, float dt, float theta, float eps, hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!std::isfinite(dt)) return fail(c, BH_EINVAL, "dt must be finite");
    if (!valid_theta(theta)) return fail(c, BH_EINVAL, "theta must be in (0, 1]");
    if (!valid_eps(eps)) return fail(c, BH_EINVAL, "eps must be finite and >= 0");
    if (!c->built) return fail(c, BH_ESTATE, "leapfrog_step before tree_build");
    uint32_t n = (uint32_t)c->n;
    record_event(c, 6, s);
    if (!c->have_acc || theta != c->acc_theta || eps != c->acc_eps) force(c, theta, eps, s);
    launch_kick_drift(c, 0.5f * dt, dt, n, s);
    rebuild(c, n, s, false);
    force(c, theta, eps, s);
    launch_kick(c, 0.5f * dt, n, s);
    record_event(c, 7, s);
    BH_HIP(c, hipGetLastError());
    return BH_OK;
}

int bh_get_state(bh_ctx *c, float *pos, float *vel, hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!c->built) return fail(c, BH_ESTATE, "no state");
    if (pos || vel) launch_state_out(c, pos, vel, (uint32_t)c->n, s);
    BH_HIP(c, hipStreamSynchronize(s));
    return check_status(c);
}

int bh_diagnostics(bh_ctx *c, double *out, hipStream_t s) {
    if (!c || !out) return BH_EINVAL;
    if (!c->built) return fail(c, BH_ESTATE, "no state");
    launch_diagnostics(c, s);
    BH_HIP(c, hipGetLastError());
    BH_HIP(c, hipMemcpyAsync(out, c->diag + (size_t)kDiagBlocks * kDiagN, kDiagN * sizeof(double),
                             hipMemcpyDeviceToHost, s));
    BH_HIP(c, hipStreamSynchronize(s));
    if (!c->have_acc) out[2] = std::nan("");
    return check_status(c);
}

int bh_sync(bh_ctx *c, hipStream_t s) {
    if (!c) return BH_EINVAL;
    BH_HIP(c, hipStreamSynchronize(s));
    return check_status(c);
}

static double elapsed(bh_ctx *c, int a, int b) {
    if (!c->ev_rec[a] || !c->ev_rec[b]) return 0.0;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[a], c->ev[b]) != hipSuccess) {
        (void)hipGetLastError();
        return 0.0;
    }
    return ms;
}

int bh_stats_get(bh_ctx *c, bh_stats *out, hipStream_t s) {
    if (!c || !out) return BH_EINVAL;
    std::memset(out, 0, sizeof(*out));
    if (c->built) launch_count_leaves(c, s);  // the leaves of the current tree, on demand
    BH_HIP(c, hipStreamSynchronize(s));
    out->n = c->n;
    if (c->built) {
        uint32_t ls[kLsSize], ng = 0;
        unsigned long long tot[3] = {0, 0, 0};
        BH_HIP(c, hipMemcpy(ls, c->cells.ls, sizeof(ls), hipMemcpyDeviceToHost));
        BH_HIP(c, hipMemcpy(&ng, c->groups.count_dev, sizeof(ng), hipMemcpyDeviceToHost));
        BH_HIP(c, hipMemcpy(tot, c->totals, sizeof(tot), hipMemcpyDeviceToHost));
        out->ncells = ls[kLevels];
        out->ngroups = ng;
        for (int l = 0; l < kLevels; ++l)
            if (ls[l + 1] > ls[l]) out->depth = l;
        if (c->counts_valid) {
            out->n_pp = (int64_t)tot[0];
            out->n_pc = (int64_t)tot[1];
        }
        out->nleaves = (int64_t)tot[2];  // counted on the device above
    }
    out->ms_sort = elapsed(c, 0, 1);
    out->ms_build = elapsed(c, 1, 2);
    out->ms_moments = elapsed(c, 2, 3);
    out->ms_walk = elapsed(c, 4, 5);
    out->ms_step = elapsed(c, 6, 7);
    out->ms_walk_vjp = elapsed(c, 8, 9);
    return check_status(c);
}

int bh_export(bh_ctx *c, int array, void *dst, int64_t cap_bytes, int64_t *nbytes,
              hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!dst) return fail(c, BH_EINVAL, "null destination");
    if (!c->built) return fail(c, BH_ESTATE, "nothing built");
    BH_HIP(c, hipStreamSynchronize(s));
    uint32_t ls[kLsSize], ng = 0;
    BH_HIP(c, hipMemcpy(ls, c->cells.ls, sizeof(ls), hipMemcpyDeviceToHost));
    BH_HIP(c, hipMemcpy(&ng, c->groups.count_dev, sizeof(ng), hipMemcpyDeviceToHost));
    const size_t n = (size_t)c->n, nc = ls[kLevels];
    const Cells &q = c->cells;
    const Groups &g = c->groups;
    const void *src = nullptr;
    size_t bytes = 0;
    switch (array) {
        case BH_ARR_KEYS: src = c->sort.key[0]; bytes = 8 * n; break;
        case BH_ARR_PERM: src = c->st[c->cur].cid; bytes = 4 * n; break;
        case BH_ARR_BOX: src = c->box; bytes = 4 * 5; break;
        case BH_ARR_LEVEL_START: src = q.ls; bytes = 4 * (kLevels + 1); break;
        case BH_ARR_CELL_LEVEL: src = q.level; bytes = 4 * nc; break;
        case BH_ARR_CELL_PREFIX: src = q.prefix; bytes = 8 * nc; break;
        case BH_ARR_CELL_BEGIN: src = q.begin; bytes = 4 * nc; break;
        case BH_ARR_CELL_COUNT: src = q.count; bytes = 4 * nc; break;
        case BH_ARR_CELL_CHILD0: src = q.child0; bytes = 4 * nc; break;
        case BH_ARR_CELL_NCHILD: src = q.nchild; bytes = 4 * nc; break;
        case BH_ARR_CELL_PARENT: src = q.parent; bytes = 4 * nc; break;
        case BH_ARR_MOM_M: src = q.M; bytes = 8 * nc; break;
        case BH_ARR_MOM_COM:
            launch_com(c, s);
            BH_HIP(c, hipStreamSynchronize(s));
            src = q.com; bytes = 24 * nc; break;
        case BH_ARR_MOM_Q: src = q.Q; bytes = 48 * nc; break;
        case BH_ARR_CELL_COMF: src = q.wA; bytes = 16 * nc; break;
        case BH_ARR_CELL_SIZE: src = q.size; bytes = 8 * nc; break;
        case BH_ARR_GROUP_BEGIN: src = g.begin; bytes = 4 * (size_t)ng; break;
        case BH_ARR_GROUP_COUNT: {
            bytes = 4 * (size_t)ng;
            if ((int64_t)bytes > cap_bytes) return fail(c, BH_ECAPACITY, "export buffer too small");
            uint32_t *b = new (std::nothrow) uint32_t[(size_t)ng + 1];
            if (!b) return fail(c, BH_ENOMEM, "host allocation");
            hipError_t e = hipMemcpy(b, g.begin, 4 * ((size_t)ng + 1), hipMemcpyDeviceToHost);
            if (e == hipSuccess)
                for (uint32_t k = 0; k < ng; ++k) ((uint32_t *)dst)[k] = b[k + 1] - b[k];
            delete[] b;
            BH_HIP(c, e);
            if (nbytes) *nbytes = (int64_t)bytes;
            return check_status(c);
        }
        case BH_ARR_GROUP_BOX: src = g.box; bytes = 32 * (size_t)ng; break;
        case BH_ARR_GROUP_NPP: src = g.npp; bytes = 4 * (size_t)ng; break;
        case BH_ARR_GROUP_NPC: src = g.npc; bytes = 4 * (size_t)ng; break;
        case BH_ARR_ACC_SORTED: src = c->acc; bytes = 16 * n; break;
        case BH_ARR_BOUNDARY_FLAG:
        case BH_ARR_BOUNDARY_CELLS:
        case BH_ARR_BOUNDARY_BOX:
            if (!c->bnd.valid) return fail(c, BH_ESTATE, "no boundary tree");
            if (array == BH_ARR_BOUNDARY_FLAG) { src = c->bnd.flag; bytes = 4 * nc; }
            if (array == BH_ARR_BOUNDARY_CELLS) { src = c->bnd.ids; bytes = 4 * (size_t)c->bnd.nterm; }
            if (array == BH_ARR_BOUNDARY_BOX) { src = c->bnd.box; bytes = 32 * (size_t)c->bnd.nterm; }
            break;
        case BH_ARR_LET_ORIGIN:
        case BH_ARR_LET_NODE:
        case BH_ARR_LET_COMF:
            if (!c->let.valid) return fail(c, BH_ESTATE, "no local essential tree");
            if (array == BH_ARR_LET_ORIGIN) { src = c->let.origin; bytes = 8 * (size_t)c->let.ncell; }
            if (array == BH_ARR_LET_NODE) { src = c->let.wN; bytes = 8 * (size_t)c->let.ncell; }
            if (array == BH_ARR_LET_COMF) { src = c->let.wA; bytes = 16 * (size_t)c->let.ncell; }
            break;
        default: return fail(c, BH_EINVAL, "unknown export id");
    }
    if ((int64_t)bytes > cap_bytes) return fail(c, BH_ECAPACITY, "export buffer too small");
    if (bytes) BH_HIP(c, hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
    if (nbytes) *nbytes = (int64_t)bytes;
    return check_status(c);
}

int bh_export_keys(bh_ctx *c, uint64_t *keys, uint32_t *perm, hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!c->built) return fail(c, BH_ESTATE, "nothing built");
    BH_HIP(c, hipStreamSynchronize(s));
    const size_t n = (size_t)c->n;
    if (keys && n) BH_HIP(c, hipMemcpy(keys, c->sort.key[0], 8 * n, hipMemcpyDeviceToHost));
    if (perm && n) BH_HIP(c, hipMemcpy(perm, c->st[c->cur].cid, 4 * n, hipMemcpyDeviceToHost));
    return check_status(c);
}

int bh_export_tree(bh_ctx *c, bh_tree_view *out, hipStream_t s) {
    if (!c || !out) return BH_EINVAL;
    if (!c->built) return fail(c, BH_ESTATE, "nothing built");
    BH_HIP(c, hipStreamSynchronize(s));
    uint32_t ls[kLsSize], ng = 0;
    BH_HIP(c, hipMemcpy(ls, c->cells.ls, sizeof(ls), hipMemcpyDeviceToHost));
    BH_HIP(c, hipMemcpy(&ng, c->groups.count_dev, sizeof(ng), hipMemcpyDeviceToHost));
    const Cells &q = c->cells;
    bh_tree_view v{};
    v.n = c->n;
    v.ncells = ls[kLevels];
    v.ngroups = ng;
    v.level_start = q.ls;
    v.prefix = q.prefix;
    v.level = q.level; v.begin = q.begin; v.count = q.count;
    v.child0 = q.child0; v.nchild = q.nchild; v.parent = q.parent;
    v.M = q.M; v.S = q.S; v.Q = q.Q;
    v.group_begin = c->groups.begin;
    *out = v;
    return check_status(c);
}

int tree_force_vjp(bh_ctx *c, float theta, float eps, const float *u, float coef,
                   float *g_pos, float *g_mass, hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!valid_theta(theta)) return fail(c, BH_EINVAL, "theta must be in (0, 1]");
    if (!valid_eps(eps)) return fail(c, BH_EINVAL, "eps must be finite and >= 0");
    if (!u || !std::isfinite(coef)) return fail(c, BH_EINVAL, "null cotangent or bad coef");
    if (!c->p.adjoint) return fail(c, BH_EINVAL, "context created without adjoint = 1");
    if (!c->built) return fail(c, BH_ESTATE, "tree_force_vjp before tree_build");
    if (!g_pos && !g_mass) return BH_OK;
    launch_walk_prep(c, theta, s);
    launch_walk_vjp(c, eps, u, coef, g_pos, g_mass, s);
    BH_HIP(c, hipGetLastError());
    return BH_OK;
}

int tree_direct(bh_ctx *c, const int64_t *targets, int64_t nt, float eps, double *acc,
                double *pot, hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!valid_eps(eps)) return fail(c, BH_EINVAL, "eps must be finite and >= 0");
    if (nt < 0 || nt > (int64_t)UINT32_MAX / 4) return fail(c, BH_EINVAL, "bad target count");
    if (nt && (!targets || !acc || !pot)) return fail(c, BH_EINVAL, "null pointer");
    if (!c->built) return fail(c, BH_ESTATE, "tree_direct before tree_build");
    if (nt == 0) return BH_OK;
    launch_direct(c, targets, (uint32_t)nt, eps, acc, pot, s);
    BH_HIP(c, hipGetLastError());
    return BH_OK;
}

int leapfrog_vjp_drift(bh_ctx *c, float dt, const float *gx, float *gv, hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!gx || !gv || !std::isfinite(dt)) return fail(c, BH_EINVAL, "bad arguments");
    if (!c->built) return fail(c, BH_ESTATE, "no state");
    launch_axpy3(gx, gv, dt, (uint32_t)c->n, s);
    BH_HIP(c, hipGetLastError());
    return BH_OK;
}

int leapfrog_vjp_segment(bh_ctx *c, const void *snap, int64_t n, int32_t k, int32_t flags,
                         float dt, float theta, float eps, const float *gx, const float *gv,
                         float *gx0, float *gv0, float *gm, hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!snap || !gx || !gv || !gx0 || !gv0) return fail(c, BH_EINVAL, "null pointer");
    if (k < 1) return fail(c, BH_EINVAL, "k must be >= 1");
    if (flags & ~(BH_SEG_FIRST | BH_SEG_LAST)) return fail(c, BH_EINVAL, "unknown flags");
    if (!std::isfinite(dt)) return fail(c, BH_EINVAL, "dt must be finite");
    if (!valid_theta(theta)) return fail(c, BH_EINVAL, "theta must be in (0, 1]");
    if (!valid_eps(eps)) return fail(c, BH_EINVAL, "eps must be finite and >= 0");
    if (!c->p.adjoint) return fail(c, BH_EINVAL, "context created without adjoint = 1");
    int rc = check_n(c, n);
    if (rc) return rc;
    const size_t vec = 3 * sizeof(float) * (size_t)n;
    const int64_t per = n * (int64_t)(7 * sizeof(float) + sizeof(uint32_t) +
                                      (c->p.pos_fp64 ? 3 * sizeof(double) : 0));
    std::string err;
    if (k > 1 && !grow(&c->seg, c->seg_cap, (int64_t)(k - 1) * per, err))
        return fail(c, BH_ENOMEM, err);
    if (gx0 != gx) BH_HIP(c, hipMemcpyAsync(gx0, gx, vec, hipMemcpyDeviceToDevice, s));
    if (gv0 != gv) BH_HIP(c, hipMemcpyAsync(gv0, gv, vec, hipMemcpyDeviceToDevice, s));
    const float h = 0.5f * dt;
    const bool last = (flags & BH_SEG_LAST) != 0;
    // recompute the segment: state j (j = 1 .. k - 1) into seg[j - 1]
    if ((rc = bh_load_state(c, snap, n, s))) return rc;
    for (int32_t j = 1; j < k; ++j) {
        if ((rc = leapfrog_step(c, dt, theta, eps, s))) return rc;
        if ((rc = bh_save_state(c, c->seg + (size_t)(j - 1) * (size_t)per, s))) return rc;
    }
    if (last) {  // the closing half kick of the final step, at x_k
        if ((rc = leapfrog_step(c, dt, theta, eps, s))) return rc;
        if ((rc = tree_force_vjp(c, theta, eps, gv0, h, gx0, gm, s))) return rc;
    }
    for (int32_t j = k - 1; j >= 0; --j) {
        if ((rc = leapfrog_vjp_drift(c, dt, gx0, gv0, s))) return rc;
        // the context holds state k - 1 after the recompute unless it went on to x_k
        if (j < k - 1 || last) {
            const void *src = j == 0 ? snap : (const void *)(c->seg + (size_t)(j - 1) * (size_t)per);
            if ((rc = bh_load_state(c, src, n, s))) return rc;
        }
        const float coef = (j == 0 && (flags & BH_SEG_FIRST)) ? h : dt;
        if ((rc = tree_force_vjp(c, theta, eps, gv0, coef, gx0, gm, s))) return rc;
    }
    BH_HIP(c, hipGetLastError());
    return BH_OK;
}

int64_t bh_state_bytes(const bh_ctx *c) {
    if (!c || !c->built) return 0;
    return c->n * (int64_t)(7 * sizeof(float) + sizeof(uint32_t) +
                            (c->p.pos_fp64 ? 3 * sizeof(double) : 0));
}

int bh_save_state(bh_ctx *c, void *dst, hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!dst) return fail(c, BH_EINVAL, "null destination");
    if (!c->built) return fail(c, BH_ESTATE, "no state");
    const size_t n = (size_t)c->n;
    const State &st = c->st[c->cur];
    char *p = static_cast<char *>(dst);
    float *const fa[7] = {st.x, st.y, st.z, st.m, st.vx, st.vy, st.vz};
    for (float *f : fa) {
        BH_HIP(c, hipMemcpyAsync(p, f, n * sizeof(float), hipMemcpyDeviceToDevice, s));
        p += n * sizeof(float);
    }
    BH_HIP(c, hipMemcpyAsync(p, st.cid, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    p += n * sizeof(uint32_t);
    if (c->p.pos_fp64) {
        double *const da[3] = {st.x64, st.y64, st.z64};
        for (double *d : da) {
            BH_HIP(c, hipMemcpyAsync(p, d, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            p += n * sizeof(double);
        }
    }
    return BH_OK;
}

int bh_load_state(bh_ctx *c, const void *src, int64_t n64, hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!src) return fail(c, BH_EINVAL, "null source");
    int rc = check_n(c, n64);
    if (rc) return rc;
    const size_t n = (size_t)n64;
    c->n = n64;
    State &st = c->st[c->cur];
    const char *p = static_cast<const char *>(src);
    float *const fa[7] = {st.x, st.y, st.z, st.m, st.vx, st.vy, st.vz};
    for (float *f : fa) {
        BH_HIP(c, hipMemcpyAsync(f, p, n * sizeof(float), hipMemcpyDeviceToDevice, s));
        p += n * sizeof(float);
    }
    BH_HIP(c, hipMemcpyAsync(st.cid, p, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    p += n * sizeof(uint32_t);
    if (c->p.pos_fp64) {
        double *const da[3] = {st.x64, st.y64, st.z64};
        for (double *d : da) {
            BH_HIP(c, hipMemcpyAsync(d, p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            p += n * sizeof(double);
        }
    }
    rebuild(c, (uint32_t)n, s, true);
    c->ev_rec[6] = c->ev_rec[7] = false;
    BH_HIP(c, hipGetLastError());
    return BH_OK;
}

static int check_grid(bh_ctx *c, const bh_cic_grid *g) {
    if (!g || !(g->r_min > 0.f) || !(g->r_max > g->r_min) || !std::isfinite(g->r_max) ||
        g->n_r < 1 || g->n_phi < 1 || (int64_t)g->n_r * g->n_phi > 65536)
        return fail(c, BH_EINVAL, "bad surface-density grid");
    return BH_OK;
}

int bh_cic_density(bh_ctx *c, const float *pos, const float *mass, const uint8_t *sel,
                   int64_t n, const bh_cic_grid *grid, float *density, hipStream_t s) {
    if (!c) return BH_EINVAL;
    int rc = check_grid(c, grid);
    if (rc) return rc;
    if (!pos || !mass || !density || n < 0 || n > c->nmax)
        return fail(c, BH_EINVAL, "bad arguments");
    launch_cic(pos, mass, sel, (uint32_t)n, grid->r_min, grid->r_max, grid->n_r, grid->n_phi,
               c->cic, density, s);
    BH_HIP(c, hipGetLastError());
    return BH_OK;
}

int bh_cic_density_vjp(bh_ctx *c, const float *pos, const float *mass, const uint8_t *sel,
                       int64_t n, const bh_cic_grid *grid, const float *g_density,
                       float *g_pos, float *g_mass, hipStream_t s) {
    if (!c) return BH_EINVAL;
    int rc = check_grid(c, grid);
    if (rc) return rc;
    if (!pos || !mass || !g_density || n < 0 || n > c->nmax)
        return fail(c, BH_EINVAL, "bad arguments");
    launch_cic_vjp(pos, mass, sel, (uint32_t)n, grid->r_min, grid->r_max, grid->n_r, grid->n_phi,
                   g_density, g_pos, g_mass, s);
    BH_HIP(c, hipGetLastError());
    return BH_OK;
}

int bh_set_box(bh_ctx *c, const float *lo, float side) {
    if (!c) return BH_EINVAL;
    if (!lo) {
        c->fixed_box = false;
        return BH_OK;
    }
    if (!std::isfinite(lo[0]) || !std::isfinite(lo[1]) || !std::isfinite(lo[2]) ||
        !std::isfinite(side) || !(side > 0.f))
        return fail(c, BH_EINVAL, "box corner must be finite and side > 0");
    c->fixed_box = true;
    c->box_lo[0] = lo[0];
    c->box_lo[1] = lo[1];
    c->box_lo[2] = lo[2];
    c->box_side = side;
    return BH_OK;
}

int bh_decompose(bh_ctx *c, int32_t p, float cap, int64_t *cuts, hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!cuts) return fail(c, BH_EINVAL, "null pointer");
    if (!c->built) return fail(c, BH_ESTATE, "bh_decompose before tree_build");
    if (!c->counts_valid) return fail(c, BH_ESTATE, "bh_decompose needs a force walk");
    const int64_t n = c->n;
    if (p < 1 || p > n) return fail(c, BH_EINVAL, "p must be in [1, n]");
    if (!std::isfinite(cap) || !(cap >= 1.f)) return fail(c, BH_EINVAL, "cap must be >= 1");
    const int64_t C = cap_count(cap, n, p);
    if (C * (int64_t)p < n) return fail(c, BH_EINVAL, "cap * n / p cannot hold n particles");
    std::string err;
    if (!grow(&c->cut.S, c->cut.S_cap, n + 1, err) ||
        !grow(&c->cut.cuts, c->cut.cuts_cap, (int64_t)p + 1, err))
        return fail(c, BH_ENOMEM, err);
    launch_cut(c, p, C, c->cut.S, c->cut.cuts, s);
    BH_HIP(c, hipGetLastError());
    BH_HIP(c, hipMemcpyAsync(cuts, c->cut.cuts, 8 * ((size_t)p + 1), hipMemcpyDeviceToHost, s));
    BH_HIP(c, hipStreamSynchronize(s));
    return check_status(c);
}

int bh_decompose_sampled(bh_ctx *c, int32_t px, int32_t py, int32_t m1, int32_t m2, float cap,
                         int64_t *cuts, uint64_t *bounds, hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!cuts) return fail(c, BH_EINVAL, "null pointer");
    if (!c->built) return fail(c, BH_ESTATE, "bh_decompose_sampled before tree_build");
    if (!c->counts_valid) return fail(c, BH_ESTATE, "bh_decompose_sampled needs a force walk");
    const int64_t n = c->n;
    if (px < 1 || py < 1 || (int64_t)px * py > n || (int64_t)px * py > 65536)
        return fail(c, BH_EINVAL, "need 1 <= px py <= min(n, 65536)");
    if (m1 < 1 || m2 < 1) return fail(c, BH_EINVAL, "sample counts must be >= 1");
    const int32_t p = px * py;
    if (!std::isfinite(cap) || !(cap >= 1.f)) return fail(c, BH_EINVAL, "cap must be >= 1");
    const int64_t C = cap_count(cap, n, p);
    if (C * (int64_t)p < n) return fail(c, BH_EINVAL, "cap * n / p cannot hold n particles");
    BH_HIP(c, hipStreamSynchronize(s));
    std::vector<int64_t> cost;
    int rc = particle_costs(c, cost);
    if (rc) return rc;
    std::vector<uint64_t> skey((size_t)n);
    std::vector<uint32_t> cid((size_t)n);
    BH_HIP(c, hipMemcpy(skey.data(), c->sort.key[0], 8 * (size_t)n, hipMemcpyDeviceToHost));
    BH_HIP(c, hipMemcpy(cid.data(), c->st[c->cur].cid, 4 * (size_t)n, hipMemcpyDeviceToHost));
    // the emulated processes: caller index i is held by process floor(i p / n)
    std::vector<std::vector<uint64_t>> lk((size_t)p);
    std::vector<std::vector<int64_t>> lc((size_t)p);
    for (int64_t i = 0; i < n; ++i) {
        const size_t q = (size_t)((int64_t)cid[(size_t)i] * p / n);
        lk[q].push_back(skey[(size_t)i]);
        lc[q].push_back(cost[(size_t)i]);
    }
    std::vector<uint64_t> smp;
    int64_t W = 0;
    // level 1: every process samples, one DD process cuts into px pieces
    std::vector<std::pair<uint64_t, int64_t>> s1;
    for (int32_t q = 0; q < p; ++q) {
        draw_samples(lk[(size_t)q], lc[(size_t)q], m1, smp, W);
        for (uint64_t k : smp) s1.push_back({k, W});
    }
    std::vector<uint64_t> top;
    std::vector<char> top_have;
    weight_cuts(s1, px, top, top_have);
    std::vector<uint64_t> present;
    for (size_t t = 0; t < top.size(); ++t)
        if (top_have[t]) present.push_back(top[t]);
    // level 2: every process samples again, each sample to the piece of its
    // key; the DD process of each piece cuts it into py pieces
    std::vector<std::vector<std::pair<uint64_t, int64_t>>> bucket((size_t)px);
    for (int32_t q = 0; q < p; ++q) {
        draw_samples(lk[(size_t)q], lc[(size_t)q], m2, smp, W);
        for (uint64_t k : smp) {
            const size_t t =
                (size_t)(std::upper_bound(present.begin(), present.end(), k) - present.begin());
            bucket[t].push_back({k, W});
        }
    }
    const uint64_t kEnd = ~(uint64_t)0;  // past every key
    std::vector<uint64_t> bk;
    for (int32_t t = 0; t < px; ++t) {
        if (t > 0) bk.push_back(top_have[(size_t)t - 1] ? top[(size_t)t - 1] : kEnd);
        const uint64_t end = t < px - 1 && top_have[(size_t)t] ? top[(size_t)t] : kEnd;
        std::vector<uint64_t> sub;
        std::vector<char> sub_have;
        weight_cuts(bucket[(size_t)t], py, sub, sub_have);
        for (size_t k = 0; k < sub.size(); ++k) bk.push_back(sub_have[k] ? sub[k] : end);
    }
    cuts[0] = 0;
    for (int32_t j = 1; j < p; ++j)
        cuts[j] = (int64_t)(std::lower_bound(skey.begin(), skey.end(), bk[(size_t)j - 1]) -
                            skey.begin());
    clamp_cuts(cuts, p, n, C);
    if (bounds)
        for (int32_t j = 0; j + 1 < p; ++j) bounds[j] = bk[(size_t)j];
    return check_status(c);
}

int bh_domain_extract(bh_ctx *c, int64_t lo, int64_t hi, float *pos, float *vel, float *mass,
                      uint32_t *ids, hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!c->built) return fail(c, BH_ESTATE, "bh_domain_extract before tree_build");
    if (lo < 0 || hi < lo || hi > c->n) return fail(c, BH_EINVAL, "need 0 <= lo <= hi <= n");
    if (hi > lo) launch_range_out(c, (uint32_t)lo, (uint32_t)(hi - lo), pos, vel, mass, ids, s);
    BH_HIP(c, hipGetLastError());
    return BH_OK;
}

int tree_force_add(bh_ctx *c, bh_ctx *src, float theta, float eps, float *acc, float *pot,
                   hipStream_t s) {
    if (!c || !src) return BH_EINVAL;
    if (src == c) return fail(c, BH_EINVAL, "the source must be another context");
    if (!valid_theta(theta)) return fail(c, BH_EINVAL, "theta must be in (0, 1]");
    if (!valid_eps(eps)) return fail(c, BH_EINVAL, "eps must be finite and >= 0");
    if (!c->built || !src->built) return fail(c, BH_ESTATE, "tree_force_add before tree_build");
    if (src->device != c->device) return fail(c, BH_EINVAL, "contexts on different devices");
    launch_walk_prep(src, theta, s);
    launch_walk_view(c, own_view(src), eps, true, false, s);
    if (acc || pot) launch_unsort_add(c, acc, pot, (uint32_t)c->n, s);
    c->have_acc = false;
    c->counts_valid = false;
    BH_HIP(c, hipGetLastError());
    return BH_OK;
}

int bh_boundary(bh_ctx *c, int32_t max_cells, int32_t *level, int64_t *nterm, hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!c->built) return fail(c, BH_ESTATE, "bh_boundary before tree_build");
    if (max_cells < 1) return fail(c, BH_EINVAL, "max_cells must be >= 1");
    Boundary &b = c->bnd;
    std::string err;
    const int64_t cap = c->cap_cells + 1;
    int64_t c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0, c6 = 0, c7 = 0, c8 = 0;
    const int64_t plen = scan_part_len(cap);
    if (!b.flag) {
        if (!grow(&b.flag, c1, cap, err) || !grow(&b.scan, c2, cap, err) ||
            !grow(&b.ids, c3, cap, err) || !grow(&b.box, c4, 2 * cap, err) ||
            !grow(&b.cmin, c7, cap, err) || !grow(&b.cmax, c8, cap, err) ||
            !grow(&b.lvl, c5, kLevels, err) || !grow(&b.part, c6, plen, err)) {
            Boundary z{};
            auto f = [](void *q) { if (q) (void)hipFree(q); };
            f(b.flag); f(b.scan); f(b.ids); f(b.box); f(b.cmin); f(b.cmax); f(b.lvl); f(b.part);
            b = z;
            return fail(c, BH_ENOMEM, err);
        }
    }
    b.valid = false;
    launch_bnd_flags(c, s);
    uint32_t lvl[kLevels];
    float box[5];
    BH_HIP(c, hipStreamSynchronize(s));
    BH_HIP(c, hipMemcpy(lvl, b.lvl, sizeof(lvl), hipMemcpyDeviceToHost));
    BH_HIP(c, hipMemcpy(box, c->box, sizeof(box), hipMemcpyDeviceToHost));
    int64_t tot = 0;
    int L = -1;
    for (int l = 0; l < kLevels; ++l) {
        if (tot + (int64_t)lvl[l] > (int64_t)max_cells) break;
        tot += lvl[l];
        L = l;
    }
    if (L < 0) return fail(c, BH_EINVAL, "max_cells < 1");
    const uint32_t nc = cell_count(c, s);
    launch_bnd_terminal(c, L, s);
    launch_exclusive_scan(b.scan, b.scan, nc + 1, b.part, s);
    uint32_t nt = 0;
    BH_HIP(c, hipStreamSynchronize(s));
    BH_HIP(c, hipMemcpy(&nt, b.scan + nc, sizeof(nt), hipMemcpyDeviceToHost));
    // margin: 2^-16 of the largest coordinate magnitude the box allows
    float mabs = std::max(std::fabs(box[0]), std::max(std::fabs(box[1]), std::fabs(box[2])));
    float r = mabs + box[3];
    b.margin = r * 0x1p-16f;
    launch_bnd_boxes(c, nc, nt, s);
    BH_HIP(c, hipGetLastError());
    b.level = L;
    b.nterm = nt;
    b.valid = true;
    if (level) *level = L;
    if (nterm) *nterm = nt;
    BH_HIP(c, hipStreamSynchronize(s));
    return check_status(c);
}

int bh_let_build(bh_ctx *c, bh_ctx *const *srcs, int32_t nsrc, float theta, int64_t *info,
                 hipStream_t s) {
    if (!c) return BH_EINVAL;
    if ((!srcs && nsrc) || nsrc < 0 || nsrc > 64)
        return fail(c, BH_EINVAL, "need 0 <= nsrc <= 64 sources");
    if (!valid_theta(theta)) return fail(c, BH_EINVAL, "theta must be in (0, 1]");
    if (!c->built || !c->bnd.valid) return fail(c, BH_ESTATE, "target needs a boundary tree");
    if (nsrc == 0) {  // a single domain: nothing remote
        c->let.ncell = c->let.npart = 0;
        c->let.nsrc = 0;
        c->let.theta = theta;
        c->let.valid = true;
        return BH_OK;
    }
    for (int32_t k = 0; k < nsrc; ++k) {
        const bh_ctx *src = srcs[k];
        if (!src || src == c) return fail(c, BH_EINVAL, "sources must be other contexts");
        if (!src->built || !src->bnd.valid)
            return fail(c, BH_ESTATE, "every source needs a boundary tree");
        if (src->device != c->device) return fail(c, BH_EINVAL, "contexts on different devices");
        if (!same_box(c, src)) return fail(c, BH_EINVAL, "all domains need the same bh_set_box");
        for (int32_t q = 0; q < k; ++q)
            if (srcs[q] == src) return fail(c, BH_EINVAL, "a source is listed twice");
    }
    Let &t = c->let;
    t.valid = false;
    // virtual cells above the LET roots: levels of at most 8 children each
    int64_t lv[4] = {nsrc, 0, 0, 0};
    int nlv = 1;
    while (lv[0] > 1 || nlv == 1) {
        for (int q = nlv; q > 0; --q) lv[q] = lv[q - 1];
        lv[0] = (lv[1] + 7) / 8;
        ++nlv;
    }
    int64_t nv = 0;
    for (int q = 0; q + 1 < nlv; ++q) nv += lv[q];
    // sizes
    std::vector<uint32_t> ncs((size_t)nsrc);
    int64_t need_c = nv, need_p = 0, max_c = 0, max_p = 0;
    for (int32_t k = 0; k < nsrc; ++k) {
        ncs[(size_t)k] = cell_count(srcs[k], s);
        need_c += ncs[(size_t)k];
        need_p += srcs[k]->n;
        max_c = std::max<int64_t>(max_c, ncs[(size_t)k]);
        max_p = std::max<int64_t>(max_p, srcs[k]->n);
    }
    if (need_c >= (int64_t(1) << 29) || need_p >= (int64_t(1) << 31))
        return fail(c, BH_ECAPACITY, "local essential tree too large");
    std::string err;
    int64_t cc = t.cell_cap, c2 = cc, c3 = cc, c4 = cc, c5 = cc, c6 = cc, c7 = 2 * cc;
    int64_t pc = t.part_cap;
    if (!grow(&t.wA, cc, need_c, err) || !grow(&t.P0, c2, need_c, err) ||
        !grow(&t.P1, c3, need_c, err) || !grow(&t.P2, c4, need_c, err) ||
        !grow(&t.wN, c5, need_c, err) || !grow(&t.origin, c7, 2 * need_c, err) ||
        !grow(&t.xyzm, pc, std::max<int64_t>(need_p, 1), err)) {
        t.cell_cap = t.part_cap = 0;
        return fail(c, BH_ENOMEM, err);
    }
    (void)c6;
    t.cell_cap = need_c;
    t.part_cap = std::max<int64_t>(need_p, 1);
    int64_t s1 = t.scr_cells, s2 = s1, s0 = s1, s3 = t.scr_parts, s4 = s3, s5 = t.part_len, s6 = 1;
    const int64_t plen = scan_part_len(std::max(max_c, max_p) + 1);
    if (!grow(&t.cmark, s1, max_c + 1, err) || !grow(&t.omark, s0, max_c + 1, err) ||
        !grow(&t.cscan, s2, max_c + 1, err) ||
        !grow(&t.pmark, s3, max_p + 1, err) || !grow(&t.pscan, s4, max_p + 1, err) ||
        !grow(&t.spart, s5, plen, err) || (!t.word && !grow(&t.word, s6, 1, err))) {
        t.scr_cells = t.scr_parts = t.part_len = 0;
        return fail(c, BH_ENOMEM, err);
    }
    t.scr_cells = max_c + 1;
    t.scr_parts = max_p + 1;
    t.part_len = plen;

    uint32_t cbase = (uint32_t)(nv + nsrc), pbase = 0;
    for (int32_t k = 0; k < nsrc; ++k) {
        bh_ctx *src = srcs[k];
        const uint32_t nc = ncs[(size_t)k];
        launch_walk_prep(src, theta, s);
        launch_let_mark(c, src, nc, s);
        uint32_t word = 0;
        BH_HIP(c, hipStreamSynchronize(s));
        BH_HIP(c, hipMemcpy(&word, t.word, sizeof(word), hipMemcpyDeviceToHost));
        const bool boundary_only = word == 0u;
        launch_let_keep(c, src, nc, boundary_only, s);
        uint32_t kc = 0, kp = 0;
        BH_HIP(c, hipStreamSynchronize(s));
        BH_HIP(c, hipMemcpy(&kc, t.cscan + nc, sizeof(kc), hipMemcpyDeviceToHost));
        BH_HIP(c, hipMemcpy(&kp, t.pscan + src->n, sizeof(kp), hipMemcpyDeviceToHost));
        launch_let_emit(c, src, nc, k, boundary_only, (uint32_t)(nv + k), cbase, pbase, s);
        BH_HIP(c, hipGetLastError());
        if (info) {
            info[3 * k] = boundary_only ? 1 : 0;
            info[3 * k + 1] = kc;
            info[3 * k + 2] = kp;
        }
        cbase += kc - 1u;
        pbase += kp;
    }
    // the virtual cells: never accepted (r_open^2 = +inf), children contiguous
    std::vector<float4> vA((size_t)nv), vz((size_t)nv);
    std::vector<uint2> vN((size_t)nv);
    std::vector<uint32_t> vo(2 * (size_t)nv, kNone);
    int64_t off = 0;
    for (int q = 0; q + 1 < nlv; ++q) {
        const int64_t next = off + lv[q];
        for (int64_t i = 0; i < lv[q]; ++i) {
            const int64_t f = 8 * i, cnt = std::min<int64_t>(8, lv[q + 1] - f);
            vA[(size_t)(off + i)] = make_float4(0.f, 0.f, 0.f, INFINITY);
            vz[(size_t)(off + i)] = make_float4(0.f, 0.f, 0.f, 0.f);
            vN[(size_t)(off + i)] = make_uint2((uint32_t)(next + f), (uint32_t)cnt);
        }
        off = next;
    }
    BH_HIP(c, hipStreamSynchronize(s));
    BH_HIP(c, hipMemcpy(t.wA, vA.data(), 16 * (size_t)nv, hipMemcpyHostToDevice));
    BH_HIP(c, hipMemcpy(t.P0, vz.data(), 16 * (size_t)nv, hipMemcpyHostToDevice));
    BH_HIP(c, hipMemcpy(t.P1, vz.data(), 16 * (size_t)nv, hipMemcpyHostToDevice));
    BH_HIP(c, hipMemcpy(t.P2, vz.data(), 16 * (size_t)nv, hipMemcpyHostToDevice));
    BH_HIP(c, hipMemcpy(t.wN, vN.data(), 8 * (size_t)nv, hipMemcpyHostToDevice));
    BH_HIP(c, hipMemcpy(t.origin, vo.data(), 8 * (size_t)nv, hipMemcpyHostToDevice));
    t.ncell = cbase;
    t.npart = pbase;
    t.nsrc = nsrc;
    t.theta = theta;
    t.valid = true;
    return check_status(c);
}

int tree_force_let(bh_ctx *c, float theta, float eps, const uint32_t *rows, float *acc,
                   float *pot, hipStream_t s) {
    if (!c) return BH_EINVAL;
    if (!valid_theta(theta)) return fail(c, BH_EINVAL, "theta must be in (0, 1]");
    if (!valid_eps(eps)) return fail(c, BH_EINVAL, "eps must be finite and >= 0");
    if (!c->built) return fail(c, BH_ESTATE, "tree_force_let before tree_build");
    if (!c->let.valid) return fail(c, BH_ESTATE, "tree_force_let before bh_let_build");
    if (theta != c->let.theta) return fail(c, BH_EINVAL, "theta differs from the LET's");
    force(c, theta, eps, s);
    SrcView v;
    v.wA = c->let.wA; v.wN = c->let.wN;
    v.P0 = c->let.P0; v.P1 = c->let.P1; v.P2 = c->let.P2;
    v.xyzm = c->let.xyzm;
    if (c->let.ncell) {
        launch_walk_view(c, v, eps, true, true, s);
        launch_totals(c, (uint32_t)c->n, s);
    }
    if (acc || pot) launch_unsort(c, acc, pot, (uint32_t)c->n, s, rows);
    c->have_acc = false;  // acc holds local + remote forces
    BH_HIP(c, hipGetLastError());
    return BH_OK;
}

int tree_force_static(const float *pos, const float *mass, int64_t n, float theta, float eps,
                      float *acc, float *pot, uint32_t *status, hipStream_t s) {
    if (!pos || !mass) return BH_EINVAL;
    if (n <= 0 || !valid_theta(theta) || !valid_eps(eps)) return BH_EINVAL;
    if (n > kStaticMaxN) return BH_ECAPACITY;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return BH_EHIP;
    }
    StaticDevice d;
    int rc = static_device(dev, d);
    if (rc) return rc;
    // a context on the stack whose buffers are pieces of this device's array
    bh_ctx c;
    c.nmax = kStaticMaxN;
    c.cap_cells = kStaticMaxN + 21 * (kStaticMaxN / (16 + 1)) + 1;
    c.p.nleaf = 16;
    c.p.ncrit = 64;
    c.device = dev;
    c.cus = d.cus;
    c.walk_grid = d.walk_grid;
    if (static_layout(&c, d.ptr) > kStaticBytes) return BH_ENOMEM;
    c.n = n;
    c.cur = 0;
    // the array keeps the previous call's contents: clear the status words
    launch_fill_u32(c.status, 0u, 4, s);
    launch_ingest(&c, pos, nullptr, mass, (uint32_t)n, s);
    rebuild(&c, (uint32_t)n, s, true);
    force(&c, theta, eps, s);
    if (acc || pot) launch_unsort(&c, acc, pot, (uint32_t)n, s);
    if (status) {
        hipError_t e = hipMemcpyAsync(status, c.status, sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return BH_EHIP;
        }
    }
    if (hipGetLastError() != hipSuccess) return BH_EHIP;
    return BH_OK;
}

}  // extern "C"
