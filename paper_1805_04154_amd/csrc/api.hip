// C ABI of the powersort library: argument checks, workspace layout, the
// per-stream scratch pool and the launch sequence.
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "powersort_hip.h"
#include "common.hpp"
#include "block.hpp"
#include "internal.hpp"

namespace ps {

constexpr size_t kCountersBytes = sizeof(Counters);
constexpr int kMaskBlockA = kThreads * 16;

// ------------------------------------------------------------ small kernels

// Copies the caller's segment offsets into the workspace, less `base` (the
// first offset of a chunk of a larger batch), checking that they start at 0,
// never decrease, end at n_total and describe segments < 2^31.  Invalid
// offsets are replaced by one segment [0, n_total) and reported through the
// status word (so that no later kernel can index out of bounds).
__global__ __launch_bounds__(kThreads) void offsets_kernel(const uint64_t* __restrict__ in, uint32_t nseg,
                                                            uint64_t N, uint64_t base, uint64_t* __restrict__ out,
                                                            int32_t* __restrict__ status) {
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    int my = 0;
    for (uint32_t g = threadIdx.x; g <= nseg; g += kThreads) {
        const uint64_t v = in ? in[g] - base : (g == 0 ? 0 : N);
        if (g == 0 && v != 0) my |= 1;
        if (g == nseg && v != N) my |= 1;
        if (g > 0) {
            const uint64_t u = in ? in[g - 1] - base : 0;
            if (v < u) my |= 1;
            else if (v - u > kMaxSegment) my |= 2;
        }
    }
    if (my) atomicOr(&bad, my);
    __syncthreads();
    for (uint32_t g = threadIdx.x; g <= nseg; g += kThreads) {
        uint64_t v = in ? in[g] - base : (g == 0 ? 0 : N);
        if (bad) v = (g == 0) ? 0 : N;
        out[g] = v;
    }
    if (threadIdx.x == 0 && status)
        *status = (bad & 1) ? (int32_t)PS_ERR_INVALID_ARG : (bad & 2) ? (int32_t)PS_ERR_TOO_LARGE : (int32_t)PS_OK;
}

__global__ void copy_u64_kernel(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

__global__ void copy_u32_kernel(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

template <class T>
__global__ void copy_dyn_kernel(const T* __restrict__ src, T* __restrict__ dst, const uint32_t* __restrict__ r_dev,
                                uint32_t extra, uint32_t cap) {
    const uint32_t n = min(cap, *r_dev + extra);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

// ---------------------------------------------------- alphabetic trees
//
// Method 2' as a standalone builder (App. A): leaf weights w[0..r) become
// "runs" [S_i, S_i + w_i) with S_i = w_0 + ... + w_{i-1}, and the tree
// kernels of powersort then give the node powers, the Cartesian tree of the
// powers and the weighted depth sum.  These kernels form the S_i.

constexpr uint32_t kWeightBlock = kThreads * 8;  // weights per scan block

// Per-block sums of the weights; flags a zero weight.
__global__ __launch_bounds__(kThreads) void weight_sum_kernel(const uint32_t* __restrict__ w, uint32_t r,
                                                               uint64_t* __restrict__ bsum, uint32_t* __restrict__ flag) {
    __shared__ uint64_t sh[kWaves];
    const uint32_t base = blockIdx.x * kWeightBlock + threadIdx.x * 8;
    uint64_t s = 0;
    bool zero = false;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t x = base + i;
        if (x < r) {
            const uint32_t v = w[x];
            s += v;
            zero |= (v == 0);
        }
    }
    if (zero) atomicOr(flag, 1u);
    uint64_t total;
    (void)block_excl_sum64(s, sh, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Exclusive scan of the nb block sums in one block; flags a total of 2^31 or
// more, and publishes r, the segment [0, W) and starts[r] = W.
__global__ __launch_bounds__(kThreads) void weight_scan_kernel(uint64_t* __restrict__ bsum, uint32_t nb, uint32_t r,
                                                            uint32_t* __restrict__ flag, Counters* __restrict__ cnt,
                                                            uint64_t* __restrict__ offsets,
                                                            uint32_t* __restrict__ starts) {
    __shared__ uint64_t sh[kWaves];
    const uint32_t per = (nb + kThreads - 1) / kThreads;
    const uint32_t b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
    uint64_t s = 0;
    for (uint32_t b = b0; b < b1; ++b) s += bsum[b];
    uint64_t total;
    uint64_t run = block_excl_sum64(s, sh, &total);
    for (uint32_t b = b0; b < b1; ++b) {
        const uint64_t v = bsum[b];
        bsum[b] = run;
        run += v;
    }
    if (threadIdx.x == 0) {
        if (total > kMaxSegment) atomicOr(flag, 2u);
        const bool bad = (*flag != 0) || total > kMaxSegment;
        const uint64_t W = bad ? (uint64_t)r : total;  // invalid input: unit weights
        cnt->r = r;
        offsets[0] = 0;
        offsets[1] = W;
        starts[r] = (uint32_t)W;
    }
}

// starts[i] = sum of the weights before leaf i (unit weights if flagged).
__global__ __launch_bounds__(kThreads) void weight_starts_kernel(const uint32_t* __restrict__ w, uint32_t r,
                                                                  const uint64_t* __restrict__ bsum,
                                                                  const uint32_t* __restrict__ flag,
                                                                  uint32_t* __restrict__ starts,
                                                                  int32_t* __restrict__ status) {
    __shared__ uint64_t sh[kWaves];
    const uint32_t f = *flag;
    const uint32_t base = blockIdx.x * kWeightBlock + threadIdx.x * 8;
    uint64_t v[8];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t x = base + i;
        v[i] = (x < r) ? (f ? 1u : w[x]) : 0u;
        s += v[i];
    }
    uint64_t run = block_excl_sum64(s, sh, nullptr) + (f ? (uint64_t)blockIdx.x * kWeightBlock : bsum[blockIdx.x]);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t x = base + i;
        if (x < r) starts[x] = (uint32_t)run;
        run += v[i];
    }
    if (status && blockIdx.x == 0 && threadIdx.x == 0)
        *status = (f & 1) ? (int32_t)PS_ERR_INVALID_ARG : (f & 2) ? (int32_t)PS_ERR_TOO_LARGE : (int32_t)PS_OK;
}

// ------------------------------------------------------------------ layout

struct Layout {
    size_t total = 0;
    size_t scratch_keys, scratch_pay, offsets, tile_seg, tile_rec;
    size_t code[4], cnt[4], entry[4], offs[4];
    uint32_t ntab[4];
    int levels;
    size_t counters, starts, Q, P, leaf_depth, node_depth, aggF, aggB, inF, inB, mc, Lf, Rt, nsize;
    size_t unit_rec, unit_par, bigleaf, bigleaf_mode, biglist, bucket, node_rec, bucket_tile, leaf_tile, split, span;
    size_t child_l, child_r;
    uint32_t unit_base[3] = {0, 0, 0};  // first record of each UnitKind's list
    size_t samp = 0;  // 4-byte keys that move: one order key per kSampleSpacing positions
    uint32_t rmax;
    uint64_t split_cap = 0;
    size_t peek_f[2] = {0, 0};  // peeksort frontiers (ranges of one depth)
    uint32_t peek_cap = 0;
};

static size_t take(size_t& at, size_t bytes) {
    at = (at + 255) & ~(size_t)255;
    const size_t here = at;
    at += bytes;
    return here;
}

static Layout make_layout(uint64_t N, uint64_t nseg, size_t kb, bool hp, uint32_t w, bool moves, bool peek,
                          uint32_t nbuf) {
    Layout L;
    size_t at = 0;
    // nbuf - 1 scratch arrays of keys (and of payload), back to back
    L.scratch_keys = moves ? take(at, N * kb * (nbuf - 1)) : 0;
    L.scratch_pay = (moves && hp) ? take(at, N * 4 * (nbuf - 1)) : 0;
    L.offsets = take(at, (nseg + 1) * 8);
    const uint32_t W1 = w + 1;
    uint32_t nt = (uint32_t)((N + kPartTile - 1) / kPartTile);
    L.tile_seg = take(at, (size_t)nt * 4);
    L.tile_rec = take(at, (size_t)nt * sizeof(TileRec));
    L.levels = 0;
    while (true) {
        L.ntab[L.levels] = nt;
        L.code[L.levels] = take(at, (size_t)nt * W1);
        L.cnt[L.levels] = take(at, (size_t)nt * W1 * 4);
        L.entry[L.levels] = take(at, nt);
        L.offs[L.levels] = take(at, (size_t)nt * 4);
        L.levels++;
        if (nt <= (uint32_t)kScanGroup) break;
        nt = (nt + kScanGroup - 1) / kScanGroup;
    }
    const uint64_t per = (w < 2) ? 2 : w;
    uint64_t rmax = N / per + nseg + 1;
    if (rmax > N) rmax = N;
    L.rmax = (uint32_t)rmax;
    const size_t r1 = rmax + 1;
    const size_t nb = (rmax + kMaskBlockA - 1) / kMaskBlockA + 1;
    L.counters = take(at, kCountersBytes);
    L.starts = take(at, r1 * 4);
    L.Q = take(at, r1 * 8);
    L.P = take(at, r1 + 1);
    L.leaf_depth = take(at, r1);
    L.node_depth = take(at, r1);
    L.aggF = take(at, nb * 16);
    L.aggB = take(at, nb * 16);
    L.inF = take(at, nb * 8);
    L.inB = take(at, nb * 8);
    L.mc = take(at, (nseg + 1) * 8);
    L.Lf = take(at, r1 * 4);
    L.Rt = take(at, r1 * 4);
    L.nsize = take(at, r1 * 4);
    if (moves) {
        // fused subtrees are disjoint: at most r1 of them in all, at most
        // N / (kMaxMinRun + 1) single runs longer than any min-run, and at
        // most r1 / kFuseRadixMinLeaves with that many leaves
        const uint64_t cap_copy = std::min<uint64_t>(r1, N / (kMaxMinRun + 1) + 1);
        const uint64_t cap_radix = r1 / kFuseRadixMinLeaves + 1;
        L.unit_base[kUnitFew] = 0;
        L.unit_base[kUnitCopy] = (uint32_t)r1;
        L.unit_base[kUnitRadix] = (uint32_t)(r1 + cap_copy);
        const size_t nrec = r1 + cap_copy + cap_radix;
        L.unit_rec = take(at, nrec * sizeof(UnitRec));
        L.unit_par = take(at, nrec);
        L.bigleaf = take(at, r1 * 4);
        L.bigleaf_mode = take(at, r1);
        L.biglist = take(at, r1 * 4);
        L.bucket = take(at, r1 * 4);
        L.node_rec = take(at, r1 * sizeof(NodeRec));
        L.bucket_tile = take(at, r1 * 4);
        L.leaf_tile = take(at, r1 * 4);
        L.child_l = take(at, r1 * 4);
        L.child_r = take(at, r1 * 4);
        // Merge tiles over all passes: at most (merged elements) / (half the
        // smallest tile, the splitter spacing of two-level merges) + one per
        // merged node, and every merged node holds more than kFuse elements.
        // The merged elements are at most n per pass (a pass's nodes are
        // disjoint) and at most M <= n (lg n + 2) in all (Thm. "powersort");
        // a powersort merges in at most pfuse passes (see run()).
        const uint64_t lg = 64 - __builtin_clzll(N | 1);
        uint64_t pfuse = 1;
        while (((uint64_t)kFuse << pfuse) < 3 * N) ++pfuse;
        const uint64_t merged = N * (peek ? lg + 2 : std::min<uint64_t>(lg + 2, pfuse));
        L.split_cap = merged / kQuadSpacing + merged / kFuse + 64;
        L.split = take(at, L.split_cap * sizeof(SplitRec));
        L.span = take(at, L.split_cap * sizeof(TileSpan));
        if (kb == 4) L.samp = take(at, (N + kSampleSpacing - 1) / kSampleSpacing * 4);
    } else {
        L.unit_rec = L.unit_par = L.bigleaf = L.bigleaf_mode = L.biglist = L.bucket = L.node_rec = L.bucket_tile = L.leaf_tile = 0;
        L.child_l = L.child_r = 0;
        L.split = L.span = 0;
    }
    if (peek) {
        // ranges of one depth are disjoint and hold >= 2 leaves each
        L.peek_cap = L.rmax / 2 + 1;
        L.peek_f[0] = take(at, (size_t)L.peek_cap * sizeof(PeekRange));
        L.peek_f[1] = take(at, (size_t)L.peek_cap * sizeof(PeekRange));
    }
    L.total = take(at, 0) + 256;
    return L;
}

// -------------------------------------------------------------- scratch pool

struct PoolEntry {
    void* ptr = nullptr;
    size_t bytes = 0;
    int device = -1;
};
static std::mutex g_pool_mu;
static std::unordered_map<void*, PoolEntry> g_pool;  // keyed by stream
static uint64_t g_pool_limit = 0;                    // bytes per pool entry; 0 = no limit
static thread_local std::string g_last_error;

static ps_status fail(ps_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

static ps_status hip_fail(hipError_t e, const char* where) {
    return fail(PS_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

static ps_status get_workspace(hipStream_t st, size_t bytes, const ps_options* opt, void** out) {
    if (opt && opt->workspace) {
        if (opt->workspace_bytes < bytes) return fail(PS_ERR_INVALID_ARG, "workspace smaller than ps_workspace_bytes()");
        *out = opt->workspace;
        return PS_OK;
    }
    const size_t want = bytes + bytes / 8;  // headroom against regrowth
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (g_pool_limit && bytes > g_pool_limit)
        return fail(PS_ERR_OUT_OF_MEMORY, "scratch of " + std::to_string(bytes) + " bytes exceeds the pool limit of " +
                                              std::to_string(g_pool_limit) + " bytes (ps_set_pool_limit)");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    PoolEntry& p = g_pool[(void*)st];
    if (p.ptr && p.bytes >= bytes && p.device == dev) {
        *out = p.ptr;
        return PS_OK;
    }
    if (p.ptr) {
        // The old block may still be in use by work queued on this stream.
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        e = hipFree(p.ptr);
        p.ptr = nullptr;
        p.bytes = 0;
        if (e != hipSuccess) return hip_fail(e, "hipFree");
    }
    const size_t size = (g_pool_limit && want > g_pool_limit) ? bytes : want;
    void* ptr = nullptr;
    e = hipMalloc(&ptr, size);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PS_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(size) + " bytes failed");
    }
    p.ptr = ptr;
    p.bytes = size;
    p.device = dev;
    *out = ptr;
    return PS_OK;
}

// --------------------------------------------- fixed scratch (no allocation)
//
// ps_sort_no_alloc runs in this array instead of the pool or a caller's
// workspace.  Each device that loads the library holds its own copy until
// the process ends.  Host code never uses the array's name as an address:
// the address on each device comes from hipGetSymbolAddress, taken once per
// device with that device current.
constexpr size_t kFixedScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];  // address of `scratch` on each device

static ps_status fixed_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(PS_ERR_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(PS_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PS_OK;
}

// ------------------------------------------------------------------ tuning

static std::mutex g_tune_mu;
static Tuning g_tune;

static Tuning current_tuning() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tune;
}

// --------------------------------------------------------------- profiling

struct ProfPending {
    int group;
    int launches;
    uint64_t host_elems;
    hipEvent_t a, b;
};
struct ProfState {
    bool on = false;
    uint32_t mask = 0;  // groups timed with events
    std::vector<ProfPending> pending;
    std::vector<hipEvent_t> pool;
    ps_profile totals{};
    unsigned long long* dev = nullptr;  // device element counters per group
};
static std::mutex g_prof_mu;
static ProfState g_prof;

static hipEvent_t prof_event() {
    if (!g_prof.pool.empty()) {
        hipEvent_t e = g_prof.pool.back();
        g_prof.pool.pop_back();
        return e;
    }
    // Timing only: no system-scope fence when the event is recorded (that
    // fence writes back and invalidates caches, which slows the work after
    // it).  Results reach the caller through the stream's own completion.
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// Brackets a group of launches with events on `st` when profiling is on.
struct ProfScope {
    bool active = false;
    int group = 0, launches = 0;
    uint64_t elems = 0;
    hipEvent_t a = nullptr;
    hipStream_t st = nullptr;
    ProfScope(int g, int nl, uint64_t host_elems, hipStream_t s, bool allowed)
        : group(g), launches(nl), elems(host_elems), st(s) {
        if (!allowed) return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof.on || !((g_prof.mask >> g) & 1)) return;
        a = prof_event();
        if (a && hipEventRecord(a, st) == hipSuccess) active = true;
    }
    ~ProfScope() {
        if (!active) return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        hipEvent_t b = prof_event();
        if (b && hipEventRecord(b, st) == hipSuccess) g_prof.pending.push_back({group, launches, elems, a, b});
    }
};

// Times one launch with the start / end events of its own dispatch
// (hipExtLaunchKernel), which adds no packets between launches.
struct ProfLaunch {
    int group;
    hipEvent_t a = nullptr, b = nullptr;
    ProfLaunch(int g, bool allowed) : group(g) {
        if (!allowed) return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof.on || !((g_prof.mask >> g) & 1)) return;
        a = prof_event();
        b = prof_event();
        if (!a || !b) {
            if (a) g_prof.pool.push_back(a);
            if (b) g_prof.pool.push_back(b);
            a = b = nullptr;
        }
    }
    void done(hipError_t launched) {
        if (!a) return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (launched == hipSuccess) {
            g_prof.pending.push_back({group, 1, 0, a, b});
        } else {
            g_prof.pool.push_back(a);
            g_prof.pool.push_back(b);
        }
        a = b = nullptr;
    }
};

static bool prof_on() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    return g_prof.on;
}

// ------------------------------------------------------------------ driver

enum class Mode { Sort, Cost, Inspect };

struct Call {
    void* keys;
    uint32_t* payload;
    const uint64_t* d_offsets;  // nullable: one segment
    uint64_t nseg;
    uint64_t N;
    int kt;
    uint32_t w;
    uint64_t* d_costs;          // nullable
    int32_t* d_status;          // nullable
    ps_inspect_out* inspect;    // Mode::Inspect
    Mode mode;
    bool peek = false;          // PS_FLAG_PEEKSORT: Alg. PeekSort's tree instead of node powers
    uint32_t nbuf = 3;          // data arrays (2 with PS_FLAG_COMPACT_SCRATCH)
    uint64_t off_base = 0;      // subtracted from d_offsets (a chunk of a larger batch)
    bool prof = true;           // false: no profiling events (nothing is created or recorded)
};

static size_t key_bytes(int kt) { return (kt == KT_I64 || kt == KT_U64) ? 8 : 4; }

struct CallOpts {
    uint32_t w = 24;
    bool peek = false;
    uint32_t nbuf = 3;
};

static ps_status check_common(int kt, const ps_options* opt, CallOpts* o) {
    if (kt < KT_I32 || kt > KT_F32) return fail(PS_ERR_INVALID_ARG, "unknown key type");
    *o = CallOpts{};
    if (opt) {
        if (opt->struct_size != sizeof(ps_options)) return fail(PS_ERR_INVALID_ARG, "ps_options.struct_size mismatch");
        if (opt->flags & ~(uint32_t)(PS_FLAG_PEEKSORT | PS_FLAG_COMPACT_SCRATCH))
            return fail(PS_ERR_UNSUPPORTED, "unknown ps_options.flags bits");
        if (opt->min_run) o->w = opt->min_run;
        o->peek = (opt->flags & PS_FLAG_PEEKSORT) != 0;
        if (opt->flags & PS_FLAG_COMPACT_SCRATCH) o->nbuf = 2;
    }
    if (o->w > (uint32_t)kMaxMinRun) return fail(PS_ERR_UNSUPPORTED, "min_run above 64 is not supported");
    return PS_OK;
}

static inline uint32_t ilog2_floor(uint64_t x) {
    uint32_t l = 0;
    while (x >>= 1) ++l;
    return l;
}

static ps_status run(const Call& c, const ps_options* opt, hipStream_t st) {
    const uint32_t N = (uint32_t)c.N;
    const uint32_t nseg = (uint32_t)c.nseg;
    const bool moves = (c.mode == Mode::Sort);
    const Tuning tune = current_tuning();
    const bool hp = moves && c.payload != nullptr;
    const size_t kb = key_bytes(c.kt);
    // 8192-output tiles need 64 KiB of LDS with 4-byte keys; 8-byte keys use 4096
    const uint32_t merge_tile = (tune.merge_tile == 8192 && kb == 8) ? 4096u : tune.merge_tile;
    const Layout L = make_layout(c.N, c.nseg, kb, hp, c.w, moves, c.peek, c.nbuf);
    void* ws = nullptr;
    ps_status s = get_workspace(st, L.total, opt, &ws);
    if (s != PS_OK) return s;
    char* base = (char*)ws;
    auto at = [&](size_t off) { return (void*)(base + off); };

    uint64_t* offsets = (uint64_t*)at(L.offsets);
    hipLaunchKernelGGL(offsets_kernel, dim3(1), dim3(kThreads), 0, st, c.d_offsets, nseg, c.N, c.off_base, offsets,
                       c.d_status);
    Counters* cnt = (Counters*)at(L.counters);
    uint64_t* mc = (uint64_t*)at(L.mc);
    hipError_t e = launch_init(cnt, mc, nseg, st);
    if (e != hipSuccess) return hip_fail(e, "init launch");

    PartitionArgs pa{};
    pa.keys = c.keys;
    pa.N = N;
    pa.offsets = offsets;
    pa.nseg = nseg;
    pa.tile_seg = (uint32_t*)at(L.tile_seg);
    pa.tile_rec = (TileRec*)at(L.tile_rec);
    pa.w = c.w;
    pa.levels = L.levels;
    for (int l = 0; l < L.levels; ++l) {
        pa.code[l] = (uint8_t*)at(L.code[l]);
        pa.cnt[l] = (uint32_t*)at(L.cnt[l]);
        pa.entry[l] = (uint8_t*)at(L.entry[l]);
        pa.offs[l] = (uint32_t*)at(L.offs[l]);
        pa.ntab[l] = L.ntab[l];
    }
    pa.starts = (uint32_t*)at(L.starts);
    pa.r_dev = (uint32_t*)cnt;  // Counters.r is its first word
    pa.rmax = L.rmax;
    pa.samp = (moves && kb == 4) ? (uint32_t*)at(L.samp) : nullptr;
    {
        ProfScope ps_(PS_PROF_PARTITION, 2 + 2 * L.levels, c.N, st, c.prof);
        e = launch_partition(c.kt, pa, st);
    }
    if (e != hipSuccess) return hip_fail(e, "partition launch");

    TreeArgs ta{};
    ta.keys = c.keys;
    ta.offsets = offsets;
    ta.nseg = nseg;
    ta.rmax = L.rmax;
    ta.starts = pa.starts;
    ta.cnt = cnt;
    ta.Q = (uint64_t*)at(L.Q);
    ta.P = (uint8_t*)at(L.P);
    ta.leaf_depth = (uint8_t*)at(L.leaf_depth);
    ta.node_depth = (uint8_t*)at(L.node_depth);
    ta.aggF = (Mask2*)at(L.aggF);
    ta.aggB = (Mask2*)at(L.aggB);
    ta.inF = (uint64_t*)at(L.inF);
    ta.inB = (uint64_t*)at(L.inB);
    ta.mc = mc;
    ta.Lf = (uint32_t*)at(L.Lf);
    ta.Rt = (uint32_t*)at(L.Rt);
    ta.nsize = (uint32_t*)at(L.nsize);
    ta.merge_tile = merge_tile;
    // Peeksort: every internal node sits at depth <= 2 floor(lg n) - 1, so
    // that many + 1 levels build the whole tree (the key bound of kMaxPass).
    const uint32_t peek_levels = std::max<uint32_t>(1, 2 * ilog2_floor(c.N));
    if (c.peek) {
        ProfScope ps_(PS_PROF_TREE, 1 + (peek_levels + 1) / 2, c.N, st, c.prof);
        e = launch_peek_tree(ta, (PeekRange*)at(L.peek_f[0]), (PeekRange*)at(L.peek_f[1]), L.peek_cap, peek_levels,
                             st);
    } else {
        ProfScope ps_(PS_PROF_TREE, 4, c.N, st, c.prof);
        e = launch_tree_cost(ta, st);
    }
    if (e != hipSuccess) return hip_fail(e, "tree launch");

    if (c.mode == Mode::Inspect && !c.peek) {
        e = launch_node_ranges(ta, st);
        if (e != hipSuccess) return hip_fail(e, "node-range launch");
    }
    if (moves) {
        ta.lists.unit_rec = (UnitRec*)at(L.unit_rec);
        ta.lists.unit_par = (uint8_t*)at(L.unit_par);
        for (int k = 0; k < 3; ++k) ta.lists.unit_base[k] = L.unit_base[k];
        ta.lists.bigleaf = (uint32_t*)at(L.bigleaf);
        ta.lists.bigleaf_mode = (uint8_t*)at(L.bigleaf_mode);
        ta.lists.biglist = (uint32_t*)at(L.biglist);
        ta.lists.bucket = (uint32_t*)at(L.bucket);
        ta.lists.node_rec = (NodeRec*)at(L.node_rec);
        ta.lists.bucket_tile = (uint32_t*)at(L.bucket_tile);
        ta.lists.leaf_tile = (uint32_t*)at(L.leaf_tile);
        ta.lists.child_l = (uint32_t*)at(L.child_l);
        ta.lists.child_r = (uint32_t*)at(L.child_r);
        ta.lists.nbuf = c.nbuf;
        // two-level passes need the split pass's records (4-byte keys);
        // 8-byte keys merge one level per pass with in-kernel co-ranks
        ta.lists.levels = kb == 4 ? tune.merge_levels : 1u;
        if (c.prof && prof_on()) {
            std::lock_guard<std::mutex> lk(g_prof_mu);
            ta.prof = g_prof.dev;
        }
        {
            ProfScope ps_(PS_PROF_LISTS, c.peek ? 5 : 6, c.N, st, c.prof);
            if (!c.peek) e = launch_node_ranges(ta, st);
            if (e == hipSuccess) e = launch_tree_lists(c.kt, ta, st);
        }
        if (e != hipSuccess) return hip_fail(e, "tree-list launch");
        MoveArgs ma{};
        ma.keys[0] = c.keys;
        ma.keys[1] = at(L.scratch_keys);
        ma.keys[2] = c.nbuf == 3 ? (void*)((char*)at(L.scratch_keys) + (size_t)N * kb) : nullptr;
        ma.pay[0] = c.payload;
        ma.pay[1] = hp ? (uint32_t*)at(L.scratch_pay) : nullptr;
        ma.pay[2] = (hp && c.nbuf == 3) ? (uint32_t*)at(L.scratch_pay) + N : nullptr;
        ma.leaf_copy = leaf_copy_buf(c.nbuf);
        ma.starts = pa.starts;
        ma.P = ta.P;
        ma.Lf = ta.Lf;
        ma.Rt = ta.Rt;
        ma.node_depth = ta.node_depth;
        ma.cnt = cnt;
        ma.unit_rec = ta.lists.unit_rec;
        ma.unit_par = ta.lists.unit_par;
        for (int k = 0; k < 3; ++k) ma.unit_base[k] = L.unit_base[k];
        ma.bigleaf = ta.lists.bigleaf;
        ma.bigleaf_mode = ta.lists.bigleaf_mode;
        ma.bucket = ta.lists.bucket;
        ma.node_rec = ta.lists.node_rec;
        ma.bucket_tile = ta.lists.bucket_tile;
        ma.leaf_tile = ta.lists.leaf_tile;
        ma.split = (SplitRec*)at(L.split);
        ma.span = (TileSpan*)at(L.span);
        ma.split_cap = (uint32_t)std::min<uint64_t>(L.split_cap, 0xFFFFFFFFull);
        ma.merge_tile = merge_tile;
        ma.n = N;
        ma.samp = pa.samp;
        // Powers: by the definition of a node power, P_j <= ceil(lg(2n / (L_{j-1}
        // + L_j))), and two adjacent leaves of a segment hold at least w + 1
        // elements (only a segment's last leaf may be shorter than w), so no
        // node of a segment of at most N keys has a power above pbound.
        uint32_t pbound = 1;
        while (((uint64_t)1 << pbound) * (c.w + 1) < 2 * c.N) ++pbound;
        // Only nodes of more than kFuse elements merge in a pass (smaller ones
        // merge inside fused subtrees).  Every internal boundary of a node of
        // power p has power >= p, so its leaf midpoints share one cell of
        // width 2^(1-p) and each of its leaves is shorter than n 2^(2-p): the
        // node holds fewer than 3n / 2^(p-1) elements.  Passes with
        // kFuse 2^(p-1) >= 3N therefore hold no node.
        uint32_t pfuse = 1;
        while (((uint64_t)kFuse << pfuse) < 3 * c.N) ++pfuse;
        const uint32_t pmax = c.peek ? std::min<uint32_t>(kMaxPass, peek_levels)
                                     : std::min<uint32_t>(std::min<uint32_t>(kMaxPower, ilog2_floor(c.N) + 1),
                                                          std::min(pbound, pfuse));
        const uint64_t max_units = c.N / 2 + 1;
        const uint32_t grid_fuse = (uint32_t)std::min<uint64_t>(max_units, tune.grid_fused);
        auto stage = [&](int group, int s, uint32_t p, uint32_t grid) {
            ProfLaunch pl(group, c.prof);
            const hipError_t r = launch_move_stage(c.kt, hp, ma, s, p, grid, st, pl.a, pl.b);
            pl.done(r);
            return r;
        };
        e = stage(PS_PROF_BIG_LEAF, 0, 0, tune.grid_big_leaf);
        if (e == hipSuccess) e = stage(PS_PROF_FUSED, 5, 0, grid_fuse);  // single-run units
        if (e == hipSuccess) e = stage(PS_PROF_FUSED, 1, 0, grid_fuse);
        if (e == hipSuccess) e = stage(PS_PROF_FUSED, 4, 0, grid_fuse);
        for (uint32_t p = pmax; p >= 1 && e == hipSuccess; --p) {
            // tile co-ranks: a split pass for 4-byte keys; 8-byte keys find
            // them inside the merge pass
            if (kb == 4) e = stage(PS_PROF_SPLIT, 3, p, tune.grid_split);
            if (e == hipSuccess && ta.lists.levels == 2) e = stage(PS_PROF_SPLIT, 7, p, tune.grid_split);
            if (e == hipSuccess) e = stage(PS_PROF_MERGE, 2, p, tune.grid_merge);
            if (e == hipSuccess && ta.lists.levels == 2) e = stage(PS_PROF_MERGE, 6, p, tune.grid_merge);
        }
        if (e != hipSuccess) return hip_fail(e, "merge launch");
        if (c.prof && prof_on()) {
            std::lock_guard<std::mutex> lk(g_prof_mu);
            g_prof.totals.calls++;
        }
    }
    if (c.d_costs) {
        hipLaunchKernelGGL(copy_u64_kernel, dim3(std::min<uint32_t>(1024, (nseg + kThreads - 1) / kThreads + 1)),
                           dim3(kThreads), 0, st, mc, c.d_costs, nseg);
    }
    if (c.mode == Mode::Inspect && c.inspect) {
        const ps_inspect_out& o = *c.inspect;
        const uint32_t* r_dev = (const uint32_t*)cnt;
        const uint32_t cap = N + 1;
        const dim3 g(1024), b(kThreads);
        if (o.starts) hipLaunchKernelGGL(copy_dyn_kernel<uint32_t>, g, b, 0, st, pa.starts, o.starts, r_dev, 1u, cap);
        if (o.powers) hipLaunchKernelGGL(copy_dyn_kernel<uint8_t>, g, b, 0, st, ta.P, o.powers, r_dev, 1u, cap);
        if (o.node_left) hipLaunchKernelGGL(copy_dyn_kernel<uint32_t>, g, b, 0, st, ta.Lf, o.node_left, r_dev, 0u, N);
        if (o.node_right) hipLaunchKernelGGL(copy_dyn_kernel<uint32_t>, g, b, 0, st, ta.Rt, o.node_right, r_dev, 0u, N);
        if (o.leaf_depth)
            hipLaunchKernelGGL(copy_dyn_kernel<uint8_t>, g, b, 0, st, ta.leaf_depth, o.leaf_depth, r_dev, 0u, N);
        if (o.r) hipLaunchKernelGGL(copy_u32_kernel, dim3(1), dim3(64), 0, st, r_dev, o.r);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "launch");
    return PS_OK;
}

// Degenerate inputs (n_total == 0) still report merge costs of zero and a
// valid status, through the same small kernels.
static ps_status run_empty(const Call& c, const ps_options* opt, hipStream_t st) {
    const Layout L = make_layout(0, c.nseg, key_bytes(c.kt), false, c.w, false, false, c.nbuf);
    void* ws = nullptr;
    ps_status s = get_workspace(st, L.total, opt, &ws);
    if (s != PS_OK) return s;
    uint64_t* offsets = (uint64_t*)((char*)ws + L.offsets);
    uint64_t* mc = (uint64_t*)((char*)ws + L.mc);
    Counters* cnt = (Counters*)((char*)ws + L.counters);
    hipLaunchKernelGGL(offsets_kernel, dim3(1), dim3(kThreads), 0, st, c.d_offsets, (uint32_t)c.nseg, 0ull,
                       c.off_base, offsets, c.d_status);
    hipError_t e = launch_init(cnt, mc, (uint32_t)c.nseg, st);
    if (e != hipSuccess) return hip_fail(e, "init launch");
    if (c.d_costs)
        hipLaunchKernelGGL(copy_u64_kernel, dim3(1), dim3(kThreads), 0, st, mc, c.d_costs, (uint32_t)c.nseg);
    if (c.mode == Mode::Inspect && c.inspect && c.inspect->r)
        hipLaunchKernelGGL(copy_u32_kernel, dim3(1), dim3(64), 0, st, (const uint32_t*)cnt, c.inspect->r);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "launch");
    return PS_OK;
}

// A segmented call above kMaxTotal elements.  Every kernel indexes positions
// in u32, so the batch is cut at segment boundaries into consecutive chunks
// of at most kMaxTotal elements (greedily, left to right; every segment is
// below 2^31, so each chunk holds at least one), which run one after another
// on the stream in one workspace sized for the largest.  Choosing the cuts
// needs the offsets on the host: they are read back once, which
// synchronises the stream, and validated there (an invalid batch returns its
// error with nothing further enqueued).
static ps_status run_chunked(const Call& c, const ps_options* opt, hipStream_t st) {
    std::vector<uint64_t> h((size_t)c.nseg + 1);
    hipError_t e = hipMemcpyAsync(h.data(), c.d_offsets, h.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "reading the segment offsets");
    if (h[0] != 0 || h[c.nseg] != c.N)
        return fail(PS_ERR_INVALID_ARG, "segment offsets must start at 0 and end at n_total");
    for (uint64_t g = 0; g < c.nseg; ++g) {
        if (h[g + 1] < h[g]) return fail(PS_ERR_INVALID_ARG, "segment offsets decrease");
        if (h[g + 1] - h[g] > kMaxSegment) return fail(PS_ERR_TOO_LARGE, "a segment holds 2^31 or more elements");
    }
    const size_t kb = key_bytes(c.kt);
    const bool moves = (c.mode == Mode::Sort);
    const bool hp = moves && c.payload != nullptr;
    std::vector<std::pair<uint64_t, uint64_t>> chunks;  // segment ranges [g0, g1)
    size_t need = 0;
    for (uint64_t g0 = 0; g0 < c.nseg;) {
        uint64_t g1 = g0 + 1;
        while (g1 < c.nseg && h[g1 + 1] - h[g0] <= kMaxTotal) ++g1;
        chunks.emplace_back(g0, g1);
        need = std::max(need, make_layout(h[g1] - h[g0], g1 - g0, kb, hp, c.w, moves, c.peek, c.nbuf).total);
        g0 = g1;
    }
    void* ws = nullptr;
    ps_status s = get_workspace(st, need, opt, &ws);
    if (s != PS_OK) return s;
    ps_options one{};
    one.struct_size = sizeof(ps_options);
    one.workspace = ws;
    one.workspace_bytes = need;
    for (const auto& ch : chunks) {
        Call cc = c;
        const uint64_t base = h[ch.first];
        cc.keys = (char*)c.keys + base * kb;
        cc.payload = c.payload ? c.payload + base : nullptr;
        cc.d_offsets = c.d_offsets + ch.first;
        cc.nseg = ch.second - ch.first;
        cc.N = h[ch.second] - base;
        cc.off_base = base;
        cc.d_costs = c.d_costs ? c.d_costs + ch.first : nullptr;
        s = cc.N == 0 ? run_empty(cc, &one, st) : run(cc, &one, st);
        if (s != PS_OK) return s;
    }
    return PS_OK;
}

static ps_status dispatch(Call c, const ps_options* opt, void* stream) {
    g_last_error.clear();
    CallOpts o;
    ps_status s = check_common(c.kt, opt, &o);
    if (s != PS_OK) return s;
    c.w = o.w;
    c.peek = o.peek;
    c.nbuf = o.nbuf;
    if (c.nseg == 0) return fail(PS_ERR_INVALID_ARG, "num_segments must be at least 1");
    if (c.nseg >= kMaxTotal) return fail(PS_ERR_TOO_LARGE, "too many segments");
    if (!c.d_offsets && c.nseg != 1) return fail(PS_ERR_INVALID_ARG, "d_offsets is NULL");
    if (!c.d_offsets && c.N > kMaxSegment) return fail(PS_ERR_TOO_LARGE, "n must be below 2^31");
    if (c.N > kMaxBatch) return fail(PS_ERR_TOO_LARGE, "n_total must be below 2^63");
    if (c.N > kMaxTotal && c.mode == Mode::Inspect)
        return fail(PS_ERR_TOO_LARGE, "ps_inspect takes n_total below 2^31 (leaf starts are 32-bit)");
    if (c.N > 0 && !c.keys) return fail(PS_ERR_INVALID_ARG, "keys is NULL");
    hipStream_t st = (hipStream_t)stream;
    if (c.N == 0) return run_empty(c, opt, st);
    if (c.N > kMaxTotal) return run_chunked(c, opt, st);
    return run(c, opt, st);
}

// Workspace of ps_alphabetic_tree: the tree arrays for r leaves.
struct TreeLayout {
    size_t total = 0;
    size_t counters, offsets, starts, Q, P, leaf_depth, node_depth, aggF, aggB, inF, inB, mc, Lf, Rt, nsize, bsum, flag;
    uint32_t rmax, nb;
};

static TreeLayout make_tree_layout(uint64_t r) {
    TreeLayout L;
    size_t at = 0;
    L.rmax = (uint32_t)r + 1;
    const size_t r1 = (size_t)L.rmax + 1;
    const size_t nbm = (L.rmax + kMaskBlockA - 1) / kMaskBlockA + 1;
    L.nb = (uint32_t)((r + kWeightBlock - 1) / kWeightBlock);
    L.counters = take(at, kCountersBytes);
    L.offsets = take(at, 2 * 8);
    L.starts = take(at, r1 * 4);
    L.Q = take(at, r1 * 8);
    L.P = take(at, r1 + 1);
    L.leaf_depth = take(at, r1);
    L.node_depth = take(at, r1);
    L.aggF = take(at, nbm * 16);
    L.aggB = take(at, nbm * 16);
    L.inF = take(at, nbm * 8);
    L.inB = take(at, nbm * 8);
    L.mc = take(at, 2 * 8);
    L.Lf = take(at, r1 * 4);
    L.Rt = take(at, r1 * 4);
    L.nsize = take(at, r1 * 4);
    L.bsum = take(at, ((size_t)L.nb + 1) * 8);
    L.flag = take(at, 4);
    L.total = take(at, 0) + 256;
    return L;
}

__global__ void zero_u32_kernel(uint32_t* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

static ps_status alphabetic_tree(const uint32_t* w, uint64_t r, uint8_t* powers, uint32_t* left, uint32_t* right,
                                 uint8_t* depth, uint64_t* cost, int32_t* status, hipStream_t st) {
    const TreeLayout L = make_tree_layout(r);
    void* ws = nullptr;
    ps_status s = get_workspace(st, L.total, nullptr, &ws);
    if (s != PS_OK) return s;
    char* base = (char*)ws;
    auto at = [&](size_t off) { return (void*)(base + off); };
    Counters* cnt = (Counters*)at(L.counters);
    uint64_t* mc = (uint64_t*)at(L.mc);
    uint64_t* offsets = (uint64_t*)at(L.offsets);
    uint32_t* starts = (uint32_t*)at(L.starts);
    uint64_t* bsum = (uint64_t*)at(L.bsum);
    uint32_t* flag = (uint32_t*)at(L.flag);
    const uint32_t r32 = (uint32_t)r;
    hipError_t e = launch_init(cnt, mc, 1, st);
    if (e != hipSuccess) return hip_fail(e, "init launch");
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, st, flag);
    hipLaunchKernelGGL(weight_sum_kernel, dim3(L.nb), dim3(kThreads), 0, st, w, r32, bsum, flag);
    hipLaunchKernelGGL(weight_scan_kernel, dim3(1), dim3(kThreads), 0, st, bsum, L.nb, r32, flag, cnt, offsets,
                       starts);
    hipLaunchKernelGGL(weight_starts_kernel, dim3(L.nb), dim3(kThreads), 0, st, w, r32, bsum, flag, starts, status);
    TreeArgs ta{};
    ta.offsets = offsets;
    ta.nseg = 1;
    ta.rmax = L.rmax;
    ta.starts = starts;
    ta.cnt = cnt;
    ta.Q = (uint64_t*)at(L.Q);
    ta.P = (uint8_t*)at(L.P);
    ta.leaf_depth = (uint8_t*)at(L.leaf_depth);
    ta.node_depth = (uint8_t*)at(L.node_depth);
    ta.aggF = (Mask2*)at(L.aggF);
    ta.aggB = (Mask2*)at(L.aggB);
    ta.inF = (uint64_t*)at(L.inF);
    ta.inB = (uint64_t*)at(L.inB);
    ta.mc = mc;
    ta.Lf = (uint32_t*)at(L.Lf);
    ta.Rt = (uint32_t*)at(L.Rt);
    ta.nsize = (uint32_t*)at(L.nsize);
    e = launch_tree_cost(ta, st);
    if (e == hipSuccess && (left || right)) e = launch_node_ranges(ta, st);
    if (e != hipSuccess) return hip_fail(e, "tree launch");
    const uint32_t* r_dev = (const uint32_t*)cnt;
    const dim3 g(1024), b(kThreads);
    if (powers) hipLaunchKernelGGL(copy_dyn_kernel<uint8_t>, g, b, 0, st, ta.P, powers, r_dev, 1u, r32 + 1);
    if (left) hipLaunchKernelGGL(copy_dyn_kernel<uint32_t>, g, b, 0, st, ta.Lf, left, r_dev, 0u, r32);
    if (right) hipLaunchKernelGGL(copy_dyn_kernel<uint32_t>, g, b, 0, st, ta.Rt, right, r_dev, 0u, r32);
    if (depth) hipLaunchKernelGGL(copy_dyn_kernel<uint8_t>, g, b, 0, st, ta.leaf_depth, depth, r_dev, 0u, r32);
    if (cost) hipLaunchKernelGGL(copy_u64_kernel, dim3(1), dim3(64), 0, st, mc, cost, 1u);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "copy launch");
    return PS_OK;
}

}  // namespace ps

using namespace ps;

// A C caller may pass any int as a ps_key_type: read the argument's bytes as
// an int (a value outside the enumerators is not a valid value of the enum
// in C++); check_common then rejects unknown types.
static inline int key_int(const ps_key_type* t) {
    int v;
    memcpy(&v, t, sizeof v);
    return v;
}

extern "C" {

size_t ps_workspace_bytes(uint64_t n_total, uint64_t num_segments, ps_key_type key_type, int has_payload,
                          const ps_options* opt) {
    CallOpts o;
    if (check_common(key_int(&key_type), opt, &o) != PS_OK) return 0;
    if (n_total > kMaxBatch || num_segments == 0 || num_segments >= kMaxTotal) return 0;
    if (num_segments == 1 && n_total > kMaxSegment) return 0;
    // above kMaxTotal the batch runs in chunks of at most kMaxTotal elements
    // (ps_segmented_sort), each needing no more than this
    return make_layout(std::min(n_total, kMaxTotal), num_segments, key_bytes(key_int(&key_type)), has_payload != 0, o.w,
                       true, o.peek, o.nbuf)
        .total;
}

ps_status ps_alphabetic_tree(const uint32_t* d_weights, uint64_t num_leaves, uint8_t* d_powers,
                             uint32_t* d_node_left, uint32_t* d_node_right, uint8_t* d_leaf_depth, uint64_t* d_cost,
                             int32_t* d_status, void* stream) {
    g_last_error.clear();
    if (num_leaves == 0) return fail(PS_ERR_INVALID_ARG, "num_leaves must be at least 1");
    if (num_leaves > kMaxTreeLeaves) return fail(PS_ERR_TOO_LARGE, "num_leaves above 2^28");
    if (!d_weights) return fail(PS_ERR_INVALID_ARG, "d_weights is NULL");
    return alphabetic_tree(d_weights, num_leaves, d_powers, d_node_left, d_node_right, d_leaf_depth, d_cost, d_status,
                           (hipStream_t)stream);
}

ps_status ps_sort(void* keys, uint32_t* payload, uint64_t n, ps_key_type key_type, const ps_options* opt,
                  uint64_t* d_merge_cost, void* stream) {
    Call c{keys, payload, nullptr, 1, n, key_int(&key_type), 0, d_merge_cost, nullptr, nullptr, Mode::Sort};
    return dispatch(c, opt, stream);
}

ps_status ps_sort_no_alloc(void* keys, uint32_t* payload, uint64_t n, ps_key_type key_type, const ps_options* opt,
                           uint64_t* d_merge_cost, void* stream) {
    g_last_error.clear();
    CallOpts o;
    ps_status s = check_common(key_int(&key_type), opt, &o);
    if (s != PS_OK) return s;
    if (opt && opt->workspace)
        return fail(PS_ERR_INVALID_ARG, "ps_sort_no_alloc runs in the library's fixed scratch: "
                                        "ps_options.workspace must be NULL");
    if (n > kMaxSegment) return fail(PS_ERR_TOO_LARGE, "n must be below 2^31");
    if (n > 0 && !keys) return fail(PS_ERR_INVALID_ARG, "keys is NULL");
    const size_t need =
        make_layout(n, 1, key_bytes(key_int(&key_type)), payload != nullptr, o.w, true, o.peek, o.nbuf).total;
    if (need > kFixedScratchBytes)
        return fail(PS_ERR_TOO_LARGE, "this sort needs " + std::to_string(need) +
                                          " bytes of scratch; the fixed scratch holds " +
                                          std::to_string(kFixedScratchBytes));
    void* ptr = nullptr;
    s = fixed_scratch(&ptr);
    if (s != PS_OK) return s;
    ps_options fixed = opt ? *opt : ps_options{};
    fixed.struct_size = sizeof(ps_options);
    fixed.workspace = ptr;
    fixed.workspace_bytes = kFixedScratchBytes;
    Call c{keys, payload, nullptr, 1, n, key_int(&key_type), 0, d_merge_cost, nullptr, nullptr, Mode::Sort};
    c.prof = false;
    return dispatch(c, &fixed, stream);
}

ps_status ps_segmented_sort(void* keys, uint32_t* payload, const uint64_t* d_offsets, uint64_t num_segments,
                            uint64_t n_total, ps_key_type key_type, const ps_options* opt, uint64_t* d_merge_costs,
                            int32_t* d_status, void* stream) {
    if (!d_offsets) return fail(PS_ERR_INVALID_ARG, "d_offsets is NULL");
    Call c{keys, payload, d_offsets, num_segments, n_total, key_int(&key_type), 0, d_merge_costs, d_status, nullptr,
           Mode::Sort};
    return dispatch(c, opt, stream);
}

ps_status ps_merge_cost(const void* keys, uint64_t n, ps_key_type key_type, const ps_options* opt,
                        uint64_t* d_merge_cost, void* stream) {
    if (!d_merge_cost) return fail(PS_ERR_INVALID_ARG, "d_merge_cost is NULL");
    Call c{(void*)keys, nullptr, nullptr, 1, n, key_int(&key_type), 0, d_merge_cost, nullptr, nullptr, Mode::Cost};
    return dispatch(c, opt, stream);
}

ps_status ps_segmented_merge_cost(const void* keys, const uint64_t* d_offsets, uint64_t num_segments,
                                  uint64_t n_total, ps_key_type key_type, const ps_options* opt,
                                  uint64_t* d_merge_costs, int32_t* d_status, void* stream) {
    if (!d_offsets) return fail(PS_ERR_INVALID_ARG, "d_offsets is NULL");
    if (!d_merge_costs) return fail(PS_ERR_INVALID_ARG, "d_merge_costs is NULL");
    Call c{(void*)keys, nullptr, d_offsets, num_segments, n_total, key_int(&key_type), 0, d_merge_costs, d_status,
           nullptr, Mode::Cost};
    return dispatch(c, opt, stream);
}

ps_status ps_inspect(const void* keys, const uint64_t* d_offsets, uint64_t num_segments, uint64_t n_total,
                     ps_key_type key_type, const ps_options* opt, ps_inspect_out* out, void* stream) {
    if (!out) return fail(PS_ERR_INVALID_ARG, "out is NULL");
    Call c{(void*)keys, nullptr, d_offsets, num_segments, n_total, key_int(&key_type), 0, nullptr, nullptr, out,
           Mode::Inspect};
    return dispatch(c, opt, stream);
}

ps_status ps_set_tuning(const ps_tuning* t) {
    g_last_error.clear();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!t) {
        g_tune = Tuning{};
        return PS_OK;
    }
    if (t->struct_size != sizeof(ps_tuning)) return fail(PS_ERR_INVALID_ARG, "ps_tuning.struct_size mismatch");
    if (t->merge_tile && t->merge_tile != 2048 && t->merge_tile != 4096 && t->merge_tile != 8192)
        return fail(PS_ERR_INVALID_ARG, "merge_tile must be 2048, 4096 or 8192");
    if (t->merge_levels > 2) return fail(PS_ERR_INVALID_ARG, "merge_levels must be 1 or 2");
    const uint32_t grids[4] = {t->grid_big_leaf, t->grid_fused, t->grid_merge, t->grid_split};
    for (uint32_t g : grids)
        if (g > 65536) return fail(PS_ERR_UNSUPPORTED, "grid above 65536");
    Tuning n = g_tune;
    if (t->grid_big_leaf) n.grid_big_leaf = t->grid_big_leaf;
    if (t->grid_fused) n.grid_fused = t->grid_fused;
    if (t->grid_merge) n.grid_merge = t->grid_merge;
    if (t->grid_split) n.grid_split = t->grid_split;
    if (t->merge_tile) n.merge_tile = t->merge_tile;
    if (t->merge_levels) n.merge_levels = t->merge_levels;
    g_tune = n;
    return PS_OK;
}

ps_status ps_get_tuning(ps_tuning* out) {
    g_last_error.clear();
    if (!out || out->struct_size != sizeof(ps_tuning)) return fail(PS_ERR_INVALID_ARG, "bad ps_tuning");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    out->grid_big_leaf = g_tune.grid_big_leaf;
    out->grid_fused = g_tune.grid_fused;
    out->grid_merge = g_tune.grid_merge;
    out->grid_split = g_tune.grid_split;
    out->merge_tile = g_tune.merge_tile;
    out->merge_levels = g_tune.merge_levels;
    return PS_OK;
}

ps_status ps_profile_enable(int on) {
    g_last_error.clear();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (on && !g_prof.dev) {
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, sizeof(unsigned long long) * PS_PROF_GROUPS);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc");
        e = hipMemset(p, 0, sizeof(unsigned long long) * PS_PROF_GROUPS);
        if (e != hipSuccess) return hip_fail(e, "hipMemset");
        g_prof.dev = (unsigned long long*)p;
    }
    g_prof.on = on != 0;
    g_prof.mask = (on == 1) ? ((1u << PS_PROF_GROUPS) - 1) : (uint32_t)on;
    return PS_OK;
}

ps_status ps_profile_read(ps_profile* out, int reset) {
    g_last_error.clear();
    if (!out || out->struct_size != sizeof(ps_profile)) return fail(PS_ERR_INVALID_ARG, "bad ps_profile");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    ps_profile& T = g_prof.totals;
    for (const ProfPending& p : g_prof.pending) {
        hipError_t e = hipEventSynchronize(p.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, p.a, p.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        T.ms[p.group] += ms;
        T.launches[p.group] += p.launches;
        T.elems[p.group] += p.host_elems;
        g_prof.pool.push_back(p.a);
        g_prof.pool.push_back(p.b);
    }
    g_prof.pending.clear();
    unsigned long long dev[PS_PROF_GROUPS] = {0};
    if (g_prof.dev) {
        hipError_t e = hipMemcpy(dev, g_prof.dev, sizeof dev, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    }
    const uint32_t size = out->struct_size;
    *out = T;
    out->struct_size = size;
    for (int g = 0; g < PS_PROF_GROUPS; ++g) out->elems[g] += dev[g];
    if (reset) {
        g_prof.totals = ps_profile{};
        if (g_prof.dev) {
            hipError_t e = hipMemset(g_prof.dev, 0, sizeof dev);
            if (e != hipSuccess) return hip_fail(e, "hipMemset");
        }
    }
    return PS_OK;
}

ps_status ps_set_pool_limit(uint64_t bytes) {
    g_last_error.clear();
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_pool_limit = bytes;
    return PS_OK;
}

ps_status ps_release(void* stream) {
    g_last_error.clear();
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_pool.find(stream);
    if (it == g_pool.end()) return PS_OK;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (it->second.ptr) {
        e = hipFree(it->second.ptr);
        if (e != hipSuccess) return hip_fail(e, "hipFree");
    }
    g_pool.erase(it);
    return PS_OK;
}

const char* ps_status_string(ps_status status) {
    // A C caller may pass any int: read the argument's bytes as an int, not
    // as the enum (a value outside the enumerators is not a valid enum value
    // in C++).
    int code;
    memcpy(&code, &status, sizeof code);
    switch (code) {
    case PS_OK: return "PS_OK";
    case PS_ERR_INVALID_ARG: return "PS_ERR_INVALID_ARG: invalid argument";
    case PS_ERR_TOO_LARGE: return "PS_ERR_TOO_LARGE: input exceeds the supported size";
    case PS_ERR_OUT_OF_MEMORY: return "PS_ERR_OUT_OF_MEMORY: scratch allocation failed";
    case PS_ERR_HIP: return "PS_ERR_HIP: HIP runtime error";
    case PS_ERR_UNSUPPORTED: return "PS_ERR_UNSUPPORTED: unsupported option";
    }
    return "unknown ps_status";
}

const char* ps_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
