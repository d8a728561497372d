// Data movement: forming the leaves and the stable merges of the merge tree.
//
// Arrays: 0 is the caller's, 1 and 2 the library's scratch (2 only when the
// call has room for it).  Every tree vertex keeps its sorted result in the
// array node_buf / big_leaf_buf assign to it; a node reads its children from
// their arrays and writes its own, never one of theirs, and the root
// (depth 0) ends in the caller's array.
//
//  * big_leaf: a leaf longer than the fused-subtree capacity is a natural run
//    (only shorter leaves are min-run extended); a strictly decreasing one is
//    reversed (Sec. 2 run convention), in place or while it is copied to
//    the array its depth assigns.
//  * fused: every maximal subtree of at most kFuse elements is loaded once
//    from the caller's array, its leaves are stably sorted in LDS (the
//    reversal / insertion-sort extension of App. B.3-B.4 has the unique stable
//    result), and its internal merges are done level by level inside LDS.
//  * merge_pass: all nodes of one power p that are larger than kFuse, as one
//    flattened space of merge-path tiles.  Nodes of equal power are disjoint
//    and their children have larger powers (Lemma "Path power
//    monotonicity"), so passes p = pmax..1 respect every dependency.
// Every merge is stable: on equal keys the left run goes first (App. B.1).
#include <hip/hip_ext.h>

#include "common.hpp"
#include "block.hpp"
#include "internal.hpp"

namespace ps {


// Data array b (0, 1, 2) of a MoveArgs pointer triple.
template <class T>
__device__ __forceinline__ T* pick3(T* const (&v)[3], uint32_t b) {
    return b == 0 ? v[0] : (b == 1 ? v[1] : v[2]);
}
// The same for a b that is equal across the wave (kept in a scalar register).
template <class T>
__device__ __forceinline__ T* pick3u(T* const (&v)[3], uint32_t b) {
    return pick3(v, (uint32_t)__builtin_amdgcn_readfirstlane(b));
}

__device__ __forceinline__ uint32_t upper_bound_u32(const uint32_t* __restrict__ a, uint32_t n, uint32_t v) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t m = (lo + hi) >> 1;
        if (a[m] <= v) lo = m + 1; else hi = m;
    }
    return lo;
}

// The sample array (4-byte keys; null otherwise) keeps the order key of
// every position divisible by kSampleSpacing: each kernel that changes the
// data at a position also updates its entry.
template <class U>
__device__ __forceinline__ void put_sample(uint32_t* samp, uint32_t pos, U key) {
    if constexpr (sizeof(U) == 4) {
        if (samp && (pos & (kSampleSpacing - 1)) == 0) samp[pos / kSampleSpacing] = (uint32_t)key;
    }
}

// Padded LDS index: one pad word after every eight, so that a thread
// handling eight consecutive elements (lane L at 8 L + i) hits a different
// bank from every other lane (9 L + i).
__device__ __forceinline__ uint32_t lpad(uint32_t x) { return x + (x >> 3); }

// ------------------------------------------------------------ big leaves

template <int KT, bool HP>
__global__ __launch_bounds__(kThreads) void big_leaf_kernel(MoveArgs a) {
    using raw = typename Key<KT>::raw;
    constexpr int kB = 16;  // elements per thread in flight
    const uint32_t ntiles = a.cnt->ptiles[0];
    const uint32_t nleaf = a.cnt->nbigleaf;
    raw* k0 = (raw*)a.keys[0];
    raw* k1 = (raw*)pick3u(a.keys, a.leaf_copy);
    uint32_t* p1 = pick3u(a.pay, a.leaf_copy);
    if (nleaf == 0) return;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t k = upper_bound_u32(a.leaf_tile, nleaf, t) - 1;
        const uint32_t i = a.bigleaf[k];
        const uint8_t mode = a.bigleaf_mode[k];
        const uint32_t s = a.starts[i], L = a.starts[i + 1] - s;
        const uint32_t x0 = (t - a.leaf_tile[k]) * kLeafTile;
        if (mode == kLeafRevInPlace) {
            const uint32_t x1 = min(L / 2, x0 + kLeafTile);
            for (uint32_t xb = x0; xb < x1; xb += kB * kThreads) {
                raw kx[kB], ky[kB];
                uint32_t px[kB], py[kB];
#pragma unroll
                for (int j = 0; j < kB; ++j) {
                    const uint32_t x = xb + j * kThreads + threadIdx.x;
                    if (x < x1) {
                        kx[j] = k0[s + x];
                        ky[j] = k0[s + L - 1 - x];
                        if (HP) {
                            px[j] = a.pay[0][s + x];
                            py[j] = a.pay[0][s + L - 1 - x];
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < kB; ++j) {
                    const uint32_t x = xb + j * kThreads + threadIdx.x;
                    if (x < x1) {
                        k0[s + x] = ky[j];
                        k0[s + L - 1 - x] = kx[j];
                        put_sample(a.samp, s + x, Key<KT>::ord(ky[j]));
                        put_sample(a.samp, s + L - 1 - x, Key<KT>::ord(kx[j]));
                        if (HP) {
                            a.pay[0][s + x] = py[j];
                            a.pay[0][s + L - 1 - x] = px[j];
                        }
                    }
                }
            }
        } else {
            const uint32_t x1 = min(L, x0 + kLeafTile);
            const bool rev = (mode == kLeafRevCopy);
            for (uint32_t xb = x0; xb < x1; xb += kB * kThreads) {
                raw kv[kB];
                uint32_t pv[kB];
#pragma unroll
                for (int j = 0; j < kB; ++j) {
                    const uint32_t x = xb + j * kThreads + threadIdx.x;
                    if (x < x1) {
                        kv[j] = k0[s + x];
                        if (HP) pv[j] = a.pay[0][s + x];
                    }
                }
#pragma unroll
                for (int j = 0; j < kB; ++j) {
                    const uint32_t x = xb + j * kThreads + threadIdx.x;
                    if (x < x1) {
                        const uint32_t y = rev ? (L - 1 - x) : x;
                        k1[s + y] = kv[j];
                        if (rev) put_sample(a.samp, s + y, Key<KT>::ord(kv[j]));
                        if (HP) p1[s + y] = pv[j];
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------- fused subtrees

// Stable LSD radix sort of the n <= kFuse order keys sk[0..n) (payload sp
// alongside) held in LDS, 8 bits per pass, ping-ponging with tk/tp; passes
// whose digit is the same for every key are skipped.  Wave w ranks the
// elements [512 w, 512 w + 512) of the current order, slot q of lane L being
// element 512 w + 64 q + L: lanes holding the same digit find each other with
// eight ballots, and a per-wave counter per digit carries the count from one
// slot to the next, so ranks follow the current order (stability).  The
// per-wave counts then become destinations by a scan over (digit, wave).
// hist: kFuseWaves x 256 counters, rank: kFuse entries.  Returns true if the
// result ended in tk/tp.  Block-uniform; all threads call.
template <class U, bool HP>
__device__ __forceinline__ bool block_radix_sort(U* sk, uint32_t* sp, U* tk, uint32_t* tp, uint32_t n,
                                                 uint16_t* hist, uint16_t* rank, uint32_t* sh,
                                                 unsigned long long* red) {
    constexpr int BITS = 8 * sizeof(U);
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
    // bits in which some key differs from the first one
    U diff = 0;
    {
        const U k0 = sk[0];
        for (uint32_t x = tid; x < n; x += kFuseThreads) diff |= sk[x] ^ k0;
        unsigned long long v = (unsigned long long)diff;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v |= __shfl_xor(v, o);
        if (tid == 0) *red = 0;
        __syncthreads();
        if (lane == 0 && v) atomicOr(red, v);
        __syncthreads();
        diff = (U)*red;
        __syncthreads();
    }
    bool alt = false;
    uint16_t* hw = hist + w * 256;
    for (int s = 0; s < BITS; s += 8) {
        if (((diff >> s) & (U)0xFF) == 0) continue;  // every key has the same digit
        for (uint32_t i = lane; i < 256; i += 64) hw[i] = 0;
        __builtin_amdgcn_wave_barrier();
#pragma unroll 1
        for (int q = 0; q < kFuseItems; ++q) {
            const uint32_t x = w * 512 + q * 64 + lane;
            const bool valid = x < n;
            const uint32_t d = valid ? (uint32_t)((sk[x] >> s) & (U)0xFF) : 0u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const uint64_t bb = __ballot((d >> b) & 1u);
                peers &= ((d >> b) & 1u) ? bb : ~bb;
            }
            const uint32_t before = (uint32_t)__popcll(peers & lt);
            const uint32_t base = valid ? hw[d] : 0u;
            __builtin_amdgcn_wave_barrier();
            if (valid && before == 0) hw[d] = (uint16_t)(base + (uint32_t)__popcll(peers));
            __builtin_amdgcn_wave_barrier();
            if (valid) rank[x] = (uint16_t)(base + before);
        }
        __syncthreads();
        // hist[w][d] := elements before (digit d, wave w) in the pass's order
        uint32_t tot = 0;
        if (tid < 256) {
            for (int v = 0; v < kFuseWaves; ++v) {
                const uint32_t c = hist[v * 256 + tid];
                hist[v * 256 + tid] = (uint16_t)tot;
                tot += c;
            }
        }
        const uint32_t dbase = block_excl_sum_w<kFuseWaves>(tid < 256 ? tot : 0u, sh, nullptr);
        if (tid < 256) {
            for (int v = 0; v < kFuseWaves; ++v) hist[v * 256 + tid] = (uint16_t)(hist[v * 256 + tid] + dbase);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kFuseItems; ++q) {
            const uint32_t x = w * 512 + q * 64 + lane;
            if (x < n) {
                const U key = sk[x];
                const uint32_t dst = hw[(uint32_t)((key >> s) & (U)0xFF)] + rank[x];
                tk[dst] = key;
                if (HP) tp[dst] = sp[x];
            }
        }
        __syncthreads();
        U* t1 = sk;
        sk = tk;
        tk = t1;
        uint32_t* t2 = sp;
        sp = tp;
        tp = t2;
        alt = !alt;
    }
    return alt;
}

// LDS of fused_radix_kernel: keys and payloads twice, the per-wave digit
// counters, the ranks, and a 128-byte header (wave totals, a reduction word).
__host__ __device__ constexpr uint32_t radix_lds_bytes(uint32_t key_bytes, bool hp) {
    return 128 + 2 * kFuse * (key_bytes + (hp ? 4u : 0u)) + kFuseWaves * 256 * 2 + kFuse * 2;
}

// Fused subtrees with many leaves: every merge in a subtree is
// stable and takes the left run first, so its result is the stable sort of
// its original elements, which the block radix sort computes in a fixed
// number of passes instead of one pass per tree level.
template <int KT, bool HP>
__global__ __launch_bounds__(kFuseThreads) void fused_radix_kernel(MoveArgs a) {
    using K = Key<KT>;
    using U = typename K::ukey;
    using raw = typename K::raw;
    extern __shared__ __align__(16) unsigned char rsm[];
    uint32_t* sh = reinterpret_cast<uint32_t*>(rsm);
    unsigned long long* red = reinterpret_cast<unsigned long long*>(rsm + 64);
    U* sk = reinterpret_cast<U*>(rsm + 128);
    U* tk = sk + kFuse;
    uint32_t* sp = reinterpret_cast<uint32_t*>(tk + kFuse);
    uint32_t* tp = sp + (HP ? kFuse : 0);
    uint16_t* hist = reinterpret_cast<uint16_t*>(tp + (HP ? kFuse : 0));
    uint16_t* rank = hist + kFuseWaves * 256;
    const uint32_t nunits = a.cnt->nunit[kUnitRadix];
    const uint32_t tid = threadIdx.x;
    for (uint32_t v = blockIdx.x; v < nunits; v += gridDim.x) {
        const uint32_t u = a.unit_base[kUnitRadix] + v;
        const UnitRec ur = a.unit_rec[u];
        const uint32_t nleaves = ur.ub - ur.ua;
        const uint32_t lo = ur.lo, n = ur.hi - ur.lo;
        if (n > (uint32_t)kFuse || n == 0 || !fuse_by_radix(sizeof(U), nleaves)) continue;
        const raw* src = (const raw*)a.keys[0];
        raw* dst = (raw*)pick3u(a.keys, a.unit_par[u]);
        uint32_t* pdst = pick3u(a.pay, a.unit_par[u]);
        {
            raw kv[kFuseItems];
            uint32_t pv[kFuseItems];
#pragma unroll
            for (int i = 0; i < kFuseItems; ++i) {
                const uint32_t x = tid + i * kFuseThreads;
                if (x < n) {
                    kv[i] = src[lo + x];
                    if (HP) pv[i] = a.pay[0][lo + x];
                }
            }
#pragma unroll
            for (int i = 0; i < kFuseItems; ++i) {
                const uint32_t x = tid + i * kFuseThreads;
                if (x < n) {
                    sk[x] = K::ord(kv[i]);
                    if (HP) sp[x] = pv[i];
                }
            }
        }
        __syncthreads();
        const bool alt = block_radix_sort<U, HP>(sk, sp, tk, tp, n, hist, rank, sh, red);
        const U* ok = alt ? tk : sk;
        const uint32_t* op = alt ? tp : sp;
#pragma unroll
        for (int i = 0; i < kFuseItems; ++i) {
            const uint32_t x = tid + i * kFuseThreads;
            if (x < n) {
                dst[lo + x] = K::unord(ok[x]);
                if (HP) pdst[lo + x] = op[x];
                put_sample(a.samp, lo + x, ok[x]);
            }
        }
        __syncthreads();
    }
}

// A fused unit that is a single natural run (longer than any min-run
// extension): copied to its array, reversed if strictly decreasing, without
// LDS.  Every element is loaded before any is stored, since a run that is a
// whole segment is written in place.  Small blocks (256 threads x 16
// elements) keep more units in flight per CU; whether the run decreases comes
// from its first two elements as loaded (a flag per parity of the round, so
// that one barrier a unit suffices).
constexpr int kCopyThreads = 256;
constexpr int kCopyItems = kFuse / kCopyThreads;
template <int KT, bool HP>
__global__ __launch_bounds__(kCopyThreads) __attribute__((amdgpu_waves_per_eu(sizeof(typename Key<KT>::raw) == 4 ? 8 : 4))) void unit_copy_kernel(MoveArgs a) {
    using K = Key<KT>;
    using raw = typename K::raw;
    __shared__ uint32_t desc_sh[2];
    const uint32_t nunits = a.cnt->nunit[kUnitCopy];
    const uint32_t tid = threadIdx.x;
    const raw* src = (const raw*)a.keys[0];
    uint32_t round = 0;
    for (uint32_t v = blockIdx.x; v < nunits; v += gridDim.x, ++round) {
        const uint32_t u = a.unit_base[kUnitCopy] + v;
        const UnitRec ur = a.unit_rec[u];
        const uint32_t lo = ur.lo, n = ur.hi - ur.lo;
        if (ur.ub - ur.ua != 1 || n <= (uint32_t)kMaxMinRun || n > (uint32_t)kFuse) continue;
        raw* dst = (raw*)pick3u(a.keys, a.unit_par[u]);
        uint32_t* pdst = pick3u(a.pay, a.unit_par[u]);
        const bool in_place = (const void*)dst == (const void*)src;
        raw kv[kCopyItems];
        uint32_t pv[kCopyItems];
#pragma unroll
        for (int i = 0; i < kCopyItems; ++i) {
            const uint32_t x = tid + i * kCopyThreads;
            if (x < n) {
                kv[i] = src[lo + x];
                if (HP) pv[i] = a.pay[0][lo + x];
            }
        }
        if (tid < 64) {
            const raw k1 = __shfl(kv[0], 1);  // n > kMaxMinRun: elements 0 and 1 exist
            if (tid == 0) desc_sh[round & 1] = K::ord(k1) < K::ord(kv[0]) ? 1u : 0u;
        }
        // A run reversed in place: each wave's loads are complete before it
        // reaches the barrier, so no wave's stores can overtake another's
        // loads (the barrier alone does not wait for loads in flight).
        if (in_place) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        const bool desc = desc_sh[round & 1] != 0;
        if (desc || !in_place) {
#pragma unroll
            for (int i = 0; i < kCopyItems; ++i) {
                const uint32_t x = tid + i * kCopyThreads;
                if (x < n) {
                    const uint32_t y = desc ? n - 1 - x : x;
                    dst[lo + y] = kv[i];
                    if (HP) pdst[lo + y] = pv[i];
                    if (desc) put_sample(a.samp, lo + y, K::ord(kv[i]));
                }
            }
        }
    }
}

constexpr int kFusedNT = 1024;  // threads of fused_kernel (kFuse / kFusedNT outputs each)

// Fused subtrees of fewer than kFuseRadixMinLeaves leaves (so at most six
// merges), and single leaves of at most kMaxMinRun elements: one block per
// subtree, its data in LDS.  Leaves are formed first (R1), then the merges
// run level by level, one level per distinct node power, deepest first
// (nodes of one power are disjoint, and children have larger powers).
// Every thread produces the 8 consecutive outputs x0 .. x0 + 7 of a level:
// each node of that power covering some of them contributes a merge-path
// co-rank and up to 8 merge steps, the rest are copied.  The node table is
// block-uniform and small (read from LDS by every lane), so a level costs two
// barriers.  LDS indices are padded (lpad), so that lanes reading their
// 8-apart outputs hit different banks.
template <int KT, bool HP>
__global__ __launch_bounds__(kFusedNT) __attribute__((amdgpu_waves_per_eu(8))) void fused_kernel(MoveArgs a) {
    constexpr int NT = kFusedNT, IT = kFuse / kFusedNT;
    using K = Key<KT>;
    using U = typename K::ukey;
    using raw = typename K::raw;
    constexpr uint32_t KL = kFuseRadixMinLeaves;  // leaves per subtree stay below this
    constexpr uint32_t KN = KL - 2;               // merges per subtree: at most KL - 2
    constexpr uint32_t PADDED = kFuse + kFuse / 8;
    __shared__ U sk[PADDED];
    __shared__ uint32_t sp[HP ? PADDED : 1];
    __shared__ uint32_t lst[KL + 1];
    __shared__ uint32_t snode[KN][3];  // per merge: first leaf, end leaf, power
    const uint32_t nunits = a.cnt->nunit[kUnitFew];
    const uint32_t tid = threadIdx.x;
    const raw* src = (const raw*)a.keys[0];
    auto uni = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane(v); };
    for (uint32_t v = blockIdx.x; v < nunits; v += gridDim.x) {
        const uint32_t u = a.unit_base[kUnitFew] + v;
        const UnitRec ur = a.unit_rec[u];
        const uint32_t ua = uni(ur.ua), nl = uni(ur.ub - ur.ua);
        const uint32_t lo = uni(ur.lo), n = uni(ur.hi - ur.lo);
        if (n > (uint32_t)kFuse || nl == 0 || fuse_by_radix(sizeof(U), nl)) continue;
        if (nl == 1 && n > (uint32_t)kMaxMinRun) continue;  // unit_copy_kernel's unit
        const uint32_t nn = nl - 1;
        raw* dst = (raw*)pick3u(a.keys, a.unit_par[u]);
        uint32_t* pdst = pick3u(a.pay, a.unit_par[u]);
        U kr[IT];
        uint32_t pr[IT];
        {
            raw kv[IT];
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const uint32_t x = tid + i * NT;
                if (x < n) {
                    kv[i] = src[lo + x];
                    if (HP) pr[i] = a.pay[0][lo + x];
                }
            }
            const uint32_t st = tid <= nl ? a.starts[ua + tid] - lo : 0u;
            uint32_t nf = 0, ne = 0, np = 0;
            if (tid < nn) {
                const uint32_t j = ua + 1 + tid;
                np = a.P[j];
                nf = a.Lf[j] - ua;
                ne = a.Rt[j] - ua;
            }
            __syncthreads();  // the previous subtree's last reads are done
            if (tid <= nl) lst[tid] = st;
            if (tid < nn) {
                snode[tid][0] = nf;
                snode[tid][1] = ne;
                snode[tid][2] = np;
            }
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const uint32_t x = tid + i * NT;
                if (x < n) {
                    sk[lpad(x)] = K::ord(kv[i]);
                    if (HP) sp[lpad(x)] = pr[i];
                }
            }
        }
        __syncthreads();
        // Powers present among the merges.
        unsigned long long pm = 0;
        for (uint32_t m = 0; m < nn; ++m) pm |= 1ull << uni(snode[m][2]);

        // Leaf formation: each leaf is stably sorted in place.
        const uint32_t x0 = tid * IT;
        uint16_t np[IT];
        bool moved = false;
        {
            uint32_t l = 0;
            while (l + 1 < nl && lst[l + 1] <= x0) ++l;
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const uint32_t x = x0 + i;
                np[i] = (uint16_t)x;
                if (x < n) {
                    while (lst[l + 1] <= x) ++l;
                    const uint32_t ls = lst[l], le = lst[l + 1];
                    const U key = sk[lpad(x)];
                    uint32_t dpos;
                    if (le - ls <= (uint32_t)kMaxMinRun) {
                        uint32_t rank = 0;
#pragma unroll 1
                        for (uint32_t y = ls; y < le; ++y) {
                            const U o = sk[lpad(y)];
                            rank += (o < key) || (o == key && y < x);
                        }
                        dpos = ls + rank;
                    } else {
                        // longer than any min-run extension: a natural run
                        const bool desc = sk[lpad(ls + 1)] < sk[lpad(ls)];
                        dpos = desc ? (ls + le - 1 - x) : x;
                    }
                    kr[i] = key;
                    if (HP) pr[i] = sp[lpad(x)];
                    np[i] = (uint16_t)dpos;
                    moved |= (dpos != x);
                }
            }
        }
        if (__syncthreads_or(moved)) {
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                if (x0 + i < n) {
                    sk[lpad(np[i])] = kr[i];
                    if (HP) sp[lpad(np[i])] = pr[i];
                }
            }
            __syncthreads();
        }

        // Merges, deepest power first.
        while (pm) {
            const uint32_t p = 63 - __clzll(pm);
            pm &= ~(1ull << p);
#pragma unroll
            for (int i = 0; i < IT; ++i) np[i] = (uint16_t)(x0 + i);  // copied unless merged
#pragma unroll 1
            for (uint32_t m = 0; m < nn; ++m) {
                if (uni(snode[m][2]) != p) continue;
                // merge [nlo, nmid) with [nmid, nhi)
                const uint32_t nlo = uni(lst[snode[m][0]]), nmid = uni(lst[m + 1]), nhi = uni(lst[snode[m][1]]);
                if (nlo < x0 + IT && x0 < nhi) {
                    const uint32_t s0 = max(x0, nlo);
                    // merge-path co-rank of diagonal s0 - nlo (ties to the left run)
                    const uint32_t d = s0 - nlo, la = nmid - nlo, lb = nhi - nmid;
                    uint32_t l = d > lb ? d - lb : 0, h = min(d, la);
                    while (l < h) {
                        const uint32_t mm = (l + h) >> 1;
                        if (sk[lpad(nlo + mm)] <= sk[lpad(nmid + d - 1 - mm)]) l = mm + 1; else h = mm;
                    }
                    uint32_t ia = nlo + l, ib = nmid + (d - l);
#pragma unroll
                    for (int i = 0; i < IT; ++i) {
                        const uint32_t x = x0 + i;
                        if (x >= s0 && x < nhi) {
                            const bool take_a = (ib >= nhi) || (ia < nmid && sk[lpad(ia)] <= sk[lpad(ib)]);
                            np[i] = (uint16_t)(take_a ? ia++ : ib++);
                        }
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                if (x0 + i < n) {
                    kr[i] = sk[lpad(np[i])];
                    if (HP) pr[i] = sp[lpad(np[i])];
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                if (x0 + i < n) {
                    sk[lpad(x0 + i)] = kr[i];
                    if (HP) sp[lpad(x0 + i)] = pr[i];
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const uint32_t x = tid + i * NT;
            if (x < n) {
                const U key = sk[lpad(x)];
                dst[lo + x] = K::unord(key);
                if (HP) pdst[lo + x] = sp[lpad(x)];
                put_sample(a.samp, lo + x, key);
            }
        }
    }
}

// Direct load of one dword per lane from global memory into LDS (gfx950
// global_load_lds): lane l of the wave writes its dword to lds[l], so lds
// must be the same for the whole wave.  No VGPR holds the data, and the
// load stays in flight while the wave goes on (the next barrier after an
// s_waitcnt vmcnt(0) publishes it).
__device__ __forceinline__ void lds_dma_dword(const void* src, void* lds) {
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                     (__attribute__((address_space(3))) void*)lds, 4, 0, 0);
}
__device__ __forceinline__ void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// A block barrier for LDS work only: this wave's LDS reads and writes are
// done, then all waves meet.  Unlike __syncthreads it is no release fence,
// so it does not wait for direct loads into LDS still in flight; compiler
// fences keep memory accesses on their side of it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt at their maxima (no wait)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

constexpr int kStageMeta = 64;  // per staged subtree: starts, then Lf, Rt and P of the merges
// Staging of one fused subtree of kUnitFew (4-byte keys), all by direct
// loads that every wave issues for its own part:
//   - with data: its keys and payload, unpadded, and the tree data of its
//     leaves and merges (raw global values) in meta;
//   - the dword of unit_par that holds its destination byte (nxt[64]), and,
//     when there is one, the record of the subtree this block takes after
//     it (nxt[0..3]), so that no load waits at the top of the next round.
template <bool HP>
__device__ __forceinline__ void fused_stage(const MoveArgs& a, const UnitRec ur, bool data, uint32_t u,
                                            bool has_next, uint32_t u_next, uint32_t* stk, uint32_t* stp,
                                            uint32_t* meta, uint32_t* nxt) {
    constexpr int NT = kFusedNT, IT = kFuse / kFusedNT;
    const uint32_t lo = ur.lo, n = ur.hi - ur.lo, ua = ur.ua, nl = ur.ub - ur.ua;
    const uint32_t tid = threadIdx.x, w0 = tid & ~63u, lane = tid & 63u;
    if (data) {
        const uint32_t* ks = (const uint32_t*)a.keys[0] + lo;
        const uint32_t* ps = a.pay[0] + lo;
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            if (i * NT + w0 < n) {  // whole waves past the end load nothing
                const uint32_t x = min(i * NT + tid, n - 1);
                lds_dma_dword(ks + x, stk + i * NT + w0);
                if (HP) lds_dma_dword(ps + x, stp + i * NT + w0);
            }
        }
        if (w0 == 0) {
            lds_dma_dword(a.starts + ua + min(lane, nl), meta);
            if (nl > 1) {
                const uint32_t j = ua + 1 + min(lane, nl - 2);
                lds_dma_dword(a.Lf + j, meta + kStageMeta);
                lds_dma_dword(a.Rt + j, meta + 2 * kStageMeta);
                // the aligned dword that holds byte j of P (P sits in a
                // 256-byte aligned allocation that is not the workspace's last)
                lds_dma_dword(a.P + (j & ~3u), meta + 3 * kStageMeta);
            }
        }
    }
    if (w0 == 64) {
        // unit_par and unit_rec sit in 256-byte aligned allocations (not the
        // workspace's last), unit records are 16 bytes
        lds_dma_dword(a.unit_par + (u & ~3u), nxt + 64);
        if (has_next && lane == 0) {
            // one 16-byte record by one lane (opaque to the compiler, so that
            // no loop-invariant part of its address stays in VGPRs)
            const UnitRec* rp = a.unit_rec + u_next;
            asm volatile("" : "+s"(rp));
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)rp,
                                             (__attribute__((address_space(3))) void*)nxt, 16, 0, 0);
        }
    }
}

// fused_kernel for 4-byte keys with the next subtree's data loaded while the
// current one is merged: direct loads fill an unpadded staging copy in LDS,
// leaf formation reads it and writes the padded working copy, and the loads
// of the next subtree are issued right after.  The leaves and merges are the
// same as fused_kernel's.  LDS: about 69 KiB with a payload, two blocks per CU.
template <int KT, bool HP>
__global__ __launch_bounds__(kFusedNT) __attribute__((amdgpu_waves_per_eu(8))) void fused_staged_kernel(MoveArgs a) {
    constexpr int NT = kFusedNT, IT = kFuse / kFusedNT;
    using K = Key<KT>;
    using U = typename K::ukey;
    using raw = typename K::raw;
    static_assert(sizeof(raw) == 4 && IT == 4, "staging holds 4-byte keys, one 16-byte vector per thread");
    constexpr uint32_t KL = kFuseRadixMinLeaves;
    constexpr uint32_t KN = KL - 2;
    constexpr uint32_t PADDED = kFuse + kFuse / 8;
    __shared__ U sk[PADDED];
    __shared__ uint32_t sp[HP ? PADDED : 1];
    __shared__ __align__(16) uint32_t stk[kFuse];
    __shared__ __align__(16) uint32_t stp[HP ? kFuse : 4];
    __shared__ uint32_t meta[4 * kStageMeta];
    __shared__ uint32_t nxt[128];
    __shared__ uint4 mrg[KN];  // per merge: nlo, nmid, nhi (subtree positions), power
    const uint32_t nunits = a.cnt->nunit[kUnitFew], base = a.unit_base[kUnitFew];
    const uint32_t tid = threadIdx.x, G = gridDim.x;
    auto uni = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane(v); };
    // Units of this list hold 1 to kFuseRadixMinLeaves - 1 leaves and at most
    // kFuse elements (classify_kernel); one that does not is skipped whole.
    auto valid = [](const UnitRec& r) {
        const uint32_t nl = r.ub - r.ua, n = r.hi - r.lo;
        return nl >= 1 && nl < KL && n >= 1 && n <= (uint32_t)kFuse;
    };
    uint32_t v = blockIdx.x;
    UnitRec ur{0, 0, 0, 0};
    if (v < nunits) {
        const UnitRec r = a.unit_rec[base + v];
        ur = UnitRec{uni(r.ua), uni(r.ub), uni(r.lo), uni(r.hi)};
        fused_stage<HP>(a, ur, valid(ur), base + v, v + G < nunits, base + v + G, stk, stp, meta, nxt);
    }
    for (; v < nunits; v += G) {
        const uint32_t vn = v + G;
        const bool ok = valid(ur);
        const uint32_t ua = ur.ua, nl = ur.ub - ur.ua, lo = ur.lo, n = ur.hi - ur.lo;
        const uint32_t nn = nl - 1;
        wait_vmem();
        __syncthreads();  // staged data in LDS; the previous subtree's last reads are done
        const uint32_t par = (uni(nxt[64]) >> (8 * ((base + v) & 3))) & 0xFFu;
        const UnitRec nr = vn < nunits ? UnitRec{uni(nxt[0]), uni(nxt[1]), uni(nxt[2]), uni(nxt[3])}
                                       : UnitRec{0, 0, 0, 0};
        unsigned long long pm = 0;
        const uint32_t x0 = tid * IT;
        U kr[IT];
        uint32_t pr[IT];
        uint16_t np[IT];
        if (ok) {
            // Leaf formation (R1): staging -> padded working copy, each leaf
            // stably sorted on the way.
            const uint4 kv = *reinterpret_cast<const uint4*>(stk + x0);
            const uint32_t kw[IT] = {kv.x, kv.y, kv.z, kv.w};
            auto st = [&](uint32_t l) { return meta[l] - lo; };
            auto okey = [&](uint32_t y) { return K::ord(__builtin_bit_cast(raw, stk[y])); };
            // A leaf longer than kMaxMinRun is a natural run: kept, or
            // reversed if strictly descending.  A shorter one is sorted by
            // ranks: each of this thread's elements in such leaves counts the
            // leaf's elements ordered before it, in one pass over the union
            // of those leaves (four independent LDS reads a step).
            U key[IT];
            uint32_t dpos[IT], sb[IT];  // sb: short leaf bounds, ls | le << 16 (none: 0)
            uint32_t ys = kFuse, ye = 0;
            uint32_t l = 0;
            while (l + 1 < nl && st(l + 1) <= x0) ++l;
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const uint32_t x = x0 + i;
                key[i] = K::ord(__builtin_bit_cast(raw, kw[i]));
                dpos[i] = x;
                sb[i] = 0;
                if (x < n) {
                    while (st(l + 1) <= x) ++l;
                    const uint32_t ls = st(l), le = st(l + 1);
                    if (le - ls <= (uint32_t)kMaxMinRun) {
                        sb[i] = ls | (le << 16);
                        dpos[i] = ls;
                        ys = min(ys, ls);
                        ye = max(ye, le);
                    } else {
                        const bool desc = okey(ls + 1) < okey(ls);
                        dpos[i] = desc ? (ls + le - 1 - x) : x;
                    }
                }
            }
#pragma unroll 1
            for (uint32_t y = ys; y < ye; y += 4) {
                U o[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) o[k] = okey(min(y + k, (uint32_t)kFuse - 1));
#pragma unroll
                for (int i = 0; i < IT; ++i) {
                    const uint32_t ls = sb[i] & 0xFFFFu, le = sb[i] >> 16;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint32_t yk = y + k;
                        if (yk >= ls && yk < le)
                            dpos[i] += (o[k] < key[i]) || (o[k] == key[i] && yk < x0 + i);
                    }
                }
            }
            uint4 pv = make_uint4(0, 0, 0, 0);
            if (HP) pv = *reinterpret_cast<const uint4*>(stp + x0);
            const uint32_t pw[IT] = {pv.x, pv.y, pv.z, pv.w};
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                if (x0 + i < n) {
                    sk[lpad(dpos[i])] = key[i];
                    if (HP) sp[lpad(dpos[i])] = pw[i];
                }
            }
            // Each merge's range [nlo, nmid) + [nmid, nhi) and power, once.
            if (tid < nn) {
                const uint32_t f = meta[kStageMeta + tid] - ua, e = meta[2 * kStageMeta + tid] - ua;
                mrg[tid] = make_uint4(meta[f] - lo, meta[tid + 1] - lo, meta[e] - lo,
                                      (meta[3 * kStageMeta + tid] >> (8 * ((ua + 1 + tid) & 3))) & 0xFFu);
            }
        }
        __syncthreads();  // staging is free: stage the next subtree
        if (vn < nunits)
            fused_stage<HP>(a, nr, valid(nr), base + vn, vn + G < nunits, base + vn + G, stk, stp, meta, nxt);
        if (ok) {
            // powers of the merges, block-uniform (kNone past the last)
            uint32_t mp[KN];
#pragma unroll
            for (uint32_t m = 0; m < KN; ++m) {
                mp[m] = m < nn ? uni(mrg[m].w) : 64u;
                if (m < nn) pm |= 1ull << mp[m];
            }
            raw* dst = (raw*)pick3u(a.keys, par);
            uint32_t* pdst = pick3u(a.pay, par);
            // Merges, deepest power first.
            while (pm) {
                const uint32_t p = 63 - __clzll(pm);
                pm &= ~(1ull << p);
                uint32_t todo = 0;
#pragma unroll
                for (uint32_t m = 0; m < KN; ++m) todo |= (mp[m] == p ? 1u : 0u) << m;
#pragma unroll
                for (int i = 0; i < IT; ++i) np[i] = (uint16_t)(x0 + i);  // copied unless merged
#pragma unroll 1
                while (todo) {
                    const uint32_t m = __builtin_ctz(todo);
                    todo &= todo - 1;
                    const uint4 r = mrg[m];
                    const uint32_t nlo = uni(r.x), nmid = uni(r.y), nhi = uni(r.z);
                    if (nlo < x0 + IT && x0 < nhi) {
                        const uint32_t s0 = max(x0, nlo);
                        const uint32_t d = s0 - nlo, la = nmid - nlo, lb = nhi - nmid;
                        // merge-path co-rank of diagonal d (ties to the left
                        // run): the largest c in [lo_c, hi_c] whose element
                        // a[c - 1] is not above b[d - c], by a fixed number of
                        // halving steps (the same for the whole block)
                        uint32_t c = d > lb ? d - lb : 0;
                        const uint32_t hi_c = min(d, la);
                        const int steps = 32 - __clz((int)min(la, lb));
#pragma unroll 1
                        for (int k = steps - 1; k >= 0; --k) {
                            // (qc >= 1 keeps both reads inside the two runs
                            // when hi_c is 0; the step is then not taken)
                            const uint32_t q = c + (1u << k), qc = max(1u, min(q, hi_c));
                            if (q <= hi_c && sk[lpad(nlo + qc - 1)] <= sk[lpad(nmid + d - qc)]) c = q;
                        }
                        // merge steps: the two run heads in registers, one
                        // LDS read per step
                        uint32_t ia = nlo + c, ib = nmid + (d - c);
                        U ka = sk[lpad(ia)], kb = sk[lpad(min(ib, (uint32_t)kFuse - 1))];
#pragma unroll
                        for (int i = 0; i < IT; ++i) {
                            const uint32_t x = x0 + i;
                            if (x >= s0 && x < nhi) {
                                const bool ta = (ib >= nhi) || (ia < nmid && ka <= kb);
                                np[i] = (uint16_t)(ta ? ia : ib);
                                ia += ta ? 1u : 0u;
                                ib += ta ? 0u : 1u;
                                if (i + 1 < IT) {
                                    const U v = sk[lpad(min(ta ? ia : ib, (uint32_t)kFuse - 1))];
                                    ka = ta ? v : ka;
                                    kb = ta ? kb : v;
                                }
                            }
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < IT; ++i) {
                    if (x0 + i < n) {
                        kr[i] = sk[lpad(np[i])];
                        if (HP) pr[i] = sp[lpad(np[i])];
                    }
                }
                lds_barrier();
#pragma unroll
                for (int i = 0; i < IT; ++i) {
                    if (x0 + i < n) {
                        sk[lpad(x0 + i)] = kr[i];
                        if (HP) sp[lpad(x0 + i)] = pr[i];
                    }
                }
                lds_barrier();
            }
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const uint32_t x = tid + i * NT;
                if (x < n) {
                    const U key = sk[lpad(x)];
                    dst[lo + x] = K::unord(key);
                    if (HP) pdst[lo + x] = sp[lpad(x)];
                    put_sample(a.samp, lo + x, key);
                }
            }
        }
        ur = nr;
    }
}

// ------------------------------------------------------------ merge passes

template <int KT, int TILE>
struct MergeShared {
    using U = typename Key<KT>::ukey;
    U sk[TILE];
    uint32_t sp[TILE];
};
// LDS of the 4-byte-key merge passes, padded (lpad).
// Sample entries of a merged range [out0, out0 + nt) whose order keys are in
// padded LDS: one thread per sampled position (nt / kSampleSpacing + 1 must
// not exceed the block).
template <class U>
__device__ __forceinline__ void put_samples_lds(uint32_t* samp, const U* sk, uint32_t out0, uint32_t nt) {
    if constexpr (sizeof(U) == 4) {
        if (!samp) return;
        const uint32_t q = ((out0 + kSampleSpacing - 1) / kSampleSpacing + threadIdx.x) * kSampleSpacing;
        if (q < out0 + nt) samp[q / kSampleSpacing] = (uint32_t)sk[lpad(q - out0)];
    }
}
template <int KT, int TILE>
struct MergeSharedPad {
    using U = typename Key<KT>::ukey;
    U sk[TILE + TILE / 8];
    uint32_t sp[TILE + TILE / 8];
};

// Merge-path co-rank in padded LDS by a fixed number of halving steps (no
// divergence between lanes): the number of elements of the run
// sk[xa, xa + n1) among the first d outputs of its stable merge with the run
// sk[xb, xb + n2) (the first run first on equal keys), for n1 < 2^STEPS.
template <int STEPS, class U>
__device__ __forceinline__ uint32_t lds_corank(const U* sk, uint32_t xa, uint32_t n1, uint32_t xb, uint32_t n2,
                                               uint32_t d) {
    const uint32_t hi = min(d, n1);
    uint32_t c = d > n2 ? d - n2 : 0;
#pragma unroll
    for (int k = STEPS - 1; k >= 0; --k) {
        const uint32_t q = c + (1u << k);
        if (q <= hi && sk[lpad(xa + q - 1)] <= sk[lpad(xb + d - q)]) c = q;
    }
    return c;
}

// Key-order bounds in a sorted run: the number of run elements whose key is
// below v (lower) or not above v (upper).
template <int KT>
__device__ __forceinline__ uint32_t lower_count(const typename Key<KT>::raw* __restrict__ x, uint32_t n,
                                                typename Key<KT>::ukey v) {
    uint32_t l = 0, h = n;
    while (l < h) {
        const uint32_t m = (l + h) >> 1;
        if (Key<KT>::ord(x[m]) < v) l = m + 1; else h = m;
    }
    return l;
}
template <int KT>
__device__ __forceinline__ uint32_t upper_count(const typename Key<KT>::raw* __restrict__ x, uint32_t n,
                                                typename Key<KT>::ukey v) {
    uint32_t l = 0, h = n;
    while (l < h) {
        const uint32_t m = (l + h) >> 1;
        if (Key<KT>::ord(x[m]) <= v) l = m + 1; else h = m;
    }
    return l;
}
// Co-rank of diagonal d in the stable merge of sorted runs x (first on equal
// keys) and y: the number of x elements among the first d outputs.
template <int KT>
__device__ __forceinline__ uint32_t corank(const typename Key<KT>::raw* __restrict__ x, uint32_t nx,
                                           const typename Key<KT>::raw* __restrict__ y, uint32_t ny, uint32_t d) {
    uint32_t l = d > ny ? d - ny : 0, h = min(d, nx);
    while (l < h) {
        const uint32_t m = (l + h) >> 1;
        if (Key<KT>::ord(x[m]) <= Key<KT>::ord(y[d - 1 - m])) l = m + 1; else h = m;
    }
    return l;
}

// k-ary search by the kSplitGroup lanes of an aligned lane group: the first
// i in [l, h) with pred(i), or h if there is none, for a predicate that is
// false and then true on [l, h).  Every lane of the group calls it with the
// same l and h and gets the same result.  Each round, lane j probes the point
// l + j step, which narrows the range to below step = ceil((h - l) / G): a
// dependent chain of log_G instead of log_2 loads.
template <class Pred>
__device__ __forceinline__ uint32_t group_first(uint32_t l, uint32_t h, Pred pred) {
    constexpr uint32_t G = kSplitGroup;
    static_assert(G >= 2 && G < 64 && (G & (G - 1)) == 0, "lane groups split a wave");
    const uint32_t lane = __lane_id();
    const uint32_t gl = lane & (G - 1), g0 = lane & ~(G - 1);
    while (l < h) {
        const uint32_t step = (h - l + G - 1) / G;
        const uint32_t q = l + gl * step;
        const bool t = q >= h || pred(q);
        const uint64_t m = ((uint64_t)__ballot(t) >> g0) & ((1ull << G) - 1ull);
        if (m == 0) {
            l += (G - 1) * step + 1;  // every probe is below h and false
        } else {
            const uint32_t f = (uint32_t)__builtin_ctzll(m);
            if (f == 0) {
                h = l;
            } else {
                const uint32_t nl = l + (f - 1) * step + 1;
                h = min(l + f * step, h);
                l = nl;
            }
        }
    }
    return l;
}

// Split passes: where every merge tile of pass p starts.  Each boundary
// writes the start of its tile and the end of the previous one (the last
// boundary of a node also ends its tile at the node's end), so a merge tile
// is read as one record.
__device__ __forceinline__ void write_split(const MoveArgs& a, const NodeRec& R, uint32_t at, uint32_t idx,
                                            uint32_t last, uint32_t ca, uint32_t cb, uint32_t cc, uint32_t cd) {
    const uint32_t pa = R.lo + ca, pb = R.m1 + cb, pc = R.mid + cc, pd = R.m2 + cd;
    const uint32_t out = R.lo + ca + cb + cc + cd;
    if (at < a.split_cap) {
        SplitRec& r = a.split[at];
        r.s[0] = pa;
        r.s[1] = pb;
        r.s[2] = pc;
        r.s[3] = pd;
        r.out = out;
        r.bufs = R.bufs;
        a.span[at].start = out | (idx == 0 ? kFirstTile : 0u);
        if (idx == last) {
            r.e[0] = R.m1;
            r.e[1] = R.mid;
            r.e[2] = R.m2;
            r.e[3] = R.hi;
            a.span[at].end = R.hi;
        }
    }
    if (idx > 0 && at - 1 < a.split_cap) {
        SplitRec& q = a.split[at - 1];
        q.e[0] = pa;
        q.e[1] = pb;
        q.e[2] = pc;
        q.e[3] = pd;
        a.span[at - 1].end = out;
    }
}

// Searches of the split passes, by the kSplitGroup lanes of a lane group,
// over runs whose sampled positions (divisible by S = kSampleSpacing) keep
// their order keys in a.samp.  A run X occupies positions [xs, xe); its
// samples are smp[j0 .. j1) for the first sampled position j0 S = xs + r.
//
// Co-rank of diagonal d in the stable merge of X = [xs, xe) with the run
// Y = [ys, ye) that follows it (X first on equal keys): the sampled elements
// of X and Y keep their relative order in the merge, so the sampled
// elements among its first d outputs are the first D of the merge of the two
// samples, where D is one of the two integers next to (d - rX - rY) / S.  The
// samples' co-ranks at those two diagonals bound the number of sampled X
// elements before the split, and with it the co-rank, to fewer than 2 S
// positions; a search there ends it.
template <int KT>
__device__ __forceinline__ uint32_t group_corank(const uint32_t* __restrict__ smp, const typename Key<KT>::raw* X,
                                                 uint32_t xs, uint32_t xe, const typename Key<KT>::raw* Y,
                                                 uint32_t ys, uint32_t ye, uint32_t d) {
    using K = Key<KT>;
    constexpr uint32_t S = kSampleSpacing;
    const uint32_t nx = xe - xs, ny = ye - ys;
    const uint32_t ja = (xs + S - 1) / S, jc = (ys + S - 1) / S, je = (ye + S - 1) / S;
    const uint32_t KA = jc - ja, KC = je - jc;  // X's samples end where Y's begin (ys = xe)
    const uint32_t rA = ja * S - xs, rC = jc * S - ys;
    const int64_t E = (int64_t)d - rA - rC;  // > -2 S
    const int64_t D0 = E >= 0 ? (E + S - 1) / S : -((-E) / S);
    const uint32_t Dc = (uint32_t)min<int64_t>(max<int64_t>(D0, 0), (int64_t)(KA + KC));
    const uint32_t k0 = group_first(Dc > KC ? Dc - KC : 0u, min(Dc, KA),
                                    [&](uint32_t i) { return smp[ja + i] > smp[jc + Dc - 1 - i]; });
    uint32_t k1;  // the samples' co-rank at D0 + 1 (clamped)
    if (D0 < 0) {
        k1 = 0;
    } else if (D0 >= (int64_t)(KA + KC)) {
        k1 = KA;
    } else {
        const uint32_t m0 = Dc - k0;
        const bool take_x = k0 < KA && (m0 >= KC || smp[ja + k0] <= smp[jc + m0]);
        k1 = k0 + (take_x ? 1u : 0u);
    }
    // k0 <= (sampled X elements before the split) <= k1
    uint32_t l = k0 == 0 ? 0u : rA + (k0 - 1) * S + 1;
    uint32_t h = k1 >= KA ? nx : rA + k1 * S;
    l = max(l, d > ny ? d - ny : 0u);
    h = min(h, min(d, nx));
    // The sampled Y elements before the split are D - (sampled X elements).
    // If the (D0 + 1)-th merged sample is an X element (k1 > k0) that is
    // D0 - k0 whichever of D0, D0 + 1 D is; otherwise D0 - k0 or one more.
    // Y's sample positions rC + j S bound the split from the other side, so
    // the window searched is at most S wide when k1 > k0.
    if (D0 >= 0 && D0 < (int64_t)(KA + KC)) {
        const int64_t kyl = D0 - (int64_t)k0, kyh = k1 > k0 ? kyl : kyl + 1;
        if (kyh < (int64_t)KC) {
            // Y's sample kyh is not before the split: d - c <= rC + kyh S
            const int64_t lo_c = (int64_t)d - rC - kyh * (int64_t)S;
            if (lo_c > (int64_t)l) l = (uint32_t)lo_c;
        }
        if (kyl >= 1) {
            // Y's sample kyl - 1 is before the split: d - c > rC + (kyl - 1) S
            const int64_t hi_c = (int64_t)d - rC - (kyl - 1) * (int64_t)S - 1;
            if (hi_c < (int64_t)h) h = (uint32_t)max<int64_t>(hi_c, (int64_t)l);
        }
    }
    return group_first(l, h, [&](uint32_t i) { return K::ord(X[i]) > K::ord(Y[d - 1 - i]); });
}

// Elements of the run X = [xs, xe) whose order key is below v (or not above
// v, with le): the count of sampled elements that qualify, k, places it
// after the k-th sample and not after the (k+1)-th, a window of at most S.
template <int KT>
__device__ __forceinline__ uint32_t group_count(const uint32_t* __restrict__ smp, const typename Key<KT>::raw* X,
                                                uint32_t xs, uint32_t xe, uint32_t v, bool le) {
    using K = Key<KT>;
    constexpr uint32_t S = kSampleSpacing;
    const uint32_t nx = xe - xs;
    const uint32_t j0 = (xs + S - 1) / S, K1 = (xe + S - 1) / S - j0, r = j0 * S - xs;
    auto fails = [&](uint32_t u) { return le ? u > v : u >= v; };
    const uint32_t k = group_first(0, K1, [&](uint32_t i) { return fails(smp[j0 + i]); });
    const uint32_t l = k == 0 ? 0u : r + (k - 1) * S + 1;
    const uint32_t h = k >= K1 ? nx : r + k * S;
    return group_first(l, h, [&](uint32_t i) { return fails((uint32_t)K::ord(X[i])); });
}

// Nodes with two inputs A = [lo, mid) and C = [mid, hi) (the pass's tiles
// [0, ptq)), one group of kSplitGroup lanes per tile: the tile starting at
// output d takes the co-rank of diagonal d (A elements among the first d
// outputs, A first on equal keys).
template <int KT>
__global__ __launch_bounds__(kThreads) void split_kernel(MoveArgs a, uint32_t p) {
    using K = Key<KT>;
    using raw = typename K::raw;
    static_assert(sizeof(typename K::ukey) == 4, "the split pass serves 4-byte keys");
    constexpr uint32_t G = kSplitGroup;
    const uint32_t ntiles = a.cnt->ptq[p];
    const uint32_t nb = a.cnt->pcount[p];
    const uint32_t bbase = a.cnt->pbase[p];
    const uint32_t sb = a.cnt->sbase[p];
    if (nb == 0) return;
    const uint32_t* bt = a.bucket_tile + bbase;
    const uint32_t ngroups = gridDim.x * (kThreads / G);
    for (uint32_t t = (blockIdx.x * kThreads + threadIdx.x) / G; t < ntiles; t += ngroups) {
        const uint32_t k = group_first(0, nb, [&](uint32_t i) { return bt[i] > t; }) - 1;
        const uint32_t node = bbase + k;
        const NodeRec R = a.node_rec[node];
        const uint32_t first = a.bucket_tile[node];
        const uint32_t u = t - first;
        const raw* A = (const raw*)pick3(a.keys, (R.bufs >> 2) & 3u) + R.lo;
        const raw* C = (const raw*)pick3(a.keys, (R.bufs >> 6) & 3u) + R.mid;
        const uint32_t d = u * a.merge_tile;
        const uint32_t ca = group_corank<KT>(a.samp, A, R.lo, R.mid, C, R.mid, R.hi, d);
        if ((threadIdx.x & (G - 1)) == 0)
            write_split(a, R, sb + first + u, u, (R.hi - R.lo - 1) / a.merge_tile, ca, 0, d - ca, 0);
    }
}

// Nodes with an absorbed child (two-level passes; the pass's tiles
// [ptq, ptiles)), one lane group per tile.  Such a node merges the left child
// L = A + B with the right child R = C + D, neither written out.  Its tile
// starts are the node's start and "splitters" every g = kQuadSpacing
// positions along L and along R: splitter i of L is its element L[i] (found
// by the co-rank of i in A, B), and it starts where the R elements below its
// key end (L goes first on equal keys); splitter j of R is R[j], preceded by
// the L elements not above its key.  Consecutive starts are at most g apart
// in L and in R, so a tile holds at most 2g outputs (the merge pass packs
// consecutive tiles into groups of up to kQuadTile).  Their order in the
// result has a closed form: R's splitter m g precedes L's element L[i]
// exactly when m g < (R elements before L[i]), and vice versa, so each
// splitter's tile index is its own index plus the number of the other
// child's splitters before it.
template <int KT>
__global__ __launch_bounds__(kThreads) void split_quad_kernel(MoveArgs a, uint32_t p) {
    using K = Key<KT>;
    using raw = typename K::raw;
    using U = typename K::ukey;
    constexpr uint32_t G = kSplitGroup;
    const uint32_t ntiles = a.cnt->ptiles[p];
    const uint32_t nb = a.cnt->pcount[p];
    const uint32_t bbase = a.cnt->pbase[p];
    const uint32_t sb = a.cnt->sbase[p];
    if (nb == 0) return;
    const uint32_t g = kQuadSpacing;
    const uint32_t* bt = a.bucket_tile + bbase;
    const uint32_t ngroups = gridDim.x * (kThreads / G);
    for (uint32_t t = a.cnt->ptq[p] + (blockIdx.x * kThreads + threadIdx.x) / G; t < ntiles; t += ngroups) {
        const uint32_t k = group_first(0, nb, [&](uint32_t i) { return bt[i] > t; }) - 1;
        const uint32_t node = bbase + k;
        const NodeRec R = a.node_rec[node];
        const uint32_t first = a.bucket_tile[node];
        const uint32_t u = t - first;
        const raw* A = (const raw*)pick3(a.keys, (R.bufs >> 2) & 3u) + R.lo;
        const raw* B = (const raw*)pick3(a.keys, (R.bufs >> 4) & 3u) + R.m1;
        const raw* C = (const raw*)pick3(a.keys, (R.bufs >> 6) & 3u) + R.mid;
        const raw* D = (const raw*)pick3(a.keys, (R.bufs >> 8) & 3u) + R.m2;
        const uint32_t na = R.m1 - R.lo, nbb = R.mid - R.m1, nc = R.m2 - R.mid, nd = R.hi - R.m2;
        const uint32_t nl = na + nbb, nr = nc + nd;
        const uint32_t sl = (nl - 1) / g, sr = (nr - 1) / g;  // splitters of L and R
        uint32_t idx = 0, ca = 0, cb = 0, cc = 0, cd = 0;   // elements of A, B, C, D before the boundary
        if (u == 0) {
            idx = 0;
        } else if (u <= sl) {
            const uint32_t i = u * g;
            ca = nbb ? group_corank<KT>(a.samp, A, R.lo, R.m1, B, R.m1, R.mid, i) : i;
            cb = i - ca;
            const bool from_a = cb >= nbb || (ca < na && K::ord(A[ca]) <= K::ord(B[cb]));
            const U v = K::ord(from_a ? A[ca] : B[cb]);
            cc = group_count<KT>(a.samp, C, R.mid, R.m2, v, false);
            cd = nd ? group_count<KT>(a.samp, D, R.m2, R.hi, v, false) : 0u;
            const uint32_t before = cc + cd;
            idx = u + min(sr, before ? (before - 1) / g : 0u);
        } else {
            const uint32_t m = u - sl, j = m * g;
            cc = nd ? group_corank<KT>(a.samp, C, R.mid, R.m2, D, R.m2, R.hi, j) : j;
            cd = j - cc;
            const bool from_c = cd >= nd || (cc < nc && K::ord(C[cc]) <= K::ord(D[cd]));
            const U v = K::ord(from_c ? C[cc] : D[cd]);
            ca = group_count<KT>(a.samp, A, R.lo, R.m1, v, true);
            cb = nbb ? group_count<KT>(a.samp, B, R.m1, R.mid, v, true) : 0u;
            const uint32_t before = ca + cb;
            idx = m + min(sl, before ? (before - 1) / g : 0u);
        }
        if ((threadIdx.x & (G - 1)) == 0) write_split(a, R, sb + first + idx, idx, sl + sr, ca, cb, cc, cd);
    }
}

// One merge-path tile of merge_pass_cr_kernel: tile t of the pass belongs
// to bucket entry `node`; i0 is the co-rank at its start and i1n the one at
// the next tile's start (used when that tile is in the same node).  NT
// threads x IT outputs.
template <int KT, bool HP, int NT, int IT>
__device__ __forceinline__ void merge_tile(const MoveArgs& a, MergeShared<KT, NT * IT>& sm, uint32_t node,
                                           uint32_t t, uint32_t i0, uint32_t i1n) {
    constexpr int TILE = NT * IT;
    using K = Key<KT>;
    using U = typename K::ukey;
    using raw = typename K::raw;
    const int tid = threadIdx.x;
    const NodeRec R = a.node_rec[node];
    const uint32_t tt = t - a.bucket_tile[node];
    const uint32_t lo = R.lo, mid = R.mid, hi = R.hi;
    const uint32_t bufs = R.bufs;
    const raw* srcA = (const raw*)pick3u(a.keys, (bufs >> 2) & 3u) + lo;
    const raw* srcB = (const raw*)pick3u(a.keys, (bufs >> 6) & 3u) + mid;  // the right input C
    raw* dst = (raw*)pick3u(a.keys, bufs & 3u);
    const uint32_t* psrcA = pick3u(a.pay, (bufs >> 2) & 3u) + lo;
    const uint32_t* psrcB = pick3u(a.pay, (bufs >> 6) & 3u) + mid;
    uint32_t* pdst = pick3u(a.pay, bufs & 3u);
    const uint32_t la = mid - lo, tot = hi - lo;
    const uint32_t k0 = tt * TILE, k1 = min(tot, k0 + TILE);
    const uint32_t i1 = (k1 == tot) ? la : i1n;  // the next tile is in this node
    const uint32_t j0 = k0 - i0, j1 = k1 - i1;
    const uint32_t na = i1 - i0, nbb = j1 - j0, nt = na + nbb;
    U kr[IT];
    uint32_t pr[IT];
    {
        raw kv[IT];
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const uint32_t x = tid + i * NT;
            // two masked loads with scalar bases (not a per-lane
            // pointer select, which costs 64-bit address arithmetic)
            if (x < na) {
                kv[i] = srcA[i0 + x];
                if (HP) pr[i] = psrcA[i0 + x];
            } else if (x < nt) {
                kv[i] = srcB[j0 + x - na];
                if (HP) pr[i] = psrcB[j0 + x - na];
            }
        }
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const uint32_t x = tid + i * NT;
            if (x < nt) {
                sm.sk[x] = K::ord(kv[i]);
                if (HP) sm.sp[x] = pr[i];
            }
        }
    }
    __syncthreads();
    const uint32_t dx = tid * IT;
    if (dx < nt) {
        uint32_t l = dx > nbb ? dx - nbb : 0, h = min(dx, na);
        while (l < h) {
            const uint32_t m = (l + h) >> 1;
            if (sm.sk[m] <= sm.sk[na + dx - 1 - m]) l = m + 1; else h = m;
        }
        uint32_t ia = l, ib = na + (dx - l);
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            if (dx + i < nt) {
                const bool take_a = (ib >= nt) || (ia < na && sm.sk[ia] <= sm.sk[ib]);
                const uint32_t s = take_a ? ia++ : ib++;
                kr[i] = sm.sk[s];
                if (HP) pr[i] = sm.sp[s];
            }
        }
    }
    __syncthreads();
    if (dx < nt) {
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            if (dx + i < nt) {
                sm.sk[dx + i] = kr[i];
                if (HP) sm.sp[dx + i] = pr[i];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const uint32_t x = tid + i * NT;
        if (x < nt) {
            kr[i] = sm.sk[x];
            if (HP) pr[i] = sm.sp[x];
        }
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const uint32_t x = tid + i * NT;
        if (x < nt) {
            dst[lo + k0 + x] = K::unord(kr[i]);
            if (HP) pdst[lo + k0 + x] = pr[i];
        }
    }
    __syncthreads();
}

// Merge pass for 8-byte keys: a workgroup owns a contiguous run of tiles
// and finds their co-ranks itself (no split pass).  NT threads x IT outputs
// per tile.  4-byte keys keep merge_pass_kernel below with the split pass's
// records: there the grid-stride tile order measured faster, and its tile
// body is kept inline as it was (the shared merge_tile body compiled 3%
// slower for them).
template <int KT, bool HP, int NT, int IT>
__global__ __launch_bounds__(NT) void merge_pass_cr_kernel(MoveArgs a, uint32_t p) {
    constexpr int TILE = NT * IT;
    using K = Key<KT>;
    using raw = typename K::raw;
    __shared__ MergeShared<KT, TILE> sm;
    const int tid = threadIdx.x;
    __shared__ uint32_t cr[NT + 1];   // co-rank at the start of each tile of the step (and of the next tile)
    __shared__ uint32_t crn[NT + 1];  // its node (bucket entry)
    const uint32_t ntiles = a.cnt->ptiles[p];
    const uint32_t nb = a.cnt->pcount[p];
    const uint32_t bbase = a.cnt->pbase[p];
    if (nb == 0 || ntiles == 0) return;
    // A workgroup owns a contiguous run of tiles.  It finds the co-ranks
    // of their starts itself, one lane per tile, up to NT tiles per step:
    // the searches of workgroups that start later overlap the merging of
    // others.
    const uint32_t chunk = (ntiles + gridDim.x - 1) / gridDim.x;
    const uint32_t tb = min(ntiles, blockIdx.x * chunk), te = min(ntiles, tb + chunk);
    for (uint32_t s0 = tb; s0 < te; s0 += NT) {
        const uint32_t s1 = min(te, s0 + NT);
        // Co-rank of diagonal d in the stable merge of A = [lo, mid) and
        // B = [mid, hi): the number of A elements among the first d
        // outputs, A going first on equal keys, by binary search.  Entry
        // s1 - s0 is the next tile's start, the end of tile s1 - 1.
        for (uint32_t j = tid; j <= s1 - s0; j += NT) {
            const uint32_t t = s0 + j;
            if (t >= ntiles) continue;
            const uint32_t k = upper_bound_u32(a.bucket_tile + bbase, nb, t) - 1;
            const NodeRec Rk = a.node_rec[bbase + k];
            const raw* A = (const raw*)pick3(a.keys, (Rk.bufs >> 2) & 3u) + Rk.lo;
            const raw* B = (const raw*)pick3(a.keys, (Rk.bufs >> 6) & 3u) + Rk.mid;  // the right input C
            const uint32_t la = Rk.mid - Rk.lo, lb = Rk.hi - Rk.mid;
            const uint32_t d = (t - a.bucket_tile[bbase + k]) * TILE;
            uint32_t l = d > lb ? d - lb : 0, h = min(d, la);
            while (l < h) {
                const uint32_t m = (l + h) >> 1;
                if (K::ord(A[m]) <= K::ord(B[d - 1 - m])) l = m + 1; else h = m;
            }
            cr[j] = l;
            crn[j] = bbase + k;
        }
        __syncthreads();
        for (uint32_t t = s0; t < s1; ++t)
            merge_tile<KT, HP, NT, IT>(a, sm, crn[t - s0], t, cr[t - s0], cr[t - s0 + 1]);
    }
}

// Merges of nodes with an absorbed child (the tail part of pass p's tiles),
// NT threads x IT outputs per group of tiles.  A group reads its part of
// each input run (A, B, C, D; B or D is empty when that child is an input)
// into LDS, merges A with B and C with D (the absorbed children's parts),
// then the two results, and writes its part of the node.  Each merge step
// keeps both run heads in registers and reads only the one that advanced;
// six waves per SIMD leave room for that without spills.
template <int KT, bool HP, int NT, int IT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(6))) void merge_quad_kernel(MoveArgs a, uint32_t p) {
    constexpr int TILE = NT * IT;
    using K = Key<KT>;
    using U = typename K::ukey;
    using raw = typename K::raw;
    __shared__ MergeSharedPad<KT, TILE> sm;
    const uint32_t sb = a.cnt->sbase[p];
    // never read past the split records (the tile count is bounded by the
    // merge cost, so this only guards against inconsistent lists)
    const uint32_t ntiles = min(a.cnt->ptiles[p], a.split_cap > sb ? a.split_cap - sb : 0u);
    const uint32_t t0 = min(a.cnt->ptq[p], ntiles);
    if (t0 >= ntiles) return;
    const int tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    // Every workgroup takes a contiguous chunk of these tiles and packs
    // consecutive tiles of one node into groups of at most TILE outputs
    // (their tiles hold at most 2 kQuadSpacing <= TILE).  Every wave finds
    // the same group from the tile spans, so no barrier is needed to share
    // it.
    static_assert(2 * kQuadSpacing <= (uint32_t)TILE, "a tile of a node with absorbed children must fit");
    const uint32_t chunk = (ntiles - t0 + gridDim.x - 1) / gridDim.x;
    if (t0 + blockIdx.x * chunk >= ntiles) return;
    const uint32_t tb = t0 + blockIdx.x * chunk, te = min(ntiles, tb + chunk);
    auto uni = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane(v); };
    // tiles in the group starting at t (at least one)
    auto group_len = [&](uint32_t t) -> uint32_t {
        const uint32_t q = t + lane;
        const uint32_t base = uni(a.span[sb + t].start) & ~kFirstTile;
        bool ok = false;
        if (q < te) {
            const TileSpan sq = a.span[sb + q];
            ok = (lane == 0 || !(sq.start & kFirstTile)) && sq.end >= base && sq.end - base <= (uint32_t)TILE;
        }
        const uint64_t bad = __ballot(!ok);
        const uint32_t g = bad ? (uint32_t)__ffsll((unsigned long long)bad) - 1u : 64u;
        return uni(g > 0 ? g : 1u);
    };
    // The next group's length and records are fetched while the current
    // group is merged (kept in scalar registers: they are block-uniform).
    struct Group {
        uint32_t s[4], e[4], out, bufs;
    };
    auto group_at = [&](uint32_t t, uint32_t len) -> Group {
        const SplitRec& f = a.split[sb + t];
        const SplitRec& l = a.split[sb + t + len - 1];
        return Group{{uni(f.s[0]), uni(f.s[1]), uni(f.s[2]), uni(f.s[3])},
                     {uni(l.e[0]), uni(l.e[1]), uni(l.e[2]), uni(l.e[3])},
                     uni(f.out),
                     uni(f.bufs)};
    };
    uint32_t t = tb, glen = group_len(tb);
    Group cur = group_at(t, glen);
    while (t < te) {
        const uint32_t bufs = cur.bufs, out0 = cur.out;
        const uint32_t sa = cur.s[0], sbp = cur.s[1], sc = cur.s[2], sd = cur.s[3];
        const uint32_t ea = cur.e[0], eb = cur.e[1], ec = cur.e[2], ed = cur.e[3];
        t += glen;
        if (t < te) {
            glen = group_len(t);
            cur = group_at(t, glen);
        }
        // Consistent records have s <= e in every run, at most TILE outputs
        // and positions below n; the checks only keep inconsistent lists
        // inside the arrays and the tile.
        const uint32_t na = ea > sa ? ea - sa : 0u, nbp = eb > sbp ? eb - sbp : 0u;
        const uint32_t nc = ec > sc ? ec - sc : 0u, nd = ed > sd ? ed - sd : 0u;
        const uint32_t nl = na + nbp, ncl = nl + nc, nt = ncl + nd;
        if (nt > (uint32_t)TILE || max(max(ea, eb), max(ec, ed)) > a.n || out0 + nt > a.n) continue;
        const raw* srcA = (const raw*)pick3u(a.keys, (bufs >> 2) & 3u) + sa;
        const raw* srcB = (const raw*)pick3u(a.keys, (bufs >> 4) & 3u) + sbp;
        const raw* srcC = (const raw*)pick3u(a.keys, (bufs >> 6) & 3u) + sc;
        const raw* srcD = (const raw*)pick3u(a.keys, (bufs >> 8) & 3u) + sd;
        const uint32_t* psrcA = pick3u(a.pay, (bufs >> 2) & 3u) + sa;
        const uint32_t* psrcB = pick3u(a.pay, (bufs >> 4) & 3u) + sbp;
        const uint32_t* psrcC = pick3u(a.pay, (bufs >> 6) & 3u) + sc;
        const uint32_t* psrcD = pick3u(a.pay, (bufs >> 8) & 3u) + sd;
        raw* dst = (raw*)pick3u(a.keys, bufs & 3u) + out0;
        uint32_t* pdst = pick3u(a.pay, bufs & 3u) + out0;
        U kr[IT];
        uint32_t pr[IT];
        {
            raw kv[IT];
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const uint32_t x = tid + i * NT;
                // masked loads with scalar bases (not a per-lane pointer
                // select, which costs 64-bit address arithmetic)
                if (x < na) {
                    kv[i] = srcA[x];
                    if (HP) pr[i] = psrcA[x];
                } else if (x < nl) {
                    kv[i] = srcB[x - na];
                    if (HP) pr[i] = psrcB[x - na];
                } else if (x < ncl) {
                    kv[i] = srcC[x - nl];
                    if (HP) pr[i] = psrcC[x - nl];
                } else if (x < nt) {
                    kv[i] = srcD[x - ncl];
                    if (HP) pr[i] = psrcD[x - ncl];
                }
            }
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const uint32_t x = tid + i * NT;
                if (x < nt) {
                    sm.sk[lpad(x)] = K::ord(kv[i]);
                    if (HP) sm.sp[lpad(x)] = pr[i];
                }
            }
        }
        __syncthreads();
        const uint32_t dx = tid * IT;
        if (nbp | nd) {
            // Absorbed children: merge sk[0, na) with sk[na, nl) (the left
            // child's part) and sk[nl, ncl) with sk[ncl, nt) (the right
            // child's), each stably, first run first on equal keys.
            if (dx < nt) {
                const bool right = dx >= nl;
                const uint32_t base = right ? nl : 0u, n1 = right ? nc : na, n2 = right ? nd : nbp;
                const uint32_t dg = dx - base;
                const uint32_t l = lds_corank<kLog2QuadTile>(sm.sk, base, n1, base + n1, n2, dg);
                uint32_t i1 = base + l, e1 = base + n1, i2 = base + n1 + (dg - l), e2 = base + n1 + n2;
                // the two run heads stay in registers (reads clamped inside
                // the tile); each step reads only the head that advanced
                U k1 = sm.sk[lpad(min(i1, nt - 1))], k2 = sm.sk[lpad(min(i2, nt - 1))];
#pragma unroll
                for (int i = 0; i < IT; ++i) {
                    const uint32_t x = dx + i;
                    if (x < nt) {
                        if (x == nl) {  // this thread's outputs continue into the right child's part
                            i1 = nl;
                            e1 = ncl;
                            i2 = ncl;
                            e2 = nt;
                            k1 = sm.sk[lpad(min(i1, nt - 1))];
                            k2 = sm.sk[lpad(min(i2, nt - 1))];
                        }
                        const bool take1 = (i2 >= e2) | ((i1 < e1) & (k1 <= k2));
                        const uint32_t s = take1 ? i1 : i2;
                        kr[i] = take1 ? k1 : k2;
                        if (HP) pr[i] = sm.sp[lpad(s)];
                        i1 += take1 ? 1u : 0u;
                        i2 += take1 ? 0u : 1u;
                        if (i + 1 < IT) {
                            const U v = sm.sk[lpad(min(take1 ? i1 : i2, nt - 1))];
                            k1 = take1 ? v : k1;
                            k2 = take1 ? k2 : v;
                        }
                    }
                }
            }
            __syncthreads();
            if (dx < nt) {
#pragma unroll
                for (int i = 0; i < IT; ++i) {
                    if (dx + i < nt) {
                        sm.sk[lpad(dx + i)] = kr[i];
                        if (HP) sm.sp[lpad(dx + i)] = pr[i];
                    }
                }
            }
            __syncthreads();
        }
        // The node's merge: sk[0, nl) with sk[nl, nt), left first on equal keys.
        const uint32_t nrp = nt - nl;
        if (dx < nt) {
            const uint32_t l = lds_corank<kLog2QuadTile>(sm.sk, 0, nl, nl, nrp, dx);
            uint32_t ia = l, ib = nl + (dx - l);
            U ka = sm.sk[lpad(min(ia, nt - 1))], kb = sm.sk[lpad(min(ib, nt - 1))];
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                if (dx + i < nt) {
                    const bool take_a = (ib >= nt) | ((ia < nl) & (ka <= kb));
                    const uint32_t s = take_a ? ia : ib;
                    kr[i] = take_a ? ka : kb;
                    if (HP) pr[i] = sm.sp[lpad(s)];
                    ia += take_a ? 1u : 0u;
                    ib += take_a ? 0u : 1u;
                    if (i + 1 < IT) {
                        const U v = sm.sk[lpad(min(take_a ? ia : ib, nt - 1))];
                        ka = take_a ? v : ka;
                        kb = take_a ? kb : v;
                    }
                }
            }
        }
        __syncthreads();
        if (dx < nt) {
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                if (dx + i < nt) {
                    sm.sk[lpad(dx + i)] = kr[i];
                    if (HP) sm.sp[lpad(dx + i)] = pr[i];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const uint32_t x = tid + i * NT;
            if (x < nt) {
                kr[i] = sm.sk[lpad(x)];
                if (HP) pr[i] = sm.sp[lpad(x)];
            }
        }
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const uint32_t x = tid + i * NT;
            if (x < nt) {
                dst[x] = K::unord(kr[i]);
                if (HP) pdst[x] = pr[i];
            }
        }
        put_samples_lds(a.samp, sm.sk, out0, nt);
        __syncthreads();
    }
}

// Merges of nodes whose two children are inputs (the head part of pass p's
// tiles): NT threads x IT outputs per tile (the tile size a.merge_tile),
// tiles handed out grid-stride.
template <int KT, bool HP, int NT, int IT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8))) void merge_pass_kernel(MoveArgs a, uint32_t p) {
    constexpr int TILE = NT * IT;
    using K = Key<KT>;
    using U = typename K::ukey;
    using raw = typename K::raw;
    __shared__ MergeSharedPad<KT, TILE> sm;
    const uint32_t sb = a.cnt->sbase[p];
    // never read past the split records (the tile count is bounded by the
    // merge cost, so this only guards against inconsistent lists)
    const uint32_t ntiles = min(a.cnt->ptq[p], a.split_cap > sb ? a.split_cap - sb : 0u);
    const int tid = threadIdx.x;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        // the record is the same across the block: keep its fields scalar
        auto uni = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane(v); };
        const SplitRec rr = a.split[sb + t];
        const uint32_t bufs = uni(rr.bufs), out0 = uni(rr.out);
        const uint32_t sa = uni(rr.s[0]), sc = uni(rr.s[2]), ea = uni(rr.e[0]), ec = uni(rr.e[2]);
        // consistent records have s <= e, at most TILE outputs and positions
        // below n; the check only keeps inconsistent lists inside the arrays
        const uint32_t na = ea > sa ? ea - sa : 0u, nbb = ec > sc ? ec - sc : 0u, nt = na + nbb;
        if (nt > (uint32_t)TILE || max(ea, ec) > a.n || out0 + nt > a.n) continue;
        const raw* srcA = (const raw*)pick3u(a.keys, (bufs >> 2) & 3u) + sa;
        const raw* srcB = (const raw*)pick3u(a.keys, (bufs >> 6) & 3u) + sc;  // the right input C
        const uint32_t* psrcA = pick3u(a.pay, (bufs >> 2) & 3u) + sa;
        const uint32_t* psrcB = pick3u(a.pay, (bufs >> 6) & 3u) + sc;
        raw* dst = (raw*)pick3u(a.keys, bufs & 3u) + out0;
        uint32_t* pdst = pick3u(a.pay, bufs & 3u) + out0;
        U kr[IT];
        uint32_t pr[IT];
        {
            raw kv[IT];
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const uint32_t x = tid + i * NT;
                // two masked loads with scalar bases (not a per-lane
                // pointer select, which costs 64-bit address arithmetic)
                if (x < na) {
                    kv[i] = srcA[x];
                    if (HP) pr[i] = psrcA[x];
                } else if (x < nt) {
                    kv[i] = srcB[x - na];
                    if (HP) pr[i] = psrcB[x - na];
                }
            }
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const uint32_t x = tid + i * NT;
                if (x < nt) {
                    sm.sk[lpad(x)] = K::ord(kv[i]);
                    if (HP) sm.sp[lpad(x)] = pr[i];
                }
            }
        }
        __syncthreads();
        const uint32_t dx = tid * IT;
        if (dx < nt) {
            uint32_t l = dx > nbb ? dx - nbb : 0, h = min(dx, na);
            while (l < h) {
                const uint32_t m = (l + h) >> 1;
                if (sm.sk[lpad(m)] <= sm.sk[lpad(na + dx - 1 - m)]) l = m + 1; else h = m;
            }
            uint32_t ia = l, ib = na + (dx - l);
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                if (dx + i < nt) {
                    const bool take_a = (ib >= nt) || (ia < na && sm.sk[lpad(ia)] <= sm.sk[lpad(ib)]);
                    const uint32_t s = take_a ? ia++ : ib++;
                    kr[i] = sm.sk[lpad(s)];
                    if (HP) pr[i] = sm.sp[lpad(s)];
                }
            }
        }
        __syncthreads();
        if (dx < nt) {
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                if (dx + i < nt) {
                    sm.sk[lpad(dx + i)] = kr[i];
                    if (HP) sm.sp[lpad(dx + i)] = pr[i];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const uint32_t x = tid + i * NT;
            if (x < nt) {
                kr[i] = sm.sk[lpad(x)];
                if (HP) pr[i] = sm.sp[lpad(x)];
            }
        }
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const uint32_t x = tid + i * NT;
            if (x < nt) {
                dst[x] = K::unord(kr[i]);
                if (HP) pdst[x] = pr[i];
            }
        }
        put_samples_lds(a.samp, sm.sk, out0, nt);
        __syncthreads();
    }
}

// ------------------------------------------------------------- host launch

// Plain launch, or one timed by its own dispatch events when ev0 is set.
template <class F, class... Args>
static void launch(F kernel, uint32_t grid, uint32_t block, uint32_t lds, hipStream_t st, hipEvent_t ev0,
                   hipEvent_t ev1, Args... args) {
    if (ev0) hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), lds, st, ev0, ev1, 0, args...);
    else hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), lds, st, args...);
}

template <int KT, bool HP>
static void launch_stage_t(const MoveArgs& a, int stage, uint32_t p, uint32_t grid, hipStream_t st, hipEvent_t ev0,
                           hipEvent_t ev1) {
    if (stage == 0) launch(big_leaf_kernel<KT, HP>, grid, kThreads, 0, st, ev0, ev1, a);
    else if (stage == 1) {
        if constexpr (sizeof(typename Key<KT>::raw) == 4)
            launch(fused_staged_kernel<KT, HP>, grid, kFusedNT, 0, st, ev0, ev1, a);
        else
            launch(fused_kernel<KT, HP>, grid, kFusedNT, 0, st, ev0, ev1, a);
    }
    else if (stage == 5) launch(unit_copy_kernel<KT, HP>, grid, kCopyThreads, 0, st, ev0, ev1, a);
    else if (stage == 4) {
        const uint32_t kb = sizeof(typename Key<KT>::ukey);
        static bool rattr_set = false;
        if (!rattr_set) {
            (void)hipFuncSetAttribute((const void*)fused_radix_kernel<KT, HP>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            rattr_set = true;
        }
        launch(fused_radix_kernel<KT, HP>, grid, kFuseThreads, radix_lds_bytes(kb, HP), st, ev0, ev1, a);
    }
    else if (stage == 2) {
        constexpr bool wide = sizeof(typename Key<KT>::ukey) == 8;
        if (a.merge_tile == 2048) {
            if constexpr (wide) launch(merge_pass_cr_kernel<KT, HP, 512, 4>, grid, 512, 0, st, ev0, ev1, a, p);
            else launch(merge_pass_kernel<KT, HP, 256, 8>, grid, 256, 0, st, ev0, ev1, a, p);
        } else if (a.merge_tile == 4096) {
            // 8-byte keys: 1024 threads x 4 outputs, 11 % faster than 512 x 8
            // on a 2^28 uint64 Zipf sort; 4-byte keys keep 8 per thread
            if constexpr (wide) launch(merge_pass_cr_kernel<KT, HP, 1024, 4>, grid, 1024, 0, st, ev0, ev1, a, p);
            else launch(merge_pass_kernel<KT, HP, 512, 8>, grid, 512, 0, st, ev0, ev1, a, p);
        }
        else if constexpr (sizeof(typename Key<KT>::ukey) == 4)  // 8192: 64 KiB of LDS, 4-byte keys only
            launch(merge_pass_kernel<KT, HP, 1024, 8>, grid, 1024, 0, st, ev0, ev1, a, p);
    }
    else if (stage == 6) {  // nodes with an absorbed child (two-level passes, 4-byte keys)
        // 512 threads x 8 outputs per group, whatever the merge tile: four
        // workgroups per CU keep memory busy through the two LDS merge
        // phases (1024 x 8 with two per CU: Zipf merges 4.61 -> 4.20 ms)
        if constexpr (sizeof(typename Key<KT>::ukey) == 4)
            launch(merge_quad_kernel<KT, HP, 512, 8>, grid, 512, 0, st, ev0, ev1, a, p);
    }
    else if constexpr (sizeof(typename Key<KT>::ukey) == 4) {
        if (stage == 3) launch(split_kernel<KT>, grid, kThreads, 0, st, ev0, ev1, a, p);
        else launch(split_quad_kernel<KT>, grid, kThreads, 0, st, ev0, ev1, a, p);
    }
}

// stage 0: big leaves; 5: single-run fused units (copied); 1: fused
// subtrees (level by level); 4: fused subtrees with many leaves (radix
// sort); 2: the merge pass of power p; 6: its merges of nodes with an
// absorbed child; 3: the split pass of power p (7: its tiles of nodes with
// an absorbed child).
// ev0 / ev1: optional dispatch events.
hipError_t launch_move_stage(int kt, bool hp, const MoveArgs& a, int stage, uint32_t p, uint32_t grid,
                             hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
#define PS_STAGE(KTV)                                                            \
    if (hp) launch_stage_t<KTV, true>(a, stage, p, grid, st, ev0, ev1);          \
    else launch_stage_t<KTV, false>(a, stage, p, grid, st, ev0, ev1);            \
    break
    switch (kt) {
    case KT_I32: PS_STAGE(KT_I32);
    case KT_U32: PS_STAGE(KT_U32);
    case KT_I64: PS_STAGE(KT_I64);
    case KT_U64: PS_STAGE(KT_U64);
    case KT_F32: PS_STAGE(KT_F32);
    default: return hipErrorInvalidValue;
    }
#undef PS_STAGE
    return hipGetLastError();
}

}  // namespace ps
