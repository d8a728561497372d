// Data movement: forming the leaves and the stable merges of the merge tree.
//
// Buffers: buf 0 is the caller's array, buf 1 the library's scratch array.
// A tree vertex (leaf or node) at depth d keeps its sorted result in
// buf (d & 1); a node therefore reads both children from buf ((d+1) & 1) and
// writes buf (d & 1), and the root (depth 0) ends in the caller's array.
//
//  * big_leaf: a leaf longer than the fused-subtree capacity is a natural run
//    (only shorter leaves are min-run extended); a strictly decreasing one is
//    reversed (Sec. 2 run convention), and it is copied to buf 1 if its depth
//    is odd.
//  * fused: every maximal subtree of at most kFuse elements is loaded once
//    from the caller's array, its leaves are stably sorted in LDS (the
//    reversal / insertion-sort extension of App. B.3-B.4 has the unique stable
//    result), and its internal merges are done level by level inside LDS.
//  * merge_pass: all nodes of one power p that are larger than kFuse, as one
//    flattened space of merge-path tiles.  Nodes of equal power are disjoint
//    and their children have larger powers (Lemma "Path power
//    monotonicity"), so passes p = pmax..1 respect every dependency.
// Every merge is stable: on equal keys the left run goes first (App. B.1).
#include "common.hpp"
#include "block.hpp"
#include "internal.hpp"

namespace ps {

constexpr uint32_t kNoneM = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t upper_bound_u32(const uint32_t* __restrict__ a, uint32_t n, uint32_t v) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t m = (lo + hi) >> 1;
        if (a[m] <= v) lo = m + 1; else hi = m;
    }
    return lo;
}

// ------------------------------------------------------------ big leaves

template <int KT, bool HP>
__global__ __launch_bounds__(kThreads) void big_leaf_kernel(MoveArgs a) {
    using raw = typename Key<KT>::raw;
    const uint32_t ntiles = a.cnt->ptiles[0];
    const uint32_t nleaf = a.cnt->nbigleaf;
    raw* k0 = (raw*)a.keys[0];
    raw* k1 = (raw*)a.keys[1];
    if (nleaf == 0) return;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t k = upper_bound_u32(a.leaf_tile, nleaf, t) - 1;
        const uint32_t i = a.bigleaf[k];
        const uint8_t mode = a.bigleaf_mode[k];
        const uint32_t s = a.starts[i], L = a.starts[i + 1] - s;
        const uint32_t x0 = (t - a.leaf_tile[k]) * kLeafTile;
        if (mode == kLeafRevInPlace) {
            const uint32_t x1 = min(L / 2, x0 + kLeafTile);
            for (uint32_t x = x0 + threadIdx.x; x < x1; x += kThreads) {
                const uint32_t y = L - 1 - x;
                const raw kx = k0[s + x], ky = k0[s + y];
                k0[s + x] = ky;
                k0[s + y] = kx;
                if (HP) {
                    const uint32_t px = a.pay[0][s + x], py = a.pay[0][s + y];
                    a.pay[0][s + x] = py;
                    a.pay[0][s + y] = px;
                }
            }
        } else {
            const uint32_t x1 = min(L, x0 + kLeafTile);
            const bool rev = (mode == kLeafRevCopy);
            for (uint32_t x = x0 + threadIdx.x; x < x1; x += kThreads) {
                const uint32_t y = rev ? (L - 1 - x) : x;
                k1[s + y] = k0[s + x];
                if (HP) a.pay[1][s + y] = a.pay[0][s + x];
            }
        }
    }
}

// ------------------------------------------------------- fused subtrees

template <int KT>
struct FuseShared {
    using U = typename Key<KT>::ukey;
    U sk[kFuse];
    uint32_t sp[kFuse];
    uint16_t lst[kFuse + 1];          // leaf starts (unit-relative), lst[nleaves] = n
    uint16_t nlo[kFuseMaxNodes];      // node ranges [nlo, nhi), split at lst[m+1]
    uint16_t nhi[kFuseMaxNodes];
    uint8_t npw[kFuseMaxNodes];
    uint16_t lvl[kFuseMaxNodes];      // nodes of the current power, in position order
    uint32_t sh[kWaves];
    unsigned long long pmask;
    uint32_t nlvl;
};

template <int KT, bool HP>
__global__ __launch_bounds__(kThreads) void fused_kernel(MoveArgs a) {
    using K = Key<KT>;
    using U = typename K::ukey;
    using raw = typename K::raw;
    __shared__ FuseShared<KT> sm;
    const uint32_t nunits = a.cnt->nunits;
    const int tid = threadIdx.x;
    for (uint32_t u = blockIdx.x; u < nunits; u += gridDim.x) {
        const uint32_t ua = a.unit_a[u], ub = a.unit_b[u];
        const uint32_t lo = a.starts[ua], n = a.starts[ub] - lo;
        const uint32_t nleaves = ub - ua, nnodes = nleaves - 1;
        if (n > (uint32_t)kFuse || nleaves == 0 || nleaves > (uint32_t)kFuseMaxNodes + 1) continue;
        const raw* src = (const raw*)a.keys[0];
        raw* dst = (raw*)a.keys[a.unit_par[u]];
        if (tid == 0) sm.pmask = 0;
        for (uint32_t x = tid; x < n; x += kThreads) {
            sm.sk[x] = K::ord(src[lo + x]);
            if (HP) sm.sp[x] = a.pay[0][lo + x];
        }
        for (uint32_t k = tid; k <= nleaves; k += kThreads) sm.lst[k] = (uint16_t)(a.starts[ua + k] - lo);
        __syncthreads();
        unsigned long long pm = 0;
        for (uint32_t m = tid; m < nnodes; m += kThreads) {
            const uint32_t j = ua + 1 + m;
            const uint32_t p = a.P[j];
            sm.npw[m] = (uint8_t)p;
            sm.nlo[m] = sm.lst[a.Lf[j] - ua];
            sm.nhi[m] = sm.lst[a.Rt[j] - ua];
            pm |= 1ull << p;
        }
        if (pm) atomicOr(&sm.pmask, pm);

        // Leaf formation: each leaf is stably sorted in place.
        U kr[kFuseItems];
        uint32_t pr[kFuseItems];
        uint16_t np[kFuseItems];
        const uint32_t x0 = tid * kFuseItems;
#pragma unroll
        for (int i = 0; i < kFuseItems; ++i) {
            const uint32_t x = x0 + i;
            np[i] = 0;
            if (x < n) {
                // leaf k: lst[k] <= x < lst[k+1]
                uint32_t l = 0, h = nleaves;
                while (l + 1 < h) {
                    const uint32_t m = (l + h) >> 1;
                    if (sm.lst[m] <= x) l = m; else h = m;
                }
                const uint32_t ls = sm.lst[l], le = sm.lst[l + 1];
                const U key = sm.sk[x];
                uint32_t dst_pos;
                if (le - ls <= (uint32_t)kMaxMinRun) {
                    uint32_t rank = 0;
                    for (uint32_t y = ls; y < le; ++y) {
                        const U o = sm.sk[y];
                        rank += (o < key) || (o == key && y < x);
                    }
                    dst_pos = ls + rank;
                } else {
                    // A leaf longer than any min-run extension is a natural run.
                    const bool desc = sm.sk[ls + 1] < sm.sk[ls];
                    dst_pos = desc ? (ls + le - 1 - x) : x;
                }
                kr[i] = key;
                pr[i] = HP ? sm.sp[x] : 0u;
                np[i] = (uint16_t)dst_pos;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kFuseItems; ++i) {
            if (x0 + i < n) {
                sm.sk[np[i]] = kr[i];
                if (HP) sm.sp[np[i]] = pr[i];
            }
        }
        __syncthreads();

        // Internal merges, deepest power first.
        unsigned long long rem = sm.pmask;
        while (rem) {
            const uint32_t p = 63 - __clzll(rem);
            rem &= ~(1ull << p);
            // Nodes of power p in position order.
            constexpr int kNodeItems = kFuseMaxNodes / kThreads;
            uint32_t c = 0;
#pragma unroll
            for (int i = 0; i < kNodeItems; ++i) {
                const uint32_t m = tid * kNodeItems + i;
                c += (m < nnodes && sm.npw[m] == p);
            }
            uint32_t total;
            uint32_t pos = block_excl_sum(c, sm.sh, &total);
#pragma unroll
            for (int i = 0; i < kNodeItems; ++i) {
                const uint32_t m = tid * kNodeItems + i;
                if (m < nnodes && sm.npw[m] == p) sm.lvl[pos++] = (uint16_t)m;
            }
            __syncthreads();
            const uint32_t nl = total;
            // First node whose range ends after x0.
            uint32_t idx;
            {
                uint32_t l = 0, h = nl;
                while (l < h) {
                    const uint32_t m = (l + h) >> 1;
                    if (sm.nhi[sm.lvl[m]] <= x0) l = m + 1; else h = m;
                }
                idx = l;
            }
            bool in_node = false;
            uint32_t ia = 0, ib = 0, ea = 0, eb = 0;
            uint32_t next_lo = kNoneM;
            if (idx < nl) {
                const uint32_t m = sm.lvl[idx];
                const uint32_t nlo = sm.nlo[m], nmid = sm.lst[m + 1], nhi = sm.nhi[m];
                if (nlo <= x0 && x0 < n) {
                    // Merge-path co-rank of diagonal x0 - nlo (ties to the left run).
                    const uint32_t d = x0 - nlo, la = nmid - nlo, lb = nhi - nmid;
                    uint32_t l = d > lb ? d - lb : 0, h = min(d, la);
                    while (l < h) {
                        const uint32_t mm = (l + h) >> 1;
                        if (sm.sk[nlo + mm] <= sm.sk[nmid + d - 1 - mm]) l = mm + 1; else h = mm;
                    }
                    ia = nlo + l;
                    ib = nmid + (d - l);
                    ea = nmid;
                    eb = nhi;
                    in_node = true;
                } else {
                    next_lo = nlo;
                }
            }
#pragma unroll
            for (int i = 0; i < kFuseItems; ++i) {
                const uint32_t x = x0 + i;
                if (x < n) {
                    if (!in_node && x == next_lo) {
                        const uint32_t m = sm.lvl[idx];
                        ia = next_lo;
                        ib = ea = sm.lst[m + 1];
                        eb = sm.nhi[m];
                        in_node = true;
                    }
                    uint32_t srcpos;
                    if (in_node) {
                        const bool take_a = (ib >= eb) || (ia < ea && sm.sk[ia] <= sm.sk[ib]);
                        srcpos = take_a ? ia++ : ib++;
                        if (x + 1 == eb) {
                            in_node = false;
                            ++idx;
                            next_lo = (idx < nl) ? sm.nlo[sm.lvl[idx]] : kNoneM;
                        }
                    } else {
                        srcpos = x;
                    }
                    kr[i] = sm.sk[srcpos];
                    if (HP) pr[i] = sm.sp[srcpos];
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < kFuseItems; ++i) {
                if (x0 + i < n) {
                    sm.sk[x0 + i] = kr[i];
                    if (HP) sm.sp[x0 + i] = pr[i];
                }
            }
            __syncthreads();
        }
        for (uint32_t x = tid; x < n; x += kThreads) {
            dst[lo + x] = K::unord(sm.sk[x]);
            if (HP) a.pay[a.unit_par[u]][lo + x] = sm.sp[x];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ merge passes

template <int KT>
struct MergeShared {
    using U = typename Key<KT>::ukey;
    U sk[kMergeTile];
    uint32_t sp[kMergeTile];
    uint32_t cnt[4];
    uint32_t rng[4];
};

// Co-rank of diagonal d in the stable merge of A[0..la) and B[0..lb): the
// number of A elements among the first d outputs (A goes first on equal
// keys).  Each 128-thread half of the block searches its own diagonal; per
// round its threads probe 128 evenly spaced candidates, so the range shrinks
// 129-fold.  Both halves run the same number of rounds (block barriers).
template <class K>
__device__ uint32_t corank_kary(const typename K::raw* __restrict__ A, const typename K::raw* __restrict__ B,
                                uint32_t la, uint32_t lb, uint32_t d, uint32_t* cnt_sh) {
    const int t = threadIdx.x & 127;
    const int half = threadIdx.x >> 7;
    const int wid_in_half = (threadIdx.x >> 6) & 1;
    uint32_t lo = d > lb ? d - lb : 0, hi = min(d, la);
    while (__syncthreads_or(hi > lo)) {
        const uint32_t span = hi - lo;
        // probe g at m_g = lo + (g+1) span / 129 < hi; "taken" = A[m_g] is
        // among the first d outputs, true for a prefix of the probes
        bool taken = false;
        if (span > 0) {
            const uint32_t m = lo + (uint32_t)(((uint64_t)(t + 1) * span) / 129u);
            taken = K::ord(A[m]) <= K::ord(B[d - 1 - m]);
        }
        const uint64_t bal = __ballot(taken);
        if ((threadIdx.x & 63) == 0) cnt_sh[half * 2 + wid_in_half] = (uint32_t)__popcll(bal);
        __syncthreads();
        const uint32_t c = cnt_sh[half * 2] + cnt_sh[half * 2 + 1];
        __syncthreads();
        if (span > 0) {
            // the answer lies in (m_{c-1}, m_c]
            const uint32_t nlo = (c == 0) ? lo : lo + (uint32_t)(((uint64_t)c * span) / 129u) + 1;
            const uint32_t nhi = (c >= 128) ? hi : lo + (uint32_t)(((uint64_t)(c + 1) * span) / 129u);
            lo = nlo;
            hi = max(nlo, nhi);
        }
    }
    return lo;
}

template <int KT, bool HP>
__global__ __launch_bounds__(kThreads) void merge_pass_kernel(MoveArgs a, uint32_t p) {
    using K = Key<KT>;
    using U = typename K::ukey;
    using raw = typename K::raw;
    __shared__ MergeShared<KT> sm;
    const uint32_t ntiles = a.cnt->ptiles[p];
    const uint32_t nb = a.cnt->pcount[p];
    const uint32_t bbase = a.cnt->pbase[p];
    const int tid = threadIdx.x;
    if (nb == 0) return;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t k = upper_bound_u32(a.bucket_tile + bbase, nb, t) - 1;
        const uint32_t j = a.bucket[bbase + k];
        const uint32_t tt = t - a.bucket_tile[bbase + k];
        const uint32_t lo = a.starts[a.Lf[j]], mid = a.starts[j], hi = a.starts[a.Rt[j]];
        const uint32_t d = a.node_depth[j];
        const raw* src = (const raw*)a.keys[(d + 1) & 1];
        raw* dst = (raw*)a.keys[d & 1];
        const uint32_t* psrc = a.pay[(d + 1) & 1];
        uint32_t* pdst = a.pay[d & 1];
        const uint32_t la = mid - lo, lb = hi - mid, tot = hi - lo;
        const uint32_t k0 = tt * kMergeTile, k1 = min(tot, k0 + kMergeTile);
        const int half = tid >> 7;
        const uint32_t dd = half ? k1 : k0;
        const uint32_t ci = corank_kary<K>(src + lo, src + mid, la, lb, dd, sm.cnt);
        if ((tid & 127) == 0) sm.rng[half] = ci;
        __syncthreads();
        const uint32_t i0 = sm.rng[0], i1 = sm.rng[1];
        const uint32_t j0 = k0 - i0, j1 = k1 - i1;
        const uint32_t na = i1 - i0, nbb = j1 - j0, nt = na + nbb;
        for (uint32_t x = tid; x < nt; x += kThreads) {
            const uint32_t g = (x < na) ? (lo + i0 + x) : (mid + j0 + (x - na));
            sm.sk[x] = K::ord(src[g]);
            if (HP) sm.sp[x] = psrc[g];
        }
        __syncthreads();
        U kr[kMergeItems];
        uint32_t pr[kMergeItems];
        const uint32_t dx = tid * kMergeItems;
        if (dx < nt) {
            uint32_t l = dx > nbb ? dx - nbb : 0, h = min(dx, na);
            while (l < h) {
                const uint32_t m = (l + h) >> 1;
                if (sm.sk[m] <= sm.sk[na + dx - 1 - m]) l = m + 1; else h = m;
            }
            uint32_t ia = l, ib = na + (dx - l);
#pragma unroll
            for (int i = 0; i < kMergeItems; ++i) {
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
            for (int i = 0; i < kMergeItems; ++i) {
                if (dx + i < nt) {
                    sm.sk[dx + i] = kr[i];
                    if (HP) sm.sp[dx + i] = pr[i];
                }
            }
        }
        __syncthreads();
        for (uint32_t x = tid; x < nt; x += kThreads) {
            dst[lo + k0 + x] = K::unord(sm.sk[x]);
            if (HP) pdst[lo + k0 + x] = sm.sp[x];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- host launch

template <int KT, bool HP>
static hipError_t launch_moves_t(const MoveArgs& a, uint32_t pmax, uint32_t grid_leaf, uint32_t grid_fuse,
                                 uint32_t grid_merge, hipStream_t st) {
    hipLaunchKernelGGL((big_leaf_kernel<KT, HP>), dim3(grid_leaf), dim3(kThreads), 0, st, a);
    hipLaunchKernelGGL((fused_kernel<KT, HP>), dim3(grid_fuse), dim3(kThreads), 0, st, a);
    for (uint32_t p = pmax; p >= 1; --p)
        hipLaunchKernelGGL((merge_pass_kernel<KT, HP>), dim3(grid_merge), dim3(kThreads), 0, st, a, p);
    return hipGetLastError();
}

hipError_t launch_moves(int kt, bool hp, const MoveArgs& a, uint32_t pmax, uint32_t grid_leaf, uint32_t grid_fuse,
                        uint32_t grid_merge, hipStream_t st) {
#define PS_MOVES(KTV)                                                                                     \
    return hp ? launch_moves_t<KTV, true>(a, pmax, grid_leaf, grid_fuse, grid_merge, st)                  \
              : launch_moves_t<KTV, false>(a, pmax, grid_leaf, grid_fuse, grid_merge, st)
    switch (kt) {
    case KT_I32: PS_MOVES(KT_I32);
    case KT_U32: PS_MOVES(KT_U32);
    case KT_I64: PS_MOVES(KT_I64);
    case KT_U64: PS_MOVES(KT_U64);
    case KT_F32: PS_MOVES(KT_F32);
    }
#undef PS_MOVES
    return hipErrorInvalidValue;
}

}  // namespace ps
